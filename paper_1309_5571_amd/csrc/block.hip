// Block Davidson-Liu on the device: the b lowest eigenpairs of a superblock
// (the block version of Davidson's method, Sec. "Runtime & Parallelism": one
// corrected residual per unconverged root is added per iteration, so the
// products with H and the orthogonalization act on blocks of vectors).
//
// Per iteration, with the basis V (n x k, orthonormal), W = H V and the
// Rayleigh matrix G = V^T W kept on the device:
//   projection    WT = H T for the new block T (b slots; slots beyond the
//                 block's size are masked off)
//   k_blk_append  V(:, k:k+nnew) = T, W(:, k:k+nnew) = WT
//   k_blk_tn      partial sums of V(:, :k+nnew)^T W(:, k:k+nnew)  (FP64 MFMA)
//   k_blk_eig     the new columns of G; eigen-decomposition of G (cyclic
//                 Jacobi, one workgroup)
//   k_blk_ritz    Ritz vectors X = V Y, residuals R = W Y - X diag(theta),
//                 corrections T = R / (D - sigma) for unconverged roots,
//                 partial sums of ||r_j||^2
//   k_blk_conv    residual norms, convergence; restart when the unconverged
//                 roots' corrections would not fit in kmax
//   k_blk_restart V(:, :kkeep) = V Y(:, :kkeep), same for W (when restarting)
//   k_blk_finish  restart bookkeeping, summary for the host
//   2 x (k_blk_tn S = V^T T, k_blk_reduce, k_blk_nn T -= V S)   two classical passes
//   2 x (k_blk_tn T^T T, k_blk_chol, k_blk_nn T <- T C)          Cholesky QR twice,
//                 columns that lost their norm are dropped
// Every size the iterations change (k, the number of new vectors) lives in
// device memory, so the host enqueues iterations without waiting; it reads
// a mapped summary after each launch of `chunk` iterations.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "gemv.h"
#include "internal.h"
#include "lanes.h"

namespace dmrg {

constexpr int BB = 8;        // largest block (number of roots)
constexpr int BK = 48;       // largest basis
constexpr int BTPB = 256;    // threads of the row kernels
constexpr int TN_ROWS = 1024;  // rows per workgroup of the tall-skinny products

struct BlkState {
    int32_t k, nnew, active, iters, nproj, restarts, converged, restart;
    int32_t kmax, kkeep, b, max_iter;
    int32_t slot_on[BB];  // projection masks of the new-vector slots
    int32_t conv[BB];
    double tol, floor_, dmin, pad;
    double theta[BK];
    double rnorm[BB];
    double G[BK * BK];  // Rayleigh matrix, row-major, leading dimension BK
    double Y[BK * BK];  // its eigenvectors (columns), ascending eigenvalues
    double S[BK * BB];  // coefficients of the current tall-skinny update (row j, column c)
};

struct BlkSummary {
    double theta[BB];
    double rnorm[BB];
    int32_t active, iters, nproj, restarts, converged, pad[3];
};

struct BlockWork {
    int64_t n = 0;
    int b = 0, kmax = 0;
    double *V = nullptr, *W = nullptr, *T = nullptr, *WT = nullptr, *D = nullptr, *coef = nullptr;
    double *part = nullptr;  // [nblk][BK][BB] partial products
    int nblk = 0;
    BlkState *st = nullptr;
    BlkSummary *h_sum = nullptr, *d_sum = nullptr;
    std::vector<void *> owned;
};

// ------------------------------------------------------------------ tall-skinny products

// Column ranges of A^T B for the three products of an iteration.
enum { TN_RR = 0, TN_ORTH = 1, TN_GRAM = 2 };

struct TnArgs {
    const double *A, *B;
    int ka, kb, a0, b0;  // columns a0 .. a0 + ka of A, b0 .. b0 + kb of B
};

__device__ __forceinline__ TnArgs tn_args(int mode, const BlkState &S, const double *V, const double *W,
                                          const double *T, int b) {
    TnArgs a;
    if (mode == TN_RR) {  // V(:, :k+nnew)^T W(:, k:k+nnew)
        a = TnArgs{V, W, S.k + S.nnew, S.nnew, 0, S.k};
    } else if (mode == TN_ORTH) {  // V(:, :k)^T T
        a = TnArgs{V, T, S.k, b, 0, 0};
    } else {  // T^T T
        a = TnArgs{T, T, b, b, 0, 0};
    }
    return a;
}

typedef double v4d __attribute__((ext_vector_type(4)));

// part[blk][j][c] = sum over the block's rows e of A[e, a0 + j] B[e, b0 + c]
// (j < ka <= BK, c < kb <= BB), FP64 MFMA 16x16x4: rows of the vectors are
// the contraction; each wavefront takes a quarter of the block's rows and all
// output tiles, lane group g holding 4 consecutive rows of a 16-row step; the
// four partial tiles are added in a fixed order through LDS.
template <int MODE>
__global__ __launch_bounds__(256) void k_blk_tn(const BlkState *__restrict__ st, const double *__restrict__ V,
                                                const double *__restrict__ W, const double *__restrict__ T,
                                                int64_t n, int b, double *__restrict__ part) {
    __shared__ double red[4][BK][BB + 1];
    const BlkState &S = *st;
    if (!S.active) return;
    const TnArgs ta = tn_args(MODE, S, V, W, T, b);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, r16 = lane & 15, g = lane >> 4;
    constexpr int NT = BK / 16;  // output tiles along A's columns
    v4d acc[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[t] = v4d{0, 0, 0, 0};
    const int64_t e_begin = (int64_t)blockIdx.x * TN_ROWS + wave * (TN_ROWS / 4);
    const int64_t e_end = min(n, e_begin + TN_ROWS / 4);
    const bool cok = r16 < ta.kb;
    const double *Bc = ta.B + (int64_t)(ta.b0 + (cok ? r16 : 0)) * n;
    for (int64_t e0 = e_begin; e0 < e_end; e0 += 16) {
        double bv[4], av[NT][4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int64_t e = e0 + 4 * g + j;
            const bool ok = e < e_end;
            bv[j] = (ok && cok) ? Bc[e] : 0.0;
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                const int col = 16 * t + r16;
                av[t][j] = (ok && col < ta.ka) ? ta.A[(int64_t)(ta.a0 + col) * n + e] : 0.0;
            }
        }
#pragma unroll
        for (int t = 0; t < NT; ++t)
            if (16 * t < ta.ka) {
#pragma unroll
                for (int j = 0; j < 4; ++j) acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[t][j], bv[j], acc[t], 0, 0, 0);
            }
    }
    // accumulator value v of lane (g, c) holds D[4 v + g][c]: D row = A column, D column = B column
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int row = 16 * t + 4 * v + g;
            if (r16 < BB) red[wave][row][r16] = acc[t][v];
        }
    __syncthreads();
    for (int i = threadIdx.x; i < BK * BB; i += 256) {
        const int j = i / BB, c = i % BB;
        part[(size_t)blockIdx.x * BK * BB + i] = (red[0][j][c] + red[1][j][c]) + (red[2][j][c] + red[3][j][c]);
    }
}

// out[e] = sum over q < nblk of part[q * stride + idx(e)] for e < nent, by all
// threads of the block: each entry gets an aligned group of G lanes (the
// largest power of two with G nent <= blockDim), every lane sums every G-th
// block with four loads in flight, and the group combines its lanes by DPP.
// The order of the sums is fixed, so every call gives the same bits.
template <class Idx, class Out>
__device__ __forceinline__ void sum_partials(const double *__restrict__ part, int64_t stride, int nblk, int nent,
                                             Idx idx, Out out) {
    const int nt = blockDim.x;
    int G = 64;
    while (G > 1 && G * nent > nt) G >>= 1;
    const int per = nt / G;  // entries per pass
    const int lane_g = threadIdx.x % G, slot = threadIdx.x / G;
    for (int e0 = 0; e0 < nent; e0 += per) {
        const int e = e0 + slot;
        const bool ok = e < nent;
        const int64_t base = ok ? idx(e) : 0;
        double a[4] = {0.0, 0.0, 0.0, 0.0};
        for (int q = lane_g; q < nblk; q += 4 * G) {
            double v[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int qq = q + u * G;
                v[u] = (ok && qq < nblk) ? part[(int64_t)qq * stride + base] : 0.0;
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) a[u] += v[u];
        }
        const double sum = group_sum((a[0] + a[1]) + (a[2] + a[3]), G);
        if (ok && lane_g == 0) out(e, sum);
    }
}

// Sum of the partial products over the blocks, in block order, into S.S
// (row j, column c); one workgroup.
template <int MODE>
__global__ __launch_bounds__(256) void k_blk_reduce(BlkState *__restrict__ st, const double *__restrict__ part,
                                                    int nblk, int b) {
    BlkState &S = *st;
    if (!S.active) return;
    const int ka = MODE == TN_ORTH ? S.k : b;
    for (int i = threadIdx.x; i < BK * BB; i += 256) S.S[i] = 0.0;
    __syncthreads();
    sum_partials(part, BK * BB, nblk, ka * b, [&](int e) { return (int64_t)(e / b) * BB + e % b; },
                 [&](int e, double v) { S.S[(e / b) * BB + e % b] = v; });
}

// ------------------------------------------------------------------ row kernels

// V(:, k + j) = T_j, W(:, k + j) = WT_j for the new vectors.
__global__ __launch_bounds__(BTPB) void k_blk_append(const BlkState *__restrict__ st, double *__restrict__ V,
                                                     double *__restrict__ W, const double *__restrict__ T,
                                                     const double *__restrict__ WT, int64_t n) {
    const BlkState &S = *st;
    if (!S.active) return;
    const int k = S.k, nn = S.nnew;
    for (int64_t e = (int64_t)blockIdx.x * BTPB + threadIdx.x; e < n; e += (int64_t)gridDim.x * BTPB)
        for (int j = 0; j < nn; ++j) {
            V[(int64_t)(k + j) * n + e] = T[(int64_t)j * n + e];
            W[(int64_t)(k + j) * n + e] = WT[(int64_t)j * n + e];
        }
}

// T(:, c) <- T(:, c) - sum_j V(:, j) S[j][c]   (mode 0: orthogonalization;
//                                                 columns of converged roots become zero)
// T(:, c) <- sum_j T(:, j) S[j][c]              (mode 1: Cholesky QR; in place per row)
template <int MODE>
__global__ __launch_bounds__(BTPB) void k_blk_nn(const BlkState *__restrict__ st, const double *__restrict__ V,
                                                 double *__restrict__ T, int64_t n, int b) {
    __shared__ double Sl[BK * BB];
    __shared__ double keep[BB];
    const BlkState &S = *st;
    if (!S.active) return;
    for (int i = threadIdx.x; i < BK * BB; i += BTPB) Sl[i] = S.S[i];
    if (threadIdx.x < BB) keep[threadIdx.x] = (MODE == 0 && S.conv[threadIdx.x]) ? 0.0 : 1.0;
    __syncthreads();
    const int kk = MODE == 0 ? S.k : b;
    for (int64_t e = (int64_t)blockIdx.x * BTPB + threadIdx.x; e < n; e += (int64_t)gridDim.x * BTPB) {
        double t[BB], o[BB];
#pragma unroll
        for (int c = 0; c < BB; ++c) {
            t[c] = (c < b) ? T[(int64_t)c * n + e] : 0.0;
            o[c] = MODE == 0 ? t[c] : 0.0;
        }
        for (int j = 0; j < kk; ++j) {
            const double x = MODE == 0 ? V[(int64_t)j * n + e] : t[0];
            double xv = x;
            if (MODE == 1) {
#pragma unroll
                for (int q = 0; q < BB; ++q)
                    if (q == j) xv = t[q];
            }
#pragma unroll
            for (int c = 0; c < BB; ++c) o[c] += (MODE == 0 ? -xv : xv) * Sl[j * BB + c];
        }
#pragma unroll
        for (int c = 0; c < BB; ++c)
            if (c < b) T[(int64_t)c * n + e] = keep[c] * o[c];
    }
}

// Ritz vectors, residuals and corrections, one row per thread; partial sums
// of ||r_j||^2 per block into part[blk][j].
__global__ __launch_bounds__(BTPB) void k_blk_ritz(const BlkState *__restrict__ st, const double *__restrict__ V,
                                                   const double *__restrict__ W, const double *__restrict__ D,
                                                   double *__restrict__ X, double *__restrict__ T, int64_t n, int b,
                                                   double *__restrict__ part) {
    __shared__ double Yl[BK * BB];
    __shared__ double th[BB], sig[BB];
    __shared__ double lds[4 * BB];
    const BlkState &S = *st;
    if (!S.active) return;
    const int k = S.k;
    for (int i = threadIdx.x; i < BK * BB; i += BTPB) {
        const int r = i / BB, c = i % BB;
        Yl[i] = (r < k && c < b) ? S.Y[r * BK + c] : 0.0;
    }
    if (threadIdx.x < BB) {
        const int j = threadIdx.x;
        th[j] = j < b ? S.theta[j] : 0.0;
        sig[j] = j == 0 ? fmin(S.theta[0], S.dmin) : th[j];
    }
    __syncthreads();
    double acc[BB];
#pragma unroll
    for (int j = 0; j < BB; ++j) acc[j] = 0.0;
    for (int64_t e = (int64_t)blockIdx.x * BTPB + threadIdx.x; e < n; e += (int64_t)gridDim.x * BTPB) {
        double x[BB], ax[BB];
#pragma unroll
        for (int j = 0; j < BB; ++j) x[j] = ax[j] = 0.0;
        for (int i = 0; i < k; ++i) {
            const double v = V[(int64_t)i * n + e], w = W[(int64_t)i * n + e];
#pragma unroll
            for (int j = 0; j < BB; ++j) {
                x[j] += v * Yl[i * BB + j];
                ax[j] += w * Yl[i * BB + j];
            }
        }
        const double d = D[e];
#pragma unroll
        for (int j = 0; j < BB; ++j) {
            if (j >= b) continue;
            const double r = ax[j] - th[j] * x[j];
            acc[j] += r * r;
            double den = d - sig[j];
            if (fabs(den) < S.floor_) den = den < 0.0 ? -S.floor_ : S.floor_;
            X[(int64_t)j * n + e] = x[j];
            T[(int64_t)j * n + e] = r / den;  // dropped later if the root has converged
        }
    }
    block_reduce<BB>(acc, BB, lds);
    if (threadIdx.x == 0)
        for (int j = 0; j < BB; ++j) part[(size_t)blockIdx.x * BK * BB + j] = acc[j];
}

// Thick restart, one row per thread: V(:, :kkeep) <- V(:, :k) Y(:, :kkeep), same for W.
__global__ __launch_bounds__(BTPB) void k_blk_restart(const BlkState *__restrict__ st, double *__restrict__ V,
                                                      double *__restrict__ W, int64_t n) {
    __shared__ double Yl[BK * BK];
    const BlkState &S = *st;
    if (!S.active || !S.restart) return;
    const int k = S.k, kk = S.kkeep;
    for (int i = threadIdx.x; i < BK * BK; i += BTPB) Yl[i] = S.Y[i];
    __syncthreads();
    for (int64_t e = (int64_t)blockIdx.x * BTPB + threadIdx.x; e < n; e += (int64_t)gridDim.x * BTPB) {
        for (int pass = 0; pass < 2; ++pass) {
            double *M = pass ? W : V;
            double row[BK];
#pragma unroll
            for (int i = 0; i < BK; ++i) row[i] = (i < k) ? M[(int64_t)i * n + e] : 0.0;
            for (int q = 0; q < kk; ++q) {
                double s = 0.0;
#pragma unroll
                for (int i = 0; i < BK; ++i) s += row[i] * Yl[i * BK + q];
                M[(int64_t)q * n + e] = s;
            }
        }
    }
}

// ------------------------------------------------------------------ small dense steps (one workgroup)

// Ordering of LDS accesses between the lanes of one wavefront.
__device__ __forceinline__ void wsync() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// Cyclic Jacobi on the symmetric k x k matrix A (LDS, leading dimension
// BK + 1) with eigenvectors U, by the whole workgroup: round-robin pairs, all
// disjoint rotations of a step applied together (rows, then columns); a step
// without a rotation costs one barrier (its flag alternates with the next
// step's); rotations with |a_pq| <= 1e-15 ||A||_F are skipped; at most 40
// sweeps.  Then eigenvalues ascending (ties by index): w[r] and the column
// perm[r] of U.
__device__ void blk_jacobi(int k, double (*A)[BK + 1], double (*U)[BK + 1], double *cs, double *sn, int *perm,
                           double *w) {
    const int tid = threadIdx.x, nth = blockDim.x;
    __shared__ double fro;
    __shared__ int fl[2], swept;
    for (int i = tid; i < BK * BK; i += nth) U[i / BK][i % BK] = (i / BK == i % BK) ? 1.0 : 0.0;
    if (tid < 64) {
        double f = 0.0;
        for (int i = tid; i < k * k; i += 64) f += A[i / k][i % k] * A[i / k][i % k];
        f = group_sum<64>(f);
        if (tid == 0) {
            fro = sqrt(f);
            fl[0] = fl[1] = 0;
            swept = 0;
        }
    }
    __syncthreads();
    const double tol = 1e-15 * fro;
    const int k2 = (k + 1) & ~1, np = k2 / 2;
    int gstep = 0;
    for (int sweep = 0; sweep < 40; ++sweep) {
        for (int step = 0; step < k2 - 1; ++step, ++gstep) {
            const int f = gstep & 1;
            if (tid == 0) fl[f ^ 1] = 0;  // the next step's flag
            if (tid < np) {
                int p, q;
                if (tid == 0) {
                    p = 0;
                    q = 1 + (step % (k2 - 1));
                } else {
                    p = 1 + ((step + tid) % (k2 - 1));
                    q = 1 + ((step + k2 - 1 - tid) % (k2 - 1));
                }
                if (p > q) {
                    const int x = p;
                    p = q;
                    q = x;
                }
                double c = 1.0, s = 0.0;
                if (q < k && fabs(A[p][q]) > tol) {
                    const double d = A[q][q] - A[p][p], e2 = 2.0 * A[p][q];
                    const double u = fabs(d) + sqrt(d * d + e2 * e2);
                    const double r = 1.0 / sqrt(u * u + e2 * e2);
                    c = u * r;
                    s = (d >= 0.0 ? e2 : -e2) * r;
                    fl[f] = 1;
                    swept = 1;
                }
                perm[2 * tid] = p;
                perm[2 * tid + 1] = q;
                cs[tid] = c;
                sn[tid] = s;
            }
            __syncthreads();
            if (!fl[f]) continue;
            for (int i = tid; i < np * k; i += nth) {  // rows p, q
                const int pr = i / k, j = i % k, p = perm[2 * pr], q = perm[2 * pr + 1];
                if (q < k) {
                    const double c = cs[pr], s = sn[pr];
                    const double ap = A[p][j], aq = A[q][j];
                    A[p][j] = c * ap - s * aq;
                    A[q][j] = s * ap + c * aq;
                }
            }
            __syncthreads();
            for (int i = tid; i < np * k; i += nth) {  // columns p, q of A and of U
                const int pr = i / k, j = i % k, p = perm[2 * pr], q = perm[2 * pr + 1];
                if (q < k) {
                    const double c = cs[pr], s = sn[pr];
                    const double ap = A[j][p], aq = A[j][q];
                    A[j][p] = c * ap - s * aq;
                    A[j][q] = s * ap + c * aq;
                    const double up = U[j][p], uq = U[j][q];
                    U[j][p] = c * up - s * uq;
                    U[j][q] = s * up + c * uq;
                }
            }
            __syncthreads();
        }
        __syncthreads();
        if (!swept) break;
        __syncthreads();
        if (tid == 0) swept = 0;  // after every thread has read it, before the next sweep sets it
        __syncthreads();
    }
    if (tid < k) {
        const double x = A[tid][tid];
        int r = 0;
        for (int j = 0; j < k; ++j) {
            const double y = A[j][j];
            r += (y < x) || (y == x && j < tid);
        }
        perm[r] = tid;
        w[r] = x;
    }
    __syncthreads();
}

// New columns of G from the summed products, symmetric fill, k += nnew;
// eigen-decomposition of G; restart decision for this iteration.
__global__ __launch_bounds__(256) void k_blk_eig(BlkState *__restrict__ st, const double *__restrict__ part,
                                                 int nblk) {
    __shared__ double A[BK][BK + 1], U[BK][BK + 1], Ye[BK][BK + 1];
    __shared__ double cs[BK / 2], sn[BK / 2], w[BK];
    __shared__ int perm[BK];
    BlkState &S = *st;
    if (!S.active) return;
    const int k0 = S.k, nn = S.nnew, k = k0 + nn;
    // the products V(:, :k)^T W(:, k0:k) from the partial sums
    sum_partials(part, BK * BB, nblk, k * nn, [&](int e) { return (int64_t)(e / nn) * BB + e % nn; },
                 [&](int e, double v) { A[e / nn][e % nn] = v; });  // staging
    __syncthreads();
    for (int i = threadIdx.x; i < k * nn; i += 256) {
        const int j = i / nn, c = i % nn;
        // symmetric: the block of new columns is averaged with its transpose
        const double v = (j >= k0) ? 0.5 * (A[j][c] + A[k0 + c][j - k0]) : A[j][c];
        S.G[j * BK + k0 + c] = v;
        S.G[(k0 + c) * BK + j] = v;
    }
    __syncthreads();
    // warm start: G in the basis of the previous Ritz vectors extended by the
    // new vectors, Ye = blockdiag(Y(:k0, :k0), I), is diagonal up to its new
    // rows and columns, so the Jacobi sweeps converge in a few passes
    for (int i = threadIdx.x; i < k * k; i += 256) {
        const int r = i / k, c = i % k;
        Ye[r][c] = (r < k0 && c < k0) ? S.Y[r * BK + c] : (r == c ? 1.0 : 0.0);
        A[r][c] = S.G[r * BK + c];
    }
    __syncthreads();
    for (int i = threadIdx.x; i < k * k; i += 256) {  // U = G Ye (staging)
        const int r = i / k, c = i % k;
        double acc = 0.0;
        for (int l = 0; l < k; ++l) acc += A[r][l] * Ye[l][c];
        U[r][c] = acc;
    }
    __syncthreads();
    __syncthreads();
    for (int i = threadIdx.x; i < k * k; i += 256) {  // A = Ye^T G Ye
        const int r = i / k, c = i % k;
        double acc = 0.0;
        for (int l = 0; l < k; ++l) acc += Ye[l][r] * U[l][c];
        A[r][c] = acc;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < k * k; i += 256) {  // exactly symmetric
        const int r = i / k, c = i % k;
        if (r < c) {
            const double v = 0.5 * (A[r][c] + A[c][r]);
            A[r][c] = v;
            A[c][r] = v;
        }
    }
    __syncthreads();
    blk_jacobi(k, A, U, cs, sn, perm, w);
    for (int i = threadIdx.x; i < k * k; i += 256) {  // Y = Ye U, columns in ascending order
        const int r = i / k, c = i % k;
        double acc = 0.0;
        for (int l = 0; l < k; ++l) acc += Ye[r][l] * U[l][perm[c]];
        S.Y[r * BK + c] = acc;
    }
    for (int i = threadIdx.x; i < k; i += 256) S.theta[i] = w[i];
    if (threadIdx.x == 0) {
        S.k = k;
        S.nnew = 0;
        S.nproj += nn;
        S.iters += 1;
    }
}

// Residual norms and convergence; the restart decision: the basis is thick-
// restarted when the corrections of the unconverged roots would not fit.
__global__ __launch_bounds__(256) void k_blk_conv(BlkState *__restrict__ st, const double *__restrict__ part,
                                                 int nblk) {
    BlkState &S = *st;
    if (!S.active) return;
    sum_partials(part, BK * BB, nblk, S.b, [](int e) { return (int64_t)e; }, [&](int e, double v) {
        S.rnorm[e] = sqrt(v);
        S.conv[e] = (S.rnorm[e] <= S.tol) ? 1 : 0;
    });
    __syncthreads();
    if (threadIdx.x == 0) {
        int c = 1, open = 0;
        bool bad = !isfinite(S.theta[0]);
        for (int j = 0; j < S.b; ++j) {
            c &= S.conv[j];
            open += !S.conv[j];
            bad = bad || !isfinite(S.rnorm[j]);
        }
        S.converged = c;
        if (c || bad || S.iters >= S.max_iter) S.active = 0;
        S.restart = (S.active && S.k + open > S.kmax) ? 1 : 0;
    }
}

// After a thick restart the kept Ritz vectors are the basis: G = diag(theta),
// Y = I.  Then the per-iteration summary for the host.
__global__ __launch_bounds__(256) void k_blk_finish(BlkState *__restrict__ st, BlkSummary *__restrict__ sum) {
    BlkState &S = *st;
    if (S.active && S.restart) {
        const int kk = S.kkeep;
        for (int i = threadIdx.x; i < BK * BK; i += 256) {
            const int r = i / BK, c = i % BK;
            S.G[i] = (r == c && r < kk) ? S.theta[r] : 0.0;
            S.Y[i] = (r == c) ? 1.0 : 0.0;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            S.k = kk;
            S.restart = 0;
            S.restarts += 1;
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        BlkSummary r;
        for (int j = 0; j < BB; ++j) {
            r.theta[j] = j < S.b ? S.theta[j] : 0.0;
            r.rnorm[j] = j < S.b ? S.rnorm[j] : 0.0;
        }
        r.active = S.active;
        r.iters = S.iters;
        r.nproj = S.nproj;
        r.restarts = S.restarts;
        r.converged = S.converged;
        r.pad[0] = r.pad[1] = r.pad[2] = 0;
        *sum = r;
    }
}

// Orthonormalization of the new block from its Gram matrix T^T T (in S.S,
// rows and columns < b), column by column in order (modified Gram-Schmidt
// through the Cholesky factor R, R^T R = T^T T): the pivot of column c is its
// norm^2 left after the kept columns before it; below drop^2 = 1e-16 of its
// own norm^2 the column is dropped.  Leaves in S.S the coefficients C,
// T_new(:, m) = sum_j T(:, j) C[j][m], with the m-th kept column at m, and
// (last pass) nnew and the projection masks.  One wavefront, lane j owns
// row j of the small matrices.
__global__ __launch_bounds__(64) void k_blk_chol(BlkState *__restrict__ st, int b, int last) {
    BlkState &S = *st;
    if (!S.active) return;
    __shared__ double Gm[BB][BB], R[BB][BB], C[BB][BB];
    __shared__ double piv;
    __shared__ int keep_c[BB];
    const int lane = threadIdx.x;
    if (lane < BB * BB) {
        const int i = lane / BB, j = lane % BB;
        Gm[i][j] = (i < b && j < b) ? S.S[i * BB + j] : 0.0;
        R[i][j] = C[i][j] = 0.0;
    }
    wsync();
    for (int c = 0; c < b; ++c) {
        if (lane == 0) {
            double d = Gm[c][c];
            for (int i = 0; i < c; ++i) d -= R[i][c] * R[i][c];
            piv = (Gm[c][c] > 0.0 && d > 1e-16 * Gm[c][c]) ? sqrt(d) : 0.0;
            keep_c[c] = piv > 0.0;
        }
        wsync();
        const double rc = piv;
        if (rc > 0.0 && lane < b) {
            // row c of R (columns j > c) and column c of C = R^{-1} in column coordinates
            const int j = lane;
            if (j > c) {
                double x = Gm[c][j];
                for (int i = 0; i < c; ++i) x -= R[i][c] * R[i][j];
                R[c][j] = x / rc;
            }
            double y = (j == c) ? 1.0 : 0.0;
            for (int i = 0; i < c; ++i) y -= R[i][c] * C[j][i];
            C[j][c] = y / rc;
        }
        if (lane == 0 && rc > 0.0) R[c][c] = rc;
        wsync();
    }
    // compaction: the m-th kept column goes to position m
    if (lane < BB * BB) {
        const int j = lane / BB, m = lane % BB;
        int col = -1, cnt = 0;
        for (int c = 0; c < b; ++c)
            if (keep_c[c]) {
                if (cnt == m) col = c;
                ++cnt;
            }
        S.S[j * BB + m] = (j < b && col >= 0) ? C[j][col] : 0.0;
    }
    if (last && lane == 0) {
        int nk = 0;
        for (int c = 0; c < b; ++c) nk += keep_c[c];
        S.nnew = nk;
        for (int j = 0; j < BB; ++j) S.slot_on[j] = j < nk ? 1 : 0;
        if (nk == 0) S.active = 0;  // nothing new: the subspace stopped growing
    }
}

// Start: b columns of the caller's block, state reset.
__global__ __launch_bounds__(BTPB) void k_blk_init(BlkState *__restrict__ st, const double *__restrict__ X0,
                                                   double *__restrict__ T, int64_t n, int b, int kmax, int kkeep,
                                                   int max_iter, double tol, double floor_, const double *__restrict__ D,
                                                   double *__restrict__ part) {
    for (int64_t i = (int64_t)blockIdx.x * BTPB + threadIdx.x; i < (int64_t)b * n; i += (int64_t)gridDim.x * BTPB)
        T[i] = X0[i];
    // min D partials: block q writes part[q * BK * BB]
    double m = INFINITY;
    for (int64_t e = (int64_t)blockIdx.x * BTPB + threadIdx.x; e < n; e += (int64_t)gridDim.x * BTPB) m = fmin(m, D[e]);
    m = wave_min(m);
    __shared__ double wm[BTPB / 64];
    if ((threadIdx.x & 63) == 0) wm[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        double x = wm[0];
        for (int i = 1; i < BTPB / 64; ++i) x = fmin(x, wm[i]);
        part[(size_t)blockIdx.x * BK * BB] = x;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        BlkState &S = *st;
        S.k = 0;
        S.nnew = 0;
        S.active = 1;
        S.iters = S.nproj = S.restarts = S.converged = S.restart = 0;
        S.kmax = kmax;
        S.kkeep = kkeep;
        S.b = b;
        S.max_iter = max_iter;
        S.tol = tol;
        S.floor_ = floor_;
        for (int j = 0; j < BB; ++j) {
            S.conv[j] = 0;
            S.slot_on[j] = 0;
            S.rnorm[j] = 0.0;
        }
    }
}

__global__ void k_blk_dmin(BlkState *__restrict__ st, const double *__restrict__ part, int nblk) {
    if (threadIdx.x) return;
    double m = INFINITY;
    for (int q = 0; q < nblk; ++q) m = fmin(m, part[(size_t)q * BK * BB]);
    st->dmin = m;
}

// ------------------------------------------------------------------ host driver

static dmrg_status blk_alloc(dmrg_plan *plan, int b, int kmax, hipStream_t s) {
    BlockWork *w = plan->blk;
    if (w && w->b == b && w->kmax == kmax) return DMRG_OK;
    block_free(plan);
    w = new BlockWork();
    plan->blk = w;
    w->n = plan->n;
    w->b = b;
    w->kmax = kmax;
    const size_t n = (size_t)plan->n;
    w->nblk = (int)std::max<int64_t>(1, (plan->n + TN_ROWS - 1) / TN_ROWS);
    auto alloc = [&](void **p, size_t bytes) -> dmrg_status {
        DMRG_HIP(hipMalloc(p, std::max<size_t>(bytes, 8)));
        w->owned.push_back(*p);
        return DMRG_OK;
    };
    DMRG_TRY(alloc((void **)&w->V, (size_t)kmax * n * 8));
    DMRG_TRY(alloc((void **)&w->W, (size_t)kmax * n * 8));
    DMRG_TRY(alloc((void **)&w->T, (size_t)BB * n * 8));
    DMRG_TRY(alloc((void **)&w->WT, (size_t)BB * n * 8));
    DMRG_TRY(alloc((void **)&w->D, n * 8));
    DMRG_TRY(alloc((void **)&w->coef, std::max(plan->nterm_total, 1) * 8));
    const int rows = std::max(w->nblk, (int)std::min<int64_t>((plan->n + BTPB - 1) / BTPB, 2048));
    DMRG_TRY(alloc((void **)&w->part, (size_t)rows * BK * BB * 8));
    DMRG_TRY(alloc((void **)&w->st, sizeof(BlkState)));
    DMRG_HIP(hipHostMalloc((void **)&w->h_sum, sizeof(BlkSummary), hipHostMallocMapped | hipHostMallocCoherent));
    DMRG_HIP(hipHostGetDevicePointer((void **)&w->d_sum, w->h_sum, 0));
    DMRG_HIP(hipMemsetAsync(w->V, 0, (size_t)kmax * n * 8, s));
    DMRG_HIP(hipMemsetAsync(w->W, 0, (size_t)kmax * n * 8, s));
    DMRG_HIP(hipMemsetAsync(w->T, 0, (size_t)BB * n * 8, s));
    DMRG_HIP(hipMemsetAsync(w->WT, 0, (size_t)BB * n * 8, s));
    DMRG_HIP(hipMemsetAsync(w->st, 0, sizeof(BlkState), s));
    DMRG_HIP(hipStreamSynchronize(s));
    return DMRG_OK;
}

dmrg_status block_free(dmrg_plan *plan) {
    BlockWork *w = plan->blk;
    if (!w) return DMRG_OK;
    for (void *p : w->owned) (void)hipFree(p);
    if (w->h_sum) (void)hipHostFree(w->h_sum);
    delete w;
    plan->blk = nullptr;
    return DMRG_OK;
}

// The orthogonalization of the corrections T against V (two classical passes)
// and among themselves (Cholesky QR twice with dropping); sets nnew.
static void enqueue_orth(const BlockWork &w, dim3 rg, hipStream_t s) {
    const int b = w.b;
    for (int pass = 0; pass < 2; ++pass) {
        hipLaunchKernelGGL(k_blk_tn<TN_ORTH>, dim3(w.nblk), dim3(256), 0, s, w.st, w.V, w.W, w.T, w.n, b, w.part);
        hipLaunchKernelGGL(k_blk_reduce<TN_ORTH>, dim3(1), dim3(256), 0, s, w.st, w.part, w.nblk, b);
        hipLaunchKernelGGL(k_blk_nn<0>, rg, dim3(BTPB), 0, s, w.st, w.V, w.T, w.n, b);
    }
    for (int pass = 0; pass < 2; ++pass) {
        hipLaunchKernelGGL(k_blk_tn<TN_GRAM>, dim3(w.nblk), dim3(256), 0, s, w.st, w.V, w.W, w.T, w.n, b, w.part);
        hipLaunchKernelGGL(k_blk_reduce<TN_GRAM>, dim3(1), dim3(256), 0, s, w.st, w.part, w.nblk, b);
        hipLaunchKernelGGL(k_blk_chol, dim3(1), dim3(64), 0, s, w.st, b, pass);
        hipLaunchKernelGGL(k_blk_nn<1>, rg, dim3(BTPB), 0, s, w.st, w.V, w.T, w.n, b);
    }
}

}  // namespace dmrg

using namespace dmrg;

extern "C" {

void dmrg_block_default_opts(dmrg_block_opts *o) {
    if (!o) return;
    o->tol = 1e-10;
    o->nroots = 4;
    o->kmax = 32;
    o->kmin = 0;
    o->max_iter = 500;
    o->precond_floor = 1e-3;
    o->chunk = 4;
}

dmrg_status dmrg_block_davidson(dmrg_plan *plan, const double *coef, const dmrg_block_opts *opts, double *X,
                                double *energies, double *residuals, dmrg_block_info *info, void *stream) {
    clear_error();
    if (!plan || !X || (!coef && plan->nterm_total)) return set_error(DMRG_E_INVALID_ARG, "null argument");
    dmrg_block_opts o;
    dmrg_block_default_opts(&o);
    if (opts) o = *opts;
    if (plan->nprob != 1) return set_error(DMRG_E_UNSUPPORTED, "block Davidson takes single-superblock plans");
    const int b = o.nroots;
    if (b < 1 || b > BB) return set_error(DMRG_E_INVALID_ARG, "nroots must be 1..%d", BB);
    if (plan->n < 2 * b) return set_error(DMRG_E_INVALID_ARG, "the sector has fewer than 2 nroots states");
    const int kmax = (int)std::min<int64_t>(std::min(o.kmax, BK), plan->n);
    const int kkeep = std::min(std::max(o.kmin, 2 * b), kmax - b);
    if (kmax < 3 * b || kkeep < b)
        return set_error(DMRG_E_INVALID_ARG, "kmax must be at least 3 nroots (and at most %d)", BK);
    if (!(o.tol > 0.0) || o.max_iter < 1 || !(o.precond_floor > 0.0) || o.chunk < 1)
        return set_error(DMRG_E_INVALID_ARG, "need tol > 0, max_iter >= 1, precond_floor > 0, chunk >= 1");
    int cur = -1;
    DMRG_HIP(hipGetDevice(&cur));
    if (cur != plan->device) return set_error(DMRG_E_INVALID_ARG, "plan belongs to another device");
    hipStream_t s = (hipStream_t)stream;
    DMRG_TRY(blk_alloc(plan, b, kmax, s));
    BlockWork &w = *plan->blk;
    const int64_t n = w.n;
    const dim3 rg((unsigned)std::min<int64_t>((n + BTPB - 1) / BTPB, 2048));
    DMRG_HIP(hipMemcpyAsync(w.coef, coef, std::max(plan->nterm_total, 1) * 8, hipMemcpyDeviceToDevice, s));
    DMRG_TRY(launch_diagonal(plan, w.coef, w.D, s));
    hipLaunchKernelGGL(k_blk_init, rg, dim3(BTPB), 0, s, w.st, (const double *)X, w.T, n, b, kmax, kkeep, o.max_iter,
                       o.tol, o.precond_floor, (const double *)w.D, w.part);
    hipLaunchKernelGGL(k_blk_dmin, dim3(1), dim3(64), 0, s, w.st, (const double *)w.part, (int)rg.x);
    DMRG_HIP(hipGetLastError());
    enqueue_orth(w, rg, s);  // with k = 0: the start block orthonormalized among itself
    bool more = true;
    while (more) {
        for (int it = 0; it < o.chunk; ++it) {
            // the new block in groups of PROJ_NVEC vectors per launch (slots past the
            // block's size are masked off on the device)
            for (int j = 0; j < b; j += PROJ_NVEC)
                DMRG_TRY(launch_project_multi(plan, w.coef, w.T + (int64_t)j * n, n, w.WT + (int64_t)j * n, n,
                                              &w.st->slot_on[j], s));
            hipLaunchKernelGGL(k_blk_append, rg, dim3(BTPB), 0, s, w.st, w.V, w.W, (const double *)w.T,
                               (const double *)w.WT, n);
            hipLaunchKernelGGL(k_blk_tn<TN_RR>, dim3(w.nblk), dim3(256), 0, s, w.st, w.V, w.W, w.T, n, b, w.part);
            hipLaunchKernelGGL(k_blk_eig, dim3(1), dim3(256), 0, s, w.st, (const double *)w.part, w.nblk);
            hipLaunchKernelGGL(k_blk_ritz, rg, dim3(BTPB), 0, s, w.st, (const double *)w.V, (const double *)w.W,
                               (const double *)w.D, X, w.T, n, b, w.part);
            hipLaunchKernelGGL(k_blk_conv, dim3(1), dim3(256), 0, s, w.st, (const double *)w.part, (int)rg.x);
            hipLaunchKernelGGL(k_blk_restart, rg, dim3(BTPB), 0, s, w.st, w.V, w.W, n);
            hipLaunchKernelGGL(k_blk_finish, dim3(1), dim3(256), 0, s, w.st, w.d_sum);
            enqueue_orth(w, rg, s);
        }
        DMRG_HIP(hipGetLastError());
        DMRG_HIP(hipStreamSynchronize(s));
        more = w.h_sum->active != 0;
    }
    const BlkSummary &r = *w.h_sum;
    for (int j = 0; j < b; ++j) {
        if (energies) energies[j] = r.theta[j];
        if (residuals) residuals[j] = r.rnorm[j];
    }
    if (info) {
        info->iterations = r.iters;
        info->projections = r.nproj;
        info->restarts = r.restarts;
        info->converged = r.converged;
    }
    for (int j = 0; j < b; ++j)
        if (!std::isfinite(r.theta[j]) || !std::isfinite(r.rnorm[j]))
            return set_error(DMRG_E_NONFINITE, "non-finite Ritz value or residual");
    if (!r.converged) return set_error(DMRG_W_NOT_CONVERGED, "not converged (iterations %d)", r.iters);
    return DMRG_OK;
}

}  // extern "C"
