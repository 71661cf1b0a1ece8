// Device-resident Davidson iteration (Alg. 3) for one or many superblocks.
//
// Every member of a plan runs in lock step: all members share the subspace
// size i of an iteration, a member that has converged is masked out, so the
// host knows the kernel sequence of each iteration in advance and can replay
// captured hipGraphs of several iterations.  Per iteration:
//
//   k_rayleigh  B(:, i-1) = V^T W(:, i-1)            (Alg. 3 line 3)
//               last block per member: smallest Ritz pair of B (line 4) by a
//               warm-started parallel Jacobi in one workgroup
//   k_ritz      x = V y, r = W y - lambda x, ||r||   (lines 5-7)
//               t = r / (D - sigma) (line 10, shifted diagonal preconditioner)
//               s = V^T t (line 12, first pass) -- all in one sweep over V, W
//   k_restart   (when i = kmax) V <- V Y(:, :kmin), W <- W Y(:, :kmin), s = V^T t
//   k_orth      t <- t - V s (line 13), ||t||, and V^T t for the DGKS pass
//   k_append    V(:, i) = (t - V s2) / ||.||        (line 14)
//   projection  W(:, i) = H V(:, i)                  (line 2 of the next iteration)
//
// Reductions over the vector length are split into fixed chunks; each block
// writes its partial sums, and the last block of a member (atomic arrival
// counter, reset by that block) sums the partials in chunk order, so results
// are independent of scheduling and identical between eager and graph runs.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <tuple>

#include "gemv.h"
#include "internal.h"

namespace dmrg {

constexpr int KM = 48;  // largest supported kmax
constexpr int TPB = GEMV_THREADS;

struct DavState {
    double Bm[KM * KM];  // Rayleigh matrix, row-major, leading dimension KM
    double Y[KM * KM];   // eigenvectors of Bm (column c = Y[r * KM + c])
    double theta[KM];
    double s[KM], s2[KM];
    double lambda, sigma, dmin, rnorm, tn0, scale, tol, floor_;
    int32_t converged, breakdown, iters, nproj, restarts, dgks, nvec, max_iter, bad_start;
};

// Kernel-argument view of the Davidson workspace (plain pointers only).
struct DavArgs {
    int64_t n = 0;
    int nprob = 0;
    int nchunk = 0;
    double *V = nullptr, *W = nullptr, *T = nullptr, *D = nullptr, *coef = nullptr;
    double *dfold = nullptr;         // [n] folded diagonal terms of the current phase's pass
    double *part = nullptr;          // [nchunk][KM + 2]
    int32_t *chunk_member = nullptr;
    int64_t *chunk_begin = nullptr;  // [nchunk + 1] element ranges
    int32_t *member_chunk = nullptr; // [nprob + 1] chunk ranges
    int32_t *counter = nullptr;      // [nprob] arrival counters
    int32_t *nactive = nullptr;      // [1] members still iterating
    int32_t *active = nullptr;       // [nprob] 1 while the member iterates
    DavState *st = nullptr;          // [nprob]
};

struct DavidsonWork {
    DavArgs a;
    int kmax = 0, kmin = 0;
    int32_t *h_nactive = nullptr;  // pinned
    std::map<std::tuple<int, int, int, int>, hipGraphExec_t> graphs;
    std::vector<void *> owned;
};

// ------------------------------------------------------------------ helpers

// Element range and member of chunk c.  A single-member plan needs no lookup:
// its chunks are the consecutive TPB-element ranges.
struct Chunk {
    int member;
    int64_t e0, e1;
};
__device__ __forceinline__ Chunk chunk_of(const DavArgs &w, int c) {
    Chunk k;
    if (w.nprob == 1) {
        k.member = 0;
        k.e0 = (int64_t)c * TPB;
        k.e1 = min(w.n, k.e0 + TPB);
    } else {
        k.member = w.chunk_member[c];
        k.e0 = w.chunk_begin[c];
        k.e1 = w.chunk_begin[c + 1];
    }
    return k;
}

__device__ __forceinline__ bool last_block_of_member(int32_t *counter, int member, int nch) {
    __shared__ int is_last;
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
        int old = atomicAdd(&counter[member], 1);
        is_last = (old == nch - 1);
        if (is_last) counter[member] = 0;
    }
    __syncthreads();
    if (is_last) __threadfence();
    return is_last != 0;
}

// sum of partial column j over the member's chunks (fixed order), all threads get it
__device__ double member_sum(const double *part, int c0, int c1, int j, double *lds) {
    double v = 0.0;
    for (int c = c0 + (int)threadIdx.x; c < c1; c += TPB) v += part[(size_t)c * (KM + 2) + j];
    double r[1] = {v};
    block_reduce<1>(r, 1, lds);
    return r[0];
}

// Sums columns [0, ncols) of the member's chunk partials at once: thread t owns
// column t % ncols and every (TPB / ncols)-th chunk from t / ncols, then the
// per-thread sums of each column are added in slot order.  out: shared [ncols].
__device__ void member_sums(const double *__restrict__ part, int c0, int c1, int ncols, double *scratch,
                            double *out) {
    const int t = threadIdx.x;
    const int per = TPB / ncols;
    const int j = t % ncols, slot = t / ncols;
    double v = 0.0;
    if (slot < per) {
#pragma unroll 4
        for (int c = c0 + slot; c < c1; c += per) v += part[(size_t)c * (KM + 2) + j];
    }
    scratch[t] = v;
    __syncthreads();
    if (t < ncols) {
        double acc = 0.0;
        for (int q = 0; q < per; ++q) acc += scratch[t + q * ncols];
        out[t] = acc;
    }
    __syncthreads();
}

// ------------------------------------------------------------------ init kernels

// ||psi||^2 per member; last block stores the scale, flags zero / non-finite starts.
__global__ __launch_bounds__(TPB) void k_init_norm(const double *__restrict__ psi, DavArgs w) {
    __shared__ double lds[4 * 2];
    const int c = blockIdx.x;
    const Chunk ck = chunk_of(w, c);
    const int member = ck.member;
    double v[1] = {0.0};
    for (int64_t e = ck.e0 + threadIdx.x; e < ck.e1; e += TPB) v[0] += psi[e] * psi[e];
    block_reduce<1>(v, 1, lds);
    if (threadIdx.x == 0) w.part[(size_t)c * (KM + 2)] = v[0];
    const int c0 = w.member_chunk[member], c1 = w.member_chunk[member + 1];
    if (!last_block_of_member(w.counter, member, c1 - c0)) return;
    double s = member_sum(w.part, c0, c1, 0, lds);
    if (threadIdx.x == 0) {
        DavState &S = w.st[member];
        if (!(s > 0.0) || !isfinite(s)) {
            S.bad_start = 1;
            w.active[member] = 0;
            S.scale = 0.0;
            atomicSub(w.nactive, 1);
        } else {
            S.scale = 1.0 / sqrt(s);
        }
    }
}

// V(:,0) = psi * scale; also the diagonal's minimum per member.
__global__ __launch_bounds__(TPB) void k_init_vec(const double *__restrict__ psi, DavArgs w) {
    __shared__ double lds[4 * 2];
    __shared__ double red[TPB];
    const int c = blockIdx.x;
    const Chunk ck = chunk_of(w, c);
    const int member = ck.member;
    const double sc = w.st[member].scale;
    double mn = INFINITY;
    for (int64_t e = ck.e0 + threadIdx.x; e < ck.e1; e += TPB) {
        w.V[e] = psi[e] * sc;
        mn = fmin(mn, w.D[e]);
    }
    red[threadIdx.x] = mn;
    __syncthreads();
    for (int off = TPB / 2; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) red[threadIdx.x] = fmin(red[threadIdx.x], red[threadIdx.x + off]);
        __syncthreads();
    }
    if (threadIdx.x == 0) w.part[(size_t)c * (KM + 2)] = red[0];
    const int c0 = w.member_chunk[member], c1 = w.member_chunk[member + 1];
    if (!last_block_of_member(w.counter, member, c1 - c0)) return;
    mn = INFINITY;
    for (int q = c0 + (int)threadIdx.x; q < c1; q += TPB) mn = fmin(mn, w.part[(size_t)q * (KM + 2)]);
    red[threadIdx.x] = mn;
    __syncthreads();
    for (int off = TPB / 2; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) red[threadIdx.x] = fmin(red[threadIdx.x], red[threadIdx.x + off]);
        __syncthreads();
    }
    if (threadIdx.x == 0) w.st[member].dmin = red[0];
    (void)lds;
}

// ------------------------------------------------------------------ small eigenproblem

// Smallest-first eigen-decomposition of the member's Rayleigh matrix B[:n,:n]
// by cyclic Jacobi in parallel (round-robin) order.  Warm start: the matrix is
// first transformed by the previous eigenvectors extended with e_n, which
// makes it nearly diagonal.  Runs in one workgroup; all threads must call.
struct JacobiLds {
    double A[KM][KM + 1];
    double Vv[KM][KM + 1];
    double Tm[KM][KM + 1];
    double c[KM / 2], s[KM / 2];
    double red[4 * 2];
    int order[KM];
    int rotated;
};

__device__ void jacobi_eig(DavState &S, int n, JacobiLds &L) {
    const int tid = threadIdx.x;
    // A = B, Vv = [Y_prev 0; 0 1]
    for (int e = tid; e < n * n; e += TPB) {
        int r = e / n, c = e % n;
        L.Tm[r][c] = S.Bm[r * KM + c];
        double y;
        if (r < n - 1 && c < n - 1)
            y = S.Y[r * KM + c];
        else
            y = (r == c) ? 1.0 : 0.0;
        L.Vv[r][c] = y;
    }
    __syncthreads();
    // A = Vv^T B Vv  (Tm holds B; A = B Vv first, then Vv^T A)
    for (int e = tid; e < n * n; e += TPB) {
        int r = e / n, c = e % n;
        double acc = 0.0;
        for (int k = 0; k < n; ++k) acc += L.Tm[r][k] * L.Vv[k][c];
        L.A[r][c] = acc;
    }
    __syncthreads();
    for (int e = tid; e < n * n; e += TPB) {
        int r = e / n, c = e % n;
        double acc = 0.0;
        for (int k = 0; k < n; ++k) acc += L.Vv[k][r] * L.A[k][c];
        L.Tm[r][c] = acc;
    }
    __syncthreads();
    for (int e = tid; e < n * n; e += TPB) {
        int r = e / n, c = e % n;
        L.A[r][c] = 0.5 * (L.Tm[r][c] + L.Tm[c][r]);  // exact symmetry
    }
    __syncthreads();
    const int n2 = (n + 1) & ~1;
    const int np = n2 / 2;
    // Frobenius norm for the absolute part of the rotation threshold
    double fro = 0.0;
    for (int e = tid; e < n * n; e += TPB) fro += L.A[e / n][e % n] * L.A[e / n][e % n];
    double fv[1] = {fro};
    block_reduce<1>(fv, 1, L.red);
    const double abs_tol = 1e-18 * sqrt(fv[0]);
    // Classical threshold Jacobi: a rotation is skipped when |a_pq| is below
    // 1e-16 sqrt(|a_pp a_qq|) (or the absolute floor); stop after a sweep
    // without rotations.
    for (int sweep = 0; sweep < 30; ++sweep) {
        if (tid == 0) L.rotated = 0;
        __syncthreads();
        for (int step = 0; step < n2 - 1; ++step) {
            if (tid < np) {
                int k = tid;
                int p = (k == 0) ? 0 : ((k - 1 + step) % (n2 - 1)) + 1;
                int q = ((n2 - 2 - k + step) % (n2 - 1)) + 1;
                double cc = 1.0, ss = 0.0;
                if (p < n && q < n) {
                    double apq = L.A[p][q];
                    double app = L.A[p][p], aqq = L.A[q][q];
                    if (fabs(apq) > fmax(1e-16 * sqrt(fabs(app * aqq)), abs_tol)) {
                        double th = (aqq - app) / (2.0 * apq);
                        double t = (th >= 0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
                        cc = 1.0 / sqrt(t * t + 1.0);
                        ss = t * cc;
                        L.rotated = 1;
                    }
                }
                L.c[k] = cc;
                L.s[k] = ss;
                L.order[2 * k] = p;
                L.order[2 * k + 1] = q;
            }
            __syncthreads();
            // rows: A <- J^T A
            for (int e = tid; e < np * n; e += TPB) {
                int k = e / n, j = e % n;
                int p = L.order[2 * k], q = L.order[2 * k + 1];
                if (p < n && q < n && L.s[k] != 0.0) {
                    double cc = L.c[k], ss = L.s[k];
                    double ap = L.A[p][j], aq = L.A[q][j];
                    L.A[p][j] = cc * ap - ss * aq;
                    L.A[q][j] = ss * ap + cc * aq;
                }
            }
            __syncthreads();
            // columns: A <- A J, Vv <- Vv J
            for (int e = tid; e < np * n; e += TPB) {
                int k = e / n, j = e % n;
                int p = L.order[2 * k], q = L.order[2 * k + 1];
                if (p < n && q < n && L.s[k] != 0.0) {
                    double cc = L.c[k], ss = L.s[k];
                    double ap = L.A[j][p], aq = L.A[j][q];
                    L.A[j][p] = cc * ap - ss * aq;
                    L.A[j][q] = ss * ap + cc * aq;
                    double vp = L.Vv[j][p], vq = L.Vv[j][q];
                    L.Vv[j][p] = cc * vp - ss * vq;
                    L.Vv[j][q] = ss * vp + cc * vq;
                }
            }
            __syncthreads();
        }
        if (!L.rotated) break;  // read after the last barrier of the sweep: uniform
        __syncthreads();
    }
    // sort eigenvalues ascending (stable selection by rank)
    for (int a = tid; a < n; a += TPB) {
        double da = L.A[a][a];
        int rank = 0;
        for (int b = 0; b < n; ++b) {
            double db = L.A[b][b];
            rank += (db < da) || (db == da && b < a);
        }
        L.order[rank] = a;
    }
    __syncthreads();
    for (int e = tid; e < n * n; e += TPB) {
        int r = e / n, c = e % n;
        S.Y[r * KM + c] = L.Vv[r][L.order[c]];
    }
    for (int c = tid; c < n; c += TPB) S.theta[c] = L.A[L.order[c]][L.order[c]];
    __syncthreads();
}

// ------------------------------------------------------------------ iteration kernels

// B(:, i-1) = V(:, :i)^T W(:, i-1); last block of a member: Ritz pair.
template <int KB>
__global__ __launch_bounds__(TPB) void k_rayleigh(DavArgs w, int i) {
    extern __shared__ __align__(16) unsigned char smem[];
    JacobiLds &L = *reinterpret_cast<JacobiLds *>(smem);
    const int c = blockIdx.x;
    const Chunk ck = chunk_of(w, c);
    const int member = ck.member;
    const int act = w.active[member];  // checked after the loads are in flight
    const int64_t n = w.n;
    double acc[KB];
#pragma unroll
    for (int j = 0; j < KB; ++j) acc[j] = 0.0;
    const double *wc = w.W + (int64_t)(i - 1) * n;
    for (int64_t e = ck.e0 + threadIdx.x; e < ck.e1; e += TPB) {
        const double x = wc[e];
        double v[KB];
#pragma unroll
        for (int j = 0; j < KB; ++j) v[j] = w.V[(int64_t)min(j, i - 1) * n + e];  // clamped: no branch
#pragma unroll
        for (int j = 0; j < KB; ++j) acc[j] += (j < i ? v[j] : 0.0) * x;
    }
    if (!act) return;
    block_reduce<KB>(acc, i, &L.Tm[0][0]);  // Tm is free until the eigensolve
    if (threadIdx.x == 0)
        for (int j = 0; j < i; ++j) w.part[(size_t)c * (KM + 2) + j] = acc[j];
    const int c0 = w.member_chunk[member], c1 = w.member_chunk[member + 1];
    if (!last_block_of_member(w.counter, member, c1 - c0)) return;
    DavState &S = w.st[member];
    member_sums(w.part, c0, c1, i, &L.Tm[0][0], &L.A[0][0]);
    if ((int)threadIdx.x < i) {
        const int j = threadIdx.x;
        const double b = L.A[0][j];
        S.Bm[j * KM + (i - 1)] = b;
        S.Bm[(i - 1) * KM + j] = b;
    }
    __syncthreads();
    jacobi_eig(S, i, L);
    if (threadIdx.x == 0) {
        S.lambda = S.theta[0];
        S.sigma = fmin(S.lambda, S.dmin);
        S.iters += 1;
        S.nvec = i;
    }
}

// x = V y, r = W y - lambda x, t = r / (D - sigma); partials: ||r||^2, ||t||^2, V^T t.
template <int KB>
__global__ __launch_bounds__(TPB) void k_ritz(DavArgs w, int i, int restart) {
    __shared__ double lds[4 * (KB + 2)];
    __shared__ double scratch[TPB];
    __shared__ double sums[KB + 2];
    const int c = blockIdx.x;
    const Chunk ck = chunk_of(w, c);
    const int member = ck.member;
    const DavState &S = w.st[member];
    const int act = w.active[member];
    const int64_t n = w.n;
    double y[KB];
#pragma unroll
    for (int j = 0; j < KB; ++j) y[j] = (j < i) ? S.Y[j * KM] : 0.0;
    const double lam = S.lambda, sig = S.sigma, fl = S.floor_;
    double acc[KB + 2];
#pragma unroll
    for (int j = 0; j < KB + 2; ++j) acc[j] = 0.0;
    for (int64_t e = ck.e0 + threadIdx.x; e < ck.e1; e += TPB) {
        double v[KB], wv[KB];
        double x = 0.0, wy = 0.0;
#pragma unroll
        for (int j = 0; j < KB; ++j) {
            v[j] = w.V[(int64_t)min(j, i - 1) * n + e];
            wv[j] = w.W[(int64_t)min(j, i - 1) * n + e];
        }
#pragma unroll
        for (int j = 0; j < KB; ++j) {
            v[j] = (j < i) ? v[j] : 0.0;
            x += v[j] * y[j];
            wy += wv[j] * y[j];
        }
        const double r = wy - lam * x;
        double den = w.D[e] - sig;
        if (fabs(den) < fl) den = (den < 0.0) ? -fl : fl;
        const double t = r / den;
        if (act) w.T[e] = t;
        acc[KB] += r * r;
        acc[KB + 1] += t * t;
        if (!restart) {
#pragma unroll
            for (int j = 0; j < KB; ++j) acc[j] += v[j] * t;
        }
    }
    if (!act) return;
    block_reduce<KB + 2>(acc, KB + 2, lds);
    if (threadIdx.x == 0)
        for (int j = 0; j < KB + 2; ++j) w.part[(size_t)c * (KM + 2) + j] = acc[j];
    // note: columns KB, KB+1 of the partial row hold ||r||^2 and ||t||^2
    const int c0 = w.member_chunk[member], c1 = w.member_chunk[member + 1];
    if (!last_block_of_member(w.counter, member, c1 - c0)) return;
    DavState &Sm = w.st[member];
    member_sums(w.part, c0, c1, KB + 2, scratch, sums);
    const double rr = sums[KB];
    const double tt = sums[KB + 1];
    double ss = 0.0;
    if (!restart) {
        if ((int)threadIdx.x < i) Sm.s[threadIdx.x] = sums[threadIdx.x];
        for (int j = 0; j < i; ++j) ss += sums[j] * sums[j];
    }
    if (threadIdx.x == 0) {
        Sm.rnorm = sqrt(rr);
        Sm.tn0 = sqrt(tt);
        if (!(Sm.rnorm == Sm.rnorm) || isinf(Sm.rnorm)) {
            w.active[member] = 0;
            Sm.bad_start = 2;  // non-finite iterate
            atomicSub(w.nactive, 1);
        } else if (Sm.rnorm <= Sm.tol) {
            Sm.converged = 1;
            w.active[member] = 0;
            atomicSub(w.nactive, 1);
        } else if (Sm.iters >= Sm.max_iter) {
            w.active[member] = 0;
            atomicSub(w.nactive, 1);
        } else if (!restart) {
            Sm.dgks = (tt - ss) < 0.5 * tt;
        }
    }
}

// Thick restart: V(:, :kmin) = V(:, :i) Y(:, :kmin), same for W; then s = V^T t, ||t||^2.
template <int KB>
__global__ __launch_bounds__(TPB) void k_restart(DavArgs w, int i, int kmin) {
    __shared__ double lds[4 * (KB + 1)];
    __shared__ double Ys[KB * KB];
    __shared__ double scratch[TPB];
    __shared__ double sums[KB + 1];
    const int c = blockIdx.x;
    const Chunk ck = chunk_of(w, c);
    const int member = ck.member;
    const DavState &S = w.st[member];
    if (!w.active[member]) return;
    for (int e = threadIdx.x; e < KB * KB; e += TPB) {
        int r = e / KB, q = e % KB;
        Ys[r * KB + q] = (r < i && q < kmin) ? S.Y[r * KM + q] : 0.0;
    }
    __syncthreads();
    const int64_t n = w.n;
    double acc[KB + 1];
#pragma unroll
    for (int j = 0; j < KB + 1; ++j) acc[j] = 0.0;
    for (int64_t e = ck.e0 + threadIdx.x; e < ck.e1; e += TPB) {
        double v[KB], wv[KB];
#pragma unroll
        for (int j = 0; j < KB; ++j) {
            v[j] = w.V[(int64_t)min(j, i - 1) * n + e];
            wv[j] = w.W[(int64_t)min(j, i - 1) * n + e];
        }
#pragma unroll
        for (int j = 0; j < KB; ++j) {
            v[j] = (j < i) ? v[j] : 0.0;
            wv[j] = (j < i) ? wv[j] : 0.0;
        }
        const double t = w.T[e];
        for (int q = 0; q < kmin; ++q) {
            double a = 0.0, b = 0.0;
#pragma unroll
            for (int j = 0; j < KB; ++j) {
                a += v[j] * Ys[j * KB + q];
                b += wv[j] * Ys[j * KB + q];
            }
            w.V[(int64_t)q * n + e] = a;
            w.W[(int64_t)q * n + e] = b;
            acc[q] += a * t;
        }
        acc[KB] += t * t;
    }
    block_reduce<KB + 1>(acc, KB + 1, lds);
    if (threadIdx.x == 0)
        for (int j = 0; j < KB + 1; ++j) w.part[(size_t)c * (KM + 2) + j] = acc[j];
    const int c0 = w.member_chunk[member], c1 = w.member_chunk[member + 1];
    if (!last_block_of_member(w.counter, member, c1 - c0)) return;
    DavState &Sm = w.st[member];
    member_sums(w.part, c0, c1, KB + 1, scratch, sums);
    const double tt = sums[KB];
    double ss = 0.0;
    if ((int)threadIdx.x < kmin) Sm.s[threadIdx.x] = sums[threadIdx.x];
    for (int j = 0; j < kmin; ++j) ss += sums[j] * sums[j];
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int r = 0; r < kmin; ++r)
            for (int q = 0; q < kmin; ++q) {
                Sm.Bm[r * KM + q] = (r == q) ? Sm.theta[r] : 0.0;
                Sm.Y[r * KM + q] = (r == q) ? 1.0 : 0.0;
            }
        Sm.tn0 = sqrt(tt);
        Sm.dgks = (tt - ss) < 0.5 * tt;
        Sm.restarts += 1;
    }
}

// t <- t - V s; partials: ||t||^2 and V^T t (for the DGKS pass).
template <int KB>
__global__ __launch_bounds__(TPB) void k_orth(DavArgs w, int i) {
    __shared__ double lds[4 * (KB + 1)];
    __shared__ double scratch[TPB];
    __shared__ double sums[KB + 1];
    const int c = blockIdx.x;
    const Chunk ck = chunk_of(w, c);
    const int member = ck.member;
    const DavState &S = w.st[member];
    const int act = w.active[member];
    double s[KB];
#pragma unroll
    for (int j = 0; j < KB; ++j) s[j] = (j < i) ? S.s[j] : 0.0;
    const int64_t n = w.n;
    double acc[KB + 1];
#pragma unroll
    for (int j = 0; j < KB + 1; ++j) acc[j] = 0.0;
    for (int64_t e = ck.e0 + threadIdx.x; e < ck.e1; e += TPB) {
        double v[KB];
        double t = w.T[e];
#pragma unroll
        for (int j = 0; j < KB; ++j) v[j] = w.V[(int64_t)min(j, i - 1) * n + e];
#pragma unroll
        for (int j = 0; j < KB; ++j) {
            v[j] = (j < i) ? v[j] : 0.0;
            t -= v[j] * s[j];
        }
        if (act) w.T[e] = t;
#pragma unroll
        for (int j = 0; j < KB; ++j) acc[j] += v[j] * t;
        acc[KB] += t * t;
    }
    if (!act) return;
    block_reduce<KB + 1>(acc, KB + 1, lds);
    if (threadIdx.x == 0)
        for (int j = 0; j < KB + 1; ++j) w.part[(size_t)c * (KM + 2) + j] = acc[j];
    const int c0 = w.member_chunk[member], c1 = w.member_chunk[member + 1];
    if (!last_block_of_member(w.counter, member, c1 - c0)) return;
    DavState &Sm = w.st[member];
    member_sums(w.part, c0, c1, KB + 1, scratch, sums);
    const double tt = sums[KB];
    double ss = 0.0;
    if ((int)threadIdx.x < i) Sm.s2[threadIdx.x] = Sm.dgks ? sums[threadIdx.x] : 0.0;
    for (int j = 0; j < i; ++j) ss += sums[j] * sums[j];
    if (threadIdx.x == 0) {
        double nn = Sm.dgks ? (tt - ss) : tt;
        double nrm = sqrt(fmax(nn, 0.0));
        if (!(nrm > 1e-13 * Sm.tn0)) {
            Sm.breakdown = 1;
            w.active[member] = 0;
            atomicSub(w.nactive, 1);
        } else {
            Sm.scale = 1.0 / nrm;
        }
    }
}

// V(:, i) = (t - V s2) * scale
template <int KB>
__global__ __launch_bounds__(TPB) void k_append(DavArgs w, int i) {
    const int c = blockIdx.x;
    const Chunk ck = chunk_of(w, c);
    const int member = ck.member;
    const DavState &S = w.st[member];
    const int act = w.active[member];
    double s2[KB];
    const bool dg = S.dgks != 0;
#pragma unroll
    for (int j = 0; j < KB; ++j) s2[j] = (dg && j < i) ? S.s2[j] : 0.0;
    const double sc = S.scale;
    const int64_t n = w.n;
    for (int64_t e = ck.e0 + threadIdx.x; e < ck.e1; e += TPB) {
        double t = w.T[e];
        if (dg) {
            double v[KB];
#pragma unroll
            for (int j = 0; j < KB; ++j) v[j] = w.V[(int64_t)min(j, i - 1) * n + e];
#pragma unroll
            for (int j = 0; j < KB; ++j) t -= v[j] * s2[j];
        }
        if (act) w.V[(int64_t)i * n + e] = t * sc;
    }
    if (act && threadIdx.x == 0 && blockIdx.x == w.member_chunk[member]) w.st[member].nproj += 1;
}

// psi = V(:, :nvec) y (normalized Ritz vector of each member)
template <int KB>
__global__ __launch_bounds__(TPB) void k_finalize(DavArgs w, double *__restrict__ psi) {
    const int c = blockIdx.x;
    const Chunk ck = chunk_of(w, c);
    const int member = ck.member;
    const DavState &S = w.st[member];
    if (S.bad_start == 1) return;
    const int nv = S.nvec;
    double y[KB];
#pragma unroll
    for (int j = 0; j < KB; ++j) y[j] = (j < nv) ? S.Y[j * KM] : 0.0;
    const int64_t n = w.n;
    for (int64_t e = ck.e0 + threadIdx.x; e < ck.e1; e += TPB) {
        double v[KB];
#pragma unroll
        for (int j = 0; j < KB; ++j) v[j] = w.V[(int64_t)min(j, nv - 1) * n + e];
        double x = 0.0;
#pragma unroll
        for (int j = 0; j < KB; ++j) x += v[j] * y[j];
        psi[e] = x;
    }
}

__global__ void k_set_state(DavArgs w, double tol, double floor_, int max_iter) {
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= w.nprob) return;
    DavState &S = w.st[m];
    S.tol = tol;
    S.floor_ = floor_;
    S.max_iter = max_iter;
    w.active[m] = 1;
    S.converged = 0;
    S.breakdown = 0;
    S.bad_start = 0;
    S.dgks = 0;
    S.nvec = 1;
    S.iters = 0;  // counts are per phase; the host adds the phases
    S.nproj = 0;
    S.restarts = 0;
    S.Y[0] = 1.0;
    w.counter[m] = 0;
    if (m == 0) *w.nactive = w.nprob;
}

// ------------------------------------------------------------------ host driver

// Register bucket for kernels that keep one row of V (and W) per thread: the
// smallest of 8 / 16 / 32 / 48 columns that holds the current subspace.
template <class K>
static void set_kb(int ncols, K &&f) {
    if (ncols <= 8)
        f(std::integral_constant<int, 8>{});
    else if (ncols <= 16)
        f(std::integral_constant<int, 16>{});
    else if (ncols <= 32)
        f(std::integral_constant<int, 32>{});
    else
        f(std::integral_constant<int, KM>{});
}

static dmrg_status work_alloc(dmrg_plan *plan, int kmax, int kmin, hipStream_t s) {
    DavidsonWork *w = plan->dav;
    if (w && w->kmax == kmax && w->kmin == kmin) return DMRG_OK;
    davidson_free(plan);
    w = new DavidsonWork();
    plan->dav = w;
    w->kmax = kmax;
    w->kmin = kmin;
    DavArgs &A = w->a;
    A.n = plan->n;
    A.nprob = plan->nprob;
    // chunks: at most 2048 elements, never crossing a member boundary
    std::vector<int32_t> cm;
    std::vector<int64_t> cb;
    std::vector<int32_t> mc(1, 0);
    const int64_t CH = TPB;  // one element per thread: many blocks, every column load in flight
    for (int p = 0; p < plan->nprob; ++p) {
        int64_t b = plan->member_off[p], e = plan->member_off[p + 1];
        if (e == b) {  // empty member: one empty chunk keeps the bookkeeping uniform
            cm.push_back(p);
            cb.push_back(b);
        }
        for (int64_t x = b; x < e; x += CH) {
            cm.push_back(p);
            cb.push_back(x);
        }
        mc.push_back((int32_t)cm.size());
    }
    cb.push_back(plan->n);
    A.nchunk = (int)cm.size();
    auto alloc = [&](void **p, size_t bytes) -> dmrg_status {
        DMRG_HIP(hipMalloc(p, std::max<size_t>(bytes, 8)));
        w->owned.push_back(*p);
        return DMRG_OK;
    };
    const size_t n = (size_t)plan->n;
    DMRG_TRY(alloc((void **)&A.V, (kmax + 1) * n * 8));
    DMRG_TRY(alloc((void **)&A.W, (kmax + 1) * n * 8));
    DMRG_TRY(alloc((void **)&A.T, n * 8));
    DMRG_TRY(alloc((void **)&A.D, n * 8));
    DMRG_TRY(alloc((void **)&A.dfold, n * 8));
    DMRG_TRY(alloc((void **)&A.coef, std::max(plan->nterm_total, 1) * 8));
    DMRG_TRY(alloc((void **)&A.part, (size_t)A.nchunk * (KM + 2) * 8));
    DMRG_TRY(alloc((void **)&A.chunk_member, cm.size() * 4));
    DMRG_TRY(alloc((void **)&A.chunk_begin, cb.size() * 8));
    DMRG_TRY(alloc((void **)&A.member_chunk, mc.size() * 4));
    DMRG_TRY(alloc((void **)&A.counter, plan->nprob * 4));
    DMRG_TRY(alloc((void **)&A.nactive, 4));
    DMRG_TRY(alloc((void **)&A.st, plan->nprob * sizeof(DavState)));
    DMRG_TRY(alloc((void **)&A.active, plan->nprob * 4));
    DMRG_HIP(hipHostMalloc((void **)&w->h_nactive, 4, hipHostMallocDefault));
    DMRG_HIP(hipMemcpyAsync(A.chunk_member, cm.data(), cm.size() * 4, hipMemcpyHostToDevice, s));
    DMRG_HIP(hipMemcpyAsync(A.chunk_begin, cb.data(), cb.size() * 8, hipMemcpyHostToDevice, s));
    DMRG_HIP(hipMemcpyAsync(A.member_chunk, mc.data(), mc.size() * 4, hipMemcpyHostToDevice, s));
    DMRG_HIP(hipMemsetAsync(A.st, 0, plan->nprob * sizeof(DavState), s));
    DMRG_HIP(hipMemsetAsync(A.counter, 0, plan->nprob * 4, s));
    DMRG_HIP(hipStreamSynchronize(s));
    return DMRG_OK;
}

dmrg_status davidson_free(dmrg_plan *plan) {
    DavidsonWork *w = plan->dav;
    if (!w) return DMRG_OK;
    for (auto &kv : w->graphs) (void)hipGraphExecDestroy(kv.second);
    for (void *p : w->owned) (void)hipFree(p);
    if (w->h_nactive) (void)hipHostFree(w->h_nactive);
    delete w;
    plan->dav = nullptr;
    return DMRG_OK;
}

// Enqueue `count` iterations starting at subspace size i; returns the next i.
static dmrg_status enqueue_iters(dmrg_plan *plan, int slot, int i, int count, int *i_next, hipStream_t s) {
    DavidsonWork *w = plan->dav;
    const DavArgs &A = w->a;
    const int kmax = w->kmax, kmin = w->kmin;
    const dim3 grid(A.nchunk), block(TPB);
    for (int it = 0; it < count; ++it) {
        const bool restart = (i == kmax);
        set_kb(i, [&](auto kb) {
            constexpr int KB = decltype(kb)::value;
            hipLaunchKernelGGL(k_rayleigh<KB>, grid, block, sizeof(JacobiLds), s, A, i);
            hipLaunchKernelGGL(k_ritz<KB>, grid, block, 0, s, A, i, restart ? 1 : 0);
        });
        int ie = i;
        if (restart) {
            set_kb(i, [&](auto kb) {
                constexpr int KB = decltype(kb)::value;
                hipLaunchKernelGGL(k_restart<KB>, grid, block, 0, s, A, i, kmin);
            });
            ie = kmin;
        }
        set_kb(ie, [&](auto kb) {
            constexpr int KB = decltype(kb)::value;
            hipLaunchKernelGGL(k_orth<KB>, grid, block, 0, s, A, ie);
            hipLaunchKernelGGL(k_append<KB>, grid, block, 0, s, A, ie);
        });
        DMRG_HIP(hipGetLastError());
        DMRG_TRY(launch_project(plan, slot, A.coef, A.V + (int64_t)ie * A.n, A.W + (int64_t)ie * A.n, s, A.active,
                                A.dfold));
        i = ie + 1;
    }
    *i_next = i;
    return DMRG_OK;
}

static dmrg_status run_phase(dmrg_plan *plan, int slot, const double *psi_in, double tol, double floor_,
                             int max_iter, bool use_graph, int chunk, hipStream_t s, int *iters_out) {
    DavidsonWork *w = plan->dav;
    const DavArgs &A = w->a;
    const dim3 grid(A.nchunk), block(TPB);
    hipLaunchKernelGGL(k_set_state, dim3((A.nprob + 63) / 64), dim3(64), 0, s, A, tol, floor_, max_iter);
    hipLaunchKernelGGL(k_init_norm, grid, block, 0, s, psi_in, A);
    hipLaunchKernelGGL(k_init_vec, grid, block, 0, s, psi_in, A);
    DMRG_HIP(hipGetLastError());
    DMRG_TRY(launch_diag_fold(plan, slot, A.coef, A.dfold, s));  // coefficients are fixed for the phase
    DMRG_TRY(launch_project(plan, slot, A.coef, A.V, A.W, s, A.active, A.dfold));
    int i = 1;
    int done = 0;
    while (done < max_iter) {
        int cnt = std::min(chunk, max_iter - done);
        int inext = i;
        if (use_graph) {
            auto key = std::make_tuple(slot, i, cnt, w->kmax);
            auto it = w->graphs.find(key);
            if (it == w->graphs.end()) {
                hipStream_t cs;
                DMRG_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
                hipGraph_t g;
                DMRG_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
                dmrg_status st = enqueue_iters(plan, slot, i, cnt, &inext, cs);
                hipError_t ce = hipStreamEndCapture(cs, &g);
                (void)hipStreamDestroy(cs);
                if (st < 0) return st;
                if (ce != hipSuccess) return set_error(DMRG_E_HIP, "graph capture failed: %s", hipGetErrorString(ce));
                hipGraphExec_t ge;
                hipError_t ie = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
                (void)hipGraphDestroy(g);
                if (ie != hipSuccess)
                    return set_error(DMRG_E_HIP, "graph instantiate failed: %s", hipGetErrorString(ie));
                it = w->graphs.emplace(key, ge).first;
            } else {
                // the subspace sequence is deterministic: recompute the next i
                int ii = i;
                for (int q = 0; q < cnt; ++q) ii = (ii == w->kmax ? w->kmin : ii) + 1;
                inext = ii;
            }
            DMRG_HIP(hipGraphLaunch(it->second, s));
        } else {
            DMRG_TRY(enqueue_iters(plan, slot, i, cnt, &inext, s));
        }
        i = inext;
        done += cnt;
        DMRG_HIP(hipMemcpyAsync(w->h_nactive, A.nactive, 4, hipMemcpyDeviceToHost, s));
        DMRG_HIP(hipStreamSynchronize(s));
        if (*w->h_nactive <= 0) break;
    }
    *iters_out = done;
    return DMRG_OK;
}

}  // namespace dmrg

// ================================================================== ABI

using namespace dmrg;

template <int KB>
__global__ __launch_bounds__(TPB) void k_gemv_t_part(int64_t n, int k, const double *__restrict__ V, int64_t ldv,
                                                     const double *__restrict__ x, double *__restrict__ part) {
    __shared__ double lds[4 * KB];
    double acc[KB];
#pragma unroll
    for (int j = 0; j < KB; ++j) acc[j] = 0.0;
    for (int64_t e = (int64_t)blockIdx.x * TPB + threadIdx.x; e < n; e += (int64_t)gridDim.x * TPB) {
        const double xv = x[e];
#pragma unroll
        for (int j = 0; j < KB; ++j)
            if (j < k) acc[j] += V[(int64_t)j * ldv + e] * xv;
    }
    block_reduce<KB>(acc, k, lds);
    if (threadIdx.x == 0)
        for (int j = 0; j < k; ++j) part[(size_t)blockIdx.x * KB + j] = acc[j];
}

// second stage: all k columns at once, thread t owns column t % k and every
// (TPB / k)-th block from t / k; slots are then added in order (deterministic)
template <int KB>
__global__ __launch_bounds__(TPB) void k_gemv_t_final(int nblk, int k, const double *__restrict__ part,
                                                      double *__restrict__ s) {
    __shared__ double scratch[TPB];
    const int t = threadIdx.x, per = TPB / k, j = t % k, slot = t / k;
    double v = 0.0;
    if (slot < per) {
#pragma unroll 4
        for (int b = slot; b < nblk; b += per) v += part[(size_t)b * KB + j];
    }
    scratch[t] = v;
    __syncthreads();
    if (t < k) {
        double acc = 0.0;
        for (int q = 0; q < per; ++q) acc += scratch[t + q * k];
        s[t] = acc;
    }
}

template <int KB>
__global__ __launch_bounds__(TPB) void k_gemv_n(int64_t n, int k, const double *__restrict__ V, int64_t ldv,
                                                const double *__restrict__ s, double beta, double *__restrict__ y) {
    double sv[KB];
#pragma unroll
    for (int j = 0; j < KB; ++j) sv[j] = (j < k) ? s[j] : 0.0;
    for (int64_t e = (int64_t)blockIdx.x * TPB + threadIdx.x; e < n; e += (int64_t)gridDim.x * TPB) {
        double acc = (beta == 0.0) ? 0.0 : beta * y[e];
#pragma unroll
        for (int j = 0; j < KB; ++j)
            if (j < k) acc += V[(int64_t)j * ldv + e] * sv[j];
        y[e] = acc;
    }
}

// per-device partials of dmrg_gemv_t (kept until the process ends)
struct GemvScratch {
    double *p = nullptr;
    size_t bytes = 0;
};
static std::map<int, GemvScratch> g_gemv_scratch;

extern "C" {

void dmrg_davidson_default_opts(dmrg_davidson_opts *o) {
    if (!o) return;
    o->tol = 1e-10;
    o->kmax = 32;
    o->kmin = 8;
    o->max_iter = 500;
    o->precond_floor = 1e-3;
    o->prec = DMRG_F64;
    o->tol_lowprec = 0.0;
    o->refine = 1;
    o->use_graph = 1;
    o->graph_chunk = 8;
}

dmrg_status dmrg_davidson(dmrg_plan *plan, const double *coef, const dmrg_davidson_opts *opts, double *psi,
                          double *energy, dmrg_davidson_info *info, void *stream) {
    clear_error();
    if (!plan || !psi || (!coef && plan->nterm_total)) return set_error(DMRG_E_INVALID_ARG, "null argument");
    dmrg_davidson_opts o;
    dmrg_davidson_default_opts(&o);
    if (opts) o = *opts;
    if (o.kmax < 2 || o.kmax > KM || o.kmin < 1 || o.kmin >= o.kmax)
        return set_error(DMRG_E_INVALID_ARG, "need 2 <= kmax <= %d and 1 <= kmin < kmax", KM);
    if (!(o.tol > 0.0) || o.max_iter < 1 || !(o.precond_floor > 0.0) || o.graph_chunk < 1)
        return set_error(DMRG_E_INVALID_ARG, "need tol > 0, max_iter >= 1, precond_floor > 0, graph_chunk >= 1");
    if (o.prec != DMRG_F64 && o.prec != plan->prec)
        return set_error(DMRG_E_INVALID_ARG, "precision %d not available in this plan", o.prec);
    int cur = -1;
    DMRG_HIP(hipGetDevice(&cur));
    if (cur != plan->device) return set_error(DMRG_E_INVALID_ARG, "plan belongs to another device");
    hipStream_t s = (hipStream_t)stream;
    // the subspace cannot exceed the smallest member dimension
    int64_t nmin = INT64_MAX;
    for (int p = 0; p < plan->nprob; ++p) nmin = std::min(nmin, plan->member_off[p + 1] - plan->member_off[p]);
    if (nmin < 1) return set_error(DMRG_E_INVALID_ARG, "a member has an empty target sector");
    int kmax = (int)std::min<int64_t>(o.kmax, std::max<int64_t>(nmin, 2));
    int kmin = std::min(o.kmin, kmax - 1);
    DMRG_TRY(work_alloc(plan, kmax, kmin, s));
    DavidsonWork *w = plan->dav;
    const DavArgs &A = w->a;
    if (plan->nterm_total)
        DMRG_HIP(hipMemcpyAsync(A.coef, coef, plan->nterm_total * 8, hipMemcpyDeviceToDevice, s));
    DMRG_TRY(launch_diagonal(plan, A.coef, A.D, s));

    std::vector<DavState> hs(plan->nprob);
    std::vector<int> low_iters(plan->nprob, 0);
    int done = 0;
    const bool two_phase = o.prec != DMRG_F64;
    if (two_phase) {
        double tl = o.tol_lowprec > 0 ? o.tol_lowprec : (o.prec == DMRG_F32 ? 1e-5 : 1e-3);
        tl = std::max(tl, o.tol);
        DMRG_TRY(run_phase(plan, 1, psi, tl, o.precond_floor, o.max_iter, o.use_graph != 0, o.graph_chunk, s,
                           &done));
        set_kb(kmax, [&](auto kb) {  // nvec <= kmax
            constexpr int KB = decltype(kb)::value;
            hipLaunchKernelGGL(k_finalize<KB>, dim3(A.nchunk), dim3(TPB), 0, s, A, psi);
        });
        DMRG_HIP(hipGetLastError());
        DMRG_HIP(hipMemcpyAsync(hs.data(), A.st, plan->nprob * sizeof(DavState), hipMemcpyDeviceToHost, s));
        DMRG_HIP(hipStreamSynchronize(s));
        for (int p = 0; p < plan->nprob; ++p) {
            if (hs[p].bad_start == 1) return set_error(DMRG_E_NONFINITE, "member %d: zero or non-finite start", p);
            low_iters[p] = hs[p].iters;
        }
    }
    std::vector<DavState> low = hs;
    if (!two_phase || o.refine) {
        DMRG_TRY(run_phase(plan, 0, psi, o.tol, o.precond_floor, o.max_iter, o.use_graph != 0, o.graph_chunk, s,
                           &done));
        set_kb(kmax, [&](auto kb) {  // nvec <= kmax
            constexpr int KB = decltype(kb)::value;
            hipLaunchKernelGGL(k_finalize<KB>, dim3(A.nchunk), dim3(TPB), 0, s, A, psi);
        });
        DMRG_HIP(hipGetLastError());
        DMRG_HIP(hipMemcpyAsync(hs.data(), A.st, plan->nprob * sizeof(DavState), hipMemcpyDeviceToHost, s));
        DMRG_HIP(hipStreamSynchronize(s));
    }
    dmrg_status ret = DMRG_OK;
    for (int p = 0; p < plan->nprob; ++p) {
        const DavState &S = hs[p];
        if (S.bad_start == 1) return set_error(DMRG_E_NONFINITE, "member %d: zero or non-finite start vector", p);
        if (S.bad_start == 2) ret = set_error(DMRG_E_NONFINITE, "member %d: non-finite iterate", p);
        if (energy) energy[p] = S.lambda;
        if (info) {
            dmrg_davidson_info &I = info[p];
            I.energy = S.lambda;
            I.residual = S.rnorm;
            I.iterations = S.iters + (two_phase && o.refine ? low_iters[p] : 0);
            I.iterations_low = two_phase ? low_iters[p] : 0;
            I.projections = S.nproj + 1 + (two_phase && o.refine ? low[p].nproj + 1 : 0);
            I.restarts = S.restarts + (two_phase && o.refine ? low[p].restarts : 0);
            I.converged = S.converged;
            I.breakdown = S.breakdown;
        }
        if (S.breakdown && ret == DMRG_OK)
            ret = set_error(DMRG_E_BREAKDOWN, "member %d: correction vanished after orthogonalization", p);
        else if (!S.converged && ret == DMRG_OK)
            ret = set_error(DMRG_W_NOT_CONVERGED, "member %d: not converged (residual %.3e)", p, S.rnorm);
    }
    return ret;
}

dmrg_status dmrg_gemv_t(int64_t n, int32_t k, const double *V, int64_t ldv, const double *x, double *s,
                        void *stream) {
    clear_error();
    if (n < 1 || k < 1 || k > 64 || ldv < n || !V || !x || !s)
        return set_error(DMRG_E_INVALID_ARG, "need n >= 1, 1 <= k <= 64, ldv >= n and non-null pointers");
    int nblk = (int)std::min<int64_t>((n + TPB - 1) / TPB, 1024);
    size_t need = (size_t)nblk * 64 * 8;
    int dev = 0;
    DMRG_HIP(hipGetDevice(&dev));
    GemvScratch &gs = g_gemv_scratch[dev];
    if (need > gs.bytes) {
        // the stream may still use the old buffer: let it finish before freeing
        DMRG_HIP(hipStreamSynchronize((hipStream_t)stream));
        if (gs.p) (void)hipFree(gs.p);
        gs.p = nullptr;
        gs.bytes = 0;
        DMRG_HIP(hipMalloc((void **)&gs.p, need));
        gs.bytes = need;
    }
    double *part = gs.p;
    hipStream_t st = (hipStream_t)stream;
    auto go = [&](auto kb) {
        constexpr int KB = decltype(kb)::value;
        hipLaunchKernelGGL(k_gemv_t_part<KB>, dim3(nblk), dim3(TPB), 0, st, n, k, V, ldv, x, part);
        hipLaunchKernelGGL(k_gemv_t_final<KB>, dim3(1), dim3(TPB), 0, st, nblk, k, (const double *)part, s);
    };
    if (k <= 16)
        go(std::integral_constant<int, 16>{});
    else if (k <= 32)
        go(std::integral_constant<int, 32>{});
    else
        go(std::integral_constant<int, 64>{});
    DMRG_HIP(hipGetLastError());
    return DMRG_OK;
}

dmrg_status dmrg_gemv_n(int64_t n, int32_t k, const double *V, int64_t ldv, const double *s, double beta,
                        double *y, void *stream) {
    clear_error();
    if (n < 1 || k < 1 || k > 64 || ldv < n || !V || !s || !y)
        return set_error(DMRG_E_INVALID_ARG, "need n >= 1, 1 <= k <= 64, ldv >= n and non-null pointers");
    int nblk = (int)std::min<int64_t>((n + TPB - 1) / TPB, 8192);
    hipStream_t st = (hipStream_t)stream;
    auto go = [&](auto kb) {
        constexpr int KB = decltype(kb)::value;
        hipLaunchKernelGGL(k_gemv_n<KB>, dim3(nblk), dim3(TPB), 0, st, n, k, V, ldv, s, beta, y);
    };
    if (k <= 16)
        go(std::integral_constant<int, 16>{});
    else if (k <= 32)
        go(std::integral_constant<int, 32>{});
    else
        go(std::integral_constant<int, 64>{});
    DMRG_HIP(hipGetLastError());
    return DMRG_OK;
}

}  // extern "C"
