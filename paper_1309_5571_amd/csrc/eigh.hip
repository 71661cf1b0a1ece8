// Eigen-decomposition of symmetric blocks (Alg. 1, step 6: the eigenvalues of
// each block's density matrix decide which states the block keeps).
// One workgroup per block, two methods by order d:
//
// d <= 8: cyclic two-sided Jacobi in LDS with the round-robin ("circle")
// ordering: each round pairs every index with one other, the d/2 plane
// rotations J of a round are independent, so all of them are found together
// and then applied at once, A <- J^T A J and V <- V J.  With the indices
// grouped by pair, A splits into 2x2 sub-blocks A_kl (rows of pair k, columns
// of pair l) that transform on their own, J_k^T A_kl J_l, so each thread takes
// whole sub-blocks.  A sweep is d - 1 rounds (every pair once); the method
// stops after a sweep with no rotation.
//
// 8 < d <= 2048: Householder reduction to tridiagonal form T = Q^T A Q, the
// matrix Q formed explicitly, then T's eigenpairs.  The reduction and the
// formation of Q are whole-workgroup passes over the block (in global memory,
// where it stays cache-resident).  Orders up to 512: Cuppen's divide and
// conquer on T (leaves of at most 16 by implicit QL, one wavefront each;
// merges by deflation, the secular equation on a group of lanes per root and
// Gu and Eisenstat's recomputed weights), then the eigenvectors of the block
// as Q times those of T.  Larger orders: the implicit QL iteration with
// Wilkinson's shift on T (the tql2 procedure of Bowdler, Martin, Reinsch and
// Wilkinson), whose plane rotations are applied to the columns of Q: the QL
// recurrence is sequential and runs on one lane, writing each sweep's
// rotations to LDS, which the whole workgroup then applies to the rows of Q
// (Q is stored column-major, so a rotation of columns i, i+1 is a coalesced
// read of two columns).
#include <hip/hip_runtime.h>

#include "internal.h"
#include "lanes.h"

namespace dmrg {

constexpr int EIG_TPB = 256;        // selection kernel
constexpr int EIG_TPB_SMALL = 512;  // Jacobi, blocks in LDS (a round has ~d^2/2 independent items)
constexpr int EIG_LDS_DIM = 8;  // largest order of the Jacobi kernel (larger ones are faster on the tridiagonal path)
constexpr int EIG_MAX_DIM = 2048;
constexpr int EIG_MAX_SWEEPS = 40;
constexpr int TRI_TPB = 1024;  // tridiagonal path
constexpr int TRI_WAVES = TRI_TPB / 64;
constexpr int QL_MAXIT = 60;  // QL iterations per eigenvalue before the block is reported unconverged

// Pair k of round r of the circle ordering on n' = m + 1 (even) indices:
// k = 0 pairs r with the fixed index m, k > 0 pairs r + k with r - k (mod m).
__device__ __forceinline__ void circle_pair(int r, int k, int m, int &p, int &q) {
    if (k == 0) {
        p = r;
        q = m;
    } else {
        p = (r + k) % m;
        q = (r - k + m) % m;
    }
}

__global__ __launch_bounds__(EIG_TPB_SMALL) void k_eigh_jacobi(int nblk, const int64_t *__restrict__ off,
                                                               const int32_t *__restrict__ dim,
                                                               const int64_t *__restrict__ woff, double *__restrict__ a,
                                                               double *__restrict__ w, double *__restrict__ u,
                                                               int32_t *__restrict__ info) {
    constexpr int NP = EIG_LDS_DIM / 2;  // pairs per round
    constexpr int NT = EIG_TPB_SMALL;
    __shared__ double A[EIG_LDS_DIM * (EIG_LDS_DIM + 1)];
    __shared__ double V[EIG_LDS_DIM * EIG_LDS_DIM];
    __shared__ double rc[NP], rs[NP];
    __shared__ int rp[NP], rq[NP], rf[NP];
    __shared__ double part[NT];
    __shared__ double diag[EIG_LDS_DIM];
    const int b = blockIdx.x;
    if (b >= nblk) return;
    const int d = dim[b];
    const int tid = threadIdx.x;
    if (d < 1 || d > EIG_MAX_DIM) {
        if (tid == 0 && info) info[b] = -1;  // unsupported order
        return;
    }
    if (d > EIG_LDS_DIM) return;  // the tridiagonal kernel's block
    const double *in = a + off[b];
    double *out = u + off[b];
    const int lda = d + 1;
    double fro = 0.0;
    for (int e = tid; e < d * d; e += NT) fro += in[e] * in[e];
    part[tid] = fro;
    __syncthreads();
    if (tid == 0) {
        double s = 0.0;
        for (int i = 0; i < NT; ++i) s += part[i];
        part[0] = sqrt(s);
    }
    __syncthreads();
    // rotations below this size are skipped: the off-diagonal part left is
    // at the rounding level of the matrix norm
    const double thr = part[0] * 0x1p-53 / d;
    for (int e = tid; e < d * d; e += NT) {
        const int r = e / d, c = e % d;
        A[r * lda + c] = in[e];
        V[r * d + c] = (r == c) ? 1.0 : 0.0;
    }
    __syncthreads();
    const int m = d + (d & 1) - 1;  // rounds per sweep; index m is a dummy when d is odd
    const int np = (m + 1) / 2;
    int sweep = 0;
    bool done = false;
    for (; sweep < EIG_MAX_SWEEPS && !done; ++sweep) {
        int rotated = 0;
        for (int r = 0; r < m; ++r) {
            int any = 0;
            for (int k = tid; k < np; k += NT) {
                int p, q;
                circle_pair(r, k, m, p, q);
                double c = 1.0, s = 0.0;
                bool rot = false;
                if (p < d && q < d) {
                    const double apq = A[p * lda + q];
                    if (fabs(apq) > thr) {
                        const double app = A[p * lda + p], aqq = A[q * lda + q];
                        const double tau = (aqq - app) / (2.0 * apq);
                        // the smaller root of t^2 + 2 tau t - 1 = 0 (rotation angle <= pi/4)
                        const double t = fabs(tau) > 1e150 ? 0.5 / tau
                                                            : (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
                        c = 1.0 / sqrt(1.0 + t * t);
                        s = t * c;
                        rot = true;
                    }
                }
                rc[k] = c;
                rs[k] = s;
                rp[k] = p;
                rq[k] = q;
                rf[k] = rot;
                any |= rot;
            }
            any = __syncthreads_or(any);
            if (!any) continue;
            rotated = 1;
            // A_kl <- J_k^T A_kl J_l for every pair of pairs; the rotated
            // element of a pair (k == l) is zero in exact arithmetic and is set
            // so (its rounding residue would otherwise be rotated again)
            for (int it = tid; it < np * np; it += NT) {
                const int k = it / np, l = it - k * np;
                if (!rf[k] && !rf[l]) continue;
                const int pk = rp[k], qk = rq[k], pl = rp[l], ql = rq[l];
                const bool vpk = pk < d, vqk = qk < d, vpl = pl < d, vql = ql < d;
                const int ipp = (vpk && vpl) ? pk * lda + pl : 0, ipq = (vpk && vql) ? pk * lda + ql : 0;
                const int iqp = (vqk && vpl) ? qk * lda + pl : 0, iqq = (vqk && vql) ? qk * lda + ql : 0;
                double xpp = A[ipp], xpq = A[ipq], xqp = A[iqp], xqq = A[iqq];
                xpp = (vpk && vpl) ? xpp : 0.0;
                xpq = (vpk && vql) ? xpq : 0.0;
                xqp = (vqk && vpl) ? xqp : 0.0;
                xqq = (vqk && vql) ? xqq : 0.0;
                const double ck = rc[k], sk = rs[k], cl = rc[l], sl = rs[l];
                const double tpp = ck * xpp - sk * xqp, tpq = ck * xpq - sk * xqq;  // rows (pair k)
                const double tqp = sk * xpp + ck * xqp, tqq = sk * xpq + ck * xqq;
                double ypp = cl * tpp - sl * tpq, ypq = sl * tpp + cl * tpq;  // columns (pair l)
                double yqp = cl * tqp - sl * tqq, yqq = sl * tqp + cl * tqq;
                if (k == l) ypq = yqp = 0.0;
                if (vpk && vpl) A[ipp] = ypp;
                if (vpk && vql) A[ipq] = ypq;
                if (vqk && vpl) A[iqp] = yqp;
                if (vqk && vql) A[iqq] = yqq;
            }
            // V <- V J: columns p, q of every rotated pair
            for (int it = tid; it < d * np; it += NT) {
                const int i = it / np, l = it - i * np;
                if (!rf[l]) continue;
                const int pl = rp[l], ql = rq[l];
                const double cl = rc[l], sl = rs[l];
                const double vp = V[i * d + pl], vq = V[i * d + ql];
                V[i * d + pl] = cl * vp - sl * vq;
                V[i * d + ql] = sl * vp + cl * vq;
            }
            __syncthreads();
        }
        done = !rotated;
    }
    // eigenvalues in descending order (ties by index), eigenvectors with the
    // first entry of largest magnitude positive
    for (int i = tid; i < d; i += NT) diag[i] = A[i * lda + i];
    __syncthreads();
    double *wb = w + woff[b];
    for (int i = tid; i < d; i += NT) {
        const double wi = diag[i];
        int rank = 0;
        for (int j = 0; j < d; ++j) {
            const double wj = diag[j];
            rank += (wj > wi) || (wj == wi && j < i);
        }
        int kmax = 0;
        double vmax = -1.0;
        for (int r = 0; r < d; ++r) {
            const double av = fabs(V[r * d + i]);
            if (av > vmax) {
                vmax = av;
                kmax = r;
            }
        }
        const double sg = V[kmax * d + i] < 0.0 ? -1.0 : 1.0;
        wb[rank] = wi;
        for (int r = 0; r < d; ++r) out[r * d + rank] = sg * V[r * d + i];
    }
    if (tid == 0 && info) info[b] = done ? sweep : -2;
}

// Sum over the workgroup of one value per thread, and the value `lead` of
// thread 0, both returned to every thread (the same total in every thread).
// Two barriers: after it, every thread may overwrite what the block read before.
__device__ __forceinline__ double block_sum_lead(double x, double lead, double *red, double *lead_out) {
    x = group_sum<64>(x);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0) red[wv] = x;
    if (threadIdx.x == 0) red[TRI_WAVES] = lead;
    __syncthreads();
    double t = 0.0;
    for (int i = 0; i < TRI_WAVES; ++i) t += red[i];
    *lead_out = red[TRI_WAVES];
    __syncthreads();
    return t;
}

// Sum over the workgroup with one barrier, and the value `lead` of the thread
// where `own` holds, to every thread: the caller alternates two buffers of
// TRI_WAVES + 1, so that a buffer is rewritten only after another barrier
__device__ __forceinline__ double block_sum1(double x, bool own, double lead, double *buf, double *lead_out) {
    x = group_sum<64>(x);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0) buf[wv] = x;
    if (own) buf[TRI_WAVES] = lead;
    __syncthreads();
    double t = 0.0;
    for (int i = 0; i < TRI_WAVES; ++i) t += buf[i];
    *lead_out = buf[TRI_WAVES];
    return t;
}

// sqrt(x^2 + y^2) without overflow or harmful underflow
__device__ __forceinline__ double hyp(double x, double y) {
    const double ax = fabs(x), ay = fabs(y);
    const double mx = fmax(ax, ay), mn = fmin(ax, ay);
    if (mx == 0.0) return 0.0;
    if (mx > 0x1p-500 && mx < 0x1p+500) return sqrt(x * x + y * y);
    const double q = mn / mx;
    return mx * sqrt(1.0 + q * q);
}

constexpr int TRI_UB = 16;  // rows of a column read per batch of loads (Householder step)
constexpr int QL_B = 8;     // rotations applied per batch of loads (QL; the next batch is fetched ahead)
constexpr int Q_REG = 8;    // column entries per lane kept in registers (Q formation, L <= 512)
constexpr int QB = 16;      // factors per block of the Q formation (their vectors: QB x 512 doubles of LDS)
constexpr int HH_ROWS = 36;     // rows of the block per thread (Householder reduction in registers, orders 129..)
constexpr int HH_REG_DIM = 180; // largest order reduced in registers (five groups of HH_ROWS rows)
constexpr int HH_VEC = 256;     // LDS vectors of that reduction: past the order up to the last group's end
static_assert(TRI_WAVES == 16 && 5 * HH_ROWS >= HH_REG_DIM && 8 * 16 >= 128 && 16 * 4 >= 64, "register rows");
static_assert(HH_REG_DIM + HH_ROWS <= HH_VEC && HH_REG_DIM <= 192, "register reduction vectors");

// ------------------------------------------------------------------ divide and conquer
// The symmetric tridiagonal eigenproblem of orders up to DC_MAX by Cuppen's
// divide and conquer (eigenvectors by Gu and Eisenstat's recomputed weights):
// T is torn at the boundaries of a bisection tree, T = blockdiag(T_i) + sum
// |e_b| v_b v_b^T (v_b = e_{b-1} + sign(e_b) e_b, the torn diagonals reduced by
// |e_b|); the leaves (at most DC_LEAF) are solved by implicit QL, one wavefront
// each; then the tree is merged bottom-up.  A merge of two solved halves is the
// rank-one eigenproblem D + rho z z^T (z: the last row of the left half's
// eigenvectors and the first row of the right half's): deflation of
// negligible weights and of nearly equal poles (a plane rotation), the roots
// of the secular equation 1 + rho sum z_i^2 / (d_i - lambda) = 0 from the
// nearer pole (a group of lanes per root: a two-pole rational model,
// bracketed), the weights recomputed from the roots, and the rows of the
// merged block of eigenvectors multiplied by the merge's eigenvector matrix
// (two rows per wavefront, in place).
constexpr int DC_MAX = 512;
constexpr int DC_LEAF = 16;
constexpr int DC_ITMAX = 100;  // root-finder steps per root (they end at the resolution, typically after 3-8)

// Product over aligned groups of G lanes (G a power of two, 1 <= G <= 64), the
// same bits on every lane of a group (as group_sum); all lanes active
template <int G>
__device__ __forceinline__ double group_prod(double v) {
    if (G >= 2) v *= dpp_f64<DPP_XOR1>(v);
    if (G >= 4) v *= dpp_f64<DPP_XOR2>(v);
    if (G >= 8) v *= dpp_f64<DPP_HALF_MIRROR>(v);
    if (G >= 16) v *= dpp_f64<DPP_MIRROR>(v);
    if (G == 32) v *= __shfl_xor(v, 16, 64);
    if (G == 64) v = (readlane_f64(v, 0) * readlane_f64(v, 16)) * (readlane_f64(v, 32) * readlane_f64(v, 48));
    return v;
}
__device__ __forceinline__ double group_prod(double v, int G) {
    switch (G) {
    case 1: return v;
    case 2: return group_prod<2>(v);
    case 4: return group_prod<4>(v);
    case 8: return group_prod<8>(v);
    case 16: return group_prod<16>(v);
    case 32: return group_prod<32>(v);
    default: return group_prod<64>(v);
    }
}

// LDS writes of a wavefront's lanes are visible to its other lanes after it
__device__ __forceinline__ void wave_sync_lds() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// 1/x: the hardware reciprocal refined by one Newton step
__device__ __forceinline__ double rcpd(double x) {
    const double r = __builtin_amdgcn_rcp(x);
    return fma(fma(-x, r, 1.0), r, r);
}
constexpr int DC_NLEAF = 32;    // most leaves: orders <= DC_MAX need at most 2^5 of at most DC_LEAF
constexpr int DC_STAGE = 224;   // LDS staging of a row per wavefront (the pool's last 16 x 224)
static_assert((DC_MAX + DC_NLEAF - 1) / DC_NLEAF <= DC_LEAF, "leaf count");
// the pool (5 EIG_MAX_DIM doubles) holds the leaves, then the scratch of a merge
static_assert(DC_NLEAF * DC_LEAF * (DC_LEAF + 1) + TRI_WAVES * (2 * DC_LEAF + 2) <= 5 * EIG_MAX_DIM, "leaf scratch");
static_assert(13 * DC_MAX + 16 * DC_STAGE <= 5 * EIG_MAX_DIM, "merge scratch");
static_assert(QB * 64 * Q_REG <= 4 * EIG_MAX_DIM, "Q formation: factor vectors in the pool past the factors' t");

// Implicit QL (as the large-order path) on a leaf of order m <= DC_LEAF, one
// wavefront: d (LDS, length m) becomes its eigenvalues, e (length m,
// e[m-1] = 0) is destroyed, Zl (row-major m x m, LDS, row stride DC_LEAF) its
// eigenvectors.  Lane 0 runs each iteration's chase and leaves its rotations
// in rot (cosines, then sines, by index); then lane r applies them, in the
// chase's order, to row r of Zl.  wctl: four ints of LDS.  Every lane returns
// the iteration count, or -1 if an eigenvalue needed more than QL_MAXIT.
__device__ __forceinline__ int ql_leaf(int m, double *d, double *e, double *Zl, double *rot, int *wctl) {
    const int lane = threadIdx.x & 63;
    for (int i = lane; i < m * DC_LEAF; i += 64) Zl[i] = i / DC_LEAF == i % DC_LEAF ? 1.0 : 0.0;
    double *rc = rot, *rs = rot + DC_LEAF;
    int l = 0, it_l = 0, its = 0;
    double tol = 0.0;
    if (lane == 0) {
        double anorm = 0.0;
        for (int i = 0; i < m; ++i) anorm = fmax(anorm, fabs(d[i]) + fabs(e[i]) + (i ? fabs(e[i - 1]) : 0.0));
        tol = anorm * 0x1p-53;
    }
    for (;;) {
        if (lane == 0) {
            // the next iteration: status 0 and the rotation range [lo, hi], 1 when
            // every eigenvalue has converged, -1 when one did not
            int status = 1, lo = 0, hi = -1;
            while (l < m) {
                int mm = l;
                while (mm < m - 1 && fabs(e[mm]) > tol) ++mm;
                if (mm == l) {
                    ++l;
                    it_l = 0;
                    continue;
                }
                if (it_l >= QL_MAXIT) {
                    status = -1;
                    break;
                }
                ++it_l;
                ++its;
                double g = (d[l + 1] - d[l]) / (2.0 * e[l]);
                double r = hyp(g, 1.0);
                g = d[mm] - d[l] + e[l] / (g + copysign(r, g));
                double s = 1.0, c = 1.0, p = 0.0;
                bool early = false;
                int i = mm - 1;
                for (; i >= l; --i) {
                    const double f = s * e[i], bb = c * e[i];
                    r = hyp(f, g);
                    e[i + 1] = r;
                    if (r == 0.0) {
                        d[i + 1] -= p;
                        e[mm] = 0.0;
                        early = true;
                        break;
                    }
                    s = f / r;
                    c = g / r;
                    g = d[i + 1] - p;
                    r = (d[i] - g) * s + 2.0 * c * bb;
                    p = s * r;
                    d[i + 1] = g + p;
                    g = c * r - bb;
                    rc[i] = c;
                    rs[i] = s;
                }
                if (!early) {
                    d[l] -= p;
                    e[l] = g;
                    e[mm] = 0.0;
                }
                status = 0;
                lo = i + 1;  // (l when the chase ran through)
                hi = mm - 1;
                break;
            }
            wctl[0] = status;
            wctl[1] = lo;
            wctl[2] = hi;
            wctl[3] = its;
        }
        wave_sync_lds();
        const int status = wctl[0], lo = wctl[1], hi = wctl[2];
        if (status != 0) {
            const int n_its = wctl[3];
            wave_sync_lds();  // (wctl is rewritten by the next leaf of this wavefront)
            return status < 0 ? -1 : n_its;
        }
        if (lane < m) {
            double *zr = Zl + lane * DC_LEAF;
            for (int i = hi; i >= lo; --i) {
                const double c = rc[i], s = rs[i], h = zr[i + 1];
                zr[i + 1] = s * zr[i] + c * h;
                zr[i] = c * zr[i] - s * h;
            }
        }
        wave_sync_lds();  // the next chase rewrites rc, rs
    }
}

// Scratch of one merge (LDS, carved from the pool): doubles of length DC_MAX
struct DcScratch {
    double *zz, *ds, *rc, *rs, *delta, *zeta, *tau, *zhat, *invn, *lamn;
    double *stage;  // [TRI_WAVES][DC_STAGE]: one row's weighted entries per wavefront
    int *perm, *defl, *rj, *ri, *nd, *tmp, *org;
};

// Merge of the solved halves [lo, mid) and [mid, hi) coupled by rho.  Zt:
// column-major n x n eigenvectors of T (rows and columns of the block only).
__device__ __forceinline__ void dc_merge(int n, int lo, int mid, int hi, double rho, double *sd, double *Zt, const DcScratch &S,
                         double *red, int *ctl) {
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const size_t N = (size_t)n;
    const int m = hi - lo;
    // z: row mid - 1 of the left half's eigenvectors, row mid of the right half's
    double part = 0.0;
    for (int c = tid; c < m; c += TRI_TPB) {
        const int col = lo + c;
        double v = col < mid ? Zt[col * N + (mid - 1)] : Zt[col * N + mid];
        if (col >= mid && rho < 0.0) v = -v;
        S.zz[c] = v;
        part += v * v;
    }
    double unused;
    const double nz2 = block_sum_lead(part, 0.0, red, &unused);
    const double rh = fabs(rho) * nz2;  // rho of the normalized z
    if (!(rh > 0.0)) return;            // no coupling: the halves are already solved
    const double inz = 1.0 / sqrt(nz2);
    // ascending order of the poles (ties by index)
    for (int c = tid; c < m; c += TRI_TPB) {
        const double x = sd[lo + c];
        int rk = 0;
        for (int j = 0; j < m; ++j) {
            const double y = sd[lo + j];
            rk += (y < x) || (y == x && j < c);
        }
        S.perm[rk] = c;
    }
    __syncthreads();
    for (int t = tid; t < m; t += TRI_TPB) {
        S.ds[t] = sd[lo + S.perm[t]];
        S.zeta[t] = S.zz[S.perm[t]] * inz;  // (zeta used as the sorted z during deflation)
    }
    __syncthreads();
    // deflation (one thread, in pole order): a negligible weight leaves its pole;
    // two poles closer than the resolution are rotated so that one weight vanishes.
    // The poles and weights are read eight at a time; the pole kept from the last
    // step (prev) is carried in registers, and the rotation test |(d_t - d_p) c s|
    // <= tol is taken as |d_t - d_p| |z_t z_p| <= tol (z_p^2 + z_t^2) (no root: the
    // weights left are above tol / rh >= 8u, so the squares do not underflow).  A
    // pole joins the list of kept ones once the next one can no longer deflate it.
    if (tid == 0) {
        double *zs = S.zeta, *ds = S.ds;
        const double tol = 8.0 * 0x1p-53 * fmax(fmax(fabs(ds[0]), fabs(ds[m - 1])), rh);
        int nrot = 0, prev = -1, k = 0;
        double zp = 0.0, dp = 0.0;  // weight and pole of prev
        for (int t0 = 0; t0 < m; t0 += 8) {
            double zb[8], db[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int t = min(t0 + u, m - 1);
                zb[u] = zs[t];
                db[u] = ds[t];
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int t = t0 + u;
                if (t >= m) break;
                double zt = zb[u], dt = db[u];
                if (rh * fabs(zt) <= tol) {
                    S.defl[t] = 1;
                    continue;
                }
                S.defl[t] = 0;
                bool rotated = false;
                if (prev >= 0 && fabs(dt - dp) * fabs(zt * zp) <= tol * (zp * zp + zt * zt)) {
                    const double tt = hyp(zp, zt);
                    const double c = zt / tt, sn = -zp / tt;
                    const double dpn = dp * c * c + dt * sn * sn;
                    const double dtn = dp * sn * sn + dt * c * c;
                    zs[t] = tt;
                    zs[prev] = 0.0;
                    ds[prev] = dpn;
                    ds[t] = dtn;
                    S.rj[nrot] = prev;
                    S.ri[nrot] = t;
                    S.rc[nrot] = c;
                    S.rs[nrot] = sn;
                    ++nrot;
                    S.defl[prev] = 1;
                    zt = tt;
                    dt = dtn;
                    rotated = true;
                }
                if (prev >= 0 && !rotated) S.tmp[k++] = prev;  // prev is final
                prev = t;
                zp = zt;
                dp = dt;
            }
        }
        if (prev >= 0) S.tmp[k++] = prev;
        ctl[0] = k;
        ctl[1] = nrot;
    }
    __syncthreads();
    const int k = ctl[0], nrot = ctl[1];
    // the non-deflated poles in ascending order (a rotation may move one by a rounding)
    for (int j = tid; j < k; j += TRI_TPB) {
        const double x = S.ds[S.tmp[j]];
        int rk = 0;
        for (int i = 0; i < k; ++i) {
            const double y = S.ds[S.tmp[i]];
            rk += (y < x) || (y == x && i < j);
        }
        S.nd[rk] = S.tmp[j];
    }
    __syncthreads();
    for (int j = tid; j < k; j += TRI_TPB) {
        S.delta[j] = S.ds[S.nd[j]];
        S.zz[j] = S.zeta[S.nd[j]];  // zz: the weights of the non-deflated poles
    }
    __syncthreads();
    // roots of the secular equation: root j lies between delta[j] and delta[j+1]
    // (the last one below delta[k-1] + rh sum z^2), in coordinates centred on
    // the nearer pole.  Each step fits the sums over the poles below and above
    // the gap with one pole each (value and slope at the iterate) and moves to
    // the root of that model; a step that leaves the bracket bisects instead.
    // G lanes per root (aligned groups inside a wavefront) split the sums over
    // the poles and combine them with group sums, so every lane of a group
    // holds the same values and takes the same steps; a wavefront iterates
    // until all of its roots have stopped, finished roots keeping their value.
    const double *dl = S.delta, *zw = S.zz;
    int G = 64;
    while (G > 1 && G * k > TRI_TPB) G >>= 1;
    if (64 * wv < G * k) {  // wavefronts past the last root's group have nothing to do
        const int g = lane & (G - 1), jr = tid / G, j = min(jr, k - 1);
        double part = 0.0;
        for (int i = g; i < k; i += G) part += zw[i] * zw[i];
        const double zsum = group_sum(part, G);
        const bool last = j + 1 == k;
        const double lo_d = dl[j], hi_d = last ? dl[j] + rh * zsum : dl[j + 1];
        const double half = 0.5 * (hi_d - lo_d);
        part = 0.0;
        for (int i = g; i < k; i += G) part += zw[i] * zw[i] * rcpd(dl[i] - (lo_d + half));
        const double f = 1.0 + rh * group_sum(part, G);
        int o;
        double a, bnd;
        if (last || f >= 0.0) {
            o = j;
            a = 0.0;
            bnd = last ? hi_d - lo_d : half;
        } else {
            o = j + 1;
            a = -half;
            bnd = 0.0;
        }
        const double dorg = dl[o];
        const double dj = dl[j] - dorg, dj1 = last ? 0.0 : dl[j + 1] - dorg;
        double x = 0.5 * (a + bnd);
        bool done = false;
        for (int it = 0; it < DC_ITMAX; ++it) {
            if (__builtin_amdgcn_ballot_w64(!done) == 0) break;  // every root of the wavefront has stopped
            double psi = 0.0, dpsi = 0.0, phi = 0.0, dphi = 0.0;
            for (int i = g; i < k; i += G) {
                const double r = rcpd((dl[i] - dorg) - x);
                const double t = zw[i] * zw[i] * r;
                const bool below = i <= j;
                psi += below ? t : 0.0;
                dpsi += below ? t * r : 0.0;
                phi += below ? 0.0 : t;
                dphi += below ? 0.0 : t * r;
            }
            psi = group_sum(psi, G);
            dpsi = group_sum(dpsi, G);
            phi = group_sum(phi, G);
            dphi = group_sum(dphi, G);
            if (done) continue;
            const double fx = 1.0 + rh * (psi + phi);
            if (fx > 0.0)
                bnd = x;
            else
                a = x;
            const double err = 8.0 * 0x1p-53 * (1.0 + rh * (fabs(psi) + fabs(phi)) + fabs(x) * rh * (dpsi + dphi));
            if (fabs(fx) <= err || bnd - a <= 2.0 * 0x1p-53 * fmax(fabs(a), fabs(bnd))) {
                done = true;
                continue;
            }
            const double u = dj - x, qq = dpsi * u * u, pp = psi - dpsi * u;
            double xn;
            if (!last) {
                const double v = dj1 - x, ss = dphi * v * v, rr = phi - dphi * v;
                const double C = 1.0 + rh * (pp + rr), A1 = rh * qq, A2 = rh * ss;
                // C (u - eta)(v - eta) + A1 (v - eta) + A2 (u - eta) = 0, root inside the gap
                const double qb = -(C * (u + v) + A1 + A2), qc = C * u * v + A1 * v + A2 * u;
                double eta;
                if (C == 0.0) {
                    eta = -qc / qb;
                } else {
                    const double sq = sqrt(fmax(qb * qb - 4.0 * C * qc, 0.0));
                    const double q1 = -0.5 * (qb + copysign(sq, qb));
                    const double e1 = q1 / C, e2 = q1 != 0.0 ? qc / q1 : e1;
                    eta = (dj < x + e1 && x + e1 < dj1) ? e1 : e2;
                }
                xn = x + eta;
            } else {
                const double C = 1.0 + rh * (pp + phi);
                xn = C != 0.0 ? dj + rh * qq / C : bnd;
            }
            x = (a < xn && xn < bnd) ? xn : 0.5 * (a + bnd);
        }
        if (jr < k && g == 0) {
            S.org[j] = o;
            S.tau[j] = x;
        }
    }
    __syncthreads();
    // weights recomputed from the roots (their signs kept), then the norms of
    // the eigenvectors zhat_i / (delta_i - lambda_j); G lanes per weight (per
    // norm) split the product (the sum) over the poles, as for the roots
    if (64 * wv < G * k) {
        const int g = lane & (G - 1), ir = tid / G, i = min(ir, k - 1);
        double prod = 1.0;
        for (int j = g; j < k; j += G)
            if (j != i) prod *= ((dl[S.org[j]] - dl[i]) + S.tau[j]) * rcpd(dl[j] - dl[i]);
        prod = group_prod(prod, G) * (((dl[S.org[i]] - dl[i]) + S.tau[i]) / rh);
        if (ir < k && g == 0) S.zhat[i] = copysign(sqrt(fmax(prod, 0.0)), zw[i]);
    }
    __syncthreads();
    if (64 * wv < G * k) {
        const int g = lane & (G - 1), jr = tid / G, j = min(jr, k - 1);
        const double dj = dl[S.org[j]], tj = S.tau[j];
        double q = 0.0;
        for (int i = g; i < k; i += G) {
            const double x = S.zhat[i] * rcpd((dl[i] - dj) - tj);
            q += x * x;
        }
        q = group_sum(q, G);
        if (jr < k && g == 0) {
            S.invn[j] = 1.0 / sqrt(q);
            S.lamn[j] = dj + tj;
        }
    }
    __syncthreads();
    // the deflation rotations on the columns of the block (in pole order)
    for (int q = 0; q < nrot; ++q) {
        const size_t cj = (size_t)(lo + S.perm[S.rj[q]]) * N, ci = (size_t)(lo + S.perm[S.ri[q]]) * N;
        const double c = S.rc[q], sn = S.rs[q];
        for (int r = lo + tid; r < hi; r += TRI_TPB) {
            const double yj = Zt[cj + r], yi = Zt[ci + r];
            Zt[cj + r] = c * yj + sn * yi;
            Zt[ci + r] = c * yi - sn * yj;
        }
        __syncthreads();
    }
    // rows of the block times the merge's eigenvectors: slot t of the block takes
    // pole t (in pole order); a deflated slot keeps its column, the slot of the
    // non-deflated pole nd[j] gets root j's eigenvector.  One wavefront per two
    // rows: their weighted entries y_i zhat_i are staged in LDS and read by every
    // lane, each lane accumulating the outputs of its roots j = lane + 64 q, one
    // reciprocal serving both rows.
    constexpr int NQ = DC_MAX / 64;
    constexpr int CH = DC_STAGE / 2;  // entries of each row per staging round
    double djr[NQ], tjr[NQ];  // origin pole and offset of this lane's roots
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        const int j = lane + 64 * q;
        djr[q] = j < k ? dl[S.org[j]] : 0.0;
        tjr[q] = j < k ? S.tau[j] : -1.0;  // (past k: a finite, unused difference)
    }
    double *st = S.stage + wv * DC_STAGE;  // [CH][2]
    for (int r = lo + 2 * wv; r < hi; r += 2 * TRI_WAVES) {
        const bool two = r + 1 < hi;  // uniform
        double yd[2][NQ], acc[2][NQ];
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            const int t = lane + 64 * q;
            acc[0][q] = acc[1][q] = 0.0;
            yd[0][q] = (64 * q < m && t < m) ? Zt[(size_t)(lo + S.perm[t]) * N + r] : 0.0;
            yd[1][q] = (two && 64 * q < m && t < m) ? Zt[(size_t)(lo + S.perm[t]) * N + r + 1] : 0.0;
        }
        for (int c0 = 0; c0 < k; c0 += CH) {
            const int cnt = min(CH, k - c0);
            for (int e = lane; e < cnt; e += 64) {
                const int i = c0 + e;
                const double *src = Zt + (size_t)(lo + S.perm[S.nd[i]]) * N;
                const double zh = S.zhat[i];
                st[2 * e] = src[r] * zh;
                st[2 * e + 1] = two ? src[r + 1] * zh : 0.0;
            }
            wave_sync_lds();
            for (int e = 0; e < cnt; ++e) {
                const double ya = st[2 * e], yb = st[2 * e + 1], di = dl[c0 + e];
#pragma unroll
                for (int q = 0; q < NQ; ++q) {
                    if (64 * q >= k) break;  // uniform: the root slots past k are not computed
                    const double rc = rcpd((di - djr[q]) - tjr[q]);
                    acc[0][q] += ya * rc;
                    acc[1][q] += yb * rc;
                }
            }
            wave_sync_lds();  // the next chunk rewrites the staging slice
        }
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            if (h == 1 && !two) break;
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
                const int i = lane + 64 * q;
                if (64 * q < m) {
                    if (i < k) Zt[(size_t)(lo + S.nd[i]) * N + r + h] = acc[h][q] * S.invn[i];
                    if (i < m && S.defl[i]) Zt[(size_t)(lo + i) * N + r + h] = yd[h][q];
                }
            }
        }
    }
    __syncthreads();
    for (int t = tid; t < m; t += TRI_TPB)
        if (S.defl[t]) sd[lo + t] = S.ds[t];
    for (int j = tid; j < k; j += TRI_TPB) sd[lo + S.nd[j]] = S.lamn[j];
    __syncthreads();
}

// The whole tridiagonal solve: sd becomes the eigenvalues of T (unordered) and
// Zt (n x n global, column-major: u) its eigenvectors.  ctl[2]: set to 1 if a
// leaf did not converge; ctl[3]: leaf QL iterations + merges.
__device__ __forceinline__ void dc_solve(int n, double *sd, double *se, double *pool, int *ipool, double *Zt,
                                         double *red, int *ctl) {
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const size_t N = (size_t)n;
    // leaves of at most 8 below order 65 (their QL chases are serial on one
    // lane; measured faster there), of at most DC_LEAF above (fewer merges)
    const int lmax = n <= 64 ? 8 : DC_LEAF;
    int T = 0;
    while (((n + (1 << T) - 1) >> T) > lmax) ++T;
    const int nleaf = 1 << T;
    auto bnd = [&](int t, int i) { return (n * i) >> t; };
    for (int c = wv; c < n; c += TRI_WAVES)
        for (int r = lane; r < n; r += 64) Zt[c * N + r] = 0.0;
    // tear at the leaf boundaries (leaves hold at least 4 rows: no index is shared)
    if (tid >= 1 && tid < nleaf) {
        const int b0 = bnd(T, tid);
        const double r = fabs(se[b0 - 1]);
        sd[b0 - 1] -= r;
        sd[b0] -= r;
    }
    if (tid == 0) ctl[3] = 0;
    __syncthreads();
    // leaves: one wavefront each (its lane 0), eigenvectors in LDS, then into Zt
    double *leafZ = pool;                              // [nleaf][DC_LEAF][DC_LEAF]
    double *leafE = pool + DC_NLEAF * DC_LEAF * DC_LEAF;  // [nleaf][DC_LEAF]
    double *leafR = leafE + DC_NLEAF * DC_LEAF + wv * 2 * DC_LEAF;  // this wavefront's rotations
    int *leafC = (int *)(leafE + DC_NLEAF * DC_LEAF + TRI_WAVES * 2 * DC_LEAF) + 4 * wv;
    for (int lf = wv; lf < nleaf; lf += TRI_WAVES) {
        const int lo = bnd(T, lf), m = bnd(T, lf + 1) - lo;
        double *el = leafE + lf * DC_LEAF;
        for (int i = lane; i < m; i += 64) el[i] = i + 1 < m ? se[lo + i] : 0.0;
        wave_sync_lds();
        const int it = ql_leaf(m, sd + lo, el, leafZ + lf * DC_LEAF * DC_LEAF, leafR, leafC);
        if (lane == 0) {
            if (it < 0) ctl[2] = 1;
            else atomicAdd(&ctl[3], it);
        }
    }
    __syncthreads();
    for (int lf = wv; lf < nleaf; lf += TRI_WAVES) {
        const int lo = bnd(T, lf), m = bnd(T, lf + 1) - lo;
        const double *Zl = leafZ + lf * DC_LEAF * DC_LEAF;
        for (int e = lane; e < m * m; e += 64) {
            const int r = e / m, c = e % m;
            Zt[(size_t)(lo + c) * N + lo + r] = Zl[r * DC_LEAF + c];
        }
    }
    __syncthreads();
    // merges, deepest level first
    DcScratch S;
    S.zz = pool;
    S.ds = pool + DC_MAX;
    S.rc = pool + 2 * DC_MAX;
    S.rs = pool + 3 * DC_MAX;
    S.delta = pool + 4 * DC_MAX;
    S.zeta = pool + 5 * DC_MAX;
    S.tau = pool + 6 * DC_MAX;
    S.zhat = pool + 7 * DC_MAX;
    S.invn = pool + 8 * DC_MAX;
    S.lamn = pool + 9 * DC_MAX;
    int *ip = (int *)(pool + 10 * DC_MAX);
    S.perm = ip;
    S.defl = ip + DC_MAX;
    S.rj = ip + 2 * DC_MAX;
    S.ri = ip + 3 * DC_MAX;
    S.nd = ip + 4 * DC_MAX;
    S.tmp = ip + 5 * DC_MAX;
    S.org = ipool;
    S.stage = pool + 13 * DC_MAX;
    for (int t = T - 1; t >= 0; --t)
        for (int i = 0; i < (1 << t); ++i) {
            const int lo = bnd(t, i), mid = bnd(t + 1, 2 * i + 1), hi = bnd(t, i + 1);
            if (lo < mid && mid < hi) dc_merge(n, lo, mid, hi, se[mid - 1], sd, Zt, S, red, ctl);
            if (tid == 0) ++ctl[3];
        }
    __syncthreads();
}

// Householder reduction with the block in registers, R rows per thread: the
// wavefront wv keeps the entries (j, c) of the rows j0 <= j < j0 + R of its
// group g = wv / CB and of the column c = 64 (wv % CB) + lane, so that only
// vectors pass through LDS (zero past the order, so that rows past it add
// nothing).  Step k: column k (left in scol by the previous step's pass, with
// step k - 1's update still to apply: (v', w') pairs in cur) gives the
// diagonal and the reflector (v into nxt, also stored in row k beyond k + 1
// for the Q formation); then rows and columns k + 1.. take step k - 1's
// update and are multiplied by v in one pass, which also leaves column k + 1
// in scol; the groups' partial products meet in LDS (spart) as p = t A v, and
// w = p - K v goes next to v in nxt, the next step's pending update.  Each
// entry is updated by its own thread (A(i, j) and A(j, i) may differ by
// roundings; every step reads the block by columns).
template <int R>
__device__ __forceinline__ void hh_reduce(int d, const double *Z, double *A, double *wb, double2 *P0, double2 *P1,
                                          double *scol, double *spart, double *red, double *red2) {
    const int tid = threadIdx.x, lane = tid & 63;
    const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);  // (so that the rows, and their tests, are scalar)
    const size_t D = (size_t)d;
    const int CB = (d + 63) >> 6, G = (d + R - 1) / R;
    const int g = wv / CB, cb = wv % CB, c = cb * 64 + lane;
    const bool act = g < G;  // (uniform: the wavefronts past the groups only join the reductions)
    const int j0 = g * R;
    const int jv = ((tid >> 6) / CB) * R;  // j0 in a vector register: LDS rows at immediate offsets from it
    double a[R];
#pragma unroll
    for (int q = 0; q < R; ++q) a[q] = (act && j0 + q < d && c < d) ? Z[(size_t)(j0 + q) * D + c] : 0.0;
    for (int j = tid; j < HH_VEC; j += TRI_TPB) {
        P0[j] = make_double2(0.0, 0.0);  // no update pending before step 0
        P1[j] = make_double2(0.0, 0.0);
        scol[j] = j < d ? Z[(size_t)j * D] : 0.0;  // column 0
    }
    __syncthreads();
    double2 *cur = P0, *nxt = P1;
    for (int k = 0; k + 2 < d; ++k) {
        // column k after step k - 1's update: the diagonal, and x into nxt
        double part = 0.0, lead = 0.0;
        bool own = false;
        {
            const double2 pk = cur[k];
            for (int j = k + tid; j < d; j += TRI_TPB) {
                const double2 pj = cur[j];
                const double x = fma(-pj.x, pk.y, fma(-pj.y, pk.x, scol[j]));
                if (j == k) {
                    wb[k] = x;
                } else {
                    nxt[j].x = x;
                    if (j == k + 1) {
                        own = true;
                        lead = x;
                    } else {
                        part += x * x;
                    }
                }
            }
        }
        double alpha;  // x(0), handed over by its thread (nxt[k + 1] is rewritten below)
        const double sigma = block_sum1(part, own, lead, red2, &alpha);
        double t = 0.0;
        if (sigma == 0.0) {  // the column is already reduced: t = 0
            for (int j = k + 1 + tid; j < d; j += TRI_TPB) {
                nxt[j].x = j == k + 1 ? 1.0 : 0.0;
                if (j > k + 1) A[k * D + j] = 0.0;
            }
            if (tid == 0) {
                A[(k + 1) * D + k] = alpha;
                A[(k + 2) * D + k] = 0.0;
            }
        } else {
            const double beta = -copysign(sqrt(alpha * alpha + sigma), alpha);
            t = (beta - alpha) / beta;
            const double scale = 1.0 / (alpha - beta);
            for (int j = k + 1 + tid; j < d; j += TRI_TPB) {
                const double vj = j == k + 1 ? 1.0 : nxt[j].x * scale;
                nxt[j].x = vj;
                if (j > k + 1) A[k * D + j] = vj;
            }
            if (tid == 0) {
                A[(k + 1) * D + k] = beta;
                A[(k + 2) * D + k] = t;
            }
        }
        __syncthreads();
        // rows and columns k + 1..: step k - 1's update, and the product with v;
        // column k + 1 into scol
        double acc = 0.0;
        if (act && cb * 64 + 63 > k) {  // (uniform: a column block left of k + 1 is finished)
            const double2 pc = cur[c];
            const double2 *pr = cur + jv, *pn = nxt + jv;
            double *sc = scol + jv;
            const bool next = c == k + 1;
            // the rows past k form a suffix; each row's LDS reads are issued one
            // row ahead, so that their latency overlaps the previous row's work
            const int qs = max(0, min(R, k + 1 - j0));
            double2 nr = qs < R ? pr[qs] : make_double2(0.0, 0.0);
            double nv = qs < R ? pn[qs].x : 0.0;
#pragma unroll
            for (int q = 0; q < R; ++q) {
                if (j0 + q > k) {  // (uniform)
                    const double2 pj = nr;
                    const double vq = nv;
                    if (q + 1 < R) {
                        nr = pr[q + 1];
                        nv = pn[q + 1].x;
                    }
                    const double x = fma(-pj.x, pc.y, fma(-pj.y, pc.x, a[q]));
                    a[q] = x;
                    acc = fma(x, vq, acc);
                    if (next) sc[q] = x;
                }
            }
        }
        spart[tid] = acc;
        __syncthreads();
        // p = t A v (column tid), K = t p.v / 2, w = p - K v
        const bool mine = tid > k && tid < d;
        double pc = 0.0, pv = 0.0, vt = 0.0;
        if (mine) {
            double sum = 0.0;
            for (int gg = 0; gg < G; ++gg) sum += spart[(gg * CB + (tid >> 6)) * 64 + (tid & 63)];
            pc = t * sum;
            vt = nxt[tid].x;
            pv = pc * vt;
        }
        double unused;
        const double K = 0.5 * t * block_sum1(pv, false, 0.0, red, &unused);
        if (mine) nxt[tid].y = pc - K * vt;
        double2 *tmp = cur;  // (v, w) of this step is the next step's pending update
        cur = nxt;
        nxt = tmp;
        __syncthreads();
    }
    // the trailing 2 x 2 after the last step's update: column d - 2 from scol,
    // the entry (d - 1, d - 1) from its thread
    const int k = d - 2;
    if (tid < 2) {
        const int j = k + tid;
        const double2 pk = cur[k], pj = cur[j];
        const double x = fma(-pj.x, pk.y, fma(-pj.y, pk.x, scol[j]));
        if (tid == 0)
            wb[k] = x;
        else
            A[(k + 1) * D + k] = x;
    }
    if (act && c == d - 1) {
        double ad = 0.0;
        bool has = false;
#pragma unroll
        for (int q = 0; q < R; ++q)
            if (j0 + q == d - 1) {
                ad = a[q];
                has = true;
            }
        const double2 pd = cur[d - 1];
        if (has) wb[d - 1] = fma(-pd.x, pd.y, fma(-pd.y, pd.x, ad));
    }
}

// Householder reduction of the blocks of orders EIG_LDS_DIM + 1 .. HH_REG_DIM to
// tridiagonal form T = Q^T A Q (Q = H_0 ... H_{d-3}, H_k = I - t_k v_k v_k^T on
// indices k + 1.., v_k(k + 1) = 1), one workgroup per block, the block held in
// registers.  Output for k_eigh_tri: the diagonal of T in w (block b's slice),
// T(k + 1, k) at u(k + 1, k), t_k at u(k + 2, k), and v_k(j) at u(k, j) for
// j >= k + 2 (u row-major, block b at off[b]); a is only read.
__global__ __launch_bounds__(TRI_TPB) void k_eigh_hh(int nblk, const int64_t *__restrict__ off,
                                                     const int32_t *__restrict__ dim, const int64_t *__restrict__ woff,
                                                     const double *__restrict__ a, double *__restrict__ w,
                                                     double *__restrict__ u) {
    __shared__ double2 P0[HH_VEC], P1[HH_VEC];  // (v, w) of two steps
    __shared__ double scol[HH_VEC];
    __shared__ double spart[TRI_TPB];
    __shared__ double red[TRI_WAVES + 1], red2[TRI_WAVES + 1];
    const int b = blockIdx.x;
    if (b >= nblk) return;
    const int d = dim[b];
    if (d <= EIG_LDS_DIM || d > HH_REG_DIM) return;
    const double *Z = a + off[b];
    double *A = u + off[b], *wb = w + woff[b];
    // rows per thread: 4, 16 or 36 for one, two or three column blocks of 64
    if (d <= 64)
        hh_reduce<4>(d, Z, A, wb, P0, P1, scol, spart, red, red2);
    else if (d <= 128)
        hh_reduce<16>(d, Z, A, wb, P0, P1, scol, spart, red, red2);
    else
        hh_reduce<HH_ROWS>(d, Z, A, wb, P0, P1, scol, spart, red, red2);
}

// Tridiagonal path of the orders EIG_LDS_DIM + 1 .. EIG_MAX_DIM, one workgroup
// per block: T handed over by k_eigh_hh (orders up to HH_REG_DIM) or reduced
// here in global memory.  Orders up to DC_MAX: divide and conquer on T, which
// leaves the eigenvectors of T in u, its eigenvalues (unordered) in w and the
// reflectors in a, for k_eigh_back and k_eigh_out.  Larger orders: Q formed,
// implicit QL on T applied to it, and the ordered output written here.
__global__ __launch_bounds__(TRI_TPB) void k_eigh_tri(int nblk, const int64_t *__restrict__ off,
                                                      const int32_t *__restrict__ dim, const int64_t *__restrict__ woff,
                                                      double *__restrict__ a, double *__restrict__ w,
                                                      double *__restrict__ u, int32_t *__restrict__ info) {
    __shared__ double sd[EIG_MAX_DIM];  // diagonal of T, then the eigenvalues
    __shared__ double se[EIG_MAX_DIM];  // se[i] couples i and i + 1
    __shared__ double pool[5 * EIG_MAX_DIM];
    double *sq = pool;                     // Householder factors; QL: cosines (second buffer)
    double *sx = pool + EIG_MAX_DIM;       // Householder vector; QL: cosines (first buffer)
    double *sy = pool + 2 * EIG_MAX_DIM;   // p, then w = p - K v; QL: sines (first buffer)
    double *sz = pool + 3 * EIG_MAX_DIM;   // QL: sines (second buffer)
    double *spart = pool + 4 * EIG_MAX_DIM;  // row-group partial sums of p
    // (after Q is formed, the divide-and-conquer path uses the whole pool)
    __shared__ int srank[EIG_MAX_DIM];
    __shared__ double red[TRI_WAVES + 1];
    __shared__ double red2[TRI_WAVES + 1];  // second buffer of the reductions of the Householder steps
    __shared__ int ctl[4];
    const int b = blockIdx.x;
    if (b >= nblk) return;
    const int d = dim[b];
    if (d <= EIG_LDS_DIM || d > EIG_MAX_DIM) return;  // the Jacobi kernel's block (or rejected there)
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const size_t D = (size_t)d;
    double *A = u + off[b];  // working matrix (row-major, both triangles), then Householder vectors
    double *Z = a + off[b];  // Q, then the eigenvectors; column-major: Z[c * d + r] = Q(r, c)
    if (d <= HH_REG_DIM) {
        // reduced by k_eigh_hh: the diagonal in w, the off-diagonal and the
        // factors t below the diagonal of u, the reflectors in its rows
        const double *wb = w + woff[b];
        for (int j = tid; j < d; j += TRI_TPB) {
            sd[j] = wb[j];
            se[j] = j + 1 < d ? A[(j + 1) * D + j] : 0.0;
            if (j + 2 < d) sq[j] = A[(j + 2) * D + j];
        }
        __syncthreads();
    } else {
        for (int r = wv; r < d; r += TRI_WAVES)
            for (int c = lane; c < d; c += 64) A[r * D + c] = Z[r * D + c];
        __syncthreads();

        // ---- Householder reduction: step k zeroes A(k, k+2..) and A(k+2.., k) with
        // H = I - t v v^T acting on indices k+1.., v(0) = 1 (stored in row k beyond it).
        // A stays symmetric up to roundings (the two products of an update may be
        // fused differently for A(i, j) and A(j, i)), so column i of the trailing
        // block is read as its row i: each thread owns columns (coalesced across
        // the threads of a row).  Step k
        // needs p = t A22 v, w = p - K v and A22 -= v w^T + w v^T; the update of
        // step k and the product of step k + 1 are one pass over the block: row
        // k + 1 is updated first (it yields the next reflector), then every other
        // element is updated, stored and multiplied by the next v at once.
        // sv: v of the current step, sn: v of the next one, sy: p, then w.
        double *sv = sx, *sn = sz;
        double t = 0.0;  // the current step's factor
        {
            // step 0's reflector from row 0 and its product p = t A22 v
            const int L = d - 1;
            double part = 0.0;
            for (int j = tid; j < L; j += TRI_TPB) {
                const double x = A[1 + j];
                sv[j] = x;
                if (j) part += x * x;
            }
            double alpha;
            const double sigma = block_sum_lead(part, tid == 0 ? A[1] : 0.0, red, &alpha);
            if (sigma == 0.0) {
                if (tid == 0) {
                    sd[0] = A[0];
                    se[0] = alpha;
                    sq[0] = 0.0;
                }
                for (int j = tid; j < L; j += TRI_TPB) sv[j] = j ? 0.0 : 1.0;  // with t = 0: no reflection
            } else {
                const double beta = -copysign(sqrt(alpha * alpha + sigma), alpha);
                t = (beta - alpha) / beta;
                const double scale = 1.0 / (alpha - beta);
                for (int j = tid; j < L; j += TRI_TPB) sv[j] = j ? sv[j] * scale : 1.0;
                if (tid == 0) {
                    sd[0] = A[0];
                    se[0] = beta;
                    sq[0] = t;
                }
            }
            __syncthreads();
            const int G = max(1, min(TRI_TPB / L, 32)), R = (L + G - 1) / G;
            for (int q = tid; q < G * L; q += TRI_TPB) {
                const int i = q % L, g = q / L;
                const int j0 = g * R, j1 = min(L, j0 + R);
                const double *col = A + D + 1 + i;
                double acc = 0.0;
                for (int jb = j0; jb < j1; jb += TRI_UB) {
                    double av[TRI_UB];
    #pragma unroll
                    for (int u = 0; u < TRI_UB; ++u) av[u] = col[min(jb + u, j1 - 1) * D];
    #pragma unroll
                    for (int u = 0; u < TRI_UB; ++u)
                        if (jb + u < j1) acc += av[u] * sv[jb + u];
                }
                spart[q] = acc;
            }
            __syncthreads();
        }
        for (int k = 0; k + 2 < d; ++k) {
            const int L = d - k - 1, G = max(1, min(TRI_TPB / L, 32));
            // p and w of step k (the groups' partial products meet in LDS)
            double pv = 0.0;
            for (int i = tid; i < L; i += TRI_TPB) {
                double acc = 0.0;
                for (int g = 0; g < G; ++g) acc += spart[g * L + i];
                const double pi = t * acc;
                sy[i] = pi;
                pv += pi * sv[i];
            }
            double unused;
            const double K = 0.5 * t * block_sum1(pv, false, 0.0, red, &unused);
            for (int j = tid; j < L; j += TRI_TPB) sy[j] -= K * sv[j];  // w
            __syncthreads();
            for (int j = 1 + tid; j < L; j += TRI_TPB) A[k * D + k + 1 + j] = sv[j];
            // row k + 1 after step k's update (the same expression as for the
            // rest of the block): its diagonal, and the vector x of step k + 1 into sn
            const bool next = k + 3 < d;
            double part = 0.0, diag = 0.0, lead = 0.0;
            for (int i = tid; i < L; i += TRI_TPB) {
                const double val = A[(k + 1) * D + k + 1 + i] - __dadd_rn(__dmul_rn(sv[0], sy[i]), __dmul_rn(sy[0], sv[i]));
                if (i == 0) diag = val;
                if (i == 1) lead = val;
                if (i >= 1) sn[i - 1] = val;
                if (i >= 2) part += val * val;
            }
            double alpha;  // x(0), handed over by the thread that formed it (sn[0] is rescaled below)
            const double sigma = block_sum1(part, tid == 1, lead, red2, &alpha);
            double tn = 0.0;
            if (!next) {  // the trailing 2 x 2: no reflector
                if (tid == 0) {
                    sd[k + 1] = diag;
                    se[k + 1] = alpha;
                }
            } else if (sigma == 0.0) {  // the column is already reduced
                if (tid == 0) {
                    sd[k + 1] = diag;
                    se[k + 1] = alpha;
                    sq[k + 1] = 0.0;
                }
                for (int j = tid; j < L - 1; j += TRI_TPB) sn[j] = j ? 0.0 : 1.0;  // with t = 0: no reflection
            } else {
                const double beta = -copysign(sqrt(alpha * alpha + sigma), alpha);
                tn = (beta - alpha) / beta;
                const double scale = 1.0 / (alpha - beta);
                for (int j = tid; j < L - 1; j += TRI_TPB) sn[j] = j ? sn[j] * scale : 1.0;
                if (tid == 0) {
                    sd[k + 1] = diag;
                    se[k + 1] = beta;
                    sq[k + 1] = tn;
                }
            }
            __syncthreads();
            // the rest of A22 (indices k + 2..): updated, stored, and (with a next
            // step) summed into that step's p; thread (i, g) on the rows of group g
            // of column i, loads in batches
            const int L1 = L - 1, G1 = max(1, min(TRI_TPB / L1, 32)), R1 = (L1 + G1 - 1) / G1;
            for (int q = tid; q < G1 * L1; q += TRI_TPB) {
                const int i = q % L1, g = q / L1;
                const int j0 = g * R1, j1 = min(L1, j0 + R1);
                double *col = A + (k + 2) * D + k + 2 + i;
                const double vi = sv[i + 1], wi = sy[i + 1];
                double acc = 0.0;
                for (int jb = j0; jb < j1; jb += TRI_UB) {
                    double av[TRI_UB];
    #pragma unroll
                    for (int u = 0; u < TRI_UB; ++u) av[u] = col[min(jb + u, j1 - 1) * D];
    #pragma unroll
                    for (int u = 0; u < TRI_UB; ++u) {
                        const int j = jb + u;
                        if (j < j1) {
                            const double val = av[u] - __dadd_rn(__dmul_rn(sv[j + 1], wi), __dmul_rn(sy[j + 1], vi));
                            col[j * D] = val;
                            acc += val * sn[j];
                        }
                    }
                }
                if (next) spart[q] = acc;
            }
            __syncthreads();
            double *tmp = sv;  // the next step's v becomes the current one
            sv = sn;
            sn = tmp;
            t = tn;
        }
        if (tid == 0) {
            sd[d - 1] = A[(d - 1) * D + d - 1];
            se[d - 1] = 0.0;
        }
    }
    if (d <= DC_MAX) {
        // the reflectors (rows of u beyond k + 1) and their factors t (at
        // (k + 2, k)) to a, which the input no longer needs: k_eigh_back applies
        // them to the eigenvectors of T; divide and conquer on T, its
        // eigenvectors into u and its eigenvalues, unordered, into w
        for (int k = wv; k + 2 < d; k += TRI_WAVES) {
            for (int j = k + 2 + lane; j < d; j += 64) Z[k * D + j] = A[k * D + j];
            if (lane == 0) Z[(k + 2) * D + k] = sq[k];
        }
        __syncthreads();
        if (tid == 0) ctl[2] = 0;
        dc_solve(d, sd, se, pool, (int *)srank, A, red, ctl);
        double *wb = w + woff[b];
        for (int i = tid; i < d; i += TRI_TPB) wb[i] = sd[i];
        if (tid == 0 && info) info[b] = ctl[2] ? -2 : 1 + ctl[3];
        return;
    }
    // ---- Q = H_0 H_1 ... H_{d-3}, accumulated from the last factor; H_k Q only
    // changes the trailing block from index k + 1: y_c = v^T Q(:, c), then
    // Q(:, c) -= t y_c v.
    for (int c = wv; c < d; c += TRI_WAVES)
        for (int r = lane; r < d; r += 64) Z[c * D + r] = r == c ? 1.0 : 0.0;
    __syncthreads();
    if (d - 1 <= 64 * Q_REG) {
        // QB factors at a time: their vectors staged in LDS (rows from the
        // block's first touched index r0 = klo + 1, zero above each factor's
        // own start), then every wave applies all of them, last first, to four
        // columns at a time held in registers: one load and one store of each
        // column per block instead of per factor.  A factor meets zeros in the
        // rows and columns it does not reach, which leaves them unchanged.
        double *sv = sx;  // [QB][L0] (the pool past the factors' t)
        for (int khi = d - 3; khi >= 0; khi -= QB) {
            const int klo = max(0, khi - QB + 1), r0 = klo + 1, L0 = d - r0;
            for (int i = tid; i < (khi - klo + 1) * L0; i += TRI_TPB) {
                const int kk = i / L0, j = i - kk * L0, k = klo + kk, r = r0 + j;
                sv[i] = r == k + 1 ? 1.0 : (r > k + 1 ? A[k * D + r] : 0.0);
            }
            __syncthreads();
            for (int c0 = 4 * wv; c0 < L0; c0 += 4 * TRI_WAVES) {
                double cv[4][Q_REG];
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const double *col = Z + (r0 + min(c0 + e, L0 - 1)) * D + r0;
#pragma unroll
                    for (int q = 0; q < Q_REG; ++q) {
                        if (64 * q >= L0) break;  // uniform: the row slots past L0 are not used
                        cv[e][q] = col[min(lane + 64 * q, L0 - 1)];
                    }
                }
                for (int k = khi; k >= klo; --k) {
                    const double t = sq[k];
                    if (t == 0.0) continue;
                    const double *v = sv + (k - klo) * L0;
                    double acc[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
                    for (int q = 0; q < Q_REG; ++q) {
                        if (64 * q >= L0) break;
                        const int r = lane + 64 * q;
                        const double vr = r < L0 ? v[r] : 0.0;
#pragma unroll
                        for (int e = 0; e < 4; ++e) acc[e] += vr * cv[e][q];
                    }
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        const double ty = t * group_sum<64>(acc[e]);
#pragma unroll
                        for (int q = 0; q < Q_REG; ++q) {
                            if (64 * q >= L0) break;
                            const int r = lane + 64 * q;
                            if (r < L0) cv[e][q] -= ty * v[r];
                        }
                    }
                }
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    if (c0 + e < L0) {
                        double *col = Z + (r0 + c0 + e) * D + r0;
#pragma unroll
                        for (int q = 0; q < Q_REG; ++q) {
                            const int r = lane + 64 * q;
                            if (r < L0) col[r] = cv[e][q];
                        }
                    }
            }
            __syncthreads();  // the next block reads these columns and rewrites sv
        }
    } else {
        // one factor at a time, one wave per column (or four columns)
        for (int k = d - 3; k >= 0; --k) {
            const double t = sq[k];
            if (t == 0.0) continue;
            const int L = d - k - 1;
            for (int j = tid; j < L; j += TRI_TPB) sx[j] = j ? A[k * D + k + 1 + j] : 1.0;
            __syncthreads();
            if (L <= 64 * Q_REG) {
                // four columns per wave at a time: all their loads in flight together
                for (int c0 = 4 * wv; c0 < L; c0 += 4 * TRI_WAVES) {
                    double cv[4][Q_REG];
                    double acc[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        const double *col = Z + (k + 1 + min(c0 + e, L - 1)) * D + k + 1;
#pragma unroll
                        for (int q = 0; q < Q_REG; ++q) cv[e][q] = col[min(lane + 64 * q, L - 1)];
                    }
#pragma unroll
                    for (int e = 0; e < 4; ++e)
#pragma unroll
                        for (int q = 0; q < Q_REG; ++q) {
                            const int r = lane + 64 * q;
                            if (r < L) acc[e] += sx[r] * cv[e][q];
                        }
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        const double ty = t * group_sum<64>(acc[e]);
                        if (c0 + e < L) {
                            double *col = Z + (k + 1 + c0 + e) * D + k + 1;
#pragma unroll
                            for (int q = 0; q < Q_REG; ++q) {
                                const int r = lane + 64 * q;
                                if (r < L) col[r] = cv[e][q] - ty * sx[r];
                            }
                        }
                    }
                }
            } else {
                for (int c = wv; c < L; c += TRI_WAVES) {
                    double *col = Z + (k + 1 + c) * D + k + 1;
                    double acc = 0.0;
                    for (int r = lane; r < L; r += 64) acc += sx[r] * col[r];
                    const double ty = t * group_sum<64>(acc);
                    for (int r = lane; r < L; r += 64) col[r] -= ty * sx[r];
                }
            }
            __syncthreads();
        }
    }

    int its = 0, bad = 0;
    {
    // ---- implicit QL on T (sd, se).  Lane 0 of wave 0 runs the recurrence and
    // leaves each iteration's rotations (indices lo..hi) in one of two LDS
    // buffers; in the same interval the other waves apply the previous
    // iteration's rotations to the rows of Z.
    int l = 0, it_l = 0;
    double tol = 0.0;
    // one QL iteration into buffer `buf` (lane 0 of wave 0 only); ctl[2 buf] = lo,
    // ctl[2 buf + 1] = hi, lo = -1 when every eigenvalue has converged
    auto ql_next = [&](int buf) {
        int lo = -1, hi = -1;
        double *rc = buf ? sq : sx, *rs = buf ? sz : sy;
        while (l < d) {
            // m: the first index >= l whose coupling counts as zero (se[d - 1] = 0);
            // eight couplings tested per round of LDS loads
            int m = l;
            for (;;) {
                double ev[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) ev[u] = se[min(m + u, d - 1)];
                int found = -1;
#pragma unroll
                for (int u = 7; u >= 0; --u)
                    if (fabs(ev[u]) <= tol || m + u >= d - 1) found = min(m + u, d - 1);
                if (found >= 0) {
                    m = found;
                    break;
                }
                m += 8;
            }
            if (m == l) {  // sd[l] is an eigenvalue
                ++l;
                it_l = 0;
                continue;
            }
            if (++it_l > QL_MAXIT) {
                bad = 1;
                l = d;
                break;
            }
            ++its;
            // shift: the eigenvalue of the leading 2 x 2 of the segment nearer sd[l]
            const double dl = sd[l];
            double g = (sd[l + 1] - dl) / (2.0 * se[l]);
            double r = hyp(g, 1.0);
            g = sd[m] - dl + se[l] / (g + copysign(r, g));
            double s = 1.0, c = 1.0, p = 0.0;
            // every value read below is still the one from before this iteration
            // (iteration i writes index i + 1), so the next ones are fetched ahead
            double dip1 = sd[m], di = sd[m - 1], ei = se[m - 1];
            int i = m - 1;
            bool early = false;
            for (; i >= l; --i) {
                const int in = i > l ? i - 1 : i;
                const double dn = sd[in], en = se[in];
                const double f = s * ei, bb = c * ei;
                // T is scaled to a norm in [1, 2), so f and g cannot overflow; a
                // rotation norm below 2^-500 (135 orders of magnitude below the
                // deflation threshold) counts as zero: the chase splits there and
                // the iteration is repeated on the shorter segment
                const double r2 = f * f + g * g;
                if (__builtin_expect(r2 <= 0x1p-1000, 0)) {
                    se[i + 1] = 0.0;
                    sd[i + 1] = dip1 - p;
                    se[m] = 0.0;
                    early = true;
                    break;
                }
                const double ir = rsqrt(r2);
                r = r2 * ir;
                se[i + 1] = r;
                s = f * ir;
                c = g * ir;
                g = dip1 - p;
                r = (di - g) * s + 2.0 * c * bb;
                p = s * r;
                sd[i + 1] = g + p;
                g = c * r - bb;
                rc[i] = c;
                rs[i] = s;
                dip1 = di;
                di = dn;
                ei = en;
            }
            if (!early) {
                sd[l] -= p;
                se[l] = g;
                se[m] = 0.0;
            }
            lo = early ? i + 1 : l;
            hi = m - 1;
            break;
        }
        ctl[2 * buf] = lo;
        ctl[2 * buf + 1] = hi;
    };
    double scale = 1.0;  // power of two: T * scale has a norm in [1, 2) (exact)
    if (tid == 0) {
        double anorm = 0.0;
        for (int i = 0; i < d; ++i)
            anorm = fmax(anorm, fabs(sd[i]) + fabs(se[i]) + (i ? fabs(se[i - 1]) : 0.0));
        if (anorm > 0.0 && isfinite(anorm)) {
            scale = ldexp(1.0, -ilogb(anorm));
            for (int i = 0; i < d; ++i) {
                sd[i] *= scale;
                se[i] *= scale;
            }
            anorm *= scale;
        }
        tol = anorm * 0x1p-53;
        ql_next(0);
    }
    __syncthreads();
    for (int step = 0;; ++step) {
        const int cur = step & 1;
        const int lo = ctl[2 * cur], hi = ctl[2 * cur + 1];
        if (lo < 0) break;
        if (wv == 0) {
            if (lane == 0) ql_next(cur ^ 1);
        } else if (hi >= lo) {
            // rotation i acts on columns i, i + 1, from hi down to lo: the column
            // i + 1 entering rotation i is the one rotation i + 1 left (carried),
            // column i is still the old one (fetched ahead in batches)
            const double *rc = cur ? sq : sx, *rs = cur ? sz : sy;
            for (int r = tid - 64; r < d; r += TRI_TPB - 64) {
                double carry = Z[(hi + 1) * D + r];
                double zv[QL_B], zn[QL_B];
#pragma unroll
                for (int q = 0; q < QL_B; ++q) zv[q] = Z[max(hi - q, lo) * D + r];
                for (int i0 = hi; i0 >= lo; i0 -= QL_B) {
                    // the next batch's columns lie below every column this batch writes
#pragma unroll
                    for (int q = 0; q < QL_B; ++q) zn[q] = Z[max(i0 - QL_B - q, lo) * D + r];
#pragma unroll
                    for (int q = 0; q < QL_B; ++q) {
                        const int i = i0 - q;
                        if (i >= lo) {
                            const double c = rc[i], s = rs[i];
                            Z[(i + 1) * D + r] = s * zv[q] + c * carry;
                            carry = c * zv[q] - s * carry;
                        }
                    }
#pragma unroll
                    for (int q = 0; q < QL_B; ++q) zv[q] = zn[q];
                }
                Z[lo * D + r] = carry;
            }
        }
        __syncthreads();
    }

    if (tid == 0 && scale != 1.0) {
        const double inv = 1.0 / scale;  // a power of two: exact
        for (int i = 0; i < d; ++i) sd[i] *= inv;
    }
    }  // QL
    __syncthreads();
    // ---- descending order (ties by index), first entry of largest magnitude positive
    for (int i = tid; i < d; i += TRI_TPB) {
        const double wi = sd[i];
        int rank = 0;
        for (int j = 0; j < d; ++j) {
            const double wj = sd[j];
            rank += (wj > wi) || (wj == wi && j < i);
        }
        srank[i] = rank;
    }
    __syncthreads();
    double *wb = w + woff[b];
    for (int i = wv; i < d; i += TRI_WAVES) {
        const double *col = Z + i * D;
        double best = -1.0;
        int bi = 0;
        for (int r = lane; r < d; r += 64) {
            const double av = fabs(col[r]);
            if (av > best) {
                best = av;
                bi = r;
            }
        }
        for (int o = 32; o > 0; o >>= 1) {
            const double ob = __shfl_xor(best, o, 64);
            const int oi = __shfl_xor(bi, o, 64);
            if (ob > best || (ob == best && oi < bi)) {
                best = ob;
                bi = oi;
            }
        }
        const double sg = col[bi] < 0.0 ? -1.0 : 1.0;
        const int rk = srank[i];
        for (int r = lane; r < d; r += 64) A[r * D + rk] = sg * col[r];
        if (lane == 0) wb[rk] = sd[i];
    }
    if (tid == 0 && info) info[b] = bad ? -2 : 1 + its;
}

constexpr int BK_COLS = 16;                 // columns of a block per workgroup of k_eigh_back
constexpr int BK_PANELS = DC_MAX / BK_COLS;  // its grid's second dimension
constexpr int BK_TPB = 256;                  // four wavefronts of four columns

// Eigenvectors of the divide-and-conquer blocks (orders EIG_LDS_DIM + 1 ..
// DC_MAX): E = H_0 H_1 ... H_{d-3} Z, the reflectors (rows of a beyond k + 1,
// t_k at a(k + 2, k)) applied to the eigenvectors Z of T (u, column-major),
// the last one first.  Workgroup (b, p) owns columns [16 p, 16 p + 16) of
// block b's Z and overwrites them with E: QB reflectors at a time are staged
// in LDS (zero above each one's first row, 1 there), then each wavefront
// applies them, two at a time, to four register-resident columns (one load
// and one store of a column per QB reflectors).
__global__ __launch_bounds__(BK_TPB) void k_eigh_back(int nblk, const int64_t *__restrict__ off,
                                                      const int32_t *__restrict__ dim, const double *__restrict__ a,
                                                      double *__restrict__ u) {
    __shared__ double sv[QB * DC_MAX];  // [QB][L0]: the staged reflectors, rows r0..d-1
    __shared__ double st[QB];
    __shared__ double ss[QB / 2];  // v_{k-1}.v_k of the pairs
    const int b = blockIdx.x;
    if (b >= nblk) return;
    const int d = dim[b];
    if (d <= EIG_LDS_DIM || d > DC_MAX) return;
    const int cp = blockIdx.y * BK_COLS;
    if (cp >= d) return;
    const size_t D = (size_t)d;
    const double *H = a + off[b];
    double *Z = u + off[b];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    for (int khi = d - 3; khi >= 0; khi -= QB) {
        const int klo = max(0, khi - QB + 1), r0 = klo + 1, L0 = d - r0;
        for (int i = threadIdx.x; i < (khi - klo + 1) * L0; i += blockDim.x) {
            const int kk = i / L0, j = i - kk * L0, k = klo + kk, r = r0 + j;
            sv[i] = r == k + 1 ? 1.0 : (r > k + 1 ? H[k * D + r] : 0.0);
        }
        for (int i = threadIdx.x; i <= khi - klo; i += blockDim.x) st[i] = H[(klo + i + 2) * D + klo + i];
        __syncthreads();
        // the reflectors go in pairs (k, k - 1) from khi down: s = v_{k-1}.v_k lets
        // both products with a column be formed at once
        const int npair = (khi - klo + 1) >> 1;
        for (int pr = wave; pr < npair; pr += nw) {
            const double *v1 = sv + (khi - 2 * pr - klo) * L0, *v2 = v1 - L0;
            double part = 0.0;
            for (int r = lane; r < L0; r += 64) part += v1[r] * v2[r];
            part = group_sum<64>(part);
            if (lane == 0) ss[pr] = part;
        }
        __syncthreads();
        for (int c0 = cp + 4 * wave; c0 < min(d, cp + BK_COLS); c0 += 4 * nw) {
            double cv[4][Q_REG];
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const double *col = Z + (size_t)min(c0 + e, d - 1) * D + r0;
#pragma unroll
                for (int q = 0; q < Q_REG; ++q) {
                    if (64 * q >= L0) break;  // uniform: the row slots past L0 are not used
                    cv[e][q] = col[min(lane + 64 * q, L0 - 1)];
                }
            }
            // H_{k-1} H_k c = c - t_k y1 v_k - t_{k-1} y2 v_{k-1}, y1 = v_k.c,
            // y2 = v_{k-1}.c - t_k y1 s
            for (int pr = 0; pr < npair; ++pr) {
                const int k = khi - 2 * pr;
                const double t1 = st[k - klo], t2 = st[k - 1 - klo], sp = ss[pr];
                const double *v1 = sv + (k - klo) * L0, *v2 = v1 - L0;
                double a1[4] = {0.0, 0.0, 0.0, 0.0}, a2[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
                for (int q = 0; q < Q_REG; ++q) {
                    if (64 * q >= L0) break;
                    const int r = lane + 64 * q;
                    const double x1 = r < L0 ? v1[r] : 0.0, x2 = r < L0 ? v2[r] : 0.0;
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        a1[e] += x1 * cv[e][q];
                        a2[e] += x2 * cv[e][q];
                    }
                }
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const double y1 = group_sum<64>(a1[e]), z = group_sum<64>(a2[e]);
                    const double f1 = t1 * y1, f2 = t2 * (z - f1 * sp);
#pragma unroll
                    for (int q = 0; q < Q_REG; ++q) {
                        if (64 * q >= L0) break;
                        const int r = lane + 64 * q;
                        if (r < L0) cv[e][q] -= f1 * v1[r] + f2 * v2[r];
                    }
                }
            }
            if (((khi - klo + 1) & 1) && st[0] != 0.0) {  // the block's last reflector, klo, alone
                const double t = st[0];
                const double *v = sv;
                double acc[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
                for (int q = 0; q < Q_REG; ++q) {
                    if (64 * q >= L0) break;
                    const int r = lane + 64 * q;
                    const double vr = r < L0 ? v[r] : 0.0;
#pragma unroll
                    for (int e = 0; e < 4; ++e) acc[e] += vr * cv[e][q];
                }
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const double ty = t * group_sum<64>(acc[e]);
#pragma unroll
                    for (int q = 0; q < Q_REG; ++q) {
                        if (64 * q >= L0) break;
                        const int r = lane + 64 * q;
                        if (r < L0) cv[e][q] -= ty * v[r];
                    }
                }
            }
#pragma unroll
            for (int e = 0; e < 4; ++e)
                if (c0 + e < d) {
                    double *col = Z + (size_t)(c0 + e) * D + r0;
#pragma unroll
                    for (int q = 0; q < Q_REG; ++q) {
                        const int r = lane + 64 * q;
                        if (r < L0) col[r] = cv[e][q];
                    }
                }
        }
        __syncthreads();  // the next block restages sv
    }
}

// Output of the divide-and-conquer blocks: eigenvalues descending (ties by
// index) into w, and the columns of E (u, column-major) in that order into u
// (row-major), each with its first entry of largest magnitude positive; a is
// the staging copy.
__global__ __launch_bounds__(TRI_TPB) void k_eigh_out(int nblk, const int64_t *__restrict__ off,
                                                      const int32_t *__restrict__ dim,
                                                      const int64_t *__restrict__ woff, double *__restrict__ a,
                                                      double *__restrict__ w, double *__restrict__ u) {
    __shared__ double sv[DC_MAX], ssg[DC_MAX];
    __shared__ int srk[DC_MAX], sinv[DC_MAX];
    __shared__ double tile[32][33];
    const int b = blockIdx.x;
    if (b >= nblk) return;
    const int d = dim[b];
    if (d <= EIG_LDS_DIM || d > DC_MAX) return;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, nw = blockDim.x >> 6;
    const size_t D = (size_t)d;
    const double *E = u + off[b];
    double *S = a + off[b], *U = u + off[b], *wb = w + woff[b];
    for (int i = tid; i < d; i += blockDim.x) sv[i] = wb[i];
    __syncthreads();
    for (int i = tid; i < d; i += blockDim.x) {
        const double wi = sv[i];
        int rank = 0;
        for (int j = 0; j < d; ++j) {
            const double wj = sv[j];
            rank += (wj > wi) || (wj == wi && j < i);
        }
        srk[i] = rank;
    }
    __syncthreads();
    for (int i = wv; i < d; i += nw) {
        const double *col = E + i * D;
        double best = -1.0;
        int bi = 0;
        for (int r = lane; r < d; r += 64) {
            const double av = fabs(col[r]);
            if (av > best) {
                best = av;
                bi = r;
            }
        }
        for (int o = 32; o > 0; o >>= 1) {
            const double ob = __shfl_xor(best, o, 64);
            const int oi = __shfl_xor(bi, o, 64);
            if (ob > best || (ob == best && oi < bi)) {
                best = ob;
                bi = oi;
            }
        }
        if (lane == 0) {
            const int rk = srk[i];
            ssg[rk] = col[bi] < 0.0 ? -1.0 : 1.0;
            sinv[rk] = i;
            wb[rk] = sv[i];
        }
    }
    __syncthreads();
    // U(r, rk) = sign * E(r, i(rk)): 32 x 32 tiles through LDS, read down the
    // columns of E and written along the rows of the staging copy
    static_assert(TRI_TPB == 1024, "32 x 32 tile threads");
    const int tr = tid & 31, tc = tid >> 5;
    for (int c0 = 0; c0 < d; c0 += 32)
        for (int rr = 0; rr < d; rr += 32) {
            const int rk = c0 + tc, r = rr + tr;
            if (rk < d && r < d) tile[tc][tr] = ssg[rk] * E[(size_t)sinv[rk] * D + r];
            __syncthreads();
            const int r2 = rr + tc, rk2 = c0 + tr;
            if (r2 < d && rk2 < d) S[(size_t)r2 * D + rk2] = tile[tr][tc];
            __syncthreads();
        }
    for (size_t e = tid; e < D * D; e += blockDim.x) U[e] = S[e];
}

// State selection (Alg. 1, step 7: a block keeps its states of largest
// density-matrix eigenvalue).  One workgroup per group of sector blocks whose
// eigenvalues lie contiguous in w.  The m-th largest value is found by a radix
// select on order-preserving 64-bit keys (eight passes of 8 bits, a 256-bin
// histogram each); values above it are kept, and of the values equal to it the
// first ones in storage order (block order, then index order), by a scan.  A
// block keeps a prefix of its values because each block's values are stored
// in descending order.
constexpr int TRUNC_MAX = 16384;

// order-preserving key: a > b  <=>  key(a) > key(b), a == b  <=>  key(a) ==
// key(b) (for non-NaN values; -0 is taken as +0)
__device__ __forceinline__ uint64_t order_key(double v) {
    const uint64_t b = (uint64_t)__double_as_longlong(v == 0.0 ? 0.0 : v);
    return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}

__global__ __launch_bounds__(EIG_TPB) void k_truncate(int ngroup, const int32_t *__restrict__ gblk,
                                                      const int32_t *__restrict__ dim,
                                                      const int64_t *__restrict__ woff, const double *__restrict__ w,
                                                      const int32_t *__restrict__ m_keep, int32_t *__restrict__ keep,
                                                      double *__restrict__ discarded) {
    __shared__ unsigned char kept[TRUNC_MAX];
    __shared__ double part[EIG_TPB];
    __shared__ int hist[256];
    __shared__ int cnt[EIG_TPB];
    __shared__ uint64_t sel_key;
    __shared__ int sel_rem;
    const int g = blockIdx.x, tid = threadIdx.x;
    if (g >= ngroup) return;
    const int b0 = gblk[g], b1 = gblk[g + 1];
    if (b1 <= b0) {
        if (tid == 0 && discarded) discarded[g] = 0.0;
        return;
    }
    const int64_t base = woff[b0];
    const int64_t N64 = woff[b1 - 1] + dim[b1 - 1] - base;
    if (N64 < 0 || N64 > TRUNC_MAX) {
        for (int b = b0 + tid; b < b1; b += EIG_TPB) keep[b] = -1;
        if (tid == 0 && discarded) discarded[g] = __builtin_nan("");
        return;
    }
    const int N = (int)N64;
    const int m = m_keep[g];
    const double *wg = w + base;
    // thread tid owns values [lo, hi)
    const int per = (N + EIG_TPB - 1) / EIG_TPB;
    const int lo = min(N, tid * per), hi = min(N, lo + per);
    if (m <= 0 || m >= N) {  // nothing or everything kept
        for (int e = lo; e < hi; ++e) kept[e] = m > 0;
    } else {
        // radix select of the m-th largest key, most significant digit first
        uint64_t prefix = 0;
        int rem = m;  // rank still to be found inside the current prefix
        for (int pass = 0; pass < 8; ++pass) {
            const int shift = 56 - 8 * pass;
            for (int i = tid; i < 256; i += EIG_TPB) hist[i] = 0;
            __syncthreads();
            const uint64_t hmask = pass == 0 ? 0 : (~0ull << (shift + 8));
            for (int e = lo; e < hi; ++e) {
                const uint64_t k = order_key(wg[e]);
                if ((k & hmask) == prefix) atomicAdd(&hist[(k >> shift) & 255], 1);
            }
            __syncthreads();
            if (tid == 0) {
                int acc = 0, digit = 255;
                for (; digit > 0; --digit) {
                    if (acc + hist[digit] >= rem) break;
                    acc += hist[digit];
                }
                sel_key = prefix | ((uint64_t)digit << shift);
                sel_rem = rem - acc;
            }
            __syncthreads();
            prefix = sel_key;
            rem = sel_rem;
            __syncthreads();  // sel_* are rewritten by the next pass
        }
        // values equal to the cut: the first rem of them in storage order
        int c = 0;
        for (int e = lo; e < hi; ++e) c += order_key(wg[e]) == prefix;
        cnt[tid] = c;
        __syncthreads();
        if (tid == 0) {
            int run = 0;
            for (int i = 0; i < EIG_TPB; ++i) {
                const int t = cnt[i];
                cnt[i] = run;
                run += t;
            }
        }
        __syncthreads();
        int before = cnt[tid];
        for (int e = lo; e < hi; ++e) {
            const uint64_t k = order_key(wg[e]);
            bool keepit = k > prefix;
            if (k == prefix) keepit = before++ < rem;
            kept[e] = keepit;
        }
    }
    __syncthreads();
    double dsum = 0.0;
    for (int b = b0 + tid; b < b1; b += EIG_TPB) {
        const int64_t s = woff[b] - base;
        int kc = 0;
        for (int j = 0; j < dim[b]; ++j) {
            if (kept[s + j])
                ++kc;
            else
                dsum += wg[s + j];
        }
        keep[b] = kc;
    }
    part[tid] = dsum;
    __syncthreads();
    if (tid == 0 && discarded) {
        double t = 0.0;
        for (int i = 0; i < EIG_TPB; ++i) t += part[i];
        discarded[g] = t;
    }
}

}  // namespace dmrg

// ================================================================== ABI

using namespace dmrg;

extern "C" {

dmrg_status dmrg_eigh_blocks(int32_t nblk, const int64_t *off, const int32_t *dim, const int64_t *woff,
                             double *a, double *w, double *u, int32_t *info, void *stream) {
    clear_error();
    if (nblk < 0) return set_error(DMRG_E_INVALID_ARG, "negative block count");
    if (nblk == 0) return DMRG_OK;
    if (!off || !dim || !woff || !a || !w || !u) return set_error(DMRG_E_INVALID_ARG, "null argument");
    if (a == u || a == w || u == w) return set_error(DMRG_E_INVALID_ARG, "a, w and u must not overlap");
    hipStream_t s = (hipStream_t)stream;
    hipLaunchKernelGGL(k_eigh_jacobi, dim3(nblk), dim3(EIG_TPB_SMALL), 0, s, nblk, off, dim, woff, a, w, u, info);
    hipLaunchKernelGGL(k_eigh_hh, dim3(nblk), dim3(TRI_TPB), 0, s, nblk, off, dim, woff, a, w, u);
    hipLaunchKernelGGL(k_eigh_tri, dim3(nblk), dim3(TRI_TPB), 0, s, nblk, off, dim, woff, a, w, u, info);
    hipLaunchKernelGGL(k_eigh_back, dim3(nblk, BK_PANELS), dim3(BK_TPB), 0, s, nblk, off, dim, a, u);
    hipLaunchKernelGGL(k_eigh_out, dim3(nblk), dim3(TRI_TPB), 0, s, nblk, off, dim, woff, a, w, u);
    DMRG_HIP(hipGetLastError());
    return DMRG_OK;
}

dmrg_status dmrg_truncate(int32_t ngroup, const int32_t *gblk, const int32_t *dim, const int64_t *woff,
                          const double *w, const int32_t *m_keep, int32_t *keep, double *discarded, void *stream) {
    clear_error();
    if (ngroup < 0) return set_error(DMRG_E_INVALID_ARG, "negative group count");
    if (ngroup == 0) return DMRG_OK;
    if (!gblk || !dim || !woff || !w || !m_keep || !keep) return set_error(DMRG_E_INVALID_ARG, "null argument");
    hipLaunchKernelGGL(k_truncate, dim3(ngroup), dim3(EIG_TPB), 0, (hipStream_t)stream, ngroup, gblk, dim, woff, w,
                       m_keep, keep, discarded);
    DMRG_HIP(hipGetLastError());
    return DMRG_OK;
}

}  // extern "C"
