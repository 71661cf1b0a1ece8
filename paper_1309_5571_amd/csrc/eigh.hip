// Eigen-decomposition of symmetric blocks (Alg. 1, step 6: the eigenvalues of
// each block's density matrix decide which states the block keeps).
//
// One workgroup per block runs the cyclic two-sided Jacobi method with the
// round-robin ("circle") ordering: each round pairs every index with one
// other, the d/2 plane rotations J of a round are independent, so all of them
// are found together and then applied at once, A <- J^T A J and V <- V J.
// With the indices grouped by pair, A splits into 2x2 sub-blocks A_kl (rows of
// pair k, columns of pair l) that transform on their own, J_k^T A_kl J_l, so
// each thread takes whole sub-blocks: A is read and written once per round,
// and along a row the threads of consecutive l touch consecutive columns (the
// circle ordering puts pair l at columns r + l and r - l).  A sweep is d - 1
// rounds (every pair once); the method stops after a sweep with no rotation.
// Blocks of order <= 48 are held in LDS, larger ones (up to 2048) are worked
// on in global memory.
#include <hip/hip_runtime.h>

#include "internal.h"

namespace dmrg {

constexpr int EIG_TPB = 256;        // selection kernel
constexpr int EIG_TPB_SMALL = 512;  // Jacobi, blocks in LDS (a round has ~d^2/2 independent items)
constexpr int EIG_LDS_DIM = 48;  // A (padded rows) and V in LDS: 37 KB
constexpr int EIG_MAX_DIM = 2048;
constexpr int EIG_MAX_SWEEPS = 40;

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

template <bool SMALL>
__global__ __launch_bounds__(SMALL ? EIG_TPB_SMALL : 1024) void k_eigh(int nblk, const int64_t *__restrict__ off,
                                                  const int32_t *__restrict__ dim, const int64_t *__restrict__ woff,
                                                  double *__restrict__ a, double *__restrict__ w,
                                                  double *__restrict__ u, int32_t *__restrict__ info) {
    constexpr int NP = SMALL ? EIG_LDS_DIM / 2 : EIG_MAX_DIM / 2;  // pairs per round
    constexpr int NT = SMALL ? EIG_TPB_SMALL : 1024;                // threads
    __shared__ double sA[SMALL ? EIG_LDS_DIM * (EIG_LDS_DIM + 1) : 1];
    __shared__ double sV[SMALL ? EIG_LDS_DIM * EIG_LDS_DIM : 1];
    __shared__ double rc[NP], rs[NP];
    __shared__ int rp[NP], rq[NP], rf[NP];
    __shared__ double part[NT];
    __shared__ double diag[SMALL ? EIG_LDS_DIM : EIG_MAX_DIM];
    const int b = blockIdx.x;
    if (b >= nblk) return;
    const int d = dim[b];
    const int tid = threadIdx.x;
    if (d < 1 || d > EIG_MAX_DIM) {
        if (!SMALL && tid == 0 && info) info[b] = -1;  // unsupported order
        return;
    }
    if (SMALL != (d <= EIG_LDS_DIM)) return;  // the other kernel's block
    double *in = a + off[b], *out = u + off[b];
    // working matrices: LDS, or (large blocks) A in u and V in a
    const int lda = SMALL ? d + 1 : d;
    double *A = SMALL ? sA : out;
    double *V = SMALL ? sV : in;
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
        const double x = in[e];
        A[r * lda + c] = x;  // (large blocks: A = u written before V = a overwrites the input)
    }
    __syncthreads();
    for (int e = tid; e < d * d; e += NT) {
        const int r = e / d, c = e % d;
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
    // first entry of largest magnitude positive (the diagonal is read before
    // u, which holds A for large blocks, is overwritten)
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
    hipLaunchKernelGGL(k_eigh<true>, dim3(nblk), dim3(EIG_TPB_SMALL), 0, s, nblk, off, dim, woff, a, w, u, info);
    hipLaunchKernelGGL(k_eigh<false>, dim3(nblk), dim3(1024), 0, s, nblk, off, dim, woff, a, w, u, info);
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
