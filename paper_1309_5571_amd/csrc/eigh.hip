// Eigen-decomposition of symmetric blocks (Alg. 1, step 6: the eigenvalues of
// each block's density matrix decide which states the block keeps).
//
// One workgroup per block runs the cyclic two-sided Jacobi method with the
// round-robin ("circle") ordering: each round pairs every index with one
// other, the d/2 plane rotations of a round are independent, so all of them
// are found together, then applied to the rows, then to the columns of A and
// of V (A <- J^T A J, V <- V J).  A sweep is d - 1 rounds (every pair once);
// the method stops after a sweep with no rotation.  Blocks of order <= 48 are
// held in LDS, larger ones (up to 2048) are worked on in global memory.
#include <hip/hip_runtime.h>

#include "internal.h"

namespace dmrg {

constexpr int EIG_TPB = 256;
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
__global__ __launch_bounds__(EIG_TPB) void k_eigh(int nblk, const int64_t *__restrict__ off,
                                                  const int32_t *__restrict__ dim, const int64_t *__restrict__ woff,
                                                  double *__restrict__ a, double *__restrict__ w,
                                                  double *__restrict__ u, int32_t *__restrict__ info) {
    constexpr int NP = SMALL ? EIG_LDS_DIM / 2 : EIG_MAX_DIM / 2;  // pairs per round
    __shared__ double sA[SMALL ? EIG_LDS_DIM * (EIG_LDS_DIM + 1) : 1];
    __shared__ double sV[SMALL ? EIG_LDS_DIM * EIG_LDS_DIM : 1];
    __shared__ double rc[NP], rs[NP];
    __shared__ int rp[NP], rq[NP];
    __shared__ double part[EIG_TPB];
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
    for (int e = tid; e < d * d; e += EIG_TPB) fro += in[e] * in[e];
    part[tid] = fro;
    __syncthreads();
    if (tid == 0) {
        double s = 0.0;
        for (int i = 0; i < EIG_TPB; ++i) s += part[i];
        part[0] = sqrt(s);
    }
    __syncthreads();
    // rotations below this size are skipped: the off-diagonal part left is
    // at the rounding level of the matrix norm
    const double thr = part[0] * 0x1p-53 / d;
    for (int e = tid; e < d * d; e += EIG_TPB) {
        const int r = e / d, c = e % d;
        const double x = in[e];
        A[r * lda + c] = x;  // (large blocks: A = u written before V = a overwrites the input)
    }
    __syncthreads();
    for (int e = tid; e < d * d; e += EIG_TPB) {
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
            for (int k = tid; k < np; k += EIG_TPB) {
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
                rp[k] = rot ? p : -1;
                rq[k] = q;
                any |= rot;
            }
            any = __syncthreads_or(any);
            if (!any) continue;
            rotated = 1;
            // rows p, q of A
            for (int e = tid; e < np * d; e += EIG_TPB) {
                const int k = e / d, j = e % d;
                const int p = rp[k];
                if (p < 0) continue;
                const int q = rq[k];
                const double c = rc[k], s = rs[k];
                const double x = A[p * lda + j], y = A[q * lda + j];
                A[p * lda + j] = c * x - s * y;
                A[q * lda + j] = s * x + c * y;
            }
            __syncthreads();
            // columns p, q of A and of V
            for (int e = tid; e < np * d; e += EIG_TPB) {
                const int k = e / d, i = e % d;
                const int p = rp[k];
                if (p < 0) continue;
                const int q = rq[k];
                const double c = rc[k], s = rs[k];
                const double x = A[i * lda + p], y = A[i * lda + q];
                A[i * lda + p] = c * x - s * y;
                A[i * lda + q] = s * x + c * y;
                const double vx = V[i * d + p], vy = V[i * d + q];
                V[i * d + p] = c * vx - s * vy;
                V[i * d + q] = s * vx + c * vy;
            }
            __syncthreads();
            // the rotated pair's element is zero in exact arithmetic: set it so
            // (its rounding residue would otherwise be rotated again)
            for (int k = tid; k < np; k += EIG_TPB) {
                const int p = rp[k];
                if (p < 0) continue;
                const int q = rq[k];
                A[p * lda + q] = 0.0;
                A[q * lda + p] = 0.0;
            }
            __syncthreads();
        }
        done = !rotated;
    }
    // eigenvalues in descending order (ties by index), eigenvectors with the
    // first entry of largest magnitude positive (the diagonal is read before
    // u, which holds A for large blocks, is overwritten)
    for (int i = tid; i < d; i += EIG_TPB) diag[i] = A[i * lda + i];
    __syncthreads();
    double *wb = w + woff[b];
    for (int i = tid; i < d; i += EIG_TPB) {
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
    hipLaunchKernelGGL(k_eigh<true>, dim3(nblk), dim3(EIG_TPB), 0, s, nblk, off, dim, woff, a, w, u, info);
    hipLaunchKernelGGL(k_eigh<false>, dim3(nblk), dim3(EIG_TPB), 0, s, nblk, off, dim, woff, a, w, u, info);
    DMRG_HIP(hipGetLastError());
    return DMRG_OK;
}

}  // extern "C"
