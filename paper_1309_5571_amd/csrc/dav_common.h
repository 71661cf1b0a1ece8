// Device-side pieces shared by the Davidson kernels and the projection kernel
// (which runs the Rayleigh step of the next Davidson iteration in its tail).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "gemv.h"

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

// Arrival counting for "last block does the tail" reductions, in two levels so
// that no counter sees more than ARRIVE_G serialized device-scope atomics:
// arrival idx of count goes to group idx / ARRIVE_G; the last arrival of a group
// bumps the member's top counter; the last group's last arrival is the last one.
// Each member owns CTR_STRIDE counters ([0] top, [1 + g] groups); the arrivals
// reset them, so they are zero again for the next kernel.
constexpr int ARRIVE_G = 16;
constexpr int CTR_STRIDE = 2048;  // supports up to ARRIVE_G * (CTR_STRIDE - 1) arrivals per member

static __device__ __forceinline__ bool last_arrival(int32_t *counters, int member, int idx, int count) {
    __shared__ int is_last;
    __syncthreads();
    if (threadIdx.x == 0) {
        int32_t *base = counters + (size_t)member * CTR_STRIDE;
        const int g = idx / ARRIVE_G, ngroups = (count + ARRIVE_G - 1) / ARRIVE_G;
        const int gsize = min(ARRIVE_G, count - g * ARRIVE_G);
        __threadfence();
        int last = 0;
        if (atomicAdd(&base[1 + g], 1) == gsize - 1) {
            base[1 + g] = 0;
            __threadfence();
            if (atomicAdd(&base[0], 1) == ngroups - 1) {
                base[0] = 0;
                last = 1;
            }
        }
        is_last = last;
    }
    __syncthreads();
    if (is_last) __threadfence();
    return is_last != 0;
}

// sum of partial column j over the member's chunks (fixed order), all threads get it
static __device__ double member_sum(const double *part, int c0, int c1, int j, double *lds) {
    double v = 0.0;
    for (int c = c0 + (int)threadIdx.x; c < c1; c += TPB) v += part[(size_t)c * (KM + 2) + j];
    double r[1] = {v};
    block_reduce<1>(r, 1, lds);
    return r[0];
}

// Lanes per column for all-column reductions: the largest power of two G <= 64
// with G * ncols <= TPB, so each column is owned by an aligned group of G lanes
// inside one wavefront and combined with shuffles (fixed order, no LDS loop).
static __device__ __forceinline__ int lanes_per_column(int ncols) {
    int G = 64;
    while (G > 1 && G * ncols > TPB) G >>= 1;
    return G;
}

// Sums columns [0, ncols) over rows [c0, c1) of the member's partial rows
// (row stride KM + 2).  out: shared [ncols]; all threads must call.
static __device__ void member_sums(const double *__restrict__ part, int c0, int c1, int ncols, double *scratch,
                                   double *out) {
    (void)scratch;
    const int G = lanes_per_column(ncols);
    const int j = threadIdx.x / G, l = threadIdx.x % G;
    double v = 0.0;
    if (j < ncols) {
#pragma unroll 4
        for (int c = c0 + l; c < c1; c += G) v += part[(size_t)c * (KM + 2) + j];
    }
    for (int off = G / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    if (j < ncols && l == 0) out[j] = v;
    __syncthreads();
}

// Smallest-first eigen-decomposition of the member's Rayleigh matrix B[:n,:n]
// by cyclic Jacobi in parallel (round-robin) order, run by ONE wavefront with
// wave-level ordering of its LDS traffic (no workgroup barriers).  Warm start:
// the matrix is first transformed by the previous eigenvectors extended with
// e_n, which makes it nearly diagonal (an arrowhead).  Threshold rotations:
// |a_pq| <= 1e-15 ||A||_F (a few ulps of the matrix, above the rounding noise
// that rotations leave in the off-diagonal) is skipped; the sweeps stop after
// one without rotations.
struct JacobiLds {
    double A[KM][KM + 1];
    double Vv[KM][KM + 1];
    double Tm[KM][KM + 1];
    double c[KM / 2], s[KM / 2];
    double red[4 * 2];
    int order[KM];
    int rotated;
};

static __device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// Call from the 64 lanes of one wavefront (threadIdx.x < 64) only.
static __device__ void jacobi_eig_wave(DavState &S, int n, JacobiLds &L) {
    const int lane = threadIdx.x & 63;
    for (int e = lane; e < n * n; e += 64) {
        const int r = e / n, c = e % n;
        L.Tm[r][c] = S.Bm[r * KM + c];
        L.Vv[r][c] = (r < n - 1 && c < n - 1) ? S.Y[r * KM + c] : (r == c ? 1.0 : 0.0);
    }
    wave_sync();
    for (int e = lane; e < n * n; e += 64) {  // A = B Vv
        const int r = e / n, c = e % n;
        double acc = 0.0;
        for (int k = 0; k < n; ++k) acc += L.Tm[r][k] * L.Vv[k][c];
        L.A[r][c] = acc;
    }
    wave_sync();
    for (int e = lane; e < n * n; e += 64) {  // Tm = Vv^T A
        const int r = e / n, c = e % n;
        double acc = 0.0;
        for (int k = 0; k < n; ++k) acc += L.Vv[k][r] * L.A[k][c];
        L.Tm[r][c] = acc;
    }
    wave_sync();
    double fro = 0.0;
    for (int e = lane; e < n * n; e += 64) {
        const int r = e / n, c = e % n;
        const double a = 0.5 * (L.Tm[r][c] + L.Tm[c][r]);  // exact symmetry
        L.A[r][c] = a;
        fro += a * a;
    }
    fro = wave_reduce(fro);
    wave_sync();
    const double tol = 1e-15 * sqrt(fro);
    const int n2 = (n + 1) & ~1;
    const int np = n2 / 2;
    for (int sweep = 0; sweep < 30; ++sweep) {
        int rotated = 0;
        for (int step = 0; step < n2 - 1; ++step) {
            if (lane < np) {
                const int k = lane;
                const int p = (k == 0) ? 0 : ((k - 1 + step) % (n2 - 1)) + 1;
                const int q = ((n2 - 2 - k + step) % (n2 - 1)) + 1;
                double cc = 1.0, ss = 0.0;
                if (p < n && q < n) {
                    const double apq = L.A[p][q], app = L.A[p][p], aqq = L.A[q][q];
                    if (fabs(apq) > tol) {
                        const double th = (aqq - app) / (2.0 * apq);
                        const double t = (th >= 0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
                        cc = 1.0 / sqrt(t * t + 1.0);
                        ss = t * cc;
                        rotated = 1;
                    }
                }
                L.c[k] = cc;
                L.s[k] = ss;
                L.order[2 * k] = p;
                L.order[2 * k + 1] = q;
            }
            wave_sync();
            for (int e = lane; e < np * n; e += 64) {  // rows: A <- J^T A
                const int k = e / n, j = e % n;
                const int p = L.order[2 * k], q = L.order[2 * k + 1];
                const double ss = L.s[k];
                if (p < n && q < n && ss != 0.0) {
                    const double cc = L.c[k], ap = L.A[p][j], aq = L.A[q][j];
                    L.A[p][j] = cc * ap - ss * aq;
                    L.A[q][j] = ss * ap + cc * aq;
                }
            }
            wave_sync();
            for (int e = lane; e < np * n; e += 64) {  // columns: A <- A J, Vv <- Vv J
                const int k = e / n, j = e % n;
                const int p = L.order[2 * k], q = L.order[2 * k + 1];
                const double ss = L.s[k];
                if (p < n && q < n && ss != 0.0) {
                    const double cc = L.c[k];
                    const double ap = L.A[j][p], aq = L.A[j][q];
                    L.A[j][p] = cc * ap - ss * aq;
                    L.A[j][q] = ss * ap + cc * aq;
                    const double vp = L.Vv[j][p], vq = L.Vv[j][q];
                    L.Vv[j][p] = cc * vp - ss * vq;
                    L.Vv[j][q] = ss * vp + cc * vq;
                }
            }
            wave_sync();
        }
        if (!__any(rotated)) break;
    }
    for (int a = lane; a < n; a += 64) {  // ascending order (stable rank)
        const double da = L.A[a][a];
        int rank = 0;
        for (int b = 0; b < n; ++b) {
            const double db = L.A[b][b];
            rank += (db < da) || (db == da && b < a);
        }
        L.order[rank] = a;
    }
    wave_sync();
    for (int e = lane; e < n * n; e += 64) {
        const int r = e / n, c = e % n;
        S.Y[r * KM + c] = L.Vv[r][L.order[c]];
    }
    for (int c = lane; c < n; c += 64) S.theta[c] = L.A[L.order[c]][L.order[c]];
}

}  // namespace dmrg
