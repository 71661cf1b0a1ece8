// Tall-skinny matrix-vector building blocks (device functions) shared by the
// Davidson kernels and the dmrg_gemv_* entry points.
//
// The paper's gemv_trans kernel (Sec. "gemv_trans()", Alg. 4) gives every
// thread a register "belt" of accumulators, one per column of the tall,
// narrow V, walks the rows with a grid-stride loop so reads stay coalesced,
// and finishes with a shared-memory reduction.  On CDNA4 the same idea maps to
// one wave64 per 64 consecutive rows, up to KMAX FP64 accumulators per lane,
// a DPP wave reduction and a cross-wave reduction in LDS; blocks
// write per-block partials that a second, fixed-order stage sums, so the
// result does not depend on scheduling.
#pragma once

#include <hip/hip_runtime.h>

#include "dmrg.h"
#include "lanes.h"

namespace dmrg {

constexpr int GEMV_THREADS = 256;

__device__ __forceinline__ double wave_reduce(double v) { return group_sum<64>(v); }

// Block-wide sum of KB values per thread into red[0..KB) (valid in all threads
// after the call).  lds must hold (GEMV_THREADS / 64) * KB doubles.
template <int KB>
__device__ __forceinline__ void block_reduce(double (&v)[KB], int kact, double *lds) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int j = 0; j < KB; ++j) {
        if (j < kact) {
            double s = wave_reduce(v[j]);
            if (lane == 0) lds[w * KB + j] = s;
        }
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < KB; ++j) {
        if (j < kact) {
            double s = 0.0;
#pragma unroll
            for (int q = 0; q < GEMV_THREADS / 64; ++q) s += lds[q * KB + j];
            v[j] = s;
        }
    }
    __syncthreads();
}

// s = V[:, :k]^T x, first stage: every block writes its k partial sums
// (block b's at part[b * KB ...]).
template <int KB>
__global__ __launch_bounds__(GEMV_THREADS) void k_gemv_t_part(int64_t n, int k, const double *__restrict__ V, int64_t ldv,
                                                     const double *__restrict__ x, double *__restrict__ part) {
    __shared__ double lds[4 * KB];
    double acc[KB];
#pragma unroll
    for (int j = 0; j < KB; ++j) acc[j] = 0.0;
    for (int64_t e = (int64_t)blockIdx.x * GEMV_THREADS + threadIdx.x; e < n; e += (int64_t)gridDim.x * GEMV_THREADS) {
        const double xv = x[e];
#pragma unroll
        for (int j = 0; j < KB; ++j)
            if (j < k) acc[j] += V[(int64_t)j * ldv + e] * xv;
    }
    block_reduce<KB>(acc, k, lds);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int j = 0; j < KB; ++j)
            if (j < k) part[(size_t)blockIdx.x * KB + j] = acc[j];
    }
}

// second stage: all k columns at once, thread t owns column t % k and every
// (GEMV_THREADS / k)-th block from t / k; slots are then added in order (deterministic)
template <int KB>
__global__ __launch_bounds__(GEMV_THREADS) void k_gemv_t_final(int nblk, int k, const double *__restrict__ part,
                                                      double *__restrict__ s) {
    __shared__ double slot_sum[GEMV_THREADS];
    const int t = threadIdx.x, per = GEMV_THREADS / k, j = t % k, slot = t / k;
    double v = 0.0;
    if (slot < per) {
#pragma unroll 4
        for (int b = slot; b < nblk; b += per) v += part[(size_t)b * KB + j];
    }
    slot_sum[t] = v;
    __syncthreads();
    if (t < k) {
        double acc = 0.0;
        for (int q = 0; q < per; ++q) acc += slot_sum[t + q * k];
        s[t] = acc;
    }
}

constexpr int GEMV_PART_BLOCKS = 1024;  // grid cap of the first stage of s = V^T x
constexpr int GEMV_PART_COLS = 64;      // largest k (the KB bucket of k > 32)

}  // namespace dmrg

// Both stages of s = V^T x on stream st, the partial sums in part (at least
// min(ceil(n / GEMV_THREADS), GEMV_PART_BLOCKS) * GEMV_PART_COLS doubles).
dmrg_status gemv_t_launch(int64_t n, int32_t k, const double *V, int64_t ldv, const double *x, double *s,
                          int nblk, double *part, hipStream_t st);
