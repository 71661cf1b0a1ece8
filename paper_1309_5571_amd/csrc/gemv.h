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

}  // namespace dmrg
