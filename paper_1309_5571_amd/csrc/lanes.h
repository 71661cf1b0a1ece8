// Cross-lane sums on 64-wide wavefronts without the LDS crossbar: DPP moves
// inside each row of 16 lanes (quad permutations, then the half-row and row
// mirrors), v_readlane across the four rows.  Every lane of a group receives
// the same bits: each step adds the value of a partner lane whose own step
// adds this lane's value, and addition is commutative.  All lanes of the
// wavefront must be active.
#pragma once

#include <hip/hip_runtime.h>

namespace dmrg {

template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
    const int lo = __double2loint(v), hi = __double2hiint(v);
    return __hiloint2double(__builtin_amdgcn_mov_dpp(hi, CTRL, 0xF, 0xF, false),
                            __builtin_amdgcn_mov_dpp(lo, CTRL, 0xF, 0xF, false));
}

__device__ __forceinline__ double readlane_f64(double v, int lane) {
    const int lo = __double2loint(v), hi = __double2hiint(v);
    return __hiloint2double(__builtin_amdgcn_readlane(hi, lane), __builtin_amdgcn_readlane(lo, lane));
}

constexpr int DPP_XOR1 = 0xB1;         // quad_perm [1, 0, 3, 2]
constexpr int DPP_XOR2 = 0x4E;         // quad_perm [2, 3, 0, 1]
constexpr int DPP_HALF_MIRROR = 0x141;  // lane i <- 7 - i within each 8 lanes
constexpr int DPP_MIRROR = 0x140;       // lane i <- 15 - i within each row

// Sum over aligned groups of G lanes (G a power of two, 1 <= G <= 64).
template <int G>
__device__ __forceinline__ double group_sum(double v) {
    static_assert(G >= 1 && G <= 64 && (G & (G - 1)) == 0, "group size");
    if (G >= 2) v += dpp_f64<DPP_XOR1>(v);
    if (G >= 4) v += dpp_f64<DPP_XOR2>(v);
    if (G >= 8) v += dpp_f64<DPP_HALF_MIRROR>(v);
    if (G >= 16) v += dpp_f64<DPP_MIRROR>(v);
    if (G == 32) v += __shfl_xor(v, 16, 64);
    if (G == 64) v = (readlane_f64(v, 0) + readlane_f64(v, 16)) + (readlane_f64(v, 32) + readlane_f64(v, 48));
    return v;
}

__device__ __forceinline__ double group_sum(double v, int G) {
    switch (G) {
    case 1: return v;
    case 2: return group_sum<2>(v);
    case 4: return group_sum<4>(v);
    case 8: return group_sum<8>(v);
    case 16: return group_sum<16>(v);
    case 32: return group_sum<32>(v);
    default: return group_sum<64>(v);
    }
}

__device__ __forceinline__ double wave_min(double v) {
    v = fmin(v, dpp_f64<DPP_XOR1>(v));
    v = fmin(v, dpp_f64<DPP_XOR2>(v));
    v = fmin(v, dpp_f64<DPP_HALF_MIRROR>(v));
    v = fmin(v, dpp_f64<DPP_MIRROR>(v));
    return fmin(fmin(readlane_f64(v, 0), readlane_f64(v, 16)), fmin(readlane_f64(v, 32), readlane_f64(v, 48)));
}

}  // namespace dmrg
