// Reduced density matrices of the two blocks (Alg. 1, step 5: each block's
// density matrix is formed from the superblock's lowest eigenstate).
//
// A left sector q_L meets exactly one right sector Q - q_L inside the target,
// so the q_L block of rho_L is Psi_p Psi_p^T of that pair's row-major block
// Psi_p [d_L, d_R] of psi, and the right block's is Psi_p^T Psi_p.  Both are
// symmetric rank-K updates: FP64 MFMA 16x16x4 tiles over the lower triangle
// of 32x32 output tiles, each value written to (r, c) and (c, r), so the
// result is exactly symmetric.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "internal.h"

namespace dmrg {

typedef double v4d_rho __attribute__((ext_vector_type(4)));

// One 32x32 output tile (ti >= tj) of one block of rho.
struct RhoTask {
    int64_t in_off;   // element offset of the pair's Psi block in psi
    int64_t out_off;  // element offset of the rho block in the output
    int32_t ld;       // row length of Psi (d_R)
    int32_t dim;      // order of the rho block
    int32_t K;        // contraction length
    int16_t side;     // 0: Psi Psi^T (left block), 1: Psi^T Psi (right block)
    int16_t pad;
    int32_t ti, tj;
};

constexpr int RHO_TILE = 32;

// Element (r, k) of the contraction operand: side 0 reads Psi[r][k], side 1 Psi[k][r].
__device__ __forceinline__ int64_t rho_index(int side, int ld, int r, int k) {
    return side == 0 ? (int64_t)r * ld + k : (int64_t)k * ld + r;
}

// Four waves, one 16x16 quarter of the tile each.  Step j of a k-block of 16
// takes k = k0 + 4 j + g (g = lane / 16), so steps past K are skipped.  The
// loads are clamped to the block and zeroed after all of them are issued.
__global__ __launch_bounds__(256) void k_density(const RhoTask *__restrict__ tasks, const double *__restrict__ psi,
                                                 double *__restrict__ rho_l, double *__restrict__ rho_r) {
    const RhoTask t = tasks[blockIdx.x];
    double *out = t.side == 0 ? rho_l : rho_r;
    if (!out) return;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int r16 = lane & 15, g = lane >> 4;
    const int r0 = t.ti * RHO_TILE + 16 * (wave >> 1), c0 = t.tj * RHO_TILE + 16 * (wave & 1);
    if (r0 >= t.dim || c0 >= t.dim || r0 + 15 < c0) return;  // outside, or above the diagonal
    const double *X = psi + t.in_off;
    const int ra = min(r0 + r16, t.dim - 1), cb = min(c0 + r16, t.dim - 1);
    const bool oka = r0 + r16 < t.dim, okb = c0 + r16 < t.dim;
    v4d_rho acc = {0.0, 0.0, 0.0, 0.0};
    for (int k0 = 0; k0 < t.K; k0 += 16) {
        double a[4], b[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int k = min(k0 + 4 * j + g, t.K - 1);
            a[j] = X[rho_index(t.side, t.ld, ra, k)];
            b[j] = X[rho_index(t.side, t.ld, cb, k)];
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const bool kin = k0 + 4 * j + g < t.K;
            a[j] = (oka && kin) ? a[j] : 0.0;
            b[j] = (okb && kin) ? b[j] : 0.0;
        }
#pragma unroll
        for (int j = 0; j < 4; ++j)
            if (k0 + 4 * j < t.K) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a[j], b[j], acc, 0, 0, 0);
    }
    // accumulator value v of lane (g, c) holds D[4 v + g][c]
    double *O = out + t.out_off;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int r = r0 + 4 * v + g, c = c0 + r16;
        if (r < t.dim && c <= r) {
            O[(int64_t)r * t.dim + c] = acc[v];
            if (c < r) O[(int64_t)c * t.dim + r] = acc[v];
        }
    }
}

dmrg_status build_density(dmrg_plan *plan, hipStream_t s) {
    const size_t np = plan->pairs.size();
    std::vector<RhoTask> tasks;
    for (int side = 0; side < 2; ++side) {
        std::vector<int64_t> &off = plan->rho_off[side];
        off.assign(np + 1, 0);
        for (size_t p = 0; p < np; ++p) {
            const Pair &pr = plan->pairs[p];
            const int64_t dim = side == 0 ? pr.dl : pr.dr, K = side == 0 ? pr.dr : pr.dl;
            off[p + 1] = off[p] + dim * dim;
            const int nt = (int)((dim + RHO_TILE - 1) / RHO_TILE);
            for (int ti = 0; ti < nt; ++ti)
                for (int tj = 0; tj <= ti; ++tj) {
                    RhoTask t{};
                    t.in_off = pr.off;
                    t.out_off = off[p];
                    t.ld = (int32_t)pr.dr;
                    t.dim = (int32_t)dim;
                    t.K = (int32_t)K;
                    t.side = (int16_t)side;
                    t.ti = ti;
                    t.tj = tj;
                    tasks.push_back(t);
                }
        }
    }
    // longest contractions first
    std::stable_sort(tasks.begin(), tasks.end(), [](const RhoTask &x, const RhoTask &y) { return x.K > y.K; });
    plan->n_rho_tasks = (int32_t)tasks.size();
    plan->d_rho_tasks = nullptr;
    if (tasks.empty()) return DMRG_OK;
    void *p = nullptr;
    DMRG_HIP(hipMalloc(&p, tasks.size() * sizeof(RhoTask)));
    plan->owned.push_back(p);
    DMRG_HIP(hipMemcpyAsync(p, tasks.data(), tasks.size() * sizeof(RhoTask), hipMemcpyHostToDevice, s));
    plan->d_rho_tasks = p;
    return DMRG_OK;
}

}  // namespace dmrg

// ================================================================== ABI

using namespace dmrg;

extern "C" {

dmrg_status dmrg_density_layout(const dmrg_plan *plan, int64_t *left_off, int64_t *right_off) {
    clear_error();
    if (!plan) return set_error(DMRG_E_INVALID_ARG, "null plan");
    int64_t *dst[2] = {left_off, right_off};
    for (int side = 0; side < 2; ++side)
        if (dst[side]) std::copy(plan->rho_off[side].begin(), plan->rho_off[side].end(), dst[side]);
    return DMRG_OK;
}

dmrg_status dmrg_density(dmrg_plan *plan, const double *psi, double *rho_left, double *rho_right, void *stream) {
    clear_error();
    if (!plan || !psi) return set_error(DMRG_E_INVALID_ARG, "null plan or psi");
    if ((const double *)rho_left == psi || (const double *)rho_right == psi ||
        (rho_left && rho_left == rho_right))
        return set_error(DMRG_E_INVALID_ARG, "psi, rho_left and rho_right must not overlap");
    int cur = -1;
    DMRG_HIP(hipGetDevice(&cur));
    if (cur != plan->device)
        return set_error(DMRG_E_INVALID_ARG, "plan was created on device %d but device %d is current", plan->device,
                         cur);
    if (plan->n_rho_tasks == 0 || (!rho_left && !rho_right)) return DMRG_OK;
    hipLaunchKernelGGL(k_density, dim3(plan->n_rho_tasks), dim3(256), 0, (hipStream_t)stream,
                       (const RhoTask *)plan->d_rho_tasks, psi, rho_left, rho_right);
    DMRG_HIP(hipGetLastError());
    return DMRG_OK;
}

}  // extern "C"
