// Operator blocks in the kept basis (Alg. 1, step 7: the block's basis is
// renormalized to the states of largest density-matrix eigenvalue).
//
// Every block O (sector src -> dst) of an operator becomes
// U_dst[:, :k_dst]^T O U_src[:, :k_src], with U the eigenvector blocks of the
// density matrix.  Two batched GEMM stages: T = O U_src (or diag(o) U_src),
// then U_dst^T T; each stage runs one workgroup per 32x32 output tile, four
// waves of FP64 MFMA 16x16x4.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <vector>

#include "internal.h"

namespace dmrg {

typedef double v4d_rn __attribute__((ext_vector_type(4)));

// One 32x32 tile of C = op(A) B:  op(A)(i, k) = A[i lda + k], or A[k lda + i]
// (trans), or (i == k) A[i] (diag, then K == M);  B(k, j) = B[k ldb + j].
struct GemmTile {
    const double *A, *B;
    double *C;
    int32_t lda, ldb, ldc;
    int32_t M, N, K;
    int32_t mode;  // 0 plain, 1 transposed A, 2 diagonal A
    int32_t ti, tj;
};

constexpr int RN_TILE = 32;

__global__ __launch_bounds__(256) void k_gemm_tiles(const GemmTile *__restrict__ tiles) {
    const GemmTile t = tiles[blockIdx.x];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int r16 = lane & 15, g = lane >> 4;
    const int r0 = t.ti * RN_TILE + 16 * (wave >> 1), c0 = t.tj * RN_TILE + 16 * (wave & 1);
    if (r0 >= t.M || c0 >= t.N) return;
    if (t.mode == 2) {  // C = diag(A) B: elementwise over the wave's quarter
        for (int e = lane; e < 256; e += 64) {
            const int r = r0 + (e >> 4), c = c0 + (e & 15);
            if (r < t.M && c < t.N) t.C[(int64_t)r * t.ldc + c] = t.A[r] * t.B[(int64_t)r * t.ldb + c];
        }
        return;
    }
    const int ra = min(r0 + r16, t.M - 1), cb = min(c0 + r16, t.N - 1);
    const bool oka = r0 + r16 < t.M, okb = c0 + r16 < t.N;
    v4d_rn acc = {0.0, 0.0, 0.0, 0.0};
    for (int k0 = 0; k0 < t.K; k0 += 16) {
        double a[4], b[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {  // clamped loads, all issued before any use
            const int k = min(k0 + 4 * j + g, t.K - 1);
            a[j] = t.mode == 1 ? t.A[(int64_t)k * t.lda + ra] : t.A[(int64_t)ra * t.lda + k];
            b[j] = t.B[(int64_t)k * t.ldb + cb];
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
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int r = r0 + 4 * v + g, c = c0 + r16;
        if (r < t.M && c < t.N) t.C[(int64_t)r * t.ldc + c] = acc[v];
    }
}

// Block placement for the enlargement of a block by one site (Alg. 1, step
// 2: the enlarged block's operators are Kronecker products of block and site
// operators, so each of their sector blocks is assembled from scaled copies of
// the block operator's blocks, or of identities): one workgroup per item,
// dst[i][j] += coef * src[i][j] (or coef * (i == j)).
struct PlaceItem {
    const double *src;
    double *dst;
    int32_t rows, cols, ld_src, ld_dst;
    double coef;
    int32_t identity;
};

__global__ __launch_bounds__(256) void k_place(const PlaceItem *__restrict__ items) {
    const PlaceItem it = items[blockIdx.x];
    for (int e = threadIdx.x; e < it.rows * it.cols; e += 256) {
        const int i = e / it.cols, j = e - i * it.cols;
        const double v = it.identity ? (i == j ? 1.0 : 0.0) : it.src[(int64_t)i * it.ld_src + j];
        it.dst[(int64_t)i * it.ld_dst + j] += it.coef * v;
    }
}

static void add_tiles(std::vector<GemmTile> &out, const GemmTile &base) {
    if (base.M <= 0 || base.N <= 0) return;
    for (int ti = 0; ti * RN_TILE < base.M; ++ti)
        for (int tj = 0; tj * RN_TILE < base.N; ++tj) {
            GemmTile t = base;
            t.ti = ti;
            t.tj = tj;
            out.push_back(t);
        }
}

// Device scratch of the host-side entry points below, one buffer per (device,
// stream), grown on demand and kept: after the first calls of a DMRG run (the
// largest step's sizes) these entry points allocate nothing.  Every call ends
// with a stream synchronization, so a buffer is idle whenever a call starts;
// calls on one stream from several host threads at once are not supported.
struct StreamScratch {
    void *p = nullptr;
    size_t bytes = 0;
};
static std::mutex g_rn_mutex;
static std::map<std::pair<int, hipStream_t>, StreamScratch> g_rn_scratch;

static dmrg_status stream_scratch(hipStream_t s, size_t need, void **out) {
    int dev = 0;
    DMRG_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lock(g_rn_mutex);
    StreamScratch &sc = g_rn_scratch[{dev, s}];
    if (need > sc.bytes) {
        if (sc.p) (void)hipFree(sc.p);
        sc.p = nullptr;
        sc.bytes = 0;
        const size_t grow = std::max(need, need + need / 2);
        DMRG_HIP(hipMalloc(&sc.p, grow));
        sc.bytes = grow;
    }
    *out = sc.p;
    return DMRG_OK;
}

}  // namespace dmrg

// ================================================================== ABI

using namespace dmrg;

extern "C" {

dmrg_status dmrg_renormalize(int32_t nblk, const dmrg_renorm_block *blocks, const double *data, const double *u,
                             double *out, void *stream) {
    clear_error();
    if (nblk < 0) return set_error(DMRG_E_INVALID_ARG, "negative block count");
    if (nblk == 0) return DMRG_OK;
    if (!blocks || !data || !u || !out) return set_error(DMRG_E_INVALID_ARG, "null argument");
    if ((const double *)out == data || (const double *)out == u)
        return set_error(DMRG_E_INVALID_ARG, "out must not overlap data or u");
    int64_t tmp_len = 0;
    for (int32_t b = 0; b < nblk; ++b) {
        const dmrg_renorm_block &B = blocks[b];
        if (B.rows < 1 || B.cols < 1 || B.k_dst < 0 || B.k_dst > B.rows || B.k_src < 0 || B.k_src > B.cols ||
            B.o < 0 || B.u_dst < 0 || B.u_src < 0 || B.out < 0 || (B.diag != 0 && B.diag != 1) ||
            (B.diag && B.rows != B.cols))
            return set_error(DMRG_E_INVALID_ARG, "block %d: bad sizes, offsets or kind", b);
        tmp_len += (int64_t)B.rows * B.k_src;
    }
    hipStream_t s = (hipStream_t)stream;
    std::vector<GemmTile> st1, st2;
    // the tile lists (counted here) and the intermediate share one scratch buffer
    auto ntiles = [](int64_t M, int64_t N) -> size_t {
        return M > 0 && N > 0 ? (size_t)((M + RN_TILE - 1) / RN_TILE) * (size_t)((N + RN_TILE - 1) / RN_TILE) : 0;
    };
    size_t nt = 0;
    for (int32_t b = 0; b < nblk; ++b) nt += ntiles(blocks[b].rows, blocks[b].k_src) + ntiles(blocks[b].k_dst, blocks[b].k_src);
    const size_t tile_bytes = ws_align(std::max<size_t>(nt, 1) * sizeof(GemmTile));
    void *scratch = nullptr;
    DMRG_TRY(stream_scratch(s, tile_bytes + (size_t)std::max<int64_t>(tmp_len, 1) * sizeof(double), &scratch));
    GemmTile *d_tiles = (GemmTile *)scratch;
    double *tmp = (double *)((char *)scratch + tile_bytes);
    int64_t toff = 0;
    for (int32_t b = 0; b < nblk; ++b) {
        const dmrg_renorm_block &B = blocks[b];
        double *T = tmp + toff;
        toff += (int64_t)B.rows * B.k_src;
        GemmTile a{};  // T [rows][k_src] = O U_src[:, :k_src]
        a.A = data + B.o;
        a.B = u + B.u_src;
        a.C = T;
        a.lda = B.cols;
        a.ldb = B.cols;
        a.ldc = B.k_src;
        a.M = B.rows;
        a.N = B.k_src;
        a.K = B.cols;
        a.mode = B.diag ? 2 : 0;
        add_tiles(st1, a);
        GemmTile c{};  // out [k_dst][k_src] = U_dst[:, :k_dst]^T T
        c.A = u + B.u_dst;
        c.B = T;
        c.C = out + B.out;
        c.lda = B.rows;
        c.ldb = B.k_src;
        c.ldc = B.k_src;
        c.M = B.k_dst;
        c.N = B.k_src;
        c.K = B.rows;
        c.mode = 1;
        add_tiles(st2, c);
    }
    const size_t n1 = st1.size(), n2 = st2.size();
    if (n1 + n2 > nt) return set_error(DMRG_E_INVALID_ARG, "internal: tile count %zu above %zu", n1 + n2, nt);
    hipError_t e = hipSuccess;
    std::vector<GemmTile> all(st1);
    all.insert(all.end(), st2.begin(), st2.end());
    if (!all.empty()) e = hipMemcpyAsync(d_tiles, all.data(), all.size() * sizeof(GemmTile), hipMemcpyHostToDevice, s);
    if (e == hipSuccess && n1) {
        hipLaunchKernelGGL(k_gemm_tiles, dim3((unsigned)n1), dim3(256), 0, s, d_tiles);
        e = hipGetLastError();
    }
    if (e == hipSuccess && n2) {
        hipLaunchKernelGGL(k_gemm_tiles, dim3((unsigned)n2), dim3(256), 0, s, d_tiles + n1);
        e = hipGetLastError();
    }
    // the host tile list must outlive its copy, and the scratch is idle for the next call
    const hipError_t e2 = hipStreamSynchronize(s);
    if (e != hipSuccess) return set_error(DMRG_E_HIP, "renormalize: %s", hipGetErrorString(e));
    if (e2 != hipSuccess) return set_error(DMRG_E_HIP, "renormalize: %s", hipGetErrorString(e2));
    return DMRG_OK;
}

dmrg_status dmrg_place_blocks(int32_t n, const dmrg_place *items, const double *src, double *dst, void *stream) {
    clear_error();
    if (n < 0) return set_error(DMRG_E_INVALID_ARG, "negative item count");
    if (n == 0) return DMRG_OK;
    if (!items || !dst) return set_error(DMRG_E_INVALID_ARG, "null argument");
    std::vector<PlaceItem> it(n);
    for (int32_t i = 0; i < n; ++i) {
        const dmrg_place &P = items[i];
        if (P.rows < 0 || P.cols < 0 || P.dst < 0 || P.ld_dst < P.cols || (P.identity != 0 && P.identity != 1) ||
            (!P.identity && (!src || P.src < 0 || P.ld_src < P.cols)))
            return set_error(DMRG_E_INVALID_ARG, "item %d: bad sizes, strides, offsets or kind", i);
        it[i].src = P.identity ? nullptr : src + P.src;
        it[i].dst = dst + P.dst;
        it[i].rows = P.rows;
        it[i].cols = P.cols;
        it[i].ld_src = P.ld_src;
        it[i].ld_dst = P.ld_dst;
        it[i].coef = P.coef;
        it[i].identity = P.identity;
    }
    hipStream_t s = (hipStream_t)stream;
    void *scratch = nullptr;
    DMRG_TRY(stream_scratch(s, (size_t)n * sizeof(PlaceItem), &scratch));
    PlaceItem *d_it = (PlaceItem *)scratch;
    hipError_t e = hipMemcpyAsync(d_it, it.data(), n * sizeof(PlaceItem), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_place, dim3(n), dim3(256), 0, s, d_it);
        e = hipGetLastError();
    }
    const hipError_t e2 = hipStreamSynchronize(s);
    if (e != hipSuccess) return set_error(DMRG_E_HIP, "place_blocks: %s", hipGetErrorString(e));
    if (e2 != hipSuccess) return set_error(DMRG_E_HIP, "place_blocks: %s", hipGetErrorString(e2));
    return DMRG_OK;
}

}  // extern "C"
