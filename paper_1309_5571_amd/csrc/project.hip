// Superblock projection kernels for gfx950 (CDNA4, wave64).
//
// The projection of the LR strategy is a sum over operation records
//     Y_{jl} += c_k A_{k,i->j} X_{ik} B_{k,k->l}^T          (Eq. 10-11)
// evaluated in two launches over task lists built once per plan:
//   stage A: the intermediates T = A X (or X B^T) of two-sided records;
//   stage B: every output tile of y, summing all of its records' second
//            products, the one-sided records, and the diagonal terms, and
//            writing the tile exactly once (no atomics, fixed order).
// Both launches run the same grouped-GEMM kernel: one wavefront owns one
// output tile of up to 32 x 32 (2 x 2 MFMA sub-tiles of 16 x 16) and walks
// its list of GEMM segments.  The paper issues two cuBLAS dgemm calls per
// record on four CUDA streams (Alg. 6-7) to overlap many small GEMMs; here
// every tile of every record is one entry of a single launch instead.
//
// Operand lane layouts (checked on the device): lane l supplies A[l % 16][k]
// and B[k][l % 16] for the k of its group l / 16 (KPL consecutive k per group
// for BF16).  The accumulator layout differs: FP32/BF16 hold D[4 (l/16) + v]
// [l % 16] in value v, FP64 holds D[4 v + l/16][l % 16].
//
// Precisions: F64 uses v_mfma_f64_16x16x4; F32 uses v_mfma_f32_16x16x4 with
// FP32 accumulation inside a segment; BF16 uses v_mfma_f32_16x16x32_bf16.
// Across segments, and in the diagonal epilogue, sums are FP64.
#include <algorithm>
#include <cstdio>

#include "internal.h"
#include "lanes.h"

namespace dmrg {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

// ------------------------------------------------------------------ precision traits

__device__ __forceinline__ uint16_t f32_to_bf16_bits(float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);  // round to nearest, ties to even
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf16_bits_to_f32(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

template <int PREC>
struct Tr;

template <>
struct Tr<DMRG_F64> {
    typedef double store_t;  // operator copies / intermediates
    typedef double val_t;    // operand value in registers
    typedef v4d acc_t;
    // A k-block of 16 is four MFMA steps.  Consecutive layout: lane group g
    // holds k = kb + 4 g + j (step j), so a lane's operands are contiguous.
    // Strided layout: step j takes k = kb + 4 j + g, so the steps of a block
    // that lie beyond the contraction length can be skipped (short blocks).
    static constexpr int KPL = 4;
    template <bool STRIDED>
    __device__ static int kbase(int kb, int g) { return STRIDED ? kb + g : kb + KPL * g; }
    template <bool STRIDED>
    __device__ static constexpr int kstep() { return STRIDED ? 4 : 1; }
    template <bool STRIDED>
    __device__ static int nsteps(int rem) { return STRIDED ? min(KPL, (rem + 3) >> 2) : (rem > 0 ? KPL : 0); }
    // accumulator value v of lane (g = lane / 16, c = lane % 16) holds D[4 v + g][c]
    __device__ static int row(int g, int v) { return 4 * v + g; }
    __device__ static val_t from_in(double x) { return x; }
    __device__ static val_t from_store(store_t x) { return x; }
    __device__ static store_t to_store(double x) { return x; }
    __device__ static void mma(acc_t &c, const val_t (&a)[KPL], const val_t (&b)[KPL], int ns) {
#pragma unroll
        for (int j = 0; j < KPL; ++j)
            if (j < ns) c = __builtin_amdgcn_mfma_f64_16x16x4f64(a[j], b[j], c, 0, 0, 0);
    }
};

template <>
struct Tr<DMRG_F32> {
    typedef float store_t;
    typedef float val_t;
    typedef v4f acc_t;
    static constexpr int KPL = 4;  // k layouts as for FP64
    template <bool STRIDED>
    __device__ static int kbase(int kb, int g) { return STRIDED ? kb + g : kb + KPL * g; }
    template <bool STRIDED>
    __device__ static constexpr int kstep() { return STRIDED ? 4 : 1; }
    template <bool STRIDED>
    __device__ static int nsteps(int rem) { return STRIDED ? min(KPL, (rem + 3) >> 2) : (rem > 0 ? KPL : 0); }
    // accumulator value v of lane (g, c) holds D[4 g + v][c]
    __device__ static int row(int g, int v) { return 4 * g + v; }
    __device__ static val_t from_in(double x) { return (float)x; }
    __device__ static val_t from_store(store_t x) { return x; }
    __device__ static store_t to_store(double x) { return (float)x; }
    __device__ static void mma(acc_t &c, const val_t (&a)[KPL], const val_t (&b)[KPL], int ns) {
#pragma unroll
        for (int j = 0; j < KPL; ++j)
            if (j < ns) c = __builtin_amdgcn_mfma_f32_16x16x4f32(a[j], b[j], c, 0, 0, 0);
    }
};

template <>
struct Tr<DMRG_BF16> {
    typedef uint16_t store_t;  // bf16 bit pattern
    typedef uint16_t val_t;
    typedef v4f acc_t;
    // one 16x16x32 MFMA per k-block of 32: lane group g holds k = kb + 8 g + j
    // (one layout)
    static constexpr int KPL = 8;
    template <bool STRIDED>
    __device__ static int kbase(int kb, int g) { return kb + KPL * g; }
    template <bool STRIDED>
    __device__ static constexpr int kstep() { return 1; }
    template <bool STRIDED>
    __device__ static int nsteps(int rem) { return rem > 0 ? 1 : 0; }
    // accumulator value v of lane (g, c) holds D[4 g + v][c]
    __device__ static int row(int g, int v) { return 4 * g + v; }
    __device__ static val_t from_in(double x) { return f32_to_bf16_bits((float)x); }
    __device__ static val_t from_store(store_t x) { return x; }
    __device__ static store_t to_store(double x) { return f32_to_bf16_bits((float)x); }
    __device__ static void mma(acc_t &c, const val_t (&a)[KPL], const val_t (&b)[KPL], int ns) {
        if (ns <= 0) return;
        v8bf va, vb;
#pragma unroll
        for (int j = 0; j < KPL; ++j) {
            va[j] = __builtin_bit_cast(__bf16, a[j]);
            vb[j] = __builtin_bit_cast(__bf16, b[j]);
        }
        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(va, vb, c, 0, 0, 0);
    }
};

// ------------------------------------------------------------------ operand fetch

// P fragment: rows row (tile-local r), k = k0 + kstep j (k0: the lane's kbase)
template <int PREC, bool PIN, bool PT, bool ST = false>
__device__ __forceinline__ void load_p(typename Tr<PREC>::val_t (&v)[Tr<PREC>::KPL], const Seg &s,
                                       const double *__restrict__ in, const void *__restrict__ tmp, int row,
                                       bool row_ok, int k0, int K, double scale) {
    typedef Tr<PREC> T;
    if (PIN) {
        const double *P = in + s.p;
#pragma unroll
        for (int j = 0; j < T::KPL; ++j) {
            int k = k0 + j * T::template kstep<ST>();
            double x = 0.0;
            if (row_ok && k < K) x = PT ? P[(int64_t)k * s.ldp + row] : P[(int64_t)row * s.ldp + k];
            v[j] = T::from_in(x * scale);
        }
    } else {
        const typename T::store_t *P = (s.pkind == OPD_ABS)
                                           ? (const typename T::store_t *)(uintptr_t)s.p
                                           : (const typename T::store_t *)tmp + s.p;
#pragma unroll
        for (int j = 0; j < T::KPL; ++j) {
            int k = k0 + j * T::template kstep<ST>();
            typename T::store_t x = 0;
            if (row_ok && k < K) x = PT ? P[(int64_t)k * s.ldp + row] : P[(int64_t)row * s.ldp + k];
            v[j] = T::from_store(x);
        }
    }
}

// Q fragment: column col, k = k0 + kstep j (k0: the lane's kbase)
template <int PREC, bool QIN, bool QT, bool ST = false>
__device__ __forceinline__ void load_q(typename Tr<PREC>::val_t (&v)[Tr<PREC>::KPL], const Seg &s,
                                       const double *__restrict__ in, const void *__restrict__ tmp, int col,
                                       bool col_ok, int k0, int K, double scale) {
    typedef Tr<PREC> T;
    if (QIN) {
        const double *Q = in + s.q;
#pragma unroll
        for (int j = 0; j < T::KPL; ++j) {
            int k = k0 + j * T::template kstep<ST>();
            double x = 0.0;
            if (col_ok && k < K) x = QT ? Q[(int64_t)col * s.ldq + k] : Q[(int64_t)k * s.ldq + col];
            v[j] = T::from_in(x * scale);
        }
    } else {
        const typename T::store_t *Q = (s.qkind == OPD_ABS)
                                           ? (const typename T::store_t *)(uintptr_t)s.q
                                           : (const typename T::store_t *)tmp + s.q;
#pragma unroll
        for (int j = 0; j < T::KPL; ++j) {
            int k = k0 + j * T::template kstep<ST>();
            typename T::store_t x = 0;
            if (col_ok && k < K) x = QT ? Q[(int64_t)col * s.ldq + k] : Q[(int64_t)k * s.ldq + col];
            v[j] = T::from_store(x);
        }
    }
}

// Raw fragments for the reduced-precision paths: FP64 from the input vector,
// the stored type from operator blocks and intermediates, converted to the
// MFMA type only where consumed.  A conversion next to a guarded load makes the
// wavefront wait for that load before it issues the next one (the FP64 path
// needs no conversion and loads through load_p / load_q).
template <int PREC, bool IN>
struct RawT {
    typedef typename Tr<PREC>::store_t type;
};
template <int PREC>
struct RawT<PREC, true> {
    typedef double type;
};
template <int PREC, bool IN>
__device__ __forceinline__ void cvt_frag(typename Tr<PREC>::val_t (&v)[Tr<PREC>::KPL],
                                         const typename RawT<PREC, IN>::type (&x)[Tr<PREC>::KPL], double scale) {
#pragma unroll
    for (int j = 0; j < Tr<PREC>::KPL; ++j) {
        if constexpr (IN)
            v[j] = Tr<PREC>::from_in(x[j] * scale);
        else
            v[j] = Tr<PREC>::from_store(x[j]);
    }
}
// op(P)[row, k] (Q: op(Q)[k, col]) for k = k0 + kstep j, zero outside; the block
// at base + off, leading dimension ld, transposed when TR.
template <int PREC, bool IN, bool TR, bool ST>
__device__ __forceinline__ void load_raw(typename RawT<PREC, IN>::type (&v)[Tr<PREC>::KPL],
                                         const typename RawT<PREC, IN>::type *__restrict__ B, int ld, int rc,
                                         bool rc_ok, int k0, int K) {
    typedef typename RawT<PREC, IN>::type R;
#pragma unroll
    for (int j = 0; j < Tr<PREC>::KPL; ++j) {
        const int k = k0 + j * Tr<PREC>::template kstep<ST>();
        R x = 0;
        if (rc_ok && k < K) x = TR ? B[(int64_t)k * ld + rc] : B[(int64_t)rc * ld + k];
        v[j] = x;
    }
}
// As load_raw without a branch per load: indices outside the block are clamped
// to its element (0, 0) and the values zeroed after every load has been issued.
template <int PREC, bool IN, bool TR, bool ST>
__device__ __forceinline__ void load_raw_u(typename RawT<PREC, IN>::type (&v)[Tr<PREC>::KPL],
                                           const typename RawT<PREC, IN>::type *__restrict__ B, int ld, int rc,
                                           bool rc_ok, int k0, int K) {
    typedef typename RawT<PREC, IN>::type R;
#pragma unroll
    for (int j = 0; j < Tr<PREC>::KPL; ++j) {
        const int k = k0 + j * Tr<PREC>::template kstep<ST>();
        const bool ok = rc_ok && k < K;
        const int64_t kk = ok ? k : 0, r = ok ? rc : 0;
        v[j] = TR ? B[kk * ld + r] : B[r * ld + kk];
    }
#pragma unroll
    for (int j = 0; j < Tr<PREC>::KPL; ++j) {
        const int k = k0 + j * Tr<PREC>::template kstep<ST>();
        v[j] = (rc_ok && k < K) ? v[j] : (R)0;
    }
}
template <int PREC, bool IN>
__device__ __forceinline__ const typename RawT<PREC, IN>::type *raw_base(const double *__restrict__ in,
                                                                         const void *__restrict__ tmp, uint64_t a,
                                                                         int16_t kind) {
    typedef typename RawT<PREC, IN>::type R;
    if constexpr (IN)
        return in + a;
    else
        return (kind == OPD_ABS) ? (const R *)(uintptr_t)a : (const R *)tmp + a;
}

constexpr int PW = 4;            // wavefronts per workgroup
// dynamic LDS of the task kernel: PW partial tiles + one tile of output values
constexpr size_t TASK_LDS = (size_t)(PW * 32 * 33 + 1024) * sizeof(double);
// contraction length of one work item: 32 (8 MFMA k-blocks for FP64/FP32, one
// 16x16x32 block for BF16); DMRG_KC_WIDE=16 trades fewer operands in flight
// for more items (measured: faster on the large batch, slower on small blocks)
#ifndef DMRG_KC_WIDE
#define DMRG_KC_WIDE 32
#endif
template <int PREC>
__host__ __device__ constexpr int kc_of() { return PREC == DMRG_BF16 ? 32 : DMRG_KC_WIDE; }
constexpr int TASK_GRID_MAX = 4096;  // persistent grid cap (blocks loop over tasks)

// One work item: acc[sr][sc] += op(P)[tile rows, k0:k0+KC] op(Q)[k0:k0+KC, tile cols], KC = kc_of<PREC>().
// All operand loads of the item are issued before its MFMAs.
template <int PREC, int NS, bool PIN, bool PT, bool QIN, bool QT>
__device__ __forceinline__ void item_gemm(typename Tr<PREC>::acc_t (&acc)[2][2], const Seg &s, const Task &tk,
                                          const double *__restrict__ in, const void *__restrict__ tmp, int nsr,
                                          int nsc, int k0) {
    typedef Tr<PREC> T;
    constexpr int KB = 4 * T::KPL;  // k per MFMA block
    constexpr int NKB = kc_of<PREC>() / KB;  // blocks per item
    const int lane = threadIdx.x & 63;
    const int r16 = lane & 15, g = lane >> 4;
    int prow[NS], qcol[NS];
    bool pok[NS], qok[NS];
    double ps[NS], qs[NS];
#pragma unroll
    for (int t = 0; t < NS; ++t) {
        ps[t] = qs[t] = 1.0;
        int r = t * 16 + r16;
        pok[t] = r < tk.m;
        prow[t] = tk.row0 + (pok[t] ? r : 0);
        int c = t * 16 + r16;
        qok[t] = c < tk.n;
        qcol[t] = tk.col0 + (qok[t] ? c : 0);
        if (PIN && s.pscale && pok[t]) ps[t] = ((const double *)(uintptr_t)s.pscale)[prow[t]];
        if (QIN && s.qscale && qok[t]) qs[t] = ((const double *)(uintptr_t)s.qscale)[qcol[t]];
    }
    if constexpr (PREC == DMRG_F64) {
        typename T::val_t pv[NS][NKB][T::KPL], qv[NS][NKB][T::KPL];
        const double *P = raw_base<PREC, PIN>(in, tmp, s.p, s.pkind);
        const double *Q = raw_base<PREC, QIN>(in, tmp, s.q, s.qkind);
#pragma unroll
        for (int b = 0; b < NKB; ++b) {
            const int kk = T::template kbase<false>(k0 + b * KB, g);
#pragma unroll
            for (int t = 0; t < NS; ++t) {
                if (t < nsr) load_raw<PREC, PIN, PT, false>(pv[t][b], P, s.ldp, prow[t], pok[t], kk, s.K);
                if (t < nsc) load_raw<PREC, QIN, !QT, false>(qv[t][b], Q, s.ldq, qcol[t], qok[t], kk, s.K);
            }
        }
        // row / column scales after all loads are issued
#pragma unroll
        for (int b = 0; b < NKB; ++b)
#pragma unroll
            for (int t = 0; t < NS; ++t)
#pragma unroll
                for (int j = 0; j < T::KPL; ++j) {
                    if (PIN) pv[t][b][j] *= ps[t];
                    if (QIN) qv[t][b][j] *= qs[t];
                }
#pragma unroll
        for (int b = 0; b < NKB; ++b)
#pragma unroll
            for (int x = 0; x < NS; ++x)
#pragma unroll
                for (int y = 0; y < NS; ++y)
                    if (x < nsr && y < nsc) T::mma(acc[x][y], pv[x][b], qv[y][b], T::KPL);
    } else {
        typename RawT<PREC, PIN>::type pr[NS][NKB][T::KPL];
        typename RawT<PREC, QIN>::type qr[NS][NKB][T::KPL];
        const auto *P = raw_base<PREC, PIN>(in, tmp, s.p, s.pkind);
        const auto *Q = raw_base<PREC, QIN>(in, tmp, s.q, s.qkind);
#pragma unroll
        for (int b = 0; b < NKB; ++b) {
            const int kk = T::template kbase<false>(k0 + b * KB, g);
#pragma unroll
            for (int t = 0; t < NS; ++t) {
                if (t < nsr) load_raw<PREC, PIN, PT, false>(pr[t][b], P, s.ldp, prow[t], pok[t], kk, s.K);
                if (t < nsc) load_raw<PREC, QIN, !QT, false>(qr[t][b], Q, s.ldq, qcol[t], qok[t], kk, s.K);
            }
        }
#pragma unroll
        for (int b = 0; b < NKB; ++b) {
            typename T::val_t pv[NS][T::KPL], qv[NS][T::KPL];
#pragma unroll
            for (int t = 0; t < NS; ++t) {
                cvt_frag<PREC, PIN>(pv[t], pr[t][b], ps[t]);
                cvt_frag<PREC, QIN>(qv[t], qr[t][b], qs[t]);
            }
#pragma unroll
            for (int x = 0; x < NS; ++x)
#pragma unroll
                for (int y = 0; y < NS; ++y)
                    if (x < nsr && y < nsc) T::mma(acc[x][y], pv[x], qv[y], T::KPL);
        }
    }
}

// Wave-local ordering of LDS accesses (lanes of one wavefront exchange data
// through LDS; other wavefronts of the workgroup are not involved).
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// Fused two-sided segment on a tile of at most 16 rows:
//   Tl[r][k] = sum_i A[row0 + r][i] X[i][k]      (k < K2, MFMA, then into LDS)
//   acc[0][b] += Tl[r][:] R[col0 + c][:]^T        (second MFMA pass from LDS)
// Tl is rounded to the operand format before the second product, like the
// intermediate of the two-stage path.  tl: this wavefront's LDS slice
// (16 x 64 doubles).
template <int PREC, int NS>
__device__ __forceinline__ void fused_item(typename Tr<PREC>::acc_t (&acc)[2][2], const Seg &s, const Task &tk,
                                           const double *__restrict__ in, double *tl, int nsc) {
    typedef Tr<PREC> T;
    constexpr int KB = 4 * T::KPL;
    const int lane = threadIdx.x & 63;
    const int r16 = lane & 15, g = lane >> 4;
    const int ncs = (s.K2 + 15) >> 4;  // column sub-tiles of the intermediate (<= 4)
    const bool pok = r16 < tk.m;
    const int prow = tk.row0 + (pok ? r16 : 0);
    typename T::acc_t a1[4];
#pragma unroll
    for (int cs = 0; cs < 4; ++cs) a1[cs] = typename T::acc_t{0, 0, 0, 0};
    for (int k0 = 0; k0 < s.K; k0 += KB) {
        typename T::val_t pv[T::KPL], qv[4][T::KPL];
        const int kk = T::template kbase<true>(k0, g);
        if constexpr (T::KPL == 4 && PREC != DMRG_F64) {  // FP32: raw FP64 input, converted at the MFMA
            double qr[4][T::KPL];
            load_p<PREC, false, false, true>(pv, s, in, nullptr, prow, pok, kk, s.K, 1.0);
#pragma unroll
            for (int cs = 0; cs < 4; ++cs) {
                const int col = cs * 16 + r16;
                if (cs < ncs)
                    load_raw<PREC, true, true, true>(qr[cs], in + s.q, s.ldq, col < s.K2 ? col : 0, col < s.K2, kk,
                                                     s.K);
            }
#pragma unroll
            for (int cs = 0; cs < 4; ++cs)
                if (cs < ncs) cvt_frag<PREC, true>(qv[cs], qr[cs], 1.0);
        } else if constexpr (PREC != DMRG_F64) {  // BF16: unconditional loads, one sub-tile at a time
            load_p<PREC, false, false, true>(pv, s, in, nullptr, prow, pok, kk, s.K, 1.0);
#pragma unroll
            for (int cs = 0; cs < 4; ++cs) {
                const int col = cs * 16 + r16;
                if (cs < ncs) {
                    double qr[T::KPL];
                    load_raw_u<PREC, true, true, true>(qr, in + s.q, s.ldq, col < s.K2 ? col : 0, col < s.K2, kk,
                                                       s.K);
                    cvt_frag<PREC, true>(qv[cs], qr, 1.0);
                }
            }
        } else {
            load_p<PREC, false, false, true>(pv, s, in, nullptr, prow, pok, kk, s.K, 1.0);
#pragma unroll
            for (int cs = 0; cs < 4; ++cs) {
                const int col = cs * 16 + r16;
                if (cs < ncs)
                    load_q<PREC, true, false, true>(qv[cs], s, in, nullptr, col < s.K2 ? col : 0, col < s.K2, kk,
                                                    s.K, 1.0);
            }
        }
#pragma unroll
        for (int cs = 0; cs < 4; ++cs)
            if (cs < ncs) T::mma(a1[cs], pv, qv[cs], T::template nsteps<true>(s.K - k0));
    }
#pragma unroll
    for (int cs = 0; cs < 4; ++cs)
        if (cs < ncs) {
#pragma unroll
            for (int v = 0; v < 4; ++v) tl[T::row(g, v) * 64 + cs * 16 + r16] = (double)a1[cs][v];
        }
    wave_lds_sync();
    const typename T::store_t *R = (const typename T::store_t *)(uintptr_t)s.r;
    for (int k0 = 0; k0 < s.K2; k0 += KB) {
        typename T::val_t pv[T::KPL], qv[NS][T::KPL];
        const int kk = T::template kbase<true>(k0, g);
        if constexpr (PREC == DMRG_BF16) {  // every read first (k < 64: inside the slice), then the conversions
            double tv[T::KPL];
#pragma unroll
            for (int j = 0; j < T::KPL; ++j) tv[j] = tl[r16 * 64 + kk + j * T::template kstep<true>()];
#pragma unroll
            for (int j = 0; j < T::KPL; ++j) {
                const int k = kk + j * T::template kstep<true>();
                pv[j] = T::from_in((k < s.K2) ? tv[j] : 0.0);
            }
        } else {
#pragma unroll
            for (int j = 0; j < T::KPL; ++j) {
                const int k = kk + j * T::template kstep<true>();
                pv[j] = T::from_in((k < s.K2) ? tl[r16 * 64 + k] : 0.0);
            }
        }
#pragma unroll
        for (int b = 0; b < NS; ++b) {
            const int c = b * 16 + r16;
            const bool ok = c < tk.n;
            const int col = tk.col0 + (ok ? c : 0);
            if (b < nsc) {
#pragma unroll
                for (int j = 0; j < T::KPL; ++j) {
                    const int k = kk + j * T::template kstep<true>();
                    typename T::store_t x = 0;
                    if (ok && k < s.K2) x = R[(int64_t)col * s.ldr + k];
                    qv[b][j] = T::from_store(x);
                }
            }
        }
#pragma unroll
        for (int b = 0; b < NS; ++b)
            if (b < nsc) T::mma(acc[0][b], pv, qv[b], T::template nsteps<true>(s.K2 - k0));
    }
    wave_lds_sync();  // the slice is rewritten by this wavefront's next fused item
}

// All work items [first, nit) step PW of one segment, for one operand layout.
template <int PREC, int NS, bool PIN, bool PT, bool QIN, bool QT>
__device__ __forceinline__ void seg_items(typename Tr<PREC>::acc_t (&acc)[2][2], const Seg &s, const Task &tk,
                                       const double *__restrict__ in, const void *__restrict__ tmp, int nsr, int nsc,
                                       int first, int nit) {
    for (int it = first; it < nit; it += PW)
        item_gemm<PREC, NS, PIN, PT, QIN, QT>(acc, s, tk, in, tmp, nsr, nsc, it * kc_of<PREC>());
}

// One switch per segment on the operand layout (the task lists use 7 of the 16).
template <int PREC, int NS>
__device__ __forceinline__ void seg_dispatch(typename Tr<PREC>::acc_t (&acc)[2][2], const Seg &s, const Task &tk,
                                             const double *__restrict__ in, const void *__restrict__ tmp, int nsr,
                                             int nsc, int first, int nit) {
    const bool pin = s.pkind == OPD_IN, qin = s.qkind == OPD_IN;
    const int code = (pin ? 8 : 0) | (s.ptrans ? 4 : 0) | (qin ? 2 : 0) | (s.qtrans ? 1 : 0);
    switch (code) {
        case 0: seg_items<PREC, NS, false, false, false, false>(acc, s, tk, in, tmp, nsr, nsc, first, nit); break;
        case 1: seg_items<PREC, NS, false, false, false, true>(acc, s, tk, in, tmp, nsr, nsc, first, nit); break;
        case 2: seg_items<PREC, NS, false, false, true, false>(acc, s, tk, in, tmp, nsr, nsc, first, nit); break;
        case 3: seg_items<PREC, NS, false, false, true, true>(acc, s, tk, in, tmp, nsr, nsc, first, nit); break;
        case 4: seg_items<PREC, NS, false, true, false, false>(acc, s, tk, in, tmp, nsr, nsc, first, nit); break;
        case 5: seg_items<PREC, NS, false, true, false, true>(acc, s, tk, in, tmp, nsr, nsc, first, nit); break;
        case 6: seg_items<PREC, NS, false, true, true, false>(acc, s, tk, in, tmp, nsr, nsc, first, nit); break;
        case 7: seg_items<PREC, NS, false, true, true, true>(acc, s, tk, in, tmp, nsr, nsc, first, nit); break;
        case 8: seg_items<PREC, NS, true, false, false, false>(acc, s, tk, in, tmp, nsr, nsc, first, nit); break;
        case 9: seg_items<PREC, NS, true, false, false, true>(acc, s, tk, in, tmp, nsr, nsc, first, nit); break;
        case 10: seg_items<PREC, NS, true, false, true, false>(acc, s, tk, in, tmp, nsr, nsc, first, nit); break;
        case 11: seg_items<PREC, NS, true, false, true, true>(acc, s, tk, in, tmp, nsr, nsc, first, nit); break;
        case 12: seg_items<PREC, NS, true, true, false, false>(acc, s, tk, in, tmp, nsr, nsc, first, nit); break;
        case 13: seg_items<PREC, NS, true, true, false, true>(acc, s, tk, in, tmp, nsr, nsc, first, nit); break;
        case 14: seg_items<PREC, NS, true, true, true, false>(acc, s, tk, in, tmp, nsr, nsc, first, nit); break;
        default: seg_items<PREC, NS, true, true, true, true>(acc, s, tk, in, tmp, nsr, nsc, first, nit); break;
    }
}

__device__ __forceinline__ double wave_sum(double v) { return group_sum<64>(v); }

template <int PREC>
__device__ __forceinline__ void zero_acc(typename Tr<PREC>::acc_t (&acc)[2][2]) {
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = typename Tr<PREC>::acc_t{0, 0, 0, 0};
}

// diagonal-term contribution at output element (rr, cc) of a task's pair
__device__ __forceinline__ double diag_sum(const DiagTerm *__restrict__ diags, int d0, int d1,
                                           const double *__restrict__ coef, double x, int64_t rr, int64_t cc) {
    double val = 0.0;
    for (int d = d0; d < d1; ++d) {
        const DiagTerm dt = diags[d];
        double w = (coef ? coef[dt.coef] : 1.0) * dt.w * x;
        if (dt.vl) w *= ((const double *)(uintptr_t)dt.vl)[rr * dt.sl];
        if (dt.vr) w *= ((const double *)(uintptr_t)dt.vr)[cc * dt.sr];
        val += w;
    }
    return val;
}

// Copy segment (fused = 2) on a tile: v = pscale[r] qscale[c] X(r, c) for the
// tile's elements in the accumulator layout (zero outside the tile), X the
// input sub-matrix at s.q with rows s.ldq apart.  FP64 in every precision.
template <int PREC, int NS>
__device__ __forceinline__ void copy_item(double (&v)[NS][NS][4], const Seg &s, const Task &tk,
                                          const double *__restrict__ in) {
    const int lane = threadIdx.x & 63;
    const int r16 = lane & 15, g = lane >> 4;
    const double *X = in + s.q;
    const double *vl = (const double *)(uintptr_t)s.pscale, *vr = (const double *)(uintptr_t)s.qscale;
#pragma unroll
    for (int a = 0; a < NS; ++a)
#pragma unroll
        for (int b = 0; b < NS; ++b)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int r = a * 16 + Tr<PREC>::row(g, e), c = b * 16 + r16;
                double x = 0.0;
                if (r < tk.m && c < tk.n) {
                    const int64_t rr = tk.row0 + r, cc = tk.col0 + c;
                    x = X[rr * s.ldq + cc];
                    if (vl) x *= vl[rr];
                    if (vr) x *= vr[cc];
                }
                v[a][b][e] = x;
            }
}

// MODE 0: write the intermediate (store_t) of stage A.
// MODE 1: write FP64 output tiles with the diagonal epilogue (stage B).
// MODE 2: coefficient-gradient partials <gbar, segment product> per segment
//         and per diagonal term (stage B task list of the FP64 pass).
// A workgroup of PW wavefronts owns one output tile at a time (a persistent
// grid walks the cost-sorted task list).  In modes 0/1 the work items of a
// tile -- (segment, kc_of<PREC>()-long slice of its contraction) in list order -- are
// dealt round-robin to the wavefronts; the PW partial tiles are summed in a
// fixed order through LDS, so results do not depend on scheduling.
template <int PREC, int MODE, int NS>
__device__ __forceinline__ void tasks_run(const Task *__restrict__ tasks, int ntask, const Seg *__restrict__ segs,
                                          const DiagTerm *__restrict__ diags, const double *__restrict__ in,
                                          const void *__restrict__ tmp, void *__restrict__ out,
                                          const double *__restrict__ coef, const double *__restrict__ gbar,
                                          double *__restrict__ partials, const int32_t *__restrict__ mask,
                                          const double *__restrict__ dfold, RayArgs ray, double *smem_tasks) {
    typedef Tr<PREC> T;
    double(*red)[32][33] = reinterpret_cast<double(*)[32][33]>(smem_tasks);
    double *wtile = smem_tasks + PW * 32 * 33;  // output values of the tile (Rayleigh step)
    const int wave = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
    const int r16 = lane & 15, g = lane >> 4;
    for (int t = blockIdx.x; t < ntask; t += gridDim.x) {
        const Task tk = tasks[t];
        if (mask && !mask[tk.member]) continue;
        const int nsr = (tk.m + 15) >> 4, nsc = (tk.n + 15) >> 4;
        if (MODE == 2) {
            // one wavefront per segment: each partial slot has exactly one writer
            for (int si = tk.seg_begin + wave; si < tk.seg_end; si += PW) {
                const Seg s = segs[si];
                typename T::acc_t acc[2][2];
                double cv[NS][NS][4];
                zero_acc<PREC>(acc);
                if (s.fused == 2) {
                    copy_item<PREC, NS>(cv, s, tk, in);
                } else if (s.fused) {
                    fused_item<PREC, NS>(acc, s, tk, in, &red[wave][0][0], nsc);
                } else {
                    // one wavefront runs every work item of the segment (PW-strided item loop, 4 passes)
                    for (int f = 0; f < PW; ++f)
                        seg_dispatch<PREC, NS>(acc, s, tk, in, tmp, nsr, nsc, f, (s.K + kc_of<PREC>() - 1) / kc_of<PREC>());
                }
                double part = 0.0;
#pragma unroll
                for (int a = 0; a < NS; ++a)
#pragma unroll
                    for (int b = 0; b < NS; ++b)
#pragma unroll
                        for (int v = 0; v < 4; ++v) {
                            const int r = a * 16 + T::row(g, v), c = b * 16 + r16;
                            if (a < nsr && b < nsc && r < tk.m && c < tk.n)
                                part += (s.fused == 2 ? cv[a][b][v] : (double)acc[a][b][v]) *
                                        gbar[tk.c_off + (int64_t)(tk.row0 + r) * tk.ldc + tk.col0 + c];
                        }
                part = wave_sum(part) * s.w;
                if (lane == 0) partials[tk.part0 + (si - tk.seg_begin)] = part;
            }
            const int nseg = tk.seg_end - tk.seg_begin;
            for (int d = tk.diag_begin + wave; d < tk.diag_end; d += PW) {
                double part = 0.0;
                for (int e = lane; e < tk.m * tk.n; e += 64) {
                    const int64_t rr = tk.row0 + e / tk.n, cc = tk.col0 + e % tk.n;
                    const int64_t o = tk.c_off + rr * tk.ldc + cc;
                    part += diag_sum(diags, d, d + 1, nullptr, in[tk.x_off + rr * tk.ldc + cc], rr, cc) * gbar[o];
                }
                part = wave_sum(part);
                if (lane == 0) partials[tk.part0 + nseg + (d - tk.diag_begin)] = part;
            }
            continue;
        }
        // epilogue inputs (folded diagonal and the matching input entries) are
        // fetched before the GEMM work so their latency overlaps it
        constexpr int NQ = NS * NS;  // tile elements per thread: (16 NS)^2 / (64 PW)
        double pre_x[NQ], pre_d[NQ];
        if (MODE == 1 && dfold) {
#pragma unroll
            for (int qq = 0; qq < NQ; ++qq) {
                const int e = threadIdx.x + qq * 64 * PW;
                pre_x[qq] = pre_d[qq] = 0.0;
                if (e < tk.m * tk.n) {
                    const int64_t rr = tk.row0 + e / tk.n, cc = tk.col0 + e % tk.n;
                    pre_x[qq] = in[tk.x_off + rr * tk.ldc + cc];
                    pre_d[qq] = dfold[tk.c_off + rr * tk.ldc + cc];
                }
            }
        }
        double tot[NS][NS][4];
#pragma unroll
        for (int a = 0; a < NS; ++a)
#pragma unroll
            for (int b = 0; b < NS; ++b)
#pragma unroll
                for (int v = 0; v < 4; ++v) tot[a][b][v] = 0.0;
        int q = 0;  // work-item counter, identical in every wavefront
        for (int si = tk.seg_begin; si < tk.seg_end; ++si) {
            const int K = segs[si].K;
            const bool fused = segs[si].fused != 0;
            const int nit = fused ? 1 : (K + kc_of<PREC>() - 1) / kc_of<PREC>();  // a fused segment is one item
            const int first = (wave - q % PW + PW) % PW;  // first item of this segment owned by this wave
            if (first < nit) {
                const Seg s = segs[si];
                const double c = (s.coef >= 0 ? coef[s.coef] : 1.0) * s.w;
                if (s.fused == 2) {  // copy segment, summed in FP64
                    double cv[NS][NS][4];
                    copy_item<PREC, NS>(cv, s, tk, in);
#pragma unroll
                    for (int a = 0; a < NS; ++a)
#pragma unroll
                        for (int b = 0; b < NS; ++b)
#pragma unroll
                            for (int v = 0; v < 4; ++v) tot[a][b][v] += c * cv[a][b][v];
                } else {
                    typename T::acc_t acc[2][2];
                    zero_acc<PREC>(acc);
                    if (fused)
                        fused_item<PREC, NS>(acc, s, tk, in, &red[wave][0][0], nsc);
                    else
                        seg_dispatch<PREC, NS>(acc, s, tk, in, tmp, nsr, nsc, first, nit);
#pragma unroll
                    for (int a = 0; a < NS; ++a)
#pragma unroll
                        for (int b = 0; b < NS; ++b)
#pragma unroll
                            for (int v = 0; v < 4; ++v) tot[a][b][v] += c * (double)acc[a][b][v];
                }
            }
            q += nit;
        }
#pragma unroll
        for (int a = 0; a < NS; ++a)
#pragma unroll
            for (int b = 0; b < NS; ++b)
                if (a < nsr && b < nsc) {
#pragma unroll
                    for (int v = 0; v < 4; ++v) red[wave][a * 16 + T::row(g, v)][b * 16 + r16] = tot[a][b][v];
                }
        __syncthreads();
#pragma unroll
        for (int qq = 0; qq < NQ; ++qq) {
            const int e = threadIdx.x + qq * 64 * PW;
            if (e >= tk.m * tk.n) break;
            const int r = e / tk.n, c = e % tk.n;
            double val = 0.0;
#pragma unroll
            for (int w = 0; w < PW; ++w) val += red[w][r][c];
            const int64_t rr = tk.row0 + r, cc = tk.col0 + c;
            const int64_t o = tk.c_off + rr * tk.ldc + cc;
            if (MODE == 0) {
                ((typename T::store_t *)out)[o] = T::to_store(val);
            } else {
                if (dfold)  // sum_d c_d vl vr, folded once for fixed coefficients
                    val += pre_d[qq] * pre_x[qq];
                else if (tk.diag_end > tk.diag_begin)
                    val += diag_sum(diags, tk.diag_begin, tk.diag_end, coef, in[tk.x_off + rr * tk.ldc + cc], rr, cc);
                ((double *)out)[o] = val;
                if (MODE == 1 && ray.V) wtile[e] = val;
            }
        }
        if (MODE == 1 && ray.V) {
            // Rayleigh partials of the iteration this projection feeds: the
            // tile's share of [V(:, :i-1), x]^T y.  Wave w takes columns w, w + PW, ...;
            // its lanes run over the tile's elements (coalesced along tile rows)
            // and combine by shuffles in a fixed order.
            __syncthreads();  // wtile complete
            constexpr int JW = KM / PW;  // columns per wave
            const int ii = ray.i, cnt = tk.m * tk.n;
            double acc[JW];
#pragma unroll
            for (int jj = 0; jj < JW; ++jj) acc[jj] = 0.0;
            for (int e0 = 0; e0 < cnt; e0 += 4 * 64) {
                int64_t off[4];
                double wv[4];
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const int e = e0 + lane + 64 * k;
                    off[k] = 0;  // element 0 of the column: in bounds, weight 0
                    wv[k] = 0.0;
                    if (e < cnt) {
                        off[k] = tk.c_off + (int64_t)(tk.row0 + e / tk.n) * tk.ldc + tk.col0 + e % tk.n;
                        wv[k] = wtile[e];
                    }
                }
                // groups of 4 columns: one branch per group, loads of a group in flight together
#pragma unroll
                for (int jg = 0; jg < JW; jg += 4) {
                    if (wave + PW * jg < ii) {
#pragma unroll
                        for (int jj = jg; jj < jg + 4; ++jj) {
                            const int j = min(wave + PW * jj, ii - 1);
                            const double *Vj = (j == ii - 1) ? in : ray.V + (int64_t)j * ray.n;
#pragma unroll
                            for (int k = 0; k < 4; ++k) acc[jj] += Vj[off[k]] * wv[k];
                        }
                    }
                }
            }
#pragma unroll
            for (int jj = 0; jj < JW; ++jj) {
                const int j = wave + PW * jj;
                if (j < ii) {
                    const double v = wave_sum(acc[jj]);
                    if (lane == 0) ray.part[j * ray.ld + tk.rslot] = v;
                }
            }
        }
        __syncthreads();  // LDS is reused by the next task
    }
}

// ------------------------------------------------------------------ several vectors per launch

// NVEC vectors projected by one launch (FP64, plans whose tiles fit 16 x 16):
// each tile loads every operator fragment once and applies it to all NVEC
// vectors, so a tile's chain of dependent loads and products is shared.
constexpr int NVEC = PROJ_NVEC;
constexpr int NV_KC = 16;  // contraction length of one work item (registers: NVEC copies of one operand)

struct MultiArgs {
    int64_t in_stride = 0, out_stride = 0, tmp_stride = 0;  // elements between consecutive vectors
    const int32_t *vmask = nullptr;                         // device [NVEC]; 0 = vector not written
};

// Fused two-sided segment on a 16-row tile for NVEC vectors, the intermediate
// kept in registers: the first product is formed transposed,
//   D1 = X^T A^T  (16 columns of T as rows, the tile's rows as columns),
// so that value e of lane (g, c) holds T[c][16 cs + row(g, e)], which is what
// lane (g, c) supplies as the first operand of the second product's step e
// (rows c, contraction index 16 cs + row(g, e)); the second operand is the B
// block at the same index.  A and B fragments are loaded once per step and
// used for every vector.
template <int NV>
__device__ __forceinline__ void fused_item_nv(v4d (&acc)[NV], const Seg &s, const Task &tk,
                                              const double *__restrict__ in, int64_t stride) {
    typedef Tr<DMRG_F64> T;
    const int lane = threadIdx.x & 63;
    const int c = lane & 15, g = lane >> 4;
    const bool rok = c < tk.m;
    const int row = tk.row0 + (rok ? c : 0);
    const bool cok = c < tk.n;
    const int col = tk.col0 + (cok ? c : 0);
    const double *A = (const double *)(uintptr_t)s.p;
    const double *B = (const double *)(uintptr_t)s.r;
    const double *X = in + s.q;
    const int ncs = (s.K2 + 15) >> 4;
    for (int cs = 0; cs < ncs; ++cs) {
        v4d t1[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) t1[v] = v4d{0, 0, 0, 0};
        const int xc = cs * 16 + c;  // column of X (index of T's second dimension)
        const bool xok = xc < s.K2;
        for (int kb = 0; kb < s.K; kb += 16) {
            double a[4], x[NV][4];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int i = kb + 4 * j + g;  // strided: step j takes i = kb + 4 j + g
                const bool iok = i < s.K;
                a[j] = (rok && iok) ? A[(int64_t)row * s.ldp + i] : 0.0;
#pragma unroll
                for (int v = 0; v < NV; ++v)
                    x[v][j] = (xok && iok) ? X[v * stride + (int64_t)i * s.ldq + xc] : 0.0;
            }
            const int ns = min(4, (s.K - kb + 3) >> 2);
#pragma unroll
            for (int j = 0; j < 4; ++j)
                if (j < ns) {
#pragma unroll
                    for (int v = 0; v < NV; ++v)
                        t1[v] = __builtin_amdgcn_mfma_f64_16x16x4f64(x[v][j], a[j], t1[v], 0, 0, 0);
                }
        }
        double b[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int k = cs * 16 + T::row(g, e);
            b[e] = (cok && k < s.K2) ? B[(int64_t)col * s.ldr + k] : 0.0;
        }
#pragma unroll
        for (int e = 0; e < 4; ++e)
            if (cs * 16 + 4 * e < s.K2) {
#pragma unroll
                for (int v = 0; v < NV; ++v)
                    acc[v] = __builtin_amdgcn_mfma_f64_16x16x4f64(t1[v][e], b[e], acc[v], 0, 0, 0);
            }
    }
}

// One work item of a non-fused segment for NVEC vectors: the operand that is
// the call's input or the intermediate differs per vector (offset v stride),
// the operator block is loaded once.
template <bool PIN, bool PT, bool QIN, bool QT>
__device__ __forceinline__ void item_gemm_nv(v4d (&acc)[NVEC], const Seg &s, const Task &tk,
                                             const double *__restrict__ in, const double *__restrict__ tmp,
                                             const MultiArgs &ma, int k0) {
    typedef Tr<DMRG_F64> T;
    constexpr int KB = 16, NKB = NV_KC / 16;  // NV_KC of the contraction per item
    const int lane = threadIdx.x & 63;
    const int r16 = lane & 15, g = lane >> 4;
    const bool pok = r16 < tk.m, qok = r16 < tk.n;
    const int prow = tk.row0 + (pok ? r16 : 0), qcol = tk.col0 + (qok ? r16 : 0);
    const bool pv = s.pkind != OPD_ABS;  // which operand depends on the vector
    const double *P = (s.pkind == OPD_ABS) ? (const double *)(uintptr_t)s.p : (PIN ? in : tmp) + s.p;
    const double *Q = (s.qkind == OPD_ABS) ? (const double *)(uintptr_t)s.q : (QIN ? in : tmp) + s.q;
    const int64_t pstr = pv ? (PIN ? ma.in_stride : ma.tmp_stride) : 0;
    const int64_t qstr = pv ? 0 : (QIN ? ma.in_stride : ma.tmp_stride);
    double ps = 1.0, qs = 1.0;
    if (PIN && s.pscale && pok) ps = ((const double *)(uintptr_t)s.pscale)[prow];
    if (QIN && s.qscale && qok) qs = ((const double *)(uintptr_t)s.qscale)[qcol];
    double sh[NKB][4], pvec[NVEC][NKB][4];  // the shared operand, the per-vector one
#pragma unroll
    for (int b = 0; b < NKB; ++b) {
        const int kk = T::template kbase<false>(k0 + b * KB, g);
        if (pv) {
            load_raw<DMRG_F64, QIN, !QT, false>(sh[b], Q, s.ldq, qcol, qok, kk, s.K);
#pragma unroll
            for (int v = 0; v < NVEC; ++v)
                load_raw<DMRG_F64, PIN, PT, false>(pvec[v][b], P + v * pstr, s.ldp, prow, pok, kk, s.K);
        } else {
            load_raw<DMRG_F64, PIN, PT, false>(sh[b], P, s.ldp, prow, pok, kk, s.K);
#pragma unroll
            for (int v = 0; v < NVEC; ++v)
                load_raw<DMRG_F64, QIN, !QT, false>(pvec[v][b], Q + v * qstr, s.ldq, qcol, qok, kk, s.K);
        }
    }
#pragma unroll
    for (int b = 0; b < NKB; ++b)
#pragma unroll
        for (int v = 0; v < NVEC; ++v)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const double x = (pv ? pvec[v][b][j] : sh[b][j]) * (PIN ? ps : 1.0);
                const double y = (pv ? sh[b][j] : pvec[v][b][j]) * (QIN ? qs : 1.0);
                acc[v] = __builtin_amdgcn_mfma_f64_16x16x4f64(x, y, acc[v], 0, 0, 0);
            }
}

__device__ __forceinline__ void seg_items_nv(v4d (&acc)[NVEC], const Seg &s, const Task &tk,
                                             const double *__restrict__ in, const double *__restrict__ tmp,
                                             const MultiArgs &ma, int first, int nit) {
    const bool pin = s.pkind == OPD_IN, qin = s.qkind == OPD_IN;
    const int code = (pin ? 8 : 0) | (s.ptrans ? 4 : 0) | (qin ? 2 : 0) | (s.qtrans ? 1 : 0);
    for (int it = first; it < nit; it += PW) {
        const int k0 = it * NV_KC;
        switch (code) {
            case 0: item_gemm_nv<false, false, false, false>(acc, s, tk, in, tmp, ma, k0); break;
            case 1: item_gemm_nv<false, false, false, true>(acc, s, tk, in, tmp, ma, k0); break;
            case 2: item_gemm_nv<false, false, true, false>(acc, s, tk, in, tmp, ma, k0); break;
            case 3: item_gemm_nv<false, false, true, true>(acc, s, tk, in, tmp, ma, k0); break;
            case 4: item_gemm_nv<false, true, false, false>(acc, s, tk, in, tmp, ma, k0); break;
            case 5: item_gemm_nv<false, true, false, true>(acc, s, tk, in, tmp, ma, k0); break;
            case 8: item_gemm_nv<true, false, false, false>(acc, s, tk, in, tmp, ma, k0); break;
            case 9: item_gemm_nv<true, false, false, true>(acc, s, tk, in, tmp, ma, k0); break;
            case 12: item_gemm_nv<true, true, false, false>(acc, s, tk, in, tmp, ma, k0); break;
            default: item_gemm_nv<true, true, false, true>(acc, s, tk, in, tmp, ma, k0); break;
        }
    }
}

// The task loop for NVEC vectors (FP64, 16 x 16 tiles): MODE 0 writes the
// intermediates of stage A, MODE 1 the output tiles with the diagonal terms.
template <int MODE>
__global__ __launch_bounds__(64 * PW) __attribute__((amdgpu_waves_per_eu(2))) void k_tasks_nv(
    const Task *__restrict__ tasks, int ntask, const Seg *__restrict__ segs, const DiagTerm *__restrict__ diags,
    const double *__restrict__ in, const double *__restrict__ tmp_in, double *__restrict__ out,
    const double *__restrict__ coef, MultiArgs ma) {
    extern __shared__ __align__(16) double smem_tasks[];
    typedef Tr<DMRG_F64> T;
    double(*red)[32][33] = reinterpret_cast<double(*)[32][33]>(smem_tasks);
    const int wave = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
    const int r16 = lane & 15, g = lane >> 4;
    bool on[NVEC];
    bool any = false;
#pragma unroll
    for (int v = 0; v < NVEC; ++v) {
        on[v] = ma.vmask ? ma.vmask[v] != 0 : true;
        any = any || on[v];
    }
    if (!any) return;
    for (int t = blockIdx.x; t < ntask; t += gridDim.x) {
        const Task tk = tasks[t];
        double tot[NVEC][4];
#pragma unroll
        for (int v = 0; v < NVEC; ++v)
#pragma unroll
            for (int e = 0; e < 4; ++e) tot[v][e] = 0.0;
        int q = 0;
        for (int si = tk.seg_begin; si < tk.seg_end; ++si) {
            const int K = segs[si].K;
            const int fz = segs[si].fused;
            const int nit = fz ? 1 : (K + NV_KC - 1) / NV_KC;
            const int first = (wave - q % PW + PW) % PW;
            if (first < nit) {
                const Seg s = segs[si];
                const double cf = (s.coef >= 0 ? coef[s.coef] : 1.0) * s.w;
                if (fz == 2) {
#pragma unroll
                    for (int v = 0; v < NVEC; ++v) {
                        double cv[1][1][4];
                        copy_item<DMRG_F64, 1>(cv, s, tk, in + v * ma.in_stride);
#pragma unroll
                        for (int e = 0; e < 4; ++e) tot[v][e] += cf * cv[0][0][e];
                    }
                } else {
                    v4d acc[NVEC];
#pragma unroll
                    for (int v = 0; v < NVEC; ++v) acc[v] = v4d{0, 0, 0, 0};
                    if (fz)
                        fused_item_nv<NVEC>(acc, s, tk, in, ma.in_stride);
                    else
                        seg_items_nv(acc, s, tk, in, tmp_in, ma, first, nit);
#pragma unroll
                    for (int v = 0; v < NVEC; ++v)
#pragma unroll
                        for (int e = 0; e < 4; ++e) tot[v][e] += cf * acc[v][e];
                }
            }
            q += nit;
        }
        // per vector: partial tiles summed in a fixed order through LDS, then the epilogue
#pragma unroll
        for (int v = 0; v < NVEC; ++v) {
#pragma unroll
            for (int e = 0; e < 4; ++e) red[wave][T::row(g, e)][r16] = tot[v][e];
            __syncthreads();
            const int el = threadIdx.x;  // one element per thread (16 x 16 tiles)
            if (el < tk.m * tk.n && on[v]) {
                const int r = el / tk.n, c = el % tk.n;
                double val = 0.0;
#pragma unroll
                for (int w = 0; w < PW; ++w) val += red[w][r][c];
                const int64_t rr = tk.row0 + r, cc = tk.col0 + c;
                const int64_t o = tk.c_off + rr * tk.ldc + cc;
                if (MODE == 0) {
                    out[v * ma.tmp_stride + o] = val;
                } else {
                    if (tk.diag_end > tk.diag_begin)
                        val += diag_sum(diags, tk.diag_begin, tk.diag_end, coef,
                                        in[v * ma.in_stride + tk.x_off + rr * tk.ldc + cc], rr, cc);
                    out[v * ma.out_stride + o] = val;
                }
            }
            __syncthreads();
        }
    }
}

#define DMRG_TASK_ARGS                                                                                          \
    const Task *__restrict__ tasks, int ntask, const Seg *__restrict__ segs, const DiagTerm *__restrict__ diags, \
        const double *__restrict__ in, const void *__restrict__ tmp, void *__restrict__ out,                     \
        const double *__restrict__ coef, const double *__restrict__ gbar, double *__restrict__ partials,          \
        const int32_t *__restrict__ mask, const double *__restrict__ dfold, RayArgs ray
#define DMRG_TASK_PASS tasks, ntask, segs, diags, in, tmp, out, coef, gbar, partials, mask, dfold, ray, smem_tasks

// The task kernel.  The 16x16-tile forward variants are held to two
// workgroups per CU (at most 256 registers per lane): a pass has a few hundred
// tiles, and with one workgroup per CU the second half would wait a round.
template <int PREC, int MODE, int NS>
__global__ __launch_bounds__(64 * PW) void k_tasks(DMRG_TASK_ARGS) {
    extern __shared__ __align__(16) double smem_tasks[];
    tasks_run<PREC, MODE, NS>(DMRG_TASK_PASS);
}
template <int PREC, int MODE>
__global__ __launch_bounds__(64 * PW) __attribute__((amdgpu_waves_per_eu(2))) void k_tasks_w2(DMRG_TASK_ARGS) {
    extern __shared__ __align__(16) double smem_tasks[];
    tasks_run<PREC, MODE, 1>(DMRG_TASK_PASS);
}
#undef DMRG_TASK_ARGS
#undef DMRG_TASK_PASS

// gcoef[k] = sum of the partial slots listed for term k, in list order.
__global__ __launch_bounds__(64) void k_reduce_terms(const int32_t *__restrict__ ptr, const int32_t *__restrict__ ent,
                                                     const double *__restrict__ partials, double *__restrict__ gcoef,
                                                     int nterm) {
    const int k = blockIdx.x;
    if (k >= nterm) return;
    double s = 0.0;
    for (int i = ptr[k] + (int)threadIdx.x; i < ptr[k + 1]; i += 64) s += partials[ent[i]];
    s = wave_sum(s);
    if (threadIdx.x == 0) gcoef[k] = s;
}

// A tile's diagonal terms staged in LDS, DIAG_LDS at a time: slice addresses
// (null = ones), strides and coefficients.
constexpr int DIAG_LDS = 64;
struct DiagLds {
    const double *vl[DIAG_LDS], *vr[DIAG_LDS];
    double c[DIAG_LDS];
    int sl[DIAG_LDS], sr[DIAG_LDS];
};

// out = sum_d c_d vl[r sl] vr[c sr] over each task's diagonal terms, for
// every element of the task's tile (at most 1024 elements: 4 per thread).
// The terms are staged in LDS first, so the slice loads of several terms are
// in flight together; each element sums its terms in list order.
__global__ __launch_bounds__(256) void k_diag_terms(const Task *__restrict__ tasks, int ntask,
                                                    const DiagTerm *__restrict__ diags,
                                                    const double *__restrict__ coef, double *__restrict__ out) {
    __shared__ DiagLds D;
    for (int t = blockIdx.x; t < ntask; t += gridDim.x) {
        const Task tk = tasks[t];
        const int cnt = tk.m * tk.n;
        if (cnt <= 0) continue;
        int64_t rr[4], cc[4];
        double acc[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int e = min((int)threadIdx.x + 256 * q, cnt - 1);
            rr[q] = tk.row0 + e / tk.n;
            cc[q] = tk.col0 + e % tk.n;
            acc[q] = 0.0;
        }
        for (int d0 = tk.diag_begin; d0 < tk.diag_end; d0 += DIAG_LDS) {
            const int nt = min(DIAG_LDS, tk.diag_end - d0);
            __syncthreads();  // the previous terms are no longer read
            if ((int)threadIdx.x < nt) {
                const DiagTerm dt = diags[d0 + threadIdx.x];
                D.vl[threadIdx.x] = (const double *)(uintptr_t)dt.vl;
                D.vr[threadIdx.x] = (const double *)(uintptr_t)dt.vr;
                D.c[threadIdx.x] = coef[dt.coef] * dt.w;
                D.sl[threadIdx.x] = dt.sl;
                D.sr[threadIdx.x] = dt.sr;
            }
            __syncthreads();
#pragma unroll 4
            for (int d = 0; d < nt; ++d) {
                const double *vl = D.vl[d], *vr = D.vr[d];
                const double c = D.c[d];
                const int sl = D.sl[d], sr = D.sr[d];
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    double w = c;
                    if (vl) w *= vl[rr[q] * sl];
                    if (vr) w *= vr[cc[q] * sr];
                    acc[q] += w;
                }
            }
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int e = threadIdx.x + 256 * q;
            if (e < cnt) out[tk.c_off + rr[q] * tk.ldc + cc[q]] = acc[q];
        }
    }
}

// All operator-copy jobs of a plan in one launch: a block per job (grid-strided).
__global__ __launch_bounds__(256) void k_convert_jobs(const ConvJob *__restrict__ jobs, int njob, int prec) {
    for (int j = blockIdx.x; j < njob; j += gridDim.x) {
        const ConvJob jb = jobs[j];
        if (jb.mode == 2) {
            for (int64_t i = threadIdx.x; i < jb.rows; i += 256)
                ((double *)jb.dst)[i] = jb.src[i * (jb.rows + 1)];
            continue;
        }
        const int64_t cnt = jb.rows * jb.cols;
        for (int64_t e = threadIdx.x; e < cnt; e += 256) {
            double x = jb.src[e];
            if (jb.mode == 1 && (e / jb.cols) == (e % jb.cols)) x = 0.0;
            const float f = (float)x;
            if (prec == DMRG_F32)
                ((float *)jb.dst)[e] = f;
            else
                ((uint16_t *)jb.dst)[e] = f32_to_bf16_bits(f);
        }
    }
}

dmrg_status launch_convert_jobs(const ConvJob *jobs, int njob, int prec, hipStream_t s) {
    if (njob <= 0) return DMRG_OK;
    hipLaunchKernelGGL(k_convert_jobs, dim3(std::min(njob, 8192)), dim3(256), 0, s, jobs, njob, prec);
    DMRG_HIP(hipGetLastError());
    return DMRG_OK;
}

// ------------------------------------------------------------------ launchers

static dim3 task_grid(int ntask) { return dim3(std::min(ntask, TASK_GRID_MAX)); }

// k_tasks<PREC, MODE, NS> launch with the pass list's sub-tile count
template <int PREC, int MODE, class... Args>
static void launch_tasks(const Lists &l, size_t lds, hipStream_t s, Args... args) {
    if constexpr (MODE != 2) {
        if (l.ns == 1)
            hipLaunchKernelGGL((k_tasks_w2<PREC, MODE>), task_grid(l.ntask), dim3(64 * PW), lds, s, l.tasks,
                               l.ntask, args...);
        else
            hipLaunchKernelGGL((k_tasks<PREC, MODE, 2>), task_grid(l.ntask), dim3(64 * PW), lds, s, l.tasks,
                               l.ntask, args...);
    } else {
        if (l.ns == 1)
            hipLaunchKernelGGL((k_tasks<PREC, MODE, 1>), task_grid(l.ntask), dim3(64 * PW), lds, s, l.tasks,
                               l.ntask, args...);
        else
            hipLaunchKernelGGL((k_tasks<PREC, MODE, 2>), task_grid(l.ntask), dim3(64 * PW), lds, s, l.tasks,
                               l.ntask, args...);
    }
}

template <int PREC>
static dmrg_status run_pass(const PassSet &ps, const double *coef, const double *in, void *tmp, double *out,
                            hipStream_t s, const int32_t *mask, const double *dfold, const RayArgs *ray) {
    if (ps.stageA.ntask)
        launch_tasks<PREC, 0>(ps.stageA, TASK_LDS, s, (const Seg *)ps.segs, (const DiagTerm *)ps.diags, in,
                              (const void *)tmp, tmp, coef, (const double *)nullptr, (double *)nullptr, mask,
                              (const double *)nullptr, RayArgs{});
    if (ps.stageB.ntask) {
        const RayArgs ra = ray ? *ray : RayArgs{};
        launch_tasks<PREC, 1>(ps.stageB, TASK_LDS, s, (const Seg *)ps.segs, (const DiagTerm *)ps.diags, in,
                              (const void *)tmp, (void *)out, coef, (const double *)nullptr, (double *)nullptr, mask,
                              dfold, ra);
    }
    DMRG_HIP(hipGetLastError());
    return DMRG_OK;
}

dmrg_status launch_project(dmrg_plan *plan, int slot, const double *coef, const double *in, double *out,
                           hipStream_t s, const int32_t *mask, const double *dfold, const RayArgs *ray) {
    if (slot == 0) return run_pass<DMRG_F64>(plan->fwd[0], coef, in, plan->d_tmp, out, s, mask, dfold, ray);
    if (plan->prec == DMRG_F32)
        return run_pass<DMRG_F32>(plan->fwd[1], coef, in, plan->d_tmp, out, s, mask, dfold, ray);
    return run_pass<DMRG_BF16>(plan->fwd[1], coef, in, plan->d_tmp, out, s, mask, dfold, ray);
}

dmrg_status launch_adjoint(dmrg_plan *plan, const double *coef, const double *in, double *out, hipStream_t s) {
    return run_pass<DMRG_F64>(plan->adj[0], coef, in, plan->d_tmp, out, s, nullptr, nullptr, nullptr);
}

dmrg_status launch_diag_fold(dmrg_plan *plan, int slot, const double *coef, double *out, hipStream_t s) {
    const PassSet &ps = plan->fwd[slot];
    if (ps.stageB.ntask)
        hipLaunchKernelGGL(k_diag_terms, task_grid(ps.stageB.ntask), dim3(256), 0, s, ps.stageB.tasks,
                           ps.stageB.ntask, (const DiagTerm *)ps.diags, coef, out);
    DMRG_HIP(hipGetLastError());
    return DMRG_OK;
}

dmrg_status launch_gcoef(dmrg_plan *plan, const double *psi, const double *gbar, double *gcoef, hipStream_t s) {
    const PassSet &ps = plan->fwd[0];
    if (ps.stageA.ntask)
        launch_tasks<DMRG_F64, 0>(ps.stageA, TASK_LDS, s, (const Seg *)ps.segs, (const DiagTerm *)ps.diags, psi,
                                  (const void *)plan->d_tmp, (void *)plan->d_tmp, (const double *)nullptr,
                                  (const double *)nullptr, (double *)nullptr, (const int32_t *)nullptr,
                                  (const double *)nullptr, RayArgs{});
    if (ps.stageB.ntask)
        launch_tasks<DMRG_F64, 2>(ps.stageB, TASK_LDS, s, (const Seg *)ps.segs, (const DiagTerm *)ps.diags, psi,
                                  (const void *)plan->d_tmp, (void *)nullptr, (const double *)nullptr, gbar,
                                  plan->d_partials, (const int32_t *)nullptr, (const double *)nullptr, RayArgs{});
    if (plan->nterm_total)
        hipLaunchKernelGGL(k_reduce_terms, dim3(plan->nterm_total), dim3(64), 0, s, plan->d_term_ptr,
                           plan->d_term_ent, (const double *)plan->d_partials, gcoef, plan->nterm_total);
    DMRG_HIP(hipGetLastError());
    return DMRG_OK;
}

dmrg_status launch_diagonal(dmrg_plan *plan, const double *coef, double *diag, hipStream_t s) {
    if (plan->n_diag_tasks)
        hipLaunchKernelGGL(k_diag_terms, task_grid(plan->n_diag_tasks), dim3(256), 0, s, plan->d_diag_tasks,
                           plan->n_diag_tasks, (const DiagTerm *)plan->d_diag_terms, coef, diag);
    DMRG_HIP(hipGetLastError());
    return DMRG_OK;
}

// NVEC vectors per launch where every tile of the FP64 forward pass fits
// 16 x 16; otherwise one launch per vector.  vmask: device [NVEC] or null.
dmrg_status launch_project_multi(dmrg_plan *plan, const double *coef, const double *in, int64_t in_stride,
                                 double *out, int64_t out_stride, const int32_t *vmask, hipStream_t s) {
    const PassSet &ps = plan->fwd[0];
    if (ps.stageA.ns != 1 || ps.stageB.ns != 1) {
        for (int v = 0; v < NVEC; ++v)
            DMRG_TRY(launch_project(plan, 0, coef, in + v * in_stride, out + v * out_stride, s,
                                    vmask ? vmask + v : nullptr));
        return DMRG_OK;
    }
    MultiArgs ma;
    ma.in_stride = in_stride;
    ma.out_stride = out_stride;
    ma.tmp_stride = (ps.tmp_elems + 63) & ~(int64_t)63;
    ma.vmask = vmask;
    if (ps.stageA.ntask) {
        const size_t need = (size_t)NVEC * ma.tmp_stride * 8;
        if (need > plan->multi_tmp_bytes) {
            DMRG_HIP(hipStreamSynchronize(s));
            if (plan->d_multi_tmp) (void)hipFree(plan->d_multi_tmp);
            plan->d_multi_tmp = nullptr;
            plan->multi_tmp_bytes = 0;
            DMRG_HIP(hipMalloc(&plan->d_multi_tmp, need));
            plan->multi_tmp_bytes = need;
        }
        hipLaunchKernelGGL(k_tasks_nv<0>, task_grid(ps.stageA.ntask), dim3(64 * PW), TASK_LDS, s, ps.stageA.tasks,
                           ps.stageA.ntask, (const Seg *)ps.segs, (const DiagTerm *)ps.diags, in,
                           (const double *)plan->d_multi_tmp, (double *)plan->d_multi_tmp, coef, ma);
    }
    if (ps.stageB.ntask)
        hipLaunchKernelGGL(k_tasks_nv<1>, task_grid(ps.stageB.ntask), dim3(64 * PW), TASK_LDS, s, ps.stageB.tasks,
                           ps.stageB.ntask, (const Seg *)ps.segs, (const DiagTerm *)ps.diags, in,
                           (const double *)plan->d_multi_tmp, out, coef, ma);
    DMRG_HIP(hipGetLastError());
    return DMRG_OK;
}

}  // namespace dmrg

// ================================================================== ABI

using namespace dmrg;

static dmrg_status check_device(const dmrg_plan *plan) {
    int cur = -1;
    DMRG_HIP(hipGetDevice(&cur));
    if (cur != plan->device)
        return set_error(DMRG_E_INVALID_ARG, "plan was created on device %d but device %d is current", plan->device,
                         cur);
    return DMRG_OK;
}

extern "C" {

dmrg_status dmrg_project(dmrg_plan *plan, int32_t prec, const double *coef, const double *psi, double *y,
                         void *stream) {
    clear_error();
    if (!plan || !psi || !y || (!coef && plan->nterm_total))
        return set_error(DMRG_E_INVALID_ARG, "null plan, coef, psi or y");
    if (prec != DMRG_F64 && prec != plan->prec)
        return set_error(DMRG_E_INVALID_ARG, "precision %d not available in this plan (built for %d)", prec,
                         plan->prec);
    if (psi == y) return set_error(DMRG_E_INVALID_ARG, "psi and y must not overlap");
    DMRG_TRY(check_device(plan));
    return launch_project(plan, prec == DMRG_F64 ? 0 : 1, coef, psi, y, (hipStream_t)stream);
}

dmrg_status dmrg_project_backward(dmrg_plan *plan, const double *coef, const double *psi, const double *gbar,
                                  double *gpsi, double *gcoef, void *stream) {
    clear_error();
    if (!plan || !gbar) return set_error(DMRG_E_INVALID_ARG, "null plan or gbar");
    if (gpsi && !coef && plan->nterm_total) return set_error(DMRG_E_INVALID_ARG, "gpsi needs coef");
    if (gcoef && !psi) return set_error(DMRG_E_INVALID_ARG, "gcoef needs psi");
    if (gpsi && gpsi == gbar) return set_error(DMRG_E_INVALID_ARG, "gpsi and gbar must not overlap");
    DMRG_TRY(check_device(plan));
    hipStream_t s = (hipStream_t)stream;
    if (gcoef) DMRG_TRY(launch_gcoef(plan, psi, gbar, gcoef, s));
    if (gpsi) DMRG_TRY(launch_adjoint(plan, coef, gbar, gpsi, s));
    return DMRG_OK;
}

dmrg_status dmrg_project_block(dmrg_plan *plan, int32_t nvec, const double *coef, const double *psi,
                               int64_t ldpsi, double *y, int64_t ldy, void *stream) {
    clear_error();
    if (!plan || !psi || !y || (!coef && plan->nterm_total) || nvec < 0)
        return set_error(DMRG_E_INVALID_ARG, "null plan, coef, psi or y, or nvec < 0");
    if (ldpsi < plan->n || ldy < plan->n) return set_error(DMRG_E_INVALID_ARG, "ldpsi and ldy must be >= n");
    const double *pe = psi + (int64_t)std::max(nvec - 1, 0) * ldpsi + plan->n, *ye = y + (int64_t)std::max(nvec - 1, 0) * ldy + plan->n;
    if (nvec && psi < ye && y < pe) return set_error(DMRG_E_INVALID_ARG, "psi and y must not overlap");
    DMRG_TRY(check_device(plan));
    hipStream_t s = (hipStream_t)stream;
    int v = 0;
    for (; v + NVEC <= nvec; v += NVEC)
        DMRG_TRY(launch_project_multi(plan, coef, psi + (int64_t)v * ldpsi, ldpsi, y + (int64_t)v * ldy, ldy, nullptr,
                                      s));
    for (; v < nvec; ++v) DMRG_TRY(launch_project(plan, 0, coef, psi + (int64_t)v * ldpsi, y + (int64_t)v * ldy, s));
    return DMRG_OK;
}

dmrg_status dmrg_diagonal(dmrg_plan *plan, const double *coef, double *diag, void *stream) {
    clear_error();
    if (!plan || !diag || (!coef && plan->nterm_total)) return set_error(DMRG_E_INVALID_ARG, "null argument");
    DMRG_TRY(check_device(plan));
    return launch_diagonal(plan, coef, diag, (hipStream_t)stream);
}

}  // extern "C"
