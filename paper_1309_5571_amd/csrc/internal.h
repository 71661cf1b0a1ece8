// Internal structures of the projection/Davidson library (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "dmrg.h"

namespace dmrg {

// ---------------------------------------------------------------- status helpers
dmrg_status set_error(dmrg_status st, const char *fmt, ...);
void clear_error();

#define DMRG_HIP(call)                                                                    \
    do {                                                                                  \
        hipError_t e_ = (call);                                                           \
        if (e_ != hipSuccess)                                                             \
            return ::dmrg::set_error(e_ == hipErrorOutOfMemory ? DMRG_E_NOMEM : DMRG_E_HIP, \
                                     "%s failed: %s (%s:%d)", #call, hipGetErrorString(e_), \
                                     __FILE__, __LINE__);                                 \
    } while (0)

#define DMRG_TRY(expr)                 \
    do {                               \
        dmrg_status s_ = (expr);       \
        if (s_ < 0) return s_;         \
    } while (0)

// ---------------------------------------------------------------- device descriptors
// Where a GEMM operand lives.
enum : int16_t {
    OPD_ABS = 0,  // absolute device address (operator blocks, plan-owned copies)
    OPD_IN = 1,   // element offset into the call's input vector (psi, or gbar in the adjoint)
    OPD_TMP = 2   // element offset into the plan's intermediate buffer
};

// One GEMM contribution to an output matrix:  C += coef * op(P) op(Q)
//   P element (r, k): ptrans ? P[k * ldp + r] : P[r * ldp + k]   (r = output row)
//   Q element (k, c): qtrans ? Q[c * ldq + k] : Q[k * ldq + c]   (c = output column)
// with optional FP64 row scale pscale[r] and column scale qscale[c] applied to
// the operands on load (a diagonal factor of the term).
//
// A fused two-sided segment (fused = 1) computes, for the tile's rows, the
// intermediate slice T = P[rows, :K] Q[:K, :K2] (P = A block, Q = the input
// block, both as above) in LDS and then C += coef * T R^T with R the
// row-major B block read as R[c * ldr + k], k < K2.
// A copy segment (fused = 2) adds coef * pscale[r] qscale[c] X(r, c), X the
// input sub-matrix at element offset q with rows of ldq (a term whose block
// factors are identities or diagonals but whose input lies elsewhere in psi:
// the site factors of the l-1-1-r strategy move it).
// Every contribution is also multiplied by the constant w (the site matrix
// elements of an l-1-1-r record; 1 otherwise).
struct Seg {
    uint64_t p, q;            // address (OPD_ABS) or element offset
    uint64_t pscale, qscale;  // absolute FP64 addresses, 0 = none
    uint64_t r;               // fused: absolute address of the B block
    int32_t ldp, ldq;
    int32_t K;
    int32_t K2;   // fused: width of the intermediate
    int32_t ldr;  // fused: row length of the B block
    int16_t pkind, qkind;
    int16_t ptrans, qtrans;
    int16_t fused, pad16;
    int32_t coef;  // global coefficient index, -1 = 1.0
    int32_t term;  // global term index (for coefficient gradients), -1 = none
    double w = 1.0;  // constant factor of the contribution
};

// A purely diagonal contribution at an output pair:
//   C(r, c) += coef * vl[r] * vr[c] * X(r, c),  X = the call's input at the same pair.
//   vl / vr are read with strides sl / sr (1 for a diagonal operator; d + 1 to
//   walk the diagonal of a dense square block, used for the preconditioner).
struct DiagTerm {
    uint64_t vl, vr;  // absolute FP64 addresses of the pair's slices, 0 = ones
    int32_t coef;
    int32_t term;
    int32_t sl, sr;
    double w = 1.0;  // constant factor (1 for the LR strategy)
};

// One output tile.
struct Task {
    int32_t seg_begin, seg_end;
    int32_t diag_begin, diag_end;
    int64_t c_off;     // element offset of the output matrix (in y, gpsi or the intermediate buffer)
    int64_t x_off;     // element offset of the matching input block (diagonal terms)
    int32_t ldc;       // row length of the output matrix
    int32_t row0, col0;
    int32_t m, n;      // rows / columns of this tile (<= tile size)
    int32_t member;
    int32_t part0;     // first coefficient-gradient partial slot of this task
    int32_t rslot;     // output-tile tasks: Rayleigh partial row (member-contiguous)
};

// ---------------------------------------------------------------- host metadata
struct Pair {
    int32_t sl, sr;
    int64_t dl, dr;
    int64_t off;  // global offset in psi
};

struct OpBlock {  // resolved block of one operator (identity/diag/dense)
    int32_t src, dst;
    int32_t kind;       // DMRG_OP_*
    int64_t rows, cols; // dims of dst, src
    const double *data; // FP64 device address of the block (dense) or the diag slice (diag); null for identity
    int32_t op;         // global operator id
    int32_t blk;        // block index within the operator (dense), -1 otherwise
};

// A row-major sub-matrix of psi: rows x cols, consecutive rows ld elements apart.
struct Geo {
    int64_t off;
    int64_t rows, cols, ld;
};

struct Record {
    int32_t term;   // term index within the member
    int32_t gterm;  // global term index
    int32_t pin, pout;  // global pair indices
    OpBlock a, b;
    int32_t order;  // 0: (A X) B^T, 1: A (X B^T), 2: one-sided / diagonal
    // Y[gout] += c w A X[gin] B^T.  LR strategy: the pair blocks, w = 1;
    // l-1-1-r strategy: the [d_l x d_r] slices of fixed site indices, w the
    // product of the two site matrix elements.
    Geo gin, gout;
    int32_t oin, oout;  // indices of gin / gout in the plan's output sub-matrices
    double w;
};

struct Lists {  // device task lists of one pass
    Task *tasks = nullptr;
    int32_t ntask = 0;
    int32_t ns = 1;  // 16 x 16 sub-tiles per tile side: 1 when every tile fits 16 x 16, else 2
};

struct PassSet {  // everything one projection direction needs in one precision
    Lists stageA, stageB;
    int32_t *slot_begin = nullptr;  // [nprob + 1] Rayleigh partial rows of each member (stage B)
    Seg *segs = nullptr;
    DiagTerm *diags = nullptr;
    int32_t nseg = 0, ndiag = 0;
    int64_t tmp_elems = 0;  // intermediate buffer length (elements)
    int32_t npart = 0;      // coefficient-gradient partials (forward only)
};

// One low-precision operator copy made at plan creation.
struct ConvJob {
    const double *src;
    void *dst;
    int64_t rows, cols;
    int32_t mode;  // 0: full copy, 1: copy with a zero diagonal, 2: FP64 diagonal of a square block
    int32_t pad;
};

struct DavidsonWork;
struct BlockWork;

constexpr int KM = 48;  // largest Davidson subspace (kmax)

// Davidson context for a projection y = H x that feeds an iteration: every
// output tile writes its share of the dot products of y with V(:, 0..i-2) and
// with x itself (column i-1) as one partial row (row = the tile's rslot).  The
// rows are summed by the next kernel in the stream, so no tile waits on
// another and no device-scope fence is needed.
struct RayArgs {
    const double *V = nullptr;  // column j at V + j * n (j < i - 1); nullptr = plain projection
    int64_t n = 0;
    int i = 0;                  // columns of the partial rows; the last one is x^T y
    double *part = nullptr;     // partial rows, column-major: (row r, column j) at part[j * ld + r]
    int64_t ld = 0;
};

}  // namespace dmrg

struct dmrg_plan {
    int32_t nprob = 0;
    int32_t prec = DMRG_F64;
    int device = 0;
    int64_t n = 0;
    int64_t flop = 0;
    int64_t bytes = 0;
    int32_t nterm_total = 0;
    std::vector<int64_t> member_off;     // [nprob + 1]
    std::vector<int32_t> term_off;       // [nprob + 1]
    std::vector<dmrg::Pair> pairs;
    std::vector<int32_t> pair_member;
    std::vector<dmrg::Record> records;
    // the sub-matrices of psi that output tiles cover, in psi order (LR: the
    // pair blocks; l-1-1-r: every [d_l x d_r] slice of fixed site indices);
    // together they cover psi exactly once
    std::vector<dmrg::Geo> out_geo;
    std::vector<int32_t> out_member;
    // device pass sets: [prec slot][direction]  slot 0 = F64, slot 1 = plan precision
    dmrg::PassSet fwd[2], adj[2];
    // coefficient-gradient reduction (forward F64 pass): CSR over global terms
    int32_t *d_term_ptr = nullptr;
    int32_t *d_term_ent = nullptr;
    double *d_partials = nullptr;
    // plan-owned device memory
    std::vector<void *> owned;
    void *d_tmp = nullptr;  // intermediate buffer (max over passes, 8-byte elements)
    int64_t tmp_bytes = 0;
    void *d_multi_tmp = nullptr;  // intermediates of several vectors per launch (grown on demand)
    size_t multi_tmp_bytes = 0;
    // preconditioner diagonal tasks (elementwise): one DiagTerm list per pair
    dmrg::Task *d_diag_tasks = nullptr;
    dmrg::DiagTerm *d_diag_terms = nullptr;
    int32_t n_diag_tasks = 0;
    // reduced density matrices: output offsets per pair [npair + 1] (0 left, 1 right) and tile tasks
    std::vector<int64_t> rho_off[2];
    void *d_rho_tasks = nullptr;
    int32_t n_rho_tasks = 0;
    dmrg::DavidsonWork *dav = nullptr;
    dmrg::BlockWork *blk = nullptr;  // block Davidson-Liu workspace
    // caller workspace (null: the plan allocates its scratch itself): the
    // projection intermediate at offset 0, the coefficient-gradient partials
    // after it, the Davidson arrays for up to ws_kmax vectors at ws_dav
    char *ws = nullptr;
    size_t ws_bytes = 0;
    int32_t ws_kmax = 0;
    size_t ws_part = 0, ws_dav = 0;
};

namespace dmrg {
// plan.cpp
dmrg_status build_plan(dmrg_plan *plan, int32_t nprob, const dmrg_problem *probs, int32_t prec,
                       hipStream_t stream);
dmrg_status plan_free(dmrg_plan *plan);
int tile_for(int64_t rows, int64_t cols);
// project.hip
// mask: optional device [nprob]; tasks of members with mask[m] == 0 are skipped
// dfold: optional device [n]; the diagonal terms folded by launch_diag_fold for
// the same coefficients (replaces the per-term diagonal epilogue)
// ray: optional Davidson context (see RayArgs), stage-B tiles only
dmrg_status launch_project(dmrg_plan *plan, int slot, const double *coef, const double *in,
                           double *out, hipStream_t s, const int32_t *mask = nullptr,
                           const double *dfold = nullptr, const RayArgs *ray = nullptr);
dmrg_status launch_diag_fold(dmrg_plan *plan, int slot, const double *coef, double *out, hipStream_t s);
dmrg_status launch_adjoint(dmrg_plan *plan, const double *coef, const double *in, double *out,
                           hipStream_t s);
dmrg_status launch_gcoef(dmrg_plan *plan, const double *psi, const double *gbar, double *gcoef,
                         hipStream_t s);
dmrg_status launch_convert_jobs(const ConvJob *jobs, int njob, int prec, hipStream_t s);
dmrg_status launch_diagonal(dmrg_plan *plan, const double *coef, double *diag, hipStream_t s);
// four vectors in one launch where the plan's tiles allow it (else one launch each);
// vmask: optional device [4], a vector whose flag is 0 is not written
constexpr int PROJ_NVEC = 4;
dmrg_status launch_project_multi(dmrg_plan *plan, const double *coef, const double *in, int64_t in_stride,
                                 double *out, int64_t out_stride, const int32_t *vmask, hipStream_t s);
// davidson.hip
dmrg_status davidson_free(dmrg_plan *plan);
// bytes of the Davidson arrays of a subspace of kmax vectors (the pieces
// 256-byte aligned), for a plan whose analysis is done; tiles = the largest
// stage-B task count of its forward passes
size_t dav_workspace_bytes(const dmrg_plan *plan, int kmax, int tiles);
constexpr size_t WS_ALIGN = 256;
inline size_t ws_align(size_t b) { return (b + WS_ALIGN - 1) / WS_ALIGN * WS_ALIGN; }
// block.hip
dmrg_status block_free(dmrg_plan *plan);
// density.hip: output offsets and tile tasks of the reduced density matrices
dmrg_status build_density(dmrg_plan *plan, hipStream_t s);
}  // namespace dmrg
