// Device-resident Davidson iteration (Alg. 3) for one or many superblocks.
//
// Every member of a plan runs in lock step: all members share the subspace
// size i of an iteration, a member that has stopped is masked out, so the
// host knows the kernel sequence of each iteration in advance and can replay
// captured hipGraphs of several iterations.  Per iteration:
//
//   projection  W(:, i-1) = H V(:, i-1) (line 2); every output tile also
//               writes its partial row of V(:, :i)^T W(:, i-1)
//   k_ritz      B(:, i-1) from the tile rows (line 3) and the small
//               eigenproblem (line 4), solved redundantly in every block;
//               x = V y, r = W y - lambda x, ||r|| (lines 5-7),
//               t = r / (D - sigma) (line 10, shifted diagonal preconditioner),
//               s = V^T t (line 12, first pass): one sweep over V and W
//   k_restart   (when i = kmax) V <- V Y(:, :kmin), W <- W Y(:, :kmin), s = V^T t
//   k_orth      stop test (line 7), first Gram-Schmidt pass t' = t - V s
//               (line 13) and the rows of the second pass s2 = V^T t', ||t'||;
//               the next projection takes t' itself, and the next k_ritz
//               finishes V(:, i) = (t' - V s2) / nu (line 14) and W(:, i) by
//               linearity
//
// Reductions over the vector length never wait inside a kernel: each block
// writes one partial row, and EVERY block of the next kernel sums the rows of
// its member itself, in row order.  Results are therefore independent of
// scheduling, identical in all blocks (so every block takes the same stop and
// orthogonalization decisions), and identical between eager and graph runs.
// One block per member (the first chunk's) records the decisions in the
// member's state for the kernels that follow.  No kernel needs a device-scope
// fence: on gfx950 such a fence writes back and invalidates the L2 of the
// XCD, which would stall every other workgroup reading operator blocks.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "gemv.h"
#include "internal.h"

namespace dmrg {

constexpr int TPB = GEMV_THREADS;
constexpr int FUSED_RAYLEIGH_MAX_CHUNKS = 1024;  // see enqueue_iters
constexpr int PR_R = KM;      // partial-row column of ||r||^2
constexpr int PR_T = KM + 1;  // partial-row column of ||t||^2

// The Rayleigh matrix B = V^T H V itself is not stored: after every Rayleigh
// step Y^T B Y = diag(theta) up to the Jacobi threshold, which is all the next
// step needs (it only adds a row and column to B).
// Y and theta are double-buffered by the parity of the iteration that wrote them
// (the blocks of an iteration read the previous buffer while one of them writes).
struct DavState {
    double Y[2][KM * KM];  // eigenvectors of B (column c = Y[b][r * KM + c]), ascending
    double theta[2][KM];   // Ritz values, ascending
    double lambda, dmin, rnorm, rnorm1, tn0, tol, floor_;
    double rbest;  // smallest residual of the phase that halved the one before it
    int32_t converged, breakdown, iters, nproj, restarts, nvec, max_iter, bad_start;
    int32_t stag_window, rbest_it, stagnated;  // stagnation exit of a reduced-precision phase
};

// Per-member results copied to the host after every launch of iterations.
struct DavSummary {
    double energy, rnorm, rnorm1;  // rnorm1: residual of the phase's first iteration
    int32_t active, iters, nproj, restarts, converged, breakdown, bad_start, pad;
};

// Kernel-argument view of the Davidson workspace (plain pointers only).
struct DavArgs {
    int64_t n = 0;
    int nprob = 0;
    int nchunk = 0;
    double *V = nullptr, *W = nullptr, *T = nullptr, *D = nullptr, *coef = nullptr;
    double *dfold = nullptr;          // [n] folded diagonal terms of the current phase's pass
    // partial rows, stored column-major ([KM + 2][rows]) so that sums over rows
    // read contiguous memory
    double *pa = nullptr;             // rows of k_init_norm and k_ritz, one per chunk
    double *pb = nullptr;             // rows of k_restart
    double *pc = nullptr;             // rows of k_orth (second pass)
    double *ptile = nullptr;          // Rayleigh rows of the projection, one per output tile
    int64_t tile_ld = 0;              // rows of ptile
    int32_t *chunk_member = nullptr;
    int64_t *chunk_begin = nullptr;   // [nchunk + 1] element ranges
    int32_t *member_chunk = nullptr;  // [nprob + 1] chunk ranges
    int32_t *active = nullptr;        // [nprob] 1 while the member iterates
    DavState *st = nullptr;           // [nprob]
    const double *X0 = nullptr;       // [n] start vectors of the phase (private copy)
    DavSummary *sum = nullptr;        // [nprob] device view of pinned host memory
    // set-up gate of a phase queued behind another one: 1 when every member
    // finished the previous phase, else 0 and the phase idles (null: no gate)
    int32_t *gate = nullptr;
};

struct DavidsonWork {
    // arguments of the reduced-precision phase (a) and of the FP64 phase (a2):
    // the same basis and work buffers, each with its own activity flags,
    // folded diagonal and summary, so that the FP64 phase can be queued behind
    // the other before its outcome is known
    DavArgs a, a2;
    int kmax = 0, kmin = 0;
    int eig_solver = 0;
    DavSummary *h_sum = nullptr, *h_sum2 = nullptr;  // pinned, mapped [nprob]
    // iterations the last phase of each kind needed (first launch size of the next one);
    // kind = 4 * slot + 2 * (ends in X0) + (starts from X0)
    std::map<int, int> last_iters;
    // graphs by the key fields of each phase launch they hold, in order: slot + 2 * gated + 4 *
    // with the preconditioner diagonal, 4 * first i (0: with the phase set-up) + 2 *
    // finalize-into-X0 + parity of the first iteration, iterations, kmax, eig_solver,
    // max_iter, tol bits, floor bits
    std::map<std::vector<uint64_t>, hipGraphExec_t> graphs;
    std::vector<void *> owned;
    // set while a solve runs and cleared when every member ended with finite
    // data: a solve that stopped early, broke down or met a non-finite iterate
    // leaves the workspace dirty, and the next solve clears it first
    bool dirty = false;
    int32_t waits = 0;  // host synchronizations of the current dmrg_davidson call
    size_t rowb = 0;  // bytes of one partial-row column set per chunk / tile row
};

// ------------------------------------------------------------------ helpers

// Element range and member of chunk c, and the chunk range of that member.  A
// single-member plan needs no lookup: its chunks are consecutive TPB-element ranges.
struct Chunk {
    int member;
    int64_t e0, e1;
    int c0, c1;
};
__device__ __forceinline__ Chunk chunk_of(const DavArgs &w, int c) {
    Chunk k;
    if (w.nprob == 1) {
        k.member = 0;
        k.e0 = (int64_t)c * TPB;
        k.e1 = min(w.n, k.e0 + TPB);
        k.c0 = 0;
        k.c1 = w.nchunk;
    } else {
        k.member = w.chunk_member[c];
        k.e0 = w.chunk_begin[c];
        k.e1 = w.chunk_begin[c + 1];
        k.c0 = w.member_chunk[k.member];
        k.c1 = w.member_chunk[k.member + 1];
    }
    return k;
}

// Lanes per column for all-column reductions: the largest power of two G <= 64
// with G * ncols <= TPB, so each column is owned by an aligned group of G lanes
// inside one wavefront and combined with shuffles.
template <int NT = TPB>
static __device__ __forceinline__ int lanes_per_column(int ncols) {
    int G = 64;
    while (G > 1 && G * ncols > NT) G >>= 1;
    return G;
}

// One lane's share of a column sum: rows r, r + G, ... below r1, fetched in
// guarded batches of UMAX (UMAX / 2 for a short tail), every load of a batch
// in flight together, added into four running sums combined in a fixed order.
// Kernels that stream long vectors keep UMAX small (registers, occupancy).
template <int U>
static __device__ __forceinline__ void lane_rows(const double *__restrict__ col, int r, int r1, int G, double (&a)[4]) {
    double x[U];
#pragma unroll
    for (int u = 0; u < U; ++u) x[u] = (r + u * G < r1) ? col[r + u * G] : 0.0;
#pragma unroll
    for (int u = 0; u < U; ++u) a[u & 3] += x[u];
}
template <int UMAX>
static __device__ __forceinline__ double lane_col_sum(const double *__restrict__ col, int r, int r1, int G) {
    double a[4] = {0.0, 0.0, 0.0, 0.0};
    for (; r + (UMAX / 2) * G < r1; r += UMAX * G) lane_rows<UMAX>(col, r, r1, G, a);
    if (r < r1) lane_rows<UMAX / 2>(col, r, r1, G, a);
    return (a[0] + a[1]) + (a[2] + a[3]);
}

// out[q] = sum of partial rows [r0, r1) in column col(q), q < nq, where
// col(q) = q for q < i and KM + (q - i) beyond (the norm columns); element
// (r, col) at part[col * ld + r].  Each lane keeps 4 running sums (rows
// interleaved), combined in a fixed order; all threads must call; out is shared.
template <int NT = TPB>
static __device__ void sum_rows(const double *__restrict__ part, int64_t ld, int r0, int r1, int i, int nq,
                                double *out) {
    const int G = lanes_per_column<NT>(nq);
    const int q = threadIdx.x / G, l = threadIdx.x % G;
    double v = 0.0;
    if (q < nq) v = lane_col_sum<8>(part + (int64_t)(q < i ? q : KM + (q - i)) * ld, r0 + l, r1, G);
    v = group_sum(v, G);
    if (q < nq && l == 0) out[q] = v;
    __syncthreads();
}

// Two sums_rows at once (one barrier): columns [0, nqa) of set a, then [0, nqb)
// of set b, each mapped as in sum_rows; every lane group owns one column.
static __device__ void sum_rows2(const double *__restrict__ pa, int64_t lda, int a0, int a1, int ia, int nqa,
                                 double *outa, const double *__restrict__ pb, int64_t ldb, int b0, int b1, int ib,
                                 int nqb, double *outb) {
    const int nq = nqa + nqb;
    const int G = lanes_per_column(nq);
    const int q = threadIdx.x / G, l = threadIdx.x % G;
    double v = 0.0;
    if (q < nq) {
        const bool A = q < nqa;
        const int qq = A ? q : q - nqa, ii = A ? ia : ib;
        const double *col = (A ? pa : pb) + (int64_t)(qq < ii ? qq : KM + (qq - ii)) * (A ? lda : ldb);
        const int r0 = A ? a0 : b0, r1 = A ? a1 : b1;
        v = lane_col_sum<32>(col, r0 + l, r1, G);
    }
    v = group_sum(v, G);
    if (q < nq && l == 0) {
        if (q < nqa)
            outa[q] = v;
        else
            outb[q - nqa] = v;
    }
    __syncthreads();
}

static __device__ double block_min(double v, double *lds) {
    v = wave_min(v);
    if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = v;
    __syncthreads();
    double m = lds[0];
#pragma unroll
    for (int q = 1; q < TPB / 64; ++q) m = fmin(m, lds[q]);
    __syncthreads();
    return m;
}

static __device__ __forceinline__ void deactivate(const DavArgs &w, int member) { w.active[member] = 0; }

// Stop test on the residual norm: 0 go on, 1 converged, 2 iteration limit,
// 3 non-finite, 4 stagnated (reduced-precision phase only).  Reads only state
// written by earlier kernels, so every block of a kernel decides alike.
static __device__ __forceinline__ int stop_code(const DavState &S, double rr) {
    const double rn = sqrt(rr);
    if (!(rn == rn) || isinf(rn)) return 3;
    if (rn <= S.tol) return 1;
    if (S.iters >= S.max_iter) return 2;
    if (S.stagnated) return 4;
    return 0;
}

// Stagnation bookkeeping at the start of a Rayleigh step (one thread per
// member): the residual of the previous iteration either halves the best one
// so far or counts toward the window.
static __device__ __forceinline__ void track_stagnation(DavState &S) {
    if (S.stag_window <= 0 || S.iters < 1) return;
    if (S.rnorm < 0.5 * S.rbest) {
        S.rbest = S.rnorm;
        S.rbest_it = S.iters;
    } else if (S.iters - S.rbest_it >= S.stag_window) {
        S.stagnated = 1;
    }
}

// ------------------------------------------------------------------ init kernels

// Phase start of member m: options, flags and counters.
static __device__ void set_state(const DavArgs &w, int m, double tol, double floor_, int max_iter, int stag) {
    DavState &S = w.st[m];
    S.stag_window = stag;
    S.rbest = INFINITY;
    S.rbest_it = 0;
    S.stagnated = 0;
    S.tol = tol;
    S.floor_ = floor_;
    S.max_iter = max_iter;
    w.active[m] = 1;
    S.converged = 0;
    S.breakdown = 0;
    S.bad_start = 0;
    S.nvec = 1;
    S.iters = 0;  // counts are per phase; the host adds the phases
    S.nproj = 0;
    S.restarts = 0;
    S.rnorm = 0.0;
    S.rnorm1 = 0.0;
    S.Y[0][0] = S.Y[1][0] = 1.0;
}

// Gate of a phase queued behind another (one block): open when no member of
// the previous phase (flags prev) still iterates; closed, this phase's members
// are marked idle and its set-up leaves every shared buffer untouched.
__global__ __launch_bounds__(TPB) void k_gate(const int32_t *__restrict__ prev, DavArgs w) {
    int any = 0;
    for (int m = threadIdx.x; m < w.nprob; m += TPB) any |= prev[m];
    any = __syncthreads_or(any);
    if (threadIdx.x == 0) *w.gate = any ? 0 : 1;
    if (any)
        for (int m = threadIdx.x; m < w.nprob; m += TPB) w.active[m] = 0;
}

// Phase start (the first block of each member resets its state); partial
// rows: ||psi||^2 (column 0) and min D (column 1) of each chunk.
__global__ __launch_bounds__(TPB) void k_init_norm(const double *__restrict__ psi, DavArgs w, double tol,
                                                   double floor_, int max_iter, int stag) {
    __shared__ double lds[4];
    if (w.gate && !*w.gate) return;  // the previous phase is still running: idle
    const Chunk ck = chunk_of(w, blockIdx.x);
    if ((int)blockIdx.x == ck.c0 && threadIdx.x == 0) set_state(w, ck.member, tol, floor_, max_iter, stag);
    double ss = 0.0, mn = INFINITY;
    for (int64_t e = ck.e0 + threadIdx.x; e < ck.e1; e += TPB) {
        ss += psi[e] * psi[e];
        mn = fmin(mn, w.D[e]);
    }
    double v[1] = {ss};
    block_reduce<1>(v, 1, lds);
    mn = block_min(mn, lds);
    if (threadIdx.x == 0) {
        w.pa[blockIdx.x] = v[0];
        w.pa[(int64_t)w.nchunk + blockIdx.x] = mn;
    }
}

// V(:, 0) = psi / ||psi|| per member; flags zero or non-finite starts.
__global__ __launch_bounds__(TPB) void k_init_vec(const double *__restrict__ psi, DavArgs w) {
    __shared__ double lds[4];
    __shared__ double sums[1];
    if (w.gate && !*w.gate) return;
    const int c = blockIdx.x;
    const Chunk ck = chunk_of(w, c);
    sum_rows(w.pa, w.nchunk, ck.c0, ck.c1, 1, 1, sums);
    double mn = INFINITY;
    for (int r = ck.c0 + (int)threadIdx.x; r < ck.c1; r += TPB) mn = fmin(mn, w.pa[(int64_t)w.nchunk + r]);
    mn = block_min(mn, lds);
    const double s = sums[0];
    const bool bad = !(s > 0.0) || !isfinite(s);
    if (c == ck.c0 && threadIdx.x == 0) {
        DavState &S = w.st[ck.member];
        S.dmin = mn;
        S.tn0 = 1.0;
        if (bad) {
            S.bad_start = 1;
            deactivate(w, ck.member);
        }
    }
    if (bad) return;
    // the first basis vector goes through the same path as every later one:
    // projected as T, finalized (here: normalized once more) by the next k_ritz
    const double sc = 1.0 / sqrt(s);
    const int64_t e = ck.e0 + threadIdx.x;
    double q[1] = {0.0};
    if (e < ck.e1) {
        const double x = psi[e] * sc;
        w.T[e] = x;
        q[0] = x * x;
    }
    block_reduce<1>(q, 1, lds);
    if (threadIdx.x == 0) {
        w.pc[PR_R * (int64_t)w.nchunk + c] = 0.0;
        w.pc[PR_T * (int64_t)w.nchunk + c] = q[0];
    }
}

// ------------------------------------------------------------------ small eigenproblem

// Smallest-first eigen-decomposition of the member's Rayleigh matrix B[:n, :n].
// Warm start: in the basis of the previous Ritz vectors (extended by e_n) the
// matrix is the arrowhead A = [[diag(d), z], [z^T, beta]] with d the previous
// Ritz values (ascending), z = Y^T b and b, beta the new column of B; its
// leading block is diagonal up to the previous step's threshold
// tol = 1e-15 ||A||_F, which is dropped.
//
// Main path (all threads of the block): the arrowhead is solved directly.
// Border entries |z_j| <= tol are dropped as well, which makes (d_j, e_j) an
// eigenpair (deflation).  The other eigenvalues are the roots of the secular
// equation
//     f(x) = beta - x - sum_j z_j^2 / (d_j - x) = 0,
// exactly one in each gap of the remaining poles and one beyond each end.
// Quad r (four lanes, each summing every fourth pole) finds root r as pole +
// offset t, the pole being the nearer end of its gap (so that differences from
// the poles keep full relative accuracy).  A step goes to the root of a model
// of f that keeps the two poles bounding the gap, with weights matching the
// derivative of the terms below and above the gap (the -x term joins the far
// side), written for the correction so that it vanishes with f; the start is
// the root of f ~ C + z_o^2 / t near the origin pole when that lies inside the
// bracket.  Iterates stay in a shrinking bracket (geometric bisection as the
// safeguard) and stop once |f| is at the level of its rounding error.
// Eigenvectors are (z'_j / (d_j - x))_j extended by -1, normalized, with the
// border z' recomputed from the roots and poles (Loewner's formula for an
// arrowhead matrix: z'_j^2 = -prod_i (d_j - x_i) / prod_{l != j} (d_j - d_l)),
// which keeps them orthogonal to working precision (Gu and Eisenstat).
//
// Fallback (two remaining poles closer than 1e3 tol, or a root not found in
// 100 steps): cyclic Jacobi in parallel (round-robin) order on the arrowhead,
// rotations with |a_pq| <= tol skipped, until a sweep without rotations.  A
// step applies all of its disjoint rotations at once, block by block:
// A[{p_k,q_k}, {p_l,q_l}] <- R_k A[..] R_l^T, and Vv[:, {p_k,q_k}] <- Vv[..] R_k^T.
struct EigLds {
    double A[KM][KM + 1];   // the arrowhead; on the main path then the eigenvector matrix U
    double Vv[KM][KM + 1];  // previous eigenvectors extended by e_n
    double c[KM / 2], s[KM / 2];
    double d[KM], z[KM];               // poles and border
    double dk[KM], zk[KM], zh[KM];     // remaining poles, their border, recomputed border
    double org[KM + 1], tau[KM + 1];   // root i = org[i] + tau[i]
    double val[KM + 1];                // eigenvalue of each entry (roots, then deflated poles)
    int kidx[KM], didx[KM];            // original index of each remaining / deflated pole
    int col[KM + 1], inv[KM + 1];      // ascending position of each entry, and its inverse
    double tol;
    int k, path;
};

static __device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// round-robin pairing: pair k of a step (indices < n2; index n is a dummy for odd n)
static __device__ __forceinline__ void rr_pair(int k, int step, int n2, int &p, int &q) {
    const int h = n2 - 1;
    int a = k - 1 + step;  // in [-1, 2h)
    a = (a >= h) ? a - h : a;
    p = (k == 0) ? 0 : a + 1;
    int b = h - 1 - k + step;  // in [0, 2h)
    b = (b >= h) ? b - h : b;
    q = b + 1;
}

// One wavefront: the arrowhead's diagonal block and the extended eigenvectors.
// Independent of the new column, so it overlaps the sums that produce it.
static __device__ void eig_load(const DavState &S, int n, int ob, EigLds &L) {
    const int lane = threadIdx.x & 63;
    const int m = n - 1;
    const double *Yo = S.Y[ob], *to = S.theta[ob];
    for (int e = lane; e < n * n; e += 64) {
        const int r = e / n, c = e - r * n;
        L.A[r][c] = (r == c && r < m) ? to[r] : 0.0;
        L.Vv[r][c] = (r < m && c < m) ? Yo[r * KM + c] : (r == c ? 1.0 : 0.0);
    }
    for (int j = lane; j < m; j += 64) L.d[j] = to[j];
}

// One wavefront: border z = Y^T b and the corner, and the threshold.
// The new column of B from the raw sums of the projection y = H t': bcol[k] =
// V(:, k)^T y (k < m), bcol[m] = t'^T y, where the new basis vector is
// v = (t' - V s2) / nu (second Gram-Schmidt pass).  By linearity
//   B(k, m) = (bcol[k] - (B s2)_k) / nu,
//   B(m, m) = (bcol[m] - 2 s2^T bcol[:m] + s2^T B s2) / nu^2,
// and in the previous Ritz basis Y (B = Y diag(theta) Y^T up to the threshold)
// the border is z = (Y^T bcol[:m] - theta o Y^T s2) / nu.
static __device__ void eig_border(int n, const double *bcol, const double *s2, double nu, EigLds &L) {
    const int lane = threadIdx.x & 63;
    const int m = n - 1;
    wave_sync();
    double quad = 0.0, cross = 0.0, fro = 0.0;
    if (lane < m) {  // m < 64
        const int r = lane;
        double y = 0.0, g = 0.0;
#pragma unroll 4
        for (int k = 0; k < m; ++k) {
            y += L.Vv[k][r] * bcol[k];
            g += L.Vv[k][r] * s2[k];
        }
        const double dr = L.d[r];
        const double z = (y - dr * g) / nu;
        L.A[r][m] = z;
        L.A[m][r] = z;
        L.z[r] = z;
        quad = dr * g * g;
        cross = s2[r] * bcol[r];
        fro = dr * dr + 2.0 * z * z;  // ||A||_F^2 without the corner
    }
    quad = wave_reduce(quad);
    cross = wave_reduce(cross);
    fro = wave_reduce(fro);
    const double beta = (bcol[m] - 2.0 * cross + quad) / (nu * nu);
    if (lane == 0) {
        L.A[m][m] = beta;
        L.tol = 1e-15 * sqrt(fro + beta * beta);
    }
    wave_sync();
}

// 1/x from the hardware estimate and two Newton steps (a few ulps)
static __device__ __forceinline__ double rcp_nr(double x) {
    double r = __builtin_amdgcn_rcp(x);
    double e = fma(-x, r, 1.0);
    r = fma(r, e, r);
    e = fma(-x, r, 1.0);
    return fma(r, e, r);
}

// Sums and products over the four lanes of a quad (lanes 4r .. 4r+3); all
// four lanes get the same bits.
static __device__ __forceinline__ double quad_sum(double v) { return group_sum<4>(v); }
static __device__ __forceinline__ double quad_prod(double v) {
    v *= dpp_f64<DPP_XOR1>(v);
    return v * dpp_f64<DPP_XOR2>(v);
}
static __device__ __forceinline__ int quad_isum(int v) {
    v += __builtin_amdgcn_mov_dpp(v, DPP_XOR1, 0xF, 0xF, false);
    return v + __builtin_amdgcn_mov_dpp(v, DPP_XOR2, 0xF, 0xF, false);
}

// All threads.  Returns 1 (the same in every thread) when the fallback is
// needed (then L.A, L.Vv are untouched); else leaves U in L.A and the entries'
// values and order in L.val, L.col, L.inv.
static __device__ int eig_secular(int n, EigLds &L) {
    const int tid = threadIdx.x, lane = tid & 63;
    const int m = n - 1;
    const double tol = L.tol, beta = L.A[m][m];
    constexpr double EPS = 1.1102230246251565e-16;  // 2^-53
    // deflation (wavefront 0; m < 64): poles with |z_j| <= tol leave the secular equation
    if (tid < 64) {
        const bool live = lane < m && fabs(L.z[lane]) > tol;
        const bool dead = lane < m && !live;
        const uint64_t lm = __ballot(live), dm = __ballot(dead);
        const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
        if (live) {
            const int r = __popcll(lm & below);
            L.dk[r] = L.d[lane];
            L.zk[r] = L.z[lane];
            L.kidx[r] = lane;
        }
        if (dead) L.didx[__popcll(dm & below)] = lane;
        const int kl = __popcll(lm);
        wave_sync();
        // two remaining poles too close for the secular equation: the fallback (k = -1)
        const bool close = lane + 1 < kl && L.dk[lane + 1] - L.dk[lane] <= 1e3 * tol;
        const uint64_t cm = __ballot(close);
        if (lane == 0) L.k = cm ? -1 : kl;
    }
    __syncthreads();
    const int k = __builtin_amdgcn_readfirstlane(L.k);  // uniform: scalar loop bounds
    if (k < 0) return 1;
    const int r = tid >> 2, p = tid & 3;  // quad r; its lane p takes the poles j = p + 4u
    constexpr int RP = KM / 4;
    // this lane's poles and border entries; slots beyond k hold a zero term
    // (z = 0 at a far pole), so the sums below need no per-lane guards
    double pd[RP], pz[RP];
#pragma unroll
    for (int u = 0; u < RP; ++u) {
        const int j = 4 * u + p;
        pd[u] = (j < k) ? L.dk[j] : 1e300;
        pz[u] = (j < k) ? L.zk[j] : 0.0;
    }
    bool fail = false;
    if (r <= k) {
        const int i = r;  // root i
        double o = beta, t = 0.0;
        if (k > 0) {
            const double dL = (i > 0) ? L.dk[i - 1] : 0.0, dR = (i < k) ? L.dk[i] : 0.0;  // the gap
            const double mid = 0.5 * (dL + dR);
            // one pass: ||z||^2, f(mid) (inner gaps), and for each candidate origin the
            // rest of f at the origin with the origin's own pole left out
            double zz = 0.0, fm = 0.0, cl = 0.0, cr = 0.0;
#pragma unroll
            for (int u = 0; u < RP; ++u) {
                if (4 * u >= k) break;
                const int j = 4 * u + p;
                const double z2 = pz[u] * pz[u];
                const double tm = z2 * rcp_nr(pd[u] - mid), tl = z2 * rcp_nr(pd[u] - dL),
                             tr = z2 * rcp_nr(pd[u] - dR);
                zz += z2;
                fm += (i > 0 && i < k) ? tm : 0.0;
                cl += (i > 0 && j != i - 1) ? tl : 0.0;  // (the excluded terms may be infinite)
                cr += (i < k && j != i) ? tr : 0.0;
            }
            const double zn = sqrt(quad_sum(zz));
            fm = quad_sum(fm);
            cl = quad_sum(cl);
            cr = quad_sum(cr);
            double a, b;
            bool left;  // origin at the lower end of the gap
            if (i == 0) {
                left = false;
                o = dR;
                a = (fmin(dR, beta) - zn - tol) - o;
                b = 0.0;
            } else if (i == k) {
                left = true;
                o = dL;
                a = 0.0;
                b = (fmax(dL, beta) + zn + tol) - o;
            } else if ((beta - mid) - fm >= 0.0) {  // root between mid and the upper pole
                left = false;
                o = dR;
                a = mid - o;
                b = 0.0;
            } else {
                left = true;
                o = dL;
                a = 0.0;
                b = mid - o;
            }
            t = 0.5 * (a + b);
            {
                const double c0 = (beta - o) - (left ? cl : cr), zo = left ? L.zk[i - 1] : L.zk[i];
                const double t0 = (c0 != 0.0) ? -(zo * zo) / c0 : 0.0;
                if (t0 > a && t0 < b) t = t0;
            }
            // weights of the model's two poles: q^2 sums below / above the gap, the
            // far side taking the -x term (inner gaps)
            const double wl = (i < k && !left) ? 1.0 : 0.0, wr = (i > 0 && left) ? 1.0 : 0.0;
            bool done = false;
            for (int it = 0; it < 100 && !done; ++it) {
                // f(o + t); sums of q_j^2 over the poles below the gap (j < i) and above;
                // sum |z_j q_j| for the rounding error of f
                double fs = 0.0, pl = 0.0, pr = 0.0, er = 0.0;
#pragma unroll
                for (int u = 0; u < RP; ++u) {
                    if (4 * u >= k) break;
                    const int j = 4 * u + p;
                    const double q = pz[u] * rcp_nr((pd[u] - o) - t);
                    const double zq = pz[u] * q, qq = q * q;
                    fs += zq;
                    er += fabs(zq);
                    pl += (j < i) ? qq : 0.0;
                    pr += (j < i) ? 0.0 : qq;
                }
                fs = quad_sum(fs);
                pl = quad_sum(pl);
                pr = quad_sum(pr);
                er = quad_sum(er);
                const double fv = ((beta - o) - t) - fs;
                if (fabs(fv) <= 8.0 * EPS * (er + fabs(beta - o) + fabs(t))) {
                    done = true;
                    break;
                }
                if (fv > 0.0)
                    a = t;
                else
                    b = t;
                // model f(t + eta) ~ c - SL / (DL - eta) - SR / (DR - eta) through f(t), f'(t)
                // with SL = wL DL^2, SR = wR DR^2; its root solves qa eta^2 - qb eta + qc = 0
                double qa, qb, qc;
                if (i == 0 || i == k) {
                    const double dd = -t;  // to the origin pole; every pole on one side, -x exact
                    const double wd = (i == 0) ? pr : pl;
                    qa = 1.0;
                    qb = dd + fv + wd * dd;
                    qc = fv * dd;
                } else {
                    const double DL = (dL - o) - t, DR = (dR - o) - t;
                    const double wL = pl + wl, wR = pr + wr;
                    qa = fv + wL * DL + wR * DR;
                    qb = qa * (DL + DR) - wL * DL * DL - wR * DR * DR;
                    qc = DL * DR * fv;
                }
                const double disc = sqrt(fabs(qb * qb - 4.0 * qa * qc));
                const double den = (qb >= 0.0) ? qb + disc : qb - disc;  // the root that vanishes with f
                double tn = (den != 0.0) ? t + 2.0 * qc * rcp_nr(den) : 0.5 * (a + b);
                if (fabs(tn - t) <= 2.0 * EPS * fabs(t)) {
                    t = tn;
                    done = true;
                    break;
                }
                if (!(tn > a && tn < b)) {
                    if (a >= 0.0 && b > 0.0 && b > 4.0 * fmax(a, 1e-300 * b))
                        tn = sqrt(fmax(a, 1e-300 * b) * b);
                    else if (b <= 0.0 && a < 0.0 && -a > 4.0 * fmax(-b, -1e-300 * a))
                        tn = -sqrt(fmax(-b, -1e-300 * a) * -a);
                    else
                        tn = 0.5 * (a + b);
                }
                if (b - a <= 2.0 * EPS * fmax(fabs(a), fabs(b))) {
                    t = tn;
                    done = true;
                    break;
                }
                t = tn;
            }
            fail = !done || !isfinite(t);
        }
        if (p == 0) {
            L.org[i] = o;
            L.tau[i] = t;
        }
    }
    if (__syncthreads_or(fail)) return 1;
    // recomputed border (pairs each pole difference with a root difference); quad j takes pole j
    if (r < k) {
        const int j = r;
        const double dj = L.dk[j];
        double prod = 1.0;
#pragma unroll
        for (int u = 0; u < RP; ++u) {
            if (4 * u >= k) break;
            const int l = 4 * u + p;
            const int x = (l < j) ? l : min(l + 1, k);
            const double fct = ((dj - L.org[x]) - L.tau[x]) * rcp_nr(dj - pd[u]);
            prod *= (l < k && l != j) ? fct : 1.0;
        }
        prod = quad_prod(prod) * (-((dj - L.org[j]) - L.tau[j]) * ((dj - L.org[j + 1]) - L.tau[j + 1]));
        if (p == 0) L.zh[j] = copysign(sqrt(fmax(prod, 0.0)), L.zk[j]);
    }
    // entries: roots 0..k, then the deflated poles; ascending order, ties by entry
    for (int e = tid; e < n; e += TPB) L.val[e] = (e <= k) ? L.org[e] + L.tau[e] : L.d[L.didx[e - k - 1]];
    __syncthreads();
    if (r < n) {
        const int e = r;
        const double v = L.val[e];
        int rank = 0;
        for (int f = p; f < n; f += 4) {
            const double w = L.val[f];
            rank += (w < v) || (w == v && f < e);
        }
        rank = quad_isum(rank);
        if (p == 0) {
            L.col[e] = rank;
            L.inv[rank] = e;
        }
    }
    for (int e = tid; e < n * n; e += TPB) L.A[e / n][e % n] = 0.0;
    __syncthreads();
    // eigenvector columns of the arrowhead; quad e takes entry e
    if (r < n) {
        const int e = r, c = L.col[e];
        if (e <= k) {
            const double o = L.org[e], t = L.tau[e];
            double uv[RP], nrm = 0.0;
#pragma unroll
            for (int u = 0; u < RP; ++u) {
                uv[u] = 0.0;
                if (4 * u >= k) break;
                const int j = 4 * u + p;
                const double x = L.zh[min(j, k - 1)] * rcp_nr((pd[u] - o) - t);
                uv[u] = (j < k) ? x : 0.0;
                nrm += uv[u] * uv[u];
            }
            const double sc = 1.0 / sqrt(1.0 + quad_sum(nrm));
#pragma unroll
            for (int u = 0; u < RP; ++u) {
                if (4 * u >= k) break;
                const int j = 4 * u + p;
                if (j < k) L.A[L.kidx[j]][c] = uv[u] * sc;
            }
            if (p == 0) L.A[m][c] = -sc;
        } else if (p == 0) {
            L.A[L.didx[e - k - 1]][c] = 1.0;
        }
    }
    __syncthreads();
    return 0;
}

// Column c of the new eigenvectors: Vv U(:, c) on the main path, the rotated
// Vv's column inv[c] after Jacobi.
static __device__ __forceinline__ double eig_y(const EigLds &L, int n, int r, int c) {
    if (L.path) return L.Vv[r][L.inv[c]];
    double acc = 0.0;
    for (int q = 0; q < n; ++q) acc += L.Vv[r][q] * L.A[q][c];
    return acc;
}

// All threads of the member's first block: Y and theta into buffer nb, and the
// scalars of the iteration.
static __device__ void eig_store(DavState &S, int n, int nb, const EigLds &L) {
    for (int e = threadIdx.x; e < n * n; e += TPB) {
        const int r = e / n, c = e - r * n;
        S.Y[nb][r * KM + c] = eig_y(L, n, r, c);
    }
    for (int c = threadIdx.x; c < n; c += TPB) S.theta[nb][c] = L.val[L.inv[c]];
    if (threadIdx.x == 0) {
        S.lambda = L.val[L.inv[0]];
        S.iters += 1;
        S.nproj += 1;
        S.nvec = n;
    }
}

// One wavefront: the Jacobi fallback on the arrowhead in L.A, L.Vv; leaves the
// rotated Vv, the eigenvalues in L.val and their ascending order in L.inv.
static __device__ void eig_jacobi(int n, EigLds &L) {
    const int lane = threadIdx.x & 63;
    const double tol = L.tol;
    const int n2 = (n + 1) & ~1;
    const int np = n2 / 2;
    // lanes as an 8 x 8 grid: lane (ga, gb) updates the blocks (k, l) with
    // k = ga mod 8, l = gb mod 8, and the rows j = gb mod 8 of Vv's column pair k
    const int ga = lane >> 3, gb = lane & 7;
    for (int sweep = 0; sweep < 30; ++sweep) {
        int rotated = 0;
        for (int step = 0; step < n2 - 1; ++step) {
            bool any_rot = false;
            if (lane < np) {
                int p, q;
                rr_pair(lane, step, n2, p, q);
                // all three loads in flight together (indices < n2 <= KM stay inside the arrays)
                const double apq = L.A[p][q], app = L.A[p][p], aqq = L.A[q][q];
                double cc = 1.0, ss = 0.0;
                if (p < n && q < n && fabs(apq) > tol) {
                    // tan of the annihilating angle: t = sgn(d) e / (|d| + sqrt(d^2 + e^2)),
                    // d = a_qq - a_pp, e = 2 a_pq; then c = u / sqrt(u^2 + e^2), s = t c
                    const double d = aqq - app, e2 = 2.0 * apq;
                    const double u = fabs(d) + sqrt(d * d + e2 * e2);
                    const double wr = rsqrt(u * u + e2 * e2);
                    cc = u * wr;
                    ss = (d >= 0.0 ? e2 : -e2) * wr;
                    rotated = 1;
                    any_rot = true;
                }
                L.c[lane] = cc;
                L.s[lane] = ss;
            }
            if (!__any(any_rot)) continue;  // nothing to apply in this step
            wave_sync();
            for (int k = ga; k < np; k += 8) {
                int pk, qk;
                rr_pair(k, step, n2, pk, qk);
                const bool vk = pk < n && qk < n;
                for (int l = gb; l < np; l += 8) {
                    int pl, ql;
                    rr_pair(l, step, n2, pl, ql);
                    const bool vl = pl < n && ql < n;
                    // one batch of loads: both rotations and the 2 x 2 block
                    const double ck = L.c[k], sk = L.s[k], cl = L.c[l], sl = L.s[l];
                    const double a = L.A[pk][pl], b = L.A[pk][ql], c = L.A[qk][pl], d = L.A[qk][ql];
                    if (sk == 0.0 && sl == 0.0) continue;
                    // rows (R_k), then columns (R_l^T); with a dummy index one side is the identity
                    const double ra = ck * a - sk * c, rb = ck * b - sk * d;
                    const double rc = sk * a + ck * c, rd = sk * b + ck * d;
                    if (vk && vl) {
                        L.A[pk][pl] = cl * ra - sl * rb;
                        L.A[pk][ql] = sl * ra + cl * rb;
                        L.A[qk][pl] = cl * rc - sl * rd;
                        L.A[qk][ql] = sl * rc + cl * rd;
                    } else if (vk) {  // column pair holds the dummy index: one valid column
                        if (pl < n) {
                            L.A[pk][pl] = ra;
                            L.A[qk][pl] = rc;
                        } else {
                            L.A[pk][ql] = rb;
                            L.A[qk][ql] = rd;
                        }
                    } else if (vl) {  // row pair holds the dummy index: one valid row
                        if (pk < n) {
                            L.A[pk][pl] = cl * a - sl * b;
                            L.A[pk][ql] = sl * a + cl * b;
                        } else {
                            L.A[qk][pl] = cl * c - sl * d;
                            L.A[qk][ql] = sl * c + cl * d;
                        }
                    }
                }
                const double ck = L.c[k], sk = L.s[k];
                if (sk != 0.0) {
                    for (int j = gb; j < n; j += 8) {
                        const double vp = L.Vv[j][pk], vq = L.Vv[j][qk];
                        L.Vv[j][pk] = ck * vp - sk * vq;
                        L.Vv[j][qk] = sk * vp + ck * vq;
                    }
                }
            }
            wave_sync();
        }
        if (!__any(rotated)) break;
    }
    // ascending order (stable rank)
    for (int a = lane; a < n; a += 64) {
        const double da = L.A[a][a];
        int rank = 0;
        for (int b = 0; b < n; ++b) {
            const double db = L.A[b][b];
            rank += (db < da) || (db == da && b < a);
        }
        L.val[a] = da;
        L.inv[rank] = a;
    }
    wave_sync();
}

// ------------------------------------------------------------------ iteration kernels

// The pending basis vector from the summed second-pass rows sums[0..q) = s2 =
// V^T t' and sums[q + 1] = ||t'||^2: copies s2 and returns nu = ||t' - V s2||
// (Pythagoras; s2 is the small remainder of the first pass, nothing cancels).
// All threads call; s2 is valid after the call.
static __device__ double pending_nu(const double *sums, int q, double *s2) {
    double ss = 0.0;
    for (int j = 0; j < q; ++j) ss += sums[j] * sums[j];
    for (int j = threadIdx.x; j < q; j += TPB) s2[j] = sums[j];
    __syncthreads();
    return sqrt(fmax(sums[q + 1] - ss, 0.0));
}

// A basis vector that vanished after orthogonalization ends the member.
static __device__ __forceinline__ bool broke_down(DavState &S, const DavArgs &w, int member, bool writer, double nu) {
    if (nu > 1e-13 * S.tn0) return false;
    if (writer && threadIdx.x == 0) {
        S.breakdown = 1;
        deactivate(w, member);
    }
    return true;
}

// Small eigenproblem of the Rayleigh step for one member (all threads call):
// wavefront 0 forms the new column of B from the summed tile rows bcol
// (corrected for the second pass, see eig_border), the block solves the
// arrowhead, wavefront 0 runs the Jacobi fallback when needed.  eig_load must
// have run.  Results stay in L.
static __device__ __forceinline__ void rayleigh_solve(int i, int jacobi_only, const double *s2, double nu, EigLds &L,
                                      const double *bcol) {
    if (threadIdx.x < 64) eig_border(i, bcol, s2, nu, L);
    __syncthreads();
    const int fb = jacobi_only ? 1 : eig_secular(i, L);
    if (fb && threadIdx.x < 64) eig_jacobi(i, L);
    if (threadIdx.x == 0) L.path = fb;
    __syncthreads();
}

// Rayleigh step as its own kernel, one block per member (plans with many
// chunks per member): stores Y, theta (buffer par) and the scalars.
__global__ __launch_bounds__(TPB) void k_rayleigh(DavArgs w, const int32_t *__restrict__ slot_begin, int i, int par,
                                                  int jacobi_only) {
    __shared__ EigLds L;
    __shared__ double bcol[KM], s2[KM], pcs[KM + 2];
    const int member = blockIdx.x;
    if (!w.active[member]) return;
    DavState &S = w.st[member];
    const int c0 = w.nprob == 1 ? 0 : w.member_chunk[member];
    const int c1 = w.nprob == 1 ? w.nchunk : w.member_chunk[member + 1];
    if (threadIdx.x < 64) eig_load(S, i, par ^ 1, L);
    sum_rows2(w.pc, w.nchunk, c0, c1, i - 1, i + 1, pcs, w.ptile, w.tile_ld, slot_begin[member],
              slot_begin[member + 1], i, i, bcol);
    const double nu = pending_nu(pcs, i - 1, s2);
    if (broke_down(S, w, member, true, nu)) return;
    if (threadIdx.x == 0) track_stagnation(S);  // before this step counts itself
    rayleigh_solve(i, jacobi_only, s2, nu, L, bcol);
    eig_store(S, i, par, L);
}

// The newest basis vector and its projection are finished here, element by
// element: V(:, q) = (t' - V s2) / nu, W(:, q) = (H t' - W s2) / nu, q = i - 1.
// Then the Ritz vector, residual and correction: x = V y, r = W y - lambda x,
// t = r / (D - sigma); partial row: V^T t, ||r||^2, ||t||^2.  With SOLVE the
// Rayleigh step runs here too: every block of a member sums the member's tile
// rows and solves the small eigenproblem itself (identical inputs and order,
// hence identical results in every block) while its own rows of V and W are
// loaded, and the member's first block stores Y and theta (buffer par; the
// previous iteration's are read from par ^ 1).  Without SOLVE, y and lambda
// come from k_rayleigh.
template <int KB, bool SOLVE>
__global__ __launch_bounds__(TPB) void k_ritz(DavArgs w, const int32_t *__restrict__ slot_begin, int i, int restart,
                                              int par, int jacobi_only) {
    __shared__ EigLds L;
    __shared__ double bcol[KM], s2[KM];
    __shared__ double y0[KM];
    __shared__ double lds[4 * (KB + 2)];
    constexpr bool PRE = KB <= 16;  // keep the rows in registers across the sums and the solve
    const int c = blockIdx.x;
    const Chunk ck = chunk_of(w, c);
    const int member = ck.member;
    if (!w.active[member]) return;
    DavState &S = w.st[member];
    const bool writer = c == ck.c0;
    const int q = i - 1;  // the pending column
    const int64_t n = w.n, e = ck.e0 + threadIdx.x;
    const bool has = e < ck.e1;
    double v[KB], wv[KB], dv = 0.0;
#pragma unroll
    for (int j = 0; j < KB; ++j) v[j] = wv[j] = 0.0;
    auto load_rows = [&]() {
        if (has) {
            dv = w.D[e];
#pragma unroll
            for (int j = 0; j < KB; ++j) {
                const int jj = min(j, q);
                v[j] = (jj < q ? w.V + (int64_t)jj * n : w.T)[e];  // column q: t'
                wv[j] = w.W[(int64_t)jj * n + e];                  // column q: H t'
            }
        }
    };
    if (PRE) load_rows();
    __shared__ double pcs[KM + 2];
    if (SOLVE) {
        if (threadIdx.x < 64) eig_load(S, i, par ^ 1, L);
        sum_rows2(w.pc, w.nchunk, ck.c0, ck.c1, q, q + 2, pcs, w.ptile, w.tile_ld, slot_begin[member],
                  slot_begin[member + 1], i, i, bcol);
    } else {
        sum_rows(w.pc, w.nchunk, ck.c0, ck.c1, q, q + 2, pcs);
    }
    const double nu = pending_nu(pcs, q, s2);
    if (broke_down(S, w, member, writer, nu)) return;
    double lam;
    if (SOLVE) {
        if (writer && threadIdx.x == 0) track_stagnation(S);  // before this step counts itself
        rayleigh_solve(i, jacobi_only, s2, nu, L, bcol);
        for (int r = threadIdx.x; r < i; r += TPB) y0[r] = eig_y(L, i, r, 0);
        if (writer) eig_store(S, i, par, L);
        lam = L.val[L.inv[0]];
    } else {
        for (int r = threadIdx.x; r < i; r += TPB) y0[r] = S.Y[par][r * KM];
        lam = S.lambda;
    }
    if (!PRE) load_rows();
    __syncthreads();
    // finish column q of V and W
    double dvq = 0.0, dwq = 0.0, vq = 0.0, wq = 0.0;
#pragma unroll
    for (int j = 0; j < KB; ++j) {
        if (j < q) {
            dvq += v[j] * s2[j];
            dwq += wv[j] * s2[j];
        }
        if (j == q) {
            vq = v[j];
            wq = wv[j];
        }
    }
    vq = (vq - dvq) / nu;
    wq = (wq - dwq) / nu;
#pragma unroll
    for (int j = 0; j < KB; ++j)
        if (j == q) {
            v[j] = vq;
            wv[j] = wq;
        }
    if (has) {
        w.V[(int64_t)q * n + e] = vq;
        w.W[(int64_t)q * n + e] = wq;
    }
    const double sig = fmin(lam, S.dmin), fl = S.floor_;
    double x = 0.0, wy = 0.0;
#pragma unroll
    for (int j = 0; j < KB; ++j) {
        const double yj = (j < i) ? y0[j] : 0.0;
        v[j] = (j < i) ? v[j] : 0.0;
        x += v[j] * yj;
        wy += wv[j] * yj;
    }
    const double r = wy - lam * x;
    double den = dv - sig;
    if (fabs(den) < fl) den = (den < 0.0) ? -fl : fl;
    const double t = has ? r / den : 0.0;
    if (has) w.T[e] = t;
    double acc[KB + 2];
#pragma unroll
    for (int j = 0; j < KB; ++j) acc[j] = restart ? 0.0 : v[j] * t;
    acc[KB] = has ? r * r : 0.0;
    acc[KB + 1] = t * t;
    block_reduce<KB + 2>(acc, KB + 2, lds);
    if (threadIdx.x == 0) {
        const int64_t ld = w.nchunk;
        if (!restart) {
#pragma unroll
            for (int j = 0; j < KB; ++j)
                if (j < i) w.pa[j * ld + c] = acc[j];
        }
        w.pa[PR_R * ld + c] = acc[KB];
        w.pa[PR_T * ld + c] = acc[KB + 1];
    }
}

// Thick restart: V(:, :kmin) = V(:, :i) Y(:, :kmin), same for W; partial row:
// V^T t of the new basis (as Y(:, :kmin)^T of the old basis' V^T t), and the
// norms of k_ritz's row.  Skipped when the stop
// test (made again by k_orth from the same sums) ends the member.
template <int KB>
__global__ __launch_bounds__(TPB) void k_restart(DavArgs w, int i, int kmin, int par) {
    __shared__ double lds[4 * KB];
    __shared__ double Ys[KB * KB];
    __shared__ double sums[2];
    const int c = blockIdx.x;
    const Chunk ck = chunk_of(w, c);
    if (!w.active[ck.member]) return;
    const DavState &S = w.st[ck.member];
    sum_rows(w.pa, w.nchunk, ck.c0, ck.c1, 0, 2, sums);
    if (stop_code(S, sums[0])) return;
    for (int e = threadIdx.x; e < KB * KB; e += TPB) {
        int r = e / KB, q = e % KB;
        Ys[r * KB + q] = (r < i && q < kmin) ? S.Y[par][r * KM + q] : 0.0;
    }
    __syncthreads();
    const int64_t n = w.n;
    double acc[KB];
#pragma unroll
    for (int j = 0; j < KB; ++j) acc[j] = 0.0;
    for (int64_t e = ck.e0 + threadIdx.x; e < ck.e1; e += TPB) {
        double v[KB], wv[KB];
#pragma unroll
        for (int j = 0; j < KB; ++j) {
            v[j] = w.V[(int64_t)min(j, i - 1) * n + e];
            wv[j] = w.W[(int64_t)min(j, i - 1) * n + e];
        }
#pragma unroll
        for (int j = 0; j < KB; ++j) {
            v[j] = (j < i) ? v[j] : 0.0;
            wv[j] = (j < i) ? wv[j] : 0.0;
        }
        const double t = w.T[e];
        for (int q = 0; q < kmin; ++q) {
            double a = 0.0, b = 0.0;
#pragma unroll
            for (int j = 0; j < KB; ++j) {
                a += v[j] * Ys[j * KB + q];
                b += wv[j] * Ys[j * KB + q];
            }
            w.V[(int64_t)q * n + e] = a;
            w.W[(int64_t)q * n + e] = b;
        }
#pragma unroll
        for (int j = 0; j < KB; ++j) acc[j] += v[j] * t;  // old V^T t; the new one is Y^T of it
    }
    block_reduce<KB>(acc, i, lds);
    if (threadIdx.x == 0) {
        const int64_t ld = w.nchunk;
        for (int q = 0; q < kmin; ++q) {
            double sq = 0.0;
#pragma unroll
            for (int j = 0; j < KB; ++j) sq += Ys[j * KB + q] * acc[j];
            w.pb[q * ld + c] = sq;
        }
        w.pb[PR_R * ld + c] = w.pa[PR_R * ld + c];
        w.pb[PR_T * ld + c] = w.pa[PR_T * ld + c];
    }
}

// Stop test, then the first Gram-Schmidt pass t' = t - V s (kept in T; the
// projection takes it as is) and the partial rows of the second pass: V^T t'
// and ||t'||^2.  pin: the rows of k_ritz, or of k_restart after a restart.
template <int KB>
__global__ __launch_bounds__(TPB) void k_orth(DavArgs w, int i, const double *__restrict__ pin, int after_restart,
                                              int par) {
    __shared__ double lds[4 * (KB + 1)];
    __shared__ double sums[KM + 2];
    const int c = blockIdx.x;
    const Chunk ck = chunk_of(w, c);
    const int member = ck.member;
    if (!w.active[member]) return;
    DavState &S = w.st[member];
    // this thread's element (a chunk holds at most TPB): its loads overlap the sums
    const int64_t n = w.n, e = ck.e0 + threadIdx.x;
    const bool has = e < ck.e1;
    double t = 0.0, v[KB];
#pragma unroll
    for (int j = 0; j < KB; ++j) v[j] = 0.0;
    if (has) {
        t = w.T[e];
#pragma unroll
        for (int j = 0; j < KB; ++j) v[j] = w.V[(int64_t)min(j, i - 1) * n + e];
    }
    sum_rows(pin, w.nchunk, ck.c0, ck.c1, i, i + 2, sums);
    const double rr = sums[i], tt = sums[i + 1];
    const int code = stop_code(S, rr);
    const bool brk = !code && !(tt > 0.0);
    if (c == ck.c0 && threadIdx.x == 0) {
        S.rnorm = sqrt(rr);
        if (S.iters == 1) S.rnorm1 = S.rnorm;
        S.tn0 = sqrt(tt);
        if (code == 1) S.converged = 1;
        if (code == 3) S.bad_start = 2;  // non-finite iterate
        if (brk) S.breakdown = 1;
        if (code || brk) {
            deactivate(w, member);
        } else if (after_restart) {  // the kept Ritz vectors are the new basis: B = diag(theta), Y = I
            S.restarts += 1;
            for (int r = 0; r < i; ++r)
                for (int q = 0; q < i; ++q) S.Y[par][r * KM + q] = (r == q) ? 1.0 : 0.0;
        }
    }
    if (code || brk) return;
#pragma unroll
    for (int j = 0; j < KB; ++j) {
        v[j] = (j < i) ? v[j] : 0.0;
        t -= v[j] * ((j < i) ? sums[j] : 0.0);
    }
    if (has) w.T[e] = t;
    double acc[KB + 1];
#pragma unroll
    for (int j = 0; j < KB; ++j) acc[j] = v[j] * t;
    acc[KB] = t * t;
    block_reduce<KB + 1>(acc, KB + 1, lds);
    if (threadIdx.x == 0) {
        const int64_t ld = w.nchunk;
#pragma unroll
        for (int j = 0; j < KB; ++j)
            if (j < i) w.pc[j * ld + c] = acc[j];
        w.pc[PR_R * ld + c] = 0.0;
        w.pc[PR_T * ld + c] = acc[KB];
    }
}

// psi = V(:, :nvec) y (normalized Ritz vector of each member)
template <int KB>
__global__ __launch_bounds__(TPB) void k_finalize(DavArgs w, double *__restrict__ psi) {
    const int c = blockIdx.x;
    const Chunk ck = chunk_of(w, c);
    const int member = ck.member;
    const DavState &S = w.st[member];
    if (S.bad_start == 1) return;
    const int nv = S.nvec;
    double y[KB];
#pragma unroll
    for (int j = 0; j < KB; ++j) y[j] = (j < nv) ? S.Y[S.iters & 1][j * KM] : 0.0;
    const int64_t n = w.n;
    for (int64_t e = ck.e0 + threadIdx.x; e < ck.e1; e += TPB) {
        double v[KB];
#pragma unroll
        for (int j = 0; j < KB; ++j) v[j] = w.V[(int64_t)min(j, nv - 1) * n + e];
        double x = 0.0;
#pragma unroll
        for (int j = 0; j < KB; ++j) x += v[j] * y[j];
        psi[e] = x;
    }
}

__global__ void k_summary(DavArgs w) {
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= w.nprob) return;
    const DavState &S = w.st[m];
    DavSummary r;
    r.energy = S.lambda;
    r.rnorm = S.rnorm;
    r.rnorm1 = S.rnorm1;
    r.active = w.active[m];
    r.iters = S.iters;
    r.nproj = S.nproj;
    r.restarts = S.restarts;
    r.converged = S.converged;
    r.breakdown = S.breakdown;
    r.bad_start = S.bad_start;
    r.pad = 0;
    w.sum[m] = r;
}

// ------------------------------------------------------------------ host driver

// Register bucket for kernels that keep one row of V (and W) per thread: the
// smallest of 8 / 16 / 32 / 48 columns that holds the current subspace.
template <class K>
static void set_kb(int ncols, K &&f) {
    if (ncols <= 8)
        f(std::integral_constant<int, 8>{});
    else if (ncols <= 16)
        f(std::integral_constant<int, 16>{});
    else if (ncols <= 32)
        f(std::integral_constant<int, 32>{});
    else
        f(std::integral_constant<int, KM>{});
}

// Subspace, work vectors and partial rows to zero (outside any captured
// graph): a subspace that fills the whole space (n <= kmax) reaches columns
// and rows no iteration has written yet, where a stale value (a NaN left by a
// failed solve) would survive a zero weight.
static dmrg_status work_zero(const dmrg_plan *plan, DavidsonWork *w, hipStream_t s) {
    const DavArgs &A = w->a;
    const size_t n = (size_t)plan->n, kp = (size_t)w->kmax + 1;
    DMRG_HIP(hipMemsetAsync(A.V, 0, kp * n * 8, s));
    DMRG_HIP(hipMemsetAsync(A.W, 0, kp * n * 8, s));
    DMRG_HIP(hipMemsetAsync(A.T, 0, n * 8, s));
    DMRG_HIP(hipMemsetAsync((void *)A.X0, 0, n * 8, s));
    DMRG_HIP(hipMemsetAsync(A.pa, 0, (size_t)A.nchunk * w->rowb, s));
    DMRG_HIP(hipMemsetAsync(A.pb, 0, (size_t)A.nchunk * w->rowb, s));
    DMRG_HIP(hipMemsetAsync(A.pc, 0, (size_t)A.nchunk * w->rowb, s));
    DMRG_HIP(hipMemsetAsync(A.ptile, 0, (size_t)A.tile_ld * w->rowb, s));
    DMRG_HIP(hipStreamSynchronize(s));
    w->dirty = false;
    return DMRG_OK;
}

// Chunks of the vector kernels: at most TPB elements, never crossing a member
// boundary (an empty member gets one empty chunk, which keeps the bookkeeping
// uniform).  Returns the chunk count; the lists are filled when given.
static int dav_chunks(const dmrg_plan *plan, std::vector<int32_t> *cm, std::vector<int64_t> *cb,
                      std::vector<int32_t> *mc) {
    const int64_t CH = TPB;  // one element per thread: many blocks, every column load in flight
    int count = 0;
    if (mc) mc->assign(1, 0);
    for (int p = 0; p < plan->nprob; ++p) {
        int64_t b = plan->member_off[p], e = plan->member_off[p + 1];
        if (e == b) {
            if (cm) cm->push_back(p);
            if (cb) cb->push_back(b);
            ++count;
        }
        for (int64_t x = b; x < e; x += CH) {
            if (cm) cm->push_back(p);
            if (cb) cb->push_back(x);
            ++count;
        }
        if (mc) mc->push_back(count);
    }
    if (cb) cb->push_back(plan->n);
    return count;
}

// The Davidson arrays, in allocation order.
enum {
    DB_V, DB_W, DB_T, DB_D, DB_DFOLD, DB_COEF, DB_PA, DB_PB, DB_PC, DB_PTILE, DB_CMEM, DB_CBEG, DB_MCH, DB_ST,
    DB_ACT, DB_X0, DB_ACT2, DB_DFOLD2, DB_GATE, DB_COUNT
};

static void dav_sizes(const dmrg_plan *plan, int kmax, int nchunk, int tiles, size_t sz[DB_COUNT]) {
    const size_t n = (size_t)plan->n, rowb = (KM + 2) * 8, np = (size_t)plan->nprob;
    sz[DB_V] = sz[DB_W] = (kmax + 1) * n * 8;
    sz[DB_T] = sz[DB_D] = sz[DB_DFOLD] = sz[DB_X0] = sz[DB_DFOLD2] = n * 8;
    sz[DB_COEF] = (size_t)std::max(plan->nterm_total, 1) * 8;
    sz[DB_PA] = sz[DB_PB] = sz[DB_PC] = (size_t)nchunk * rowb;  // partial rows, one per chunk (three sets)
    sz[DB_PTILE] = (size_t)tiles * rowb;                         // one per output tile (Rayleigh rows)
    sz[DB_CMEM] = (size_t)nchunk * 4;
    sz[DB_CBEG] = (size_t)(nchunk + 1) * 8;
    sz[DB_MCH] = (np + 1) * 4;
    sz[DB_ST] = np * sizeof(DavState);
    sz[DB_ACT] = sz[DB_ACT2] = np * 4;
    sz[DB_GATE] = 8;
    for (int i = 0; i < DB_COUNT; ++i) sz[i] = std::max<size_t>(sz[i], 8);
}

size_t dav_workspace_bytes(const dmrg_plan *plan, int kmax, int tiles) {
    size_t sz[DB_COUNT], total = 0;
    dav_sizes(plan, kmax, dav_chunks(plan, nullptr, nullptr, nullptr), tiles, sz);
    for (int i = 0; i < DB_COUNT; ++i) total += ws_align(sz[i]);
    return total;
}

static dmrg_status work_alloc(dmrg_plan *plan, int kmax, int kmin, hipStream_t s) {
    DavidsonWork *w = plan->dav;
    if (w && w->kmax == kmax && w->kmin == kmin) return w->dirty ? work_zero(plan, w, s) : DMRG_OK;
    if (plan->ws && kmax > plan->ws_kmax)
        return set_error(DMRG_E_NOMEM, "the plan's workspace holds a subspace of at most %d vectors (kmax %d asked)",
                         plan->ws_kmax, kmax);
    davidson_free(plan);
    w = new DavidsonWork();
    plan->dav = w;
    w->kmax = kmax;
    w->kmin = kmin;
    DavArgs &A = w->a;
    A.n = plan->n;
    A.nprob = plan->nprob;
    std::vector<int32_t> cm, mc;
    std::vector<int64_t> cb;
    A.nchunk = dav_chunks(plan, &cm, &cb, &mc);
    const int tiles = std::max({1, plan->fwd[0].stageB.ntask, plan->fwd[1].stageB.ntask});
    A.tile_ld = tiles;
    w->rowb = (KM + 2) * 8;
    size_t sz[DB_COUNT];
    dav_sizes(plan, kmax, A.nchunk, tiles, sz);
    void *buf[DB_COUNT];
    if (plan->ws) {  // carved from the caller's workspace, in order
        char *q = plan->ws + plan->ws_dav;
        for (int i = 0; i < DB_COUNT; ++i) {
            buf[i] = q;
            q += ws_align(sz[i]);
        }
        if (q > plan->ws + plan->ws_bytes) return set_error(DMRG_E_NOMEM, "workspace too small for the Davidson arrays");
    } else {
        for (int i = 0; i < DB_COUNT; ++i) {
            DMRG_HIP(hipMalloc(&buf[i], sz[i]));
            w->owned.push_back(buf[i]);
        }
    }
    A.V = (double *)buf[DB_V];
    A.W = (double *)buf[DB_W];
    A.T = (double *)buf[DB_T];
    A.D = (double *)buf[DB_D];
    A.dfold = (double *)buf[DB_DFOLD];
    A.coef = (double *)buf[DB_COEF];
    A.pa = (double *)buf[DB_PA];
    A.pb = (double *)buf[DB_PB];
    A.pc = (double *)buf[DB_PC];
    A.ptile = (double *)buf[DB_PTILE];
    A.chunk_member = (int32_t *)buf[DB_CMEM];
    A.chunk_begin = (int64_t *)buf[DB_CBEG];
    A.member_chunk = (int32_t *)buf[DB_MCH];
    A.st = (DavState *)buf[DB_ST];
    A.active = (int32_t *)buf[DB_ACT];
    A.X0 = (double *)buf[DB_X0];
    // the summary goes straight to pinned, mapped, coherent host memory (no copy step)
    DMRG_HIP(hipHostMalloc((void **)&w->h_sum, plan->nprob * sizeof(DavSummary),
                           hipHostMallocMapped | hipHostMallocCoherent));
    DMRG_HIP(hipHostGetDevicePointer((void **)&A.sum, w->h_sum, 0));
    DavArgs &B = w->a2;  // FP64 phase: own flags, folded diagonal, gate and summary
    B = A;
    B.active = (int32_t *)buf[DB_ACT2];
    B.dfold = (double *)buf[DB_DFOLD2];
    B.gate = (int32_t *)buf[DB_GATE];
    DMRG_HIP(hipHostMalloc((void **)&w->h_sum2, plan->nprob * sizeof(DavSummary),
                           hipHostMallocMapped | hipHostMallocCoherent));
    DMRG_HIP(hipHostGetDevicePointer((void **)&B.sum, w->h_sum2, 0));
    DMRG_HIP(hipMemcpyAsync(A.chunk_member, cm.data(), cm.size() * 4, hipMemcpyHostToDevice, s));
    DMRG_HIP(hipMemcpyAsync(A.chunk_begin, cb.data(), cb.size() * 8, hipMemcpyHostToDevice, s));
    DMRG_HIP(hipMemcpyAsync(A.member_chunk, mc.data(), mc.size() * 4, hipMemcpyHostToDevice, s));
    DMRG_HIP(hipMemsetAsync(A.st, 0, plan->nprob * sizeof(DavState), s));
    DMRG_HIP(hipMemsetAsync(A.active, 0, plan->nprob * 4, s));
    DMRG_HIP(hipMemsetAsync(B.active, 0, plan->nprob * 4, s));
    return work_zero(plan, w, s);
}

dmrg_status davidson_free(dmrg_plan *plan) {
    DavidsonWork *w = plan->dav;
    if (!w) return DMRG_OK;
    for (auto &kv : w->graphs) (void)hipGraphExecDestroy(kv.second);
    for (void *p : w->owned) (void)hipFree(p);
    if (w->h_sum) (void)hipHostFree(w->h_sum);
    if (w->h_sum2) (void)hipHostFree(w->h_sum2);
    delete w;
    plan->dav = nullptr;
    return DMRG_OK;
}

// Davidson context of a projection whose output is W(:, i-1).
static RayArgs ray_args(const DavArgs &A, int i) {
    RayArgs r;
    r.V = A.V;
    r.n = A.n;
    r.i = i;
    r.part = A.ptile;
    r.ld = A.tile_ld;
    return r;
}

// Enqueue `count` iterations starting at subspace size i and iteration number
// t (1 = the phase's first; its parity selects the Y/theta buffer); returns the next i.
static dmrg_status enqueue_iters(dmrg_plan *plan, const DavArgs &A, int slot, int i, int t, int count, int *i_next,
                                 hipStream_t s) {
    DavidsonWork *w = plan->dav;
    const int kmax = w->kmax, kmin = w->kmin;
    const dim3 grid(A.nchunk), block(TPB);
    const int32_t *slot_begin = plan->fwd[slot].slot_begin;
    for (int it = 0; it < count; ++it, ++t) {
        const bool restart = (i == kmax);
        const int par = t & 1;
        // W(:, i-1) and its Rayleigh rows came from the previous projection.  The
        // Rayleigh step runs redundantly inside k_ritz while all chunk blocks fit on
        // the device at once; beyond that a block per member solves it first.
        const bool fused = A.nchunk <= FUSED_RAYLEIGH_MAX_CHUNKS;
        if (!fused)
            hipLaunchKernelGGL(k_rayleigh, dim3(A.nprob), block, 0, s, A, slot_begin, i, par, w->eig_solver);
        set_kb(i, [&](auto kb) {
            constexpr int KB = decltype(kb)::value;
            if (fused)
                hipLaunchKernelGGL((k_ritz<KB, true>), grid, block, 0, s, A, slot_begin, i, restart ? 1 : 0, par,
                                   w->eig_solver);
            else
                hipLaunchKernelGGL((k_ritz<KB, false>), grid, block, 0, s, A, slot_begin, i, restart ? 1 : 0, par,
                                   w->eig_solver);
        });
        int ie = i;
        const double *pin = A.pa;
        if (restart) {
            set_kb(i, [&](auto kb) {
                constexpr int KB = decltype(kb)::value;
                hipLaunchKernelGGL(k_restart<KB>, grid, block, 0, s, A, i, kmin, par);
            });
            ie = kmin;
            pin = A.pb;
        }
        set_kb(ie, [&](auto kb) {
            constexpr int KB = decltype(kb)::value;
            hipLaunchKernelGGL(k_orth<KB>, grid, block, 0, s, A, ie, pin, restart ? 1 : 0, par);
        });
        DMRG_HIP(hipGetLastError());
        const RayArgs ray = ray_args(A, ie + 1);
        DMRG_TRY(launch_project(plan, slot, A.coef, A.T, A.W + (int64_t)ie * A.n, s, A.active, A.dfold, &ray));
        i = ie + 1;
    }
    *i_next = i;
    return DMRG_OK;
}

// Phase set-up: state, start vector, diagonal folding (with the preconditioner
// diagonal for the first phase of a solve), and W(:, 0) with the rows of
// B(0, 0).  Reads the private copy X0 of the start vectors.  With A.gate the
// set-up first tests the previous phase (flags prev) and idles unless it has
// finished.
static dmrg_status enqueue_setup(dmrg_plan *plan, const DavArgs &A, const int32_t *prev, int slot, bool with_diag,
                                 double tol, double floor_, int max_iter, hipStream_t s) {
    const dim3 grid(A.nchunk), block(TPB);
    if (A.gate) hipLaunchKernelGGL(k_gate, dim3(1), block, 0, s, prev, A);
    // one queue, no branches: a cross-queue join inside a graph costs more than
    // the few microseconds the diagonal kernels take
    if (with_diag) DMRG_TRY(launch_diagonal(plan, A.coef, A.D, s));  // preconditioner diagonal of the solve
    DMRG_TRY(launch_diag_fold(plan, slot, A.coef, A.dfold, s));       // coefficients are fixed for the phase
    // a reduced-precision phase ends early when its residual stops halving (5 iterations)
    hipLaunchKernelGGL(k_init_norm, grid, block, 0, s, A.X0, A, tol, floor_, max_iter, slot == 0 ? 0 : 5);
    hipLaunchKernelGGL(k_init_vec, grid, block, 0, s, A.X0, A);
    DMRG_HIP(hipGetLastError());
    const RayArgs ray = ray_args(A, 1);
    return launch_project(plan, slot, A.coef, A.T, A.W, s, A.active, A.dfold, &ray);
}

static uint64_t bits_of(double x) {
    uint64_t u;
    std::memcpy(&u, &x, 8);
    return u;
}

constexpr int FIRST_CHUNK = 4;  // iterations of the first launch of a phase

// Iterations still needed by the slowest active member, from its residual
// decay over the phase so far (geometric model); cap when unknown.
static int predict_iters(const std::vector<DavSummary> &sm, double tol, int cap) {
    int need = 1;
    for (const DavSummary &r : sm) {
        if (!r.active) continue;
        int k = cap;
        if (r.iters > 1 && r.rnorm1 > 0.0 && r.rnorm > 0.0 && r.rnorm < r.rnorm1 && r.rnorm > tol) {
            const double rate = std::log(r.rnorm / r.rnorm1) / (r.iters - 1);  // < 0
            const double est = std::ceil(std::log(tol / r.rnorm) / rate);
            k = (int)std::min<double>(cap, std::max(1.0, est));
        }
        need = std::max(need, k);
    }
    return std::min(need, cap);
}

// One phase (fixed projection precision) to tolerance tol, in launches of
// iterations (captured hipGraphs when use_graph); after each launch the
// per-member summary comes back to the host and decides about the next one.
struct Phase {
    int slot = 0;                    // 1: reduced-precision projection, 0: FP64
    bool psi_in = false;             // starts from the caller's vectors (staged in X0), else from X0 as left
    bool with_diag = false;          // the set-up also computes the preconditioner diagonal
    double tol = 0.0, floor_ = 0.0;
    int max_iter = 1, chunk_max = 1;
    bool use_graph = true;
    bool fin_x0 = false;        // every launch ends with X0 = the current Ritz vectors
    bool gated = false;         // the first launch idles unless the other phase has finished
    double *fin_psi = nullptr;  // every launch ends with fin_psi = the current Ritz vectors
    int i = 0, done = 0, cnt = 0;
};

static const DavArgs &phase_args(const DavidsonWork *w, int slot) { return slot == 0 ? w->a2 : w->a; }
static int phase_kind(const Phase &P) { return 4 * P.slot + (P.fin_x0 ? 2 : 0) + (P.psi_in ? 0 : 1); }

// The caller's coefficients and start vectors into the private copies that
// the captured graphs read (one launch for both).
__global__ __launch_bounds__(TPB) void k_stage(const double *__restrict__ coef, int ncoef, double *__restrict__ cdst,
                                               const double *__restrict__ psi, int64_t n, double *__restrict__ x0) {
    const int64_t t = (int64_t)blockIdx.x * TPB + threadIdx.x, stride = (int64_t)gridDim.x * TPB;
    for (int64_t e = t; e < ncoef; e += stride) cdst[e] = coef[e];
    for (int64_t e = t; e < n; e += stride) x0[e] = psi[e];
}

// First launch: as many iterations as the last phase of this kind needed (a
// repeated solve of a plan, e.g. along a sweep, converges alike), else FIRST_CHUNK.
static void phase_begin(const DavidsonWork *w, Phase &P) {
    const auto hint = w->last_iters.find(phase_kind(P));
    P.i = 0;
    P.done = 0;
    P.cnt = std::min({P.chunk_max, P.max_iter, hint == w->last_iters.end() ? FIRST_CHUNK : hint->second});
}

// Graph key fields of a phase's next launch.
static void phase_key(const DavidsonWork *w, const Phase &P, std::vector<uint64_t> &k) {
    const bool gated = P.gated && P.i == 0, with_diag = P.with_diag && P.i == 0;
    k.insert(k.end(), {(uint64_t)(P.slot + (gated ? 2 : 0) + (with_diag ? 4 : 0)),
                       (uint64_t)(P.i * 4 + (P.fin_x0 ? 2 : 0) + ((P.done + 1) & 1)), (uint64_t)P.cnt,
                       (uint64_t)w->kmax, (uint64_t)w->eig_solver, (uint64_t)P.max_iter, bits_of(P.tol),
                       bits_of(P.floor_)});
}

// Record the next launch of P.cnt iterations of a phase (with the set-up when P.i == 0).
static dmrg_status phase_enqueue(dmrg_plan *plan, const Phase &P, hipStream_t q) {
    DavidsonWork *w = plan->dav;
    DavArgs A = phase_args(w, P.slot);
    const bool gated = P.gated && P.i == 0;
    if (!gated) A.gate = nullptr;
    const int32_t *prev = phase_args(w, 1 - P.slot).active;
    const int i0 = (P.i == 0) ? 1 : P.i;
    int inext = i0;
    if (P.i == 0) DMRG_TRY(enqueue_setup(plan, A, prev, P.slot, P.with_diag, P.tol, P.floor_, P.max_iter, q));
    DMRG_TRY(enqueue_iters(plan, A, P.slot, i0, P.done + 1, P.cnt, &inext, q));
    hipLaunchKernelGGL(k_summary, dim3((A.nprob + 63) / 64), dim3(64), 0, q, A);
    if (P.fin_x0)
        set_kb(w->kmax, [&](auto kb) {  // nvec <= kmax
            constexpr int KB = decltype(kb)::value;
            hipLaunchKernelGGL(k_finalize<KB>, dim3(A.nchunk), dim3(TPB), 0, q, A, (double *)A.X0);
        });
    DMRG_HIP(hipGetLastError());
    return DMRG_OK;
}

// Queue the next launch of each of np phases, in order, as one captured graph
// (use_graph) or directly; the caller's output (fin_psi) is written after it.
static dmrg_status launch_phases(dmrg_plan *plan, Phase *const *ph, int np, hipStream_t s) {
    DavidsonWork *w = plan->dav;
    if (ph[0]->use_graph) {
        std::vector<uint64_t> key;
        for (int j = 0; j < np; ++j) phase_key(w, *ph[j], key);
        auto it = w->graphs.find(key);
        if (it == w->graphs.end()) {
            hipStream_t cs;
            DMRG_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
            hipGraph_t g;
            DMRG_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
            dmrg_status st = DMRG_OK;
            for (int j = 0; j < np && st >= 0; ++j) st = phase_enqueue(plan, *ph[j], cs);
            hipError_t ce = hipStreamEndCapture(cs, &g);
            (void)hipStreamDestroy(cs);
            if (st < 0) return st;
            if (ce != hipSuccess) return set_error(DMRG_E_HIP, "graph capture failed: %s", hipGetErrorString(ce));
            hipGraphExec_t ge;
            hipError_t ie = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
            (void)hipGraphDestroy(g);
            if (ie != hipSuccess) return set_error(DMRG_E_HIP, "graph instantiate failed: %s", hipGetErrorString(ie));
            it = w->graphs.emplace(key, ge).first;
        }
        DMRG_HIP(hipGraphLaunch(it->second, s));
    } else {
        for (int j = 0; j < np; ++j) DMRG_TRY(phase_enqueue(plan, *ph[j], s));
    }
    for (int j = 0; j < np; ++j) {
        Phase &P = *ph[j];
        if (P.fin_psi)  // outside the graphs: the caller's buffer changes from call to call
            set_kb(w->kmax, [&](auto kb) {
                constexpr int KB = decltype(kb)::value;
                hipLaunchKernelGGL(k_finalize<KB>, dim3(w->a.nchunk), dim3(TPB), 0, s, phase_args(w, P.slot),
                                   P.fin_psi);
            });
        // the subspace sequence is deterministic: i after P.cnt iterations
        int ii = (P.i == 0) ? 1 : P.i;
        for (int q = 0; q < P.cnt; ++q) ii = (ii == w->kmax ? w->kmin : ii) + 1;
        P.i = ii;
        P.done += P.cnt;
    }
    DMRG_HIP(hipGetLastError());
    return DMRG_OK;
}

static dmrg_status phase_launch(dmrg_plan *plan, Phase &P, hipStream_t s) {
    Phase *one[1] = {&P};
    return launch_phases(plan, one, 1, s);
}

// After the stream has synchronized: the phase's summary into sm; true when
// the phase needs another launch (then P.cnt is its size).
static bool phase_more(DavidsonWork *w, Phase &P, std::vector<DavSummary> &sm) {
    const DavSummary *h = P.slot == 0 ? w->h_sum2 : w->h_sum;
    const int nprob = w->a.nprob;
    sm.assign(h, h + nprob);
    bool any = false;
    for (const DavSummary &r : sm) any = any || r.active;
    if (any && P.done < P.max_iter) {
        P.cnt = std::min(predict_iters(sm, P.tol, P.chunk_max), P.max_iter - P.done);
        return true;
    }
    int need = 1;
    for (const DavSummary &r : sm) need = std::max(need, (int)r.iters);
    w->last_iters[phase_kind(P)] = need;
    return false;
}

// The host waits for the stream (a launch's mapped summary is then readable).
static dmrg_status host_wait(DavidsonWork *w, hipStream_t s) {
    ++w->waits;
    DMRG_HIP(hipStreamSynchronize(s));
    return DMRG_OK;
}

// A whole phase, one synchronization per launch.
static dmrg_status phase_run(dmrg_plan *plan, Phase &P, hipStream_t s, std::vector<DavSummary> &sm) {
    phase_begin(plan->dav, P);
    do {
        DMRG_TRY(phase_launch(plan, P, s));
        DMRG_TRY(host_wait(plan->dav, s));  // k_summary wrote the mapped summary
    } while (phase_more(plan->dav, P, sm));
    return DMRG_OK;
}

}  // namespace dmrg

// ================================================================== ABI

using namespace dmrg;

template <int KB>
__global__ __launch_bounds__(TPB) void k_gemv_n(int64_t n, int k, const double *__restrict__ V, int64_t ldv,
                                                const double *__restrict__ s, double beta, double *__restrict__ y) {
    double sv[KB];
#pragma unroll
    for (int j = 0; j < KB; ++j) sv[j] = (j < k) ? s[j] : 0.0;
    for (int64_t e = (int64_t)blockIdx.x * TPB + threadIdx.x; e < n; e += (int64_t)gridDim.x * TPB) {
        double acc = (beta == 0.0) ? 0.0 : beta * y[e];
#pragma unroll
        for (int j = 0; j < KB; ++j)
            if (j < k) acc += V[(int64_t)j * ldv + e] * sv[j];
        y[e] = acc;
    }
}

// Partials of dmrg_gemv_t: one buffer per (device, stream), kept until the
// process ends, so calls on different streams never share one.  The map is
// guarded; a buffer only grows, after its own stream has drained.
struct GemvScratch {
    double *p = nullptr;
    size_t bytes = 0;
};
static std::map<std::pair<int, hipStream_t>, GemvScratch> g_gemv_scratch;
static std::mutex g_gemv_mutex;

// Both stages of s = V^T x with the partials in part (>= nblk * 64 doubles).
dmrg_status gemv_t_launch(int64_t n, int32_t k, const double *V, int64_t ldv, const double *x, double *s,
                                 int nblk, double *part, hipStream_t st) {
    auto go = [&](auto kb) {
        constexpr int KB = decltype(kb)::value;
        hipLaunchKernelGGL(k_gemv_t_part<KB>, dim3(nblk), dim3(TPB), 0, st, n, k, V, ldv, x, part);
        hipLaunchKernelGGL(k_gemv_t_final<KB>, dim3(1), dim3(TPB), 0, st, nblk, k, (const double *)part, s);
    };
    if (k <= 16)
        go(std::integral_constant<int, 16>{});
    else if (k <= 32)
        go(std::integral_constant<int, 32>{});
    else
        go(std::integral_constant<int, 64>{});
    DMRG_HIP(hipGetLastError());
    return DMRG_OK;
}

extern "C" {

void dmrg_davidson_default_opts(dmrg_davidson_opts *o) {
    if (!o) return;
    o->tol = 1e-10;
    o->kmax = 32;
    o->kmin = 8;
    o->max_iter = 500;
    o->precond_floor = 1e-3;
    o->prec = DMRG_F64;
    o->tol_lowprec = 0.0;
    o->refine = 1;
    o->use_graph = 1;
    o->graph_chunk = 8;
    o->eig_solver = 0;
}

dmrg_status dmrg_davidson(dmrg_plan *plan, const double *coef, const dmrg_davidson_opts *opts, double *psi,
                          double *energy, dmrg_davidson_info *info, void *stream) {
    clear_error();
    if (!plan || !psi || (!coef && plan->nterm_total)) return set_error(DMRG_E_INVALID_ARG, "null argument");
    dmrg_davidson_opts o;
    dmrg_davidson_default_opts(&o);
    if (opts) o = *opts;
    if (o.kmax < 2 || o.kmax > KM || o.kmin < 1 || o.kmin >= o.kmax)
        return set_error(DMRG_E_INVALID_ARG, "need 2 <= kmax <= %d and 1 <= kmin < kmax", KM);
    if (!(o.tol > 0.0) || o.max_iter < 1 || !(o.precond_floor > 0.0) || o.graph_chunk < 1)
        return set_error(DMRG_E_INVALID_ARG, "need tol > 0, max_iter >= 1, precond_floor > 0, graph_chunk >= 1");
    if (o.eig_solver != 0 && o.eig_solver != 1) return set_error(DMRG_E_INVALID_ARG, "eig_solver must be 0 or 1");
    if (o.prec != DMRG_F64 && o.prec != plan->prec)
        return set_error(DMRG_E_INVALID_ARG, "precision %d not available in this plan", o.prec);
    int cur = -1;
    DMRG_HIP(hipGetDevice(&cur));
    if (cur != plan->device) return set_error(DMRG_E_INVALID_ARG, "plan belongs to another device");
    hipStream_t s = (hipStream_t)stream;
    // the subspace cannot exceed the smallest member dimension
    int64_t nmin = INT64_MAX;
    for (int p = 0; p < plan->nprob; ++p) nmin = std::min(nmin, plan->member_off[p + 1] - plan->member_off[p]);
    if (nmin < 1) return set_error(DMRG_E_INVALID_ARG, "a member has an empty target sector");
    int kmax = (int)std::min<int64_t>(o.kmax, std::max<int64_t>(nmin, 2));
    int kmin = std::min(o.kmin, kmax - 1);
    DMRG_TRY(work_alloc(plan, kmax, kmin, s));
    DavidsonWork *w = plan->dav;
    w->dirty = true;  // until every member is seen to end with finite data
    w->waits = 0;
    w->eig_solver = o.eig_solver;
    const DavArgs &A = w->a;
    hipLaunchKernelGGL(k_stage, dim3((unsigned)std::min<int64_t>((A.n + TPB - 1) / TPB, 2048)), dim3(TPB), 0, s, coef,
                       plan->nterm_total, A.coef, psi, A.n, (double *)A.X0);
    DMRG_HIP(hipGetLastError());

    std::vector<DavSummary> hs, low;
    const bool two_phase = o.prec != DMRG_F64;
    Phase P1, P2;  // reduced precision, FP64
    P1.slot = 1;
    P2.slot = 0;
    for (Phase *P : {&P1, &P2}) {
        P->floor_ = o.precond_floor;
        P->max_iter = o.max_iter;
        P->chunk_max = o.graph_chunk;
        P->use_graph = o.use_graph != 0;
    }
    P1.tol = std::max(o.tol, o.tol_lowprec > 0 ? o.tol_lowprec : (o.prec == DMRG_F32 ? 1e-5 : 1e-3));
    P2.tol = o.tol;
    P2.fin_psi = psi;  // psi = V y, ordered on the stream
    if (!two_phase) {
        P2.psi_in = P2.with_diag = true;
        DMRG_TRY(phase_run(plan, P2, s, hs));
    } else if (!o.refine) {
        P1.psi_in = P1.with_diag = true;
        P1.fin_psi = psi;
        DMRG_TRY(phase_run(plan, P1, s, low));
        hs = low;
    } else {
        // the phase-1 Ritz vectors stay in X0 as the start of phase 2
        P1.psi_in = P1.with_diag = true;
        P1.fin_x0 = true;
        phase_begin(w, P1);
        // a repeated solve (both phases seen before) queues phase 2 right behind
        // the first launch of phase 1, gated on device: one synchronization fewer
        const bool chain = P1.use_graph && w->last_iters.count(phase_kind(P1)) && w->last_iters.count(phase_kind(P2));
        if (chain) {
            P2.gated = true;
            phase_begin(w, P2);
            Phase *both[2] = {&P1, &P2};  // one graph
            DMRG_TRY(launch_phases(plan, both, 2, s));
        } else {
            DMRG_TRY(phase_launch(plan, P1, s));
        }
        DMRG_TRY(host_wait(w, s));
        bool more1 = phase_more(w, P1, low);
        bool open = chain;  // phase 2 has run its first launch
        for (const DavSummary &r : low) open = open && !r.active;
        if (open) {
            while (phase_more(w, P2, hs)) {
                DMRG_TRY(phase_launch(plan, P2, s));
                DMRG_TRY(host_wait(w, s));
            }
        } else {  // finish phase 1, then phase 2 from its start (a gated launch idled)
            while (more1) {
                DMRG_TRY(phase_launch(plan, P1, s));
                DMRG_TRY(host_wait(w, s));
                more1 = phase_more(w, P1, low);
            }
            for (int p = 0; p < plan->nprob; ++p)
                if (low[p].bad_start == 1) return set_error(DMRG_E_NONFINITE, "member %d: zero or non-finite start", p);
            P2.gated = false;
            DMRG_TRY(phase_run(plan, P2, s, hs));
        }
    }
    const bool both = two_phase && o.refine;
    bool clean = true;
    for (int p = 0; p < plan->nprob; ++p)
        clean = clean && !hs[p].bad_start && !hs[p].breakdown && std::isfinite(hs[p].energy) &&
                (!both || (!low[p].bad_start && !low[p].breakdown));
    w->dirty = !clean;
    dmrg_status ret = DMRG_OK;
    for (int p = 0; p < plan->nprob; ++p) {
        const DavSummary &S = hs[p];
        if (S.bad_start == 1) return set_error(DMRG_E_NONFINITE, "member %d: zero or non-finite start vector", p);
        if (S.bad_start == 2) ret = set_error(DMRG_E_NONFINITE, "member %d: non-finite iterate", p);
        if (energy) energy[p] = S.energy;
        if (info) {
            dmrg_davidson_info &I = info[p];
            I.energy = S.energy;
            I.residual = S.rnorm;
            I.iterations = S.iters + (both ? low[p].iters : 0);
            I.iterations_low = two_phase ? low[p].iters : 0;
            I.projections = S.nproj + (both ? low[p].nproj : 0);
            I.restarts = S.restarts + (both ? low[p].restarts : 0);
            I.converged = S.converged;
            I.breakdown = S.breakdown;
            I.host_waits = w->waits;
        }
        if (S.breakdown && ret == DMRG_OK)
            ret = set_error(DMRG_E_BREAKDOWN, "member %d: correction vanished after orthogonalization", p);
        else if (!S.converged && ret == DMRG_OK)
            ret = set_error(DMRG_W_NOT_CONVERGED, "member %d: not converged (residual %.3e)", p, S.rnorm);
    }
    return ret;
}

dmrg_status dmrg_gemv_t(int64_t n, int32_t k, const double *V, int64_t ldv, const double *x, double *s,
                        void *stream) {
    clear_error();
    if (n < 1 || k < 1 || k > 64 || ldv < n || !V || !x || !s)
        return set_error(DMRG_E_INVALID_ARG, "need n >= 1, 1 <= k <= 64, ldv >= n and non-null pointers");
    const int nblk = (int)std::min<int64_t>((n + TPB - 1) / TPB, GEMV_PART_BLOCKS);
    const size_t need = (size_t)nblk * GEMV_PART_COLS * 8;
    int dev = 0;
    DMRG_HIP(hipGetDevice(&dev));
    hipStream_t st = (hipStream_t)stream;
    double *part = nullptr;
    {
        std::lock_guard<std::mutex> lock(g_gemv_mutex);
        GemvScratch &gs = g_gemv_scratch[{dev, st}];
        if (need > gs.bytes) {
            // this stream may still read the old buffer: let it finish before freeing
            DMRG_HIP(hipStreamSynchronize(st));
            if (gs.p) (void)hipFree(gs.p);
            gs.p = nullptr;
            gs.bytes = 0;
            DMRG_HIP(hipMalloc((void **)&gs.p, need));
            gs.bytes = need;
        }
        part = gs.p;
    }
    return gemv_t_launch(n, k, V, ldv, x, s, nblk, part, st);
}

dmrg_status dmrg_gemv_n(int64_t n, int32_t k, const double *V, int64_t ldv, const double *s, double beta,
                        double *y, void *stream) {
    clear_error();
    if (n < 1 || k < 1 || k > 64 || ldv < n || !V || !s || !y)
        return set_error(DMRG_E_INVALID_ARG, "need n >= 1, 1 <= k <= 64, ldv >= n and non-null pointers");
    int nblk = (int)std::min<int64_t>((n + TPB - 1) / TPB, 8192);
    hipStream_t st = (hipStream_t)stream;
    auto go = [&](auto kb) {
        constexpr int KB = decltype(kb)::value;
        hipLaunchKernelGGL(k_gemv_n<KB>, dim3(nblk), dim3(TPB), 0, st, n, k, V, ldv, s, beta, y);
    };
    if (k <= 16)
        go(std::integral_constant<int, 16>{});
    else if (k <= 32)
        go(std::integral_constant<int, 32>{});
    else
        go(std::integral_constant<int, 64>{});
    DMRG_HIP(hipGetLastError());
    return DMRG_OK;
}

}  // extern "C"
