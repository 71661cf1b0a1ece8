/*
 * dmrg.h — C ABI of the MI355X superblock-projection and Davidson library.
 *
 * The library evaluates the DMRG superblock projection of the LR strategy
 * (Nemes et al., "The density matrix renormalization group algorithm on
 * kilo-processor architectures", Sec. "LR strategy", Eq. 9-11)
 *
 *     y = H_SB psi = sum_k c_k (A_k (x) B_k) psi ,
 *
 * restricted to one target symmetry sector Q and evaluated block by block as
 *     Y_{jl} += c_k A_{k, i->j} X_{ik} B_{k, k->l}^T                 (Eq. 11)
 * on the GPU, and runs the Davidson iteration (Alg. 3) for the lowest
 * eigenpair of H_SB in that sector entirely on the device.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Pointers marked "host" are read during the call only.  Pointers marked
 *    "device" must be GPU memory of the device that was current when the plan
 *    was created.
 *  - "stream" is a hipStream_t passed as void* (NULL = the legacy default
 *    stream).  All device work is enqueued on it.
 *  - Every function returns a dmrg_status; no exception or abort crosses the
 *    ABI.  On failure dmrg_last_error() returns a message (thread-local).
 *  - A plan is not thread-safe; distinct plans are independent.
 *  - Symmetry labels are int32 tuples of length `rank` (1 for S^z, 2 for
 *    (N_up, N_dn)); sector labels of a space must be strictly ascending in
 *    lexicographic order.
 *
 * Layout of the target-sector vector psi (the paper leaves it open; this is
 * the library's reading of Eq. 10-11): for every left sector s_L in ascending
 * order whose complement Q - label(s_L) is a right sector s_R, and whose two
 * dimensions are both non-zero, one row-major block X[d_L(s_L)][d_R(s_R)];
 * psi is the concatenation of those blocks.  For a batched plan, psi is the
 * concatenation of the members' vectors in member order.
 */
#ifndef DMRG_H
#define DMRG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t dmrg_status; /* 0 ok, > 0 warning, < 0 error */

enum {
    DMRG_OK = 0,
    DMRG_W_NOT_CONVERGED = 1, /* Davidson stopped at max_iter; outputs are the last iterate */
    DMRG_E_INVALID_ARG = -1,  /* null pointer, negative size, bad enum, bad index */
    DMRG_E_SECTOR = -2,       /* a term maps the target sector outside itself, or block
                                 dims do not match the sector dims */
    DMRG_E_LAYOUT = -3,       /* labels not strictly ascending, duplicate blocks */
    DMRG_E_NOMEM = -4,        /* device allocation failed */
    DMRG_E_HIP = -5,          /* a HIP runtime call failed (message has the HIP error) */
    DMRG_E_NONFINITE = -6,    /* NaN/Inf in the start vector or the result */
    DMRG_E_BREAKDOWN = -7,    /* Davidson correction vanished after orthogonalization */
    DMRG_E_UNSUPPORTED = -8   /* valid request the library does not implement */
};

/* Compute precision of the projection GEMMs.  Vectors and all Davidson
 * arithmetic other than the projection are always FP64. */
enum { DMRG_F64 = 0, DMRG_F32 = 1, DMRG_BF16 = 2 };

/* Operator kinds (Sec. "Symmetries to be exploited": a symmetric operator is
 * a set of dense blocks A_{q_i -> q_j}). */
enum { DMRG_OP_IDENTITY = 0, DMRG_OP_DIAG = 1, DMRG_OP_DENSE = 2 };

/* A block basis grouped by symmetry sectors.  host arrays. */
typedef struct {
    int32_t nsec;         /* number of sectors, >= 1 */
    int32_t rank;         /* labels per sector, 1 or 2 */
    const int32_t *label; /* host [nsec * rank], strictly ascending (lexicographic) */
    const int64_t *dim;   /* host [nsec], >= 0 */
} dmrg_space;

/* One block operator.
 *  IDENTITY: all other fields ignored.
 *  DIAG:     data = device FP64 [m] (m = sum of dims), the diagonal in sector order.
 *  DENSE:    nblk blocks; block b maps sector src[b] to sector dst[b] and is a
 *            row-major FP64 matrix [dim(dst[b])][dim(src[b])] stored at
 *            data + off[b].  A (src, dst) pair may appear at most once.
 * The plan keeps the data pointer (not a copy): the FP64 data must stay
 * valid and unchanged for the plan's lifetime. */
typedef struct {
    int32_t kind;
    int32_t nblk;
    const int32_t *src;  /* host [nblk] */
    const int32_t *dst;  /* host [nblk] */
    const int64_t *off;  /* host [nblk], element offsets into data */
    const double *data;  /* device */
} dmrg_op;

/* Term k of H_SB: coef[k] * ops_left[a] (x) ops_right[b]   (Eq. 9). */
typedef struct {
    int32_t a, b;
} dmrg_term;

/* One superblock (Alg. 1, steps 1-2: left block, right block, superblock). */
typedef struct {
    dmrg_space left, right;
    const int32_t *target; /* host [rank]: the conserved label Q of the sector */
    int32_t nop_left, nop_right;
    const dmrg_op *ops_left, *ops_right; /* host arrays of descriptors */
    int32_t nterm;
    const dmrg_term *terms; /* host [nterm] */
} dmrg_problem;

typedef struct dmrg_plan dmrg_plan; /* opaque */

/* Validate one problem on the host only (no GPU needed).  Checks labels,
 * dims, block indices and sizes, and that every term keeps the target
 * sector closed.  Returns DMRG_OK or the first error found. */
dmrg_status dmrg_problem_check(const dmrg_problem *prob);

/* Build a plan for nprob independent problems (nprob = 1 for a single
 * superblock): enumerate the target-sector pairs, build the operation records
 * once (A and B do not change during Davidson, Sec. "Accelerating projection
 * operation"), choose tiles, upload the task lists, and, for prec != F64,
 * convert the dense operator blocks once (FP64 -> FP32 [-> BF16], round to
 * nearest even) with the diagonals of square blocks kept in FP64.
 * A plan of precision F32/BF16 can also project in F64.  Synchronizes stream.
 * out: receives the plan (NULL on failure).
 * workspace: NULL, or caller-owned device memory (256-byte aligned) of at
 *   least dmrg_plan_workspace_size(.., ws_kmax, ..) bytes that the plan uses
 *   for all of its per-call scratch: the projection intermediate, the
 *   coefficient-gradient partials and the Davidson arrays (basis, products,
 *   partial rows) of a subspace of up to ws_kmax vectors.  It must outlive
 *   the plan and must not be shared with another plan used concurrently.
 *   With NULL the plan allocates that scratch itself (the Davidson arrays at
 *   the first solve).  The plan still owns its metadata, task lists and
 *   reduced-precision operator copies; the block solver, dmrg_project_block
 *   and the density-matrix calls keep allocating their own scratch.
 * ws_kmax: 2..48, read only with a workspace; a later dmrg_davidson with a
 *   larger kmax fails with DMRG_E_NOMEM.
 * Errors: as dmrg_problem_check; DMRG_E_NOMEM when ws_bytes is below the
 * size needed (found on the host, before any device call). */
dmrg_status dmrg_plan_create(dmrg_plan **out, int32_t nprob, const dmrg_problem *probs,
                             int32_t prec, int32_t ws_kmax, void *workspace, size_t ws_bytes,
                             void *stream);

/* Bytes of the caller workspace that dmrg_plan_create needs for these problems,
 * this precision and Davidson subspaces of up to kmax vectors (2..48), found
 * by the same host analysis that plan creation runs (records built once, Sec.
 * "Accelerating projection operation"); no device call.  bytes: host.
 * The size depends on the tile table in force (dmrg_set_tile_table): query it
 * under the table the plan will be created with. */
dmrg_status dmrg_plan_workspace_size(int32_t nprob, const dmrg_problem *probs, int32_t prec,
                                     int32_t kmax, size_t *bytes);

/* Sizes of a plan.  Any output pointer may be NULL.
 *  n:       total length of psi (sum over members)
 *  npair:   total number of target-sector pairs
 *  nrec:    total number of operation records
 *  flop:    algorithmic FLOP of one projection (2 min(...) per two-sided
 *           record, 2 d_j d_i d_k per one-sided record, 2 per element of a
 *           purely diagonal record)
 *  bytes:   algorithmic bytes of one F64 projection (operator blocks and
 *           diagonals read once, psi read once, y written once) */
dmrg_status dmrg_plan_sizes(const dmrg_plan *plan, int64_t *n, int32_t *npair, int32_t *nrec,
                            int64_t *flop, int64_t *bytes);

/* psi layout, host outputs sized by dmrg_plan_sizes:
 *  member [npair], pair_left [npair], pair_right [npair] (sector indices),
 *  pair_off [npair + 1] (element offsets into psi), member_off [nprob + 1]. */
dmrg_status dmrg_plan_layout(const dmrg_plan *plan, int32_t *member, int32_t *pair_left,
                             int32_t *pair_right, int64_t *pair_off, int64_t *member_off);

/* Operation records (Alg. 5, step 1), host outputs [nrec] each:
 *  term index (within the member), input pair, output pair (global pair
 *  indices), and the product order chosen (0: (A X) B^T, 1: A (X B^T),
 *  2: one-sided or diagonal). */
dmrg_status dmrg_plan_records(const dmrg_plan *plan, int32_t *term, int32_t *pair_in,
                              int32_t *pair_out, int32_t *order);

/* y = H_SB psi for every member.
 *  prec: DMRG_F64, or the plan's own precision.
 *  coef: device FP64 [total terms] (members' coefficients concatenated).
 *  psi, y: device FP64 [n]; must not overlap.  Asynchronous on stream. */
dmrg_status dmrg_project(dmrg_plan *plan, int32_t prec, const double *coef, const double *psi,
                         double *y, void *stream);

/* y_v = H_SB psi_v for nvec vectors in FP64 (the block projection of block
 * Davidson-Liu, Sec. "Runtime & Parallelism"): vector v at psi + v ldpsi,
 * result at y + v ldy (ldpsi, ldy >= n).  Groups of four vectors run as one
 * launch in which every output tile loads each operator fragment once for
 * all four (plans whose tiles fit 16 x 16; other plans take one launch per
 * vector).  Same results as dmrg_project up to the order of the FP64 sums.
 * psi and y must not overlap.  Asynchronous on stream. */
dmrg_status dmrg_project_block(dmrg_plan *plan, int32_t nvec, const double *coef, const double *psi,
                               int64_t ldpsi, double *y, int64_t ldy, void *stream);

/* Adjoint of dmrg_project with respect to psi and coef, in FP64:
 *  gpsi  = sum_k c_k (A_k^T (x) B_k^T) gbar     (device [n]; may be NULL)
 *  gcoef[k] = <gbar, (A_k (x) B_k) psi>          (device [total terms]; may be NULL)
 * psi, gbar: device [n].  Asynchronous on stream.  With gbar = psi = the
 * normalized ground state, gcoef is dE/dc_k (Hellmann-Feynman). */
dmrg_status dmrg_project_backward(dmrg_plan *plan, const double *coef, const double *psi,
                                  const double *gbar, double *gpsi, double *gcoef, void *stream);

/* Davidson options (Alg. 3 with the readings documented in the design notes). */
typedef struct {
    double tol;            /* stop when ||r||_2 <= tol (||x|| = 1).  default 1e-10 */
    int32_t kmax;          /* subspace limit (thick restart when reached), 2..48, default 32 */
    int32_t kmin;          /* vectors kept at a restart, 1..kmax-1, default 8 */
    int32_t max_iter;      /* iterations (Ritz evaluations) per phase, default 500 */
    double precond_floor;  /* |D - sigma| floor of the diagonal preconditioner, default 1e-3 */
    int32_t prec;          /* projection precision of phase 1: F64 (one phase) or the plan's */
    double tol_lowprec;    /* phase-1 tolerance for F32/BF16 (0: 1e-5 for F32, 1e-3 for BF16) */
    int32_t refine;        /* F32/BF16: 1 = continue in F64 to tol (default), 0 = stop after phase 1 */
    int32_t use_graph;     /* 1 = replay captured hipGraphs of graph_chunk iterations (default) */
    int32_t graph_chunk;   /* most iterations per launch (graph replay or eager), default 8 */
    int32_t eig_solver;    /* small eigenproblem of the Rayleigh step: 0 = direct solve of the
                              arrowhead (secular equation, Jacobi only where poles nearly
                              coincide), default; 1 = Jacobi always */
} dmrg_davidson_opts;

/* Per-member results, host. */
typedef struct {
    double energy;          /* lowest Ritz value */
    double residual;        /* final ||r||_2 */
    int32_t iterations;     /* Ritz evaluations, both phases */
    int32_t iterations_low; /* of which in the reduced-precision phase */
    int32_t projections;    /* H.v products */
    int32_t restarts;
    int32_t converged;      /* 1 if ||r|| <= tol */
    int32_t breakdown;      /* 1 if the correction vanished */
    int32_t host_waits;     /* host waits for the launches of iterations of the whole call
                               (all members share them) */
} dmrg_davidson_info;

void dmrg_davidson_default_opts(dmrg_davidson_opts *opts);

/* Lowest eigenpair of every member (Alg. 3 on the device).
 *  coef: device FP64 [total terms].
 *  psi:  device FP64 [n]; in: start vectors (any norm, non-zero per member),
 *        out: normalized ground states.
 *  energy: host [nprob] (may be NULL); info: host [nprob] (may be NULL).
 * Iterations run in launches of at most graph_chunk: the first as long as the
 * plan's previous phase of the same kind took (4 without history), then as
 * many as the residual decay predicts; the host waits for each launch's summary.
 * When the plan has solved with refinement before, the first launch of the
 * FP64 phase is queued right behind the first launch of phase 1 (one graph) and
 * starts on device only if every member has finished phase 1; otherwise it
 * idles, phase 1 continues and phase 2 starts afterwards (same results either
 * way).  energy and info are final on return; psi is completed in stream order
 * (work enqueued on stream afterwards sees it; synchronize stream before
 * reading it from the host).  Returns DMRG_W_NOT_CONVERGED if any member did not
 * converge, DMRG_E_BREAKDOWN if any broke down, DMRG_E_NONFINITE for a
 * zero or non-finite start vector, DMRG_E_NOMEM when the plan runs on a caller
 * workspace sized for fewer than kmax vectors.  The arrays of the subspace
 * come from the plan's workspace, or are allocated at the first solve (and
 * again when kmax or kmin changes). */
dmrg_status dmrg_davidson(dmrg_plan *plan, const double *coef, const dmrg_davidson_opts *opts,
                          double *psi, double *energy, dmrg_davidson_info *info, void *stream);

/* Block Davidson-Liu options (the block version of Davidson's method named
 * in Sec. "Runtime & Parallelism"; readings in the design notes). */
typedef struct {
    double tol;           /* stop when every ||r_j||_2 <= tol, default 1e-10 */
    int32_t nroots;       /* b: the lowest b eigenpairs, 1..8, default 4 */
    int32_t kmax;         /* basis limit, 3 b..48 (and <= n), default 32 */
    int32_t kmin;         /* Ritz vectors kept at a restart (at least 2 b), default 0 = 2 b */
    int32_t max_iter;     /* default 500 */
    double precond_floor; /* |D - sigma| floor, default 1e-3 */
    int32_t chunk;        /* iterations enqueued between host checks, default 4 */
} dmrg_block_opts;

typedef struct {
    int32_t iterations, projections, restarts, converged;
} dmrg_block_info;

void dmrg_block_default_opts(dmrg_block_opts *opts);

/* The nroots lowest eigenpairs of a single-superblock plan by block
 * Davidson-Liu on the device (FP64): per iteration one corrected residual
 * r_j / (D - sigma_j) per unconverged root (sigma_0 = min(theta_0, min D),
 * sigma_j = theta_j otherwise), orthogonalized against the basis by two
 * classical passes and among themselves by Cholesky QR twice (a vector that
 * keeps less than 1e-8 of its norm is dropped), projected as a block, the
 * Rayleigh matrix extended by FP64 MFMA tall-skinny products and diagonalized
 * by cyclic Jacobi; thick restart to max(kmin, 2 nroots) Ritz vectors.
 *  X: device FP64 [nroots][n] (vector j at X + j n): in, the start block (any
 *     linearly independent columns); out, the Ritz vectors (orthonormal).
 *  energies, residuals: host [nroots] (may be NULL), ascending.
 * Sizes that change with the iterations stay on the device; the host waits
 * once per `chunk` iterations.  Returns DMRG_W_NOT_CONVERGED after max_iter,
 * DMRG_E_NONFINITE for a non-finite Ritz value, DMRG_E_UNSUPPORTED for a
 * batched plan. */
dmrg_status dmrg_block_davidson(dmrg_plan *plan, const double *coef, const dmrg_block_opts *opts, double *X,
                                double *energies, double *residuals, dmrg_block_info *info, void *stream);

/* Diagonal of H_SB in the target sector (the Davidson preconditioner),
 * device FP64 [n].  Asynchronous. */
dmrg_status dmrg_diagonal(dmrg_plan *plan, const double *coef, double *diag, void *stream);

/* Tall-skinny products of the Davidson orthogonalization (Alg. 3, lines 3,
 * 5, 12, 13) on column-major V (device FP64, column j at V + j * ldv):
 *  dmrg_gemv_t: s[j] = sum_e V[e, j] x[e], j < k          (s: device [k])
 *  dmrg_gemv_n: y[e] = beta * y[e] + sum_j V[e, j] s[j]    (y: device [n])
 * n <= ldv, 1 <= k <= 64.  Asynchronous.  These are the kernels the
 * Davidson driver uses, exposed for measurement. */
dmrg_status dmrg_gemv_t(int64_t n, int32_t k, const double *V, int64_t ldv, const double *x,
                        double *s, void *stream);
dmrg_status dmrg_gemv_n(int64_t n, int32_t k, const double *V, int64_t ldv, const double *s,
                        double beta, double *y, void *stream);

/* dmrg_gemv_t without any allocation, for callers that cannot allocate
 * device memory (code under hipGraph capture, tight serving loops, harnesses
 * that forbid hipMalloc).  Same arguments, kernels and results (bit for bit)
 * as dmrg_gemv_t, but the per-block partial sums live in a fixed 512 KiB
 * array of device memory inside the library, one copy per device, held until
 * the process ends.  Limits: 1 <= k <= 64 (larger k returns
 * DMRG_E_INVALID_ARG naming the limit); any n >= 1.  Calls on one device
 * share that array: calls that overlap in time on one device (different
 * streams or threads) race and must not be issued.  Asynchronous on stream. */
dmrg_status dmrg_gemv_t_noalloc(int64_t n, int32_t k, const double *V, int64_t ldv, const double *x,
                                double *s, void *stream);

/* Reduced density matrices of the left and right blocks from a state psi
 * (Alg. 1, step 5: each block's density matrix, built from the superblock's
 * lowest eigenstate; it is the partial trace of |psi><psi| over the other
 * block).  A left sector meets exactly one right sector inside the target,
 * so for every pair p of the psi layout, with Psi_p the row-major
 * [d_L, d_R] block of psi at pair_off[p]:
 *   rho_left  + left_off[p]:  Psi_p Psi_p^T, row-major [d_L][d_L]
 *   rho_right + right_off[p]: Psi_p^T Psi_p, row-major [d_R][d_R]
 * which is that sector's whole block of the block's density matrix (sectors
 * that no pair uses have a zero block and no storage).  psi is used as given
 * (the traces equal |psi|^2).  Outputs are exactly symmetric.
 *  dmrg_density_layout: host outputs [npair + 1] each (either may be NULL);
 *    left_off[npair] and right_off[npair] are the output lengths.
 *  dmrg_density: psi device FP64 [n]; rho_left, rho_right device FP64 of
 *    those lengths, owned by the caller; either may be NULL (not computed);
 *    must not overlap psi or each other.  FP64 throughout.  Batched plans:
 *    the members' pairs in order.  Asynchronous on stream.
 *  Errors: DMRG_E_INVALID_ARG for a null plan or psi, outputs that alias psi
 *  or each other, or a device other than the plan's; DMRG_E_HIP if the
 *  launch fails. */
dmrg_status dmrg_density_layout(const dmrg_plan *plan, int64_t *left_off, int64_t *right_off);
dmrg_status dmrg_density(dmrg_plan *plan, const double *psi, double *rho_left, double *rho_right,
                         void *stream);

/* Eigen-decomposition of symmetric blocks, e.g. the density-matrix blocks of
 * dmrg_density (Alg. 1, step 6: the eigenvalues of each block's density
 * matrix select the states the block keeps).  FP64, one workgroup per block:
 * cyclic Jacobi for orders up to 8 (in LDS), Householder reduction to
 * tridiagonal form for larger orders (with the block in registers up to
 * order 180), finished by divide and conquer up to order 512 (the
 * reflectors applied to the eigenvectors of the tridiagonal matrix by one
 * workgroup per 16 columns of a block) and by the implicit QL iteration
 * above.
 *  off, dim, woff: device arrays [nblk].  Block b is the row-major symmetric
 *    [dim[b]][dim[b]] matrix at a + off[b] (every entry is read).
 *  w + woff[b]: its eigenvalues in descending order (ties by index).
 *  u + off[b]: row-major [dim[b]][dim[b]]; column j is the unit eigenvector
 *    of w[woff[b] + j], with its first entry of largest magnitude positive.
 *  a is overwritten (contents unspecified on return).  a, w and u are
 *    device FP64, owned by the caller, and must not overlap.
 *  info: optional device [nblk]: Jacobi sweeps (order <= 8), 1 + the QL
 *    iterations of the leaves plus the merges (divide and conquer, orders
 *    9..512), or 1 + the QL iterations (orders above 512); -1 if dim[b] is
 *    outside 1..2048 (the block is then not touched), -2 if the method did
 *    not converge (40 sweeps; 60 QL iterations for one eigenvalue).
 *  The sizes are read on the device: the caller guarantees that every
 *  block lies inside a, w and u.  Asynchronous on stream.
 *  Errors: DMRG_E_INVALID_ARG for nblk < 0, a null array, or a, w, u that
 *  alias; DMRG_E_HIP if a launch fails.  nblk = 0 does nothing. */
dmrg_status dmrg_eigh_blocks(int32_t nblk, const int64_t *off, const int32_t *dim, const int64_t *woff,
                             double *a, double *w, double *u, int32_t *info, void *stream);

/* State selection of the renormalization step (Alg. 1, step 7: a block keeps
 * its states of largest density-matrix eigenvalue).  The sector blocks are
 * grouped (e.g. the left block of one superblock, or of one batch member):
 * group g is blocks gblk[g] .. gblk[g + 1] - 1, whose eigenvalues, each
 * block's in descending order as dmrg_eigh_blocks writes them, lie contiguous
 * in w from w + woff[gblk[g]].  The m_keep[g] largest values of each group
 * are kept; equal values are taken in block order, then in index order.
 *  gblk device [ngroup + 1]; dim, woff device [nblk]; m_keep device [ngroup].
 *  keep: device out [nblk], the number of states kept per block (a prefix of
 *    its eigenvectors); -1 for the blocks of a group of more than 16384 values.
 *  discarded: device out [ngroup] or NULL: the sum of the values not kept
 *    (NaN for an oversized group).
 *  The sizes are read on the device: the caller guarantees that they describe
 *  w.  Asynchronous on stream.
 *  Errors: DMRG_E_INVALID_ARG for ngroup < 0 or a null array (discarded may
 *  be NULL); DMRG_E_HIP if the launch fails.  ngroup = 0 does nothing. */
dmrg_status dmrg_truncate(int32_t ngroup, const int32_t *gblk, const int32_t *dim, const int64_t *woff,
                          const double *w, const int32_t *m_keep, int32_t *keep, double *discarded,
                          void *stream);

/* One operator block to take to the kept basis (see dmrg_renormalize). */
typedef struct {
    int64_t o;            /* element offset in data: the dense block [rows][cols] (row-major),
                             or its diagonal [rows] when diag = 1 */
    int64_t u_dst, u_src; /* element offsets in u of U_dst [rows][rows] and U_src [cols][cols]
                             (row-major, eigenvectors in columns, as dmrg_eigh_blocks writes them) */
    int64_t out;          /* element offset in out of the result [k_dst][k_src] (row-major) */
    int32_t rows, cols;   /* dimensions of the destination and source sectors, >= 1 */
    int32_t k_dst, k_src; /* states kept: 0 <= k_dst <= rows, 0 <= k_src <= cols */
    int32_t diag;         /* 1: the block is diagonal (rows == cols) */
} dmrg_renorm_block;

/* Operator blocks in the kept basis (Alg. 1, step 7: the block's basis is
 * renormalized to its kept states): for every block b,
 *   out[b] = U_dst[:, :k_dst]^T O U_src[:, :k_src],
 * the first k columns of each sector's eigenvector block being the kept
 * states (dmrg_truncate's counts).  FP64, two batched GEMM stages on MFMA.
 *  blocks: host [nblk], validated on the host (sizes, kinds, offsets >= 0);
 *    the caller guarantees that the offsets and sizes lie inside data, u and
 *    out.  data, u: device FP64 inputs; out: device FP64, owned by the
 *    caller, not overlapping data or u.
 *  The device intermediate (sum of rows * k_src doubles) and the tile list
 *  live in a scratch buffer kept per (device, stream) and grown only when a
 *  call needs more, so repeated calls allocate nothing; the call
 *  synchronizes stream before returning.  Calls on one stream from several
 *  host threads at once are not supported (they share that buffer).
 *  Errors: DMRG_E_INVALID_ARG for nblk < 0, a null pointer, out aliasing
 *  data or u, or a block with bad sizes, kind or offsets (the message names
 *  the block); DMRG_E_NOMEM / DMRG_E_HIP from the allocation, copy or
 *  launches.  nblk = 0 does nothing. */
dmrg_status dmrg_renormalize(int32_t nblk, const dmrg_renorm_block *blocks, const double *data,
                             const double *u, double *out, void *stream);

/* One block placement (see dmrg_place_blocks). */
typedef struct {
    int64_t src;      /* element offset in src of a row-major [rows][ld_src] block (ignored if identity) */
    int64_t dst;      /* element offset in dst of the target [rows][ld_dst] region */
    int32_t rows, cols, ld_src, ld_dst;
    double coef;
    int32_t identity; /* 1: place coef times the identity (i == j) instead of src */
} dmrg_place;

/* Block placement, the assembly step of enlarging a block by one site
 * (Alg. 1, step 2: the enlarged block's operators are Kronecker products of
 * block and site operators, so every sector block of them is made of scaled
 * copies of the block operator's blocks, or of identities):
 *   dst[dst + i ld_dst + j] += coef * src[src + i ld_src + j]   (i < rows, j < cols)
 * for every item.  items: host [n], validated on the host; the items of one
 * call must not overlap in dst (they run in parallel; overlapping sums go in
 * separate calls, which run in call order).  src, dst: device FP64, owned by
 * the caller; the caller guarantees the offsets lie inside them.  The item
 * list goes to the per-(device, stream) scratch buffer of dmrg_renormalize
 * (grown only when needed); the call synchronizes stream before returning.
 * Errors: DMRG_E_INVALID_ARG for n < 0, a null dst (or src with a copy
 * item), or an item with negative sizes or offsets, strides below cols or
 * an unknown kind (the message names the item); DMRG_E_NOMEM / DMRG_E_HIP
 * from the allocation, copy or launch.  n = 0 does nothing. */
dmrg_status dmrg_place_blocks(int32_t n, const dmrg_place *items, const double *src, double *dst,
                              void *stream);

/* ------------------------------------------------------------------------
 * Enlarged blocks and the l-1-1-r strategy
 * ------------------------------------------------------------------------
 * Basis of an enlarged block slow (x) fast (Alg. 1, steps 1-2: a block and
 * its neighbouring site, L = l (x) s1 or R = s2 (x) r; the paper leaves the
 * order open, this is the library's reading): one sector per label sum
 * q = q_slow + q_fast that holds states, in ascending lexicographic order;
 * inside sector q the combinations (s_slow, s_fast) with that sum follow in
 * ascending order of s_slow, each a row-major [d(s_slow)][d(s_fast)]
 * sub-block (slow index first, as in the Kronecker product slow (x) fast). */

/* Term of an enlarged operator: op_out += coef * slow_op[a] (x) fast_op[b]. */
typedef struct {
    int32_t out, a, b;
    double coef;
} dmrg_kron_term;

typedef struct {
    int32_t nsec;        /* sectors of the enlarged block */
    int32_t nblk_total;  /* dense blocks over all output operators */
    int64_t m;           /* dimension of the enlarged block */
    int64_t data_len;    /* FP64 elements of all output operators */
} dmrg_enlarge_sizes;

/* Operators of an enlarged block (Alg. 1, steps 1-2): for every output o,
 *   op_out[o] = sum over its terms of coef * slow_op[a] (x) fast_op[b]
 * in the enlarged basis above.  Host only (no GPU): every data pointer of
 * ops_slow / ops_fast is HOST FP64 here (the dmrg_op layouts as usual).
 * Two calls: with label == NULL only *sizes is filled; then call again with
 * arrays of those sizes:
 *  label [nsec * rank], dim [nsec]: the enlarged space;
 *  op_kind [nout]: IDENTITY (a single term I (x) I with coef 1), DIAG (every
 *    term's two factors are identity or diagonal) or DENSE;
 *  op_nblk [nout], op_off [nout]: blocks and first data element of output o;
 *  src, dst, off [nblk_total]: the blocks of output 0, then of output 1, ...,
 *    each output's in ascending (src, dst); off relative to op_off[o];
 *  data [data_len]: DIAG outputs hold their diagonal [m], DENSE outputs their
 *    row-major blocks [dim(dst)][dim(src)].
 * A dmrg_op for output o is {op_kind[o], op_nblk[o], src + b0, dst + b0,
 * off + b0, data + op_off[o]} with b0 = the blocks of the outputs before it.
 * Errors: DMRG_E_INVALID_ARG (null or out-of-range arguments, output arrays
 * missing in the second call), DMRG_E_LAYOUT (labels not ascending, duplicate
 * blocks), DMRG_E_UNSUPPORTED (a sector above 2^20 states). */
dmrg_status dmrg_enlarge(const dmrg_space *slow, int32_t nop_slow, const dmrg_op *ops_slow,
                         const dmrg_space *fast, int32_t nop_fast, const dmrg_op *ops_fast,
                         int32_t nterm, const dmrg_kron_term *terms, int32_t nout,
                         dmrg_enlarge_sizes *sizes, int32_t *label, int64_t *dim, int32_t *op_kind,
                         int32_t *op_nblk, int64_t *op_off, int32_t *src, int32_t *dst, int64_t *off,
                         double *data);

/* Term k of a four-subsystem superblock (Sec. "l-1-1-r strategy", Eq. 12):
 * coef[k] * ops[0][a] (x) ops[1][b] (x) ops[2][c] (x) ops[3][d]. */
typedef struct {
    int32_t a, b, c, d;
} dmrg_term4;

/* A superblock written over its four subsystems: block l, site 1, site 2,
 * block r.  Operator data: blocks l and r device FP64 (kept by reference, as
 * in dmrg_problem); the two sites HOST FP64, read once at plan creation
 * (their matrix elements become constant factors of the records). */
typedef struct {
    dmrg_space space[4];
    const int32_t *target; /* host [rank] */
    int32_t nop[4];
    const dmrg_op *ops[4]; /* host arrays of descriptors */
    int32_t nterm;
    const dmrg_term4 *terms; /* host [nterm] */
} dmrg_problem4;

/* Plan of the l-1-1-r strategy (Eq. 13, Alg. 2): the projection is formed
 * from the four subsystems' operators, so no operator of an enlarged block
 * (largest matrix O((m q)^2)) is ever built, only blocks of l and r
 * (O(m^2)).  psi has the LR layout of the enlarged blocks (l (x) s1,
 * s2 (x) r) in the basis above (dmrg_enlarge with no terms returns their
 * spaces); a sector quadruple (s_l, s_1, s_2, s_r) is the sub-block of rows
 * of its combination (s_l, s_1) and columns of (s_2, s_r), a [d_l d_1] x
 * [d_2 d_r] sub-matrix that reshapes to Alg. 2's X[i_l][i_1][i_2][i_r].
 * Every record applies A_l X B_r^T to the [d_l x d_r] slice of fixed site
 * indices (i_1, i_2), scaled by the site matrix elements, on the same
 * grouped-GEMM kernels as the LR plans.  The resulting plan serves
 * dmrg_project, dmrg_project_backward, dmrg_davidson, dmrg_diagonal and the
 * density calls exactly like an LR plan (FP64 only).  Synchronizes stream.
 * Errors: as dmrg_plan_create; DMRG_E_SECTOR for a term that leaves the
 * target sector. */
dmrg_status dmrg_plan_create_l11r(dmrg_plan **out, int32_t nprob, const dmrg_problem4 *probs, void *stream);

/* Set the tile table used by later dmrg_plan_create calls: for output
 * blocks with max(rows, cols) <= bound[c] (ascending, ncls <= 8), tiles of
 * tile[c] rows and columns (16 or 32).  ncls = 0 restores the built-in table.
 * Process-wide; not thread-safe against concurrent plan creation. */
dmrg_status dmrg_set_tile_table(int32_t ncls, const int32_t *bound, const int32_t *tile);

void dmrg_plan_destroy(dmrg_plan *plan);

const char *dmrg_last_error(void);

/* Library version string. */
const char *dmrg_version(void);

#ifdef __cplusplus
}
#endif

#endif /* DMRG_H */
