// Device-resident Davidson iteration (Alg. 3) for one or many superblocks.
//
// Every member of a plan runs in lock step: all members share the subspace
// size i of an iteration, a member that has converged is masked out, so the
// host knows the kernel sequence of each iteration in advance and can replay
// captured hipGraphs of several iterations.  Per iteration:
//
//   projection  W(:, i-1) = H V(:, i-1)                  (line 2), whose output
//               tiles also form B(:, i-1) = V^T W(:, i-1) (line 3); the last
//               tile of a member solves the small eigenproblem (line 4) by a
//               warm-started parallel Jacobi in one workgroup
//   k_ritz      x = V y, r = W y - lambda x, ||r||   (lines 5-7)
//               t = r / (D - sigma) (line 10, shifted diagonal preconditioner)
//               s = V^T t (line 12, first pass) -- all in one sweep over V, W
//   k_restart   (when i = kmax) V <- V Y(:, :kmin), W <- W Y(:, :kmin), s = V^T t
//   k_orth      t <- t - V s (line 13), ||t||, and V^T t for the DGKS pass
//   k_append    V(:, i) = (t - V s2) / ||.||  when a second pass is needed (line 14)
//
// Reductions over the vector length are split into fixed chunks; each block
// writes its partial sums, and the last block of a member (atomic arrival
// counter, reset by that block) sums the partials in chunk order, so results
// are independent of scheduling and identical between eager and graph runs.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <tuple>

#include "dav_common.h"
#include "gemv.h"
#include "internal.h"

namespace dmrg {

// Kernel-argument view of the Davidson workspace (plain pointers only).
struct DavArgs {
    int64_t n = 0;
    int nprob = 0;
    int nchunk = 0;
    double *V = nullptr, *W = nullptr, *T = nullptr, *D = nullptr, *coef = nullptr;
    double *dfold = nullptr;         // [n] folded diagonal terms of the current phase's pass
    double *part = nullptr;          // [nchunk][KM + 2]
    int32_t *chunk_member = nullptr;
    int64_t *chunk_begin = nullptr;  // [nchunk + 1] element ranges
    int32_t *member_chunk = nullptr; // [nprob + 1] chunk ranges
    int32_t *counter = nullptr;      // [nprob] arrival counters
    int32_t *nactive = nullptr;      // [1] members still iterating
    int32_t *active = nullptr;       // [nprob] 1 while the member iterates
    DavState *st = nullptr;          // [nprob]
};

struct DavidsonWork {
    DavArgs a;
    int kmax = 0, kmin = 0;
    int32_t *h_nactive = nullptr;  // pinned
    std::map<std::tuple<int, int, int, int>, hipGraphExec_t> graphs;
    std::vector<void *> owned;
};

// ------------------------------------------------------------------ helpers

// Element range and member of chunk c.  A single-member plan needs no lookup:
// its chunks are the consecutive TPB-element ranges.
struct Chunk {
    int member;
    int64_t e0, e1;
};
__device__ __forceinline__ Chunk chunk_of(const DavArgs &w, int c) {
    Chunk k;
    if (w.nprob == 1) {
        k.member = 0;
        k.e0 = (int64_t)c * TPB;
        k.e1 = min(w.n, k.e0 + TPB);
    } else {
        k.member = w.chunk_member[c];
        k.e0 = w.chunk_begin[c];
        k.e1 = w.chunk_begin[c + 1];
    }
    return k;
}

// ------------------------------------------------------------------ init kernels

// ||psi||^2 per member; last block stores the scale, flags zero / non-finite starts.
__global__ __launch_bounds__(TPB) void k_init_norm(const double *__restrict__ psi, DavArgs w) {
    __shared__ double lds[4 * 2];
    const int c = blockIdx.x;
    const Chunk ck = chunk_of(w, c);
    const int member = ck.member;
    double v[1] = {0.0};
    for (int64_t e = ck.e0 + threadIdx.x; e < ck.e1; e += TPB) v[0] += psi[e] * psi[e];
    block_reduce<1>(v, 1, lds);
    if (threadIdx.x == 0) w.part[(size_t)c * (KM + 2)] = v[0];
    const int c0 = w.nprob == 1 ? 0 : w.member_chunk[member];
    const int c1 = w.nprob == 1 ? w.nchunk : w.member_chunk[member + 1];
    if (!last_arrival(w.counter, member, c - c0, c1 - c0)) return;
    double s = member_sum(w.part, c0, c1, 0, lds);
    if (threadIdx.x == 0) {
        DavState &S = w.st[member];
        if (!(s > 0.0) || !isfinite(s)) {
            S.bad_start = 1;
            w.active[member] = 0;
            S.scale = 0.0;
            atomicSub(w.nactive, 1);
        } else {
            S.scale = 1.0 / sqrt(s);
        }
    }
}

// V(:,0) = psi * scale; also the diagonal's minimum per member.
__global__ __launch_bounds__(TPB) void k_init_vec(const double *__restrict__ psi, DavArgs w) {
    __shared__ double lds[4 * 2];
    __shared__ double red[TPB];
    const int c = blockIdx.x;
    const Chunk ck = chunk_of(w, c);
    const int member = ck.member;
    const double sc = w.st[member].scale;
    double mn = INFINITY;
    for (int64_t e = ck.e0 + threadIdx.x; e < ck.e1; e += TPB) {
        w.V[e] = psi[e] * sc;
        mn = fmin(mn, w.D[e]);
    }
    red[threadIdx.x] = mn;
    __syncthreads();
    for (int off = TPB / 2; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) red[threadIdx.x] = fmin(red[threadIdx.x], red[threadIdx.x + off]);
        __syncthreads();
    }
    if (threadIdx.x == 0) w.part[(size_t)c * (KM + 2)] = red[0];
    const int c0 = w.nprob == 1 ? 0 : w.member_chunk[member];
    const int c1 = w.nprob == 1 ? w.nchunk : w.member_chunk[member + 1];
    if (!last_arrival(w.counter, member, c - c0, c1 - c0)) return;
    mn = INFINITY;
    for (int q = c0 + (int)threadIdx.x; q < c1; q += TPB) mn = fmin(mn, w.part[(size_t)q * (KM + 2)]);
    red[threadIdx.x] = mn;
    __syncthreads();
    for (int off = TPB / 2; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) red[threadIdx.x] = fmin(red[threadIdx.x], red[threadIdx.x + off]);
        __syncthreads();
    }
    if (threadIdx.x == 0) w.st[member].dmin = red[0];
    (void)lds;
}

// ------------------------------------------------------------------ small eigenproblem

// ------------------------------------------------------------------ iteration kernels

// x = V y, r = W y - lambda x, t = r / (D - sigma); partials: ||r||^2, ||t||^2, V^T t.
template <int KB>
__global__ __launch_bounds__(TPB) void k_ritz(DavArgs w, int i, int restart) {
    __shared__ double lds[4 * (KB + 2)];
    __shared__ double scratch[TPB];
    __shared__ double sums[KB + 2];
    const int c = blockIdx.x;
    const Chunk ck = chunk_of(w, c);
    const int member = ck.member;
    const DavState &S = w.st[member];
    const int act = w.active[member];
    const int64_t n = w.n;
    double y[KB];
#pragma unroll
    for (int j = 0; j < KB; ++j) y[j] = (j < i) ? S.Y[j * KM] : 0.0;
    const double lam = S.lambda, sig = S.sigma, fl = S.floor_;
    double acc[KB + 2];
#pragma unroll
    for (int j = 0; j < KB + 2; ++j) acc[j] = 0.0;
    for (int64_t e = ck.e0 + threadIdx.x; e < ck.e1; e += TPB) {
        double v[KB], wv[KB];
        double x = 0.0, wy = 0.0;
#pragma unroll
        for (int j = 0; j < KB; ++j) {
            v[j] = w.V[(int64_t)min(j, i - 1) * n + e];
            wv[j] = w.W[(int64_t)min(j, i - 1) * n + e];
        }
#pragma unroll
        for (int j = 0; j < KB; ++j) {
            v[j] = (j < i) ? v[j] : 0.0;
            x += v[j] * y[j];
            wy += wv[j] * y[j];
        }
        const double r = wy - lam * x;
        double den = w.D[e] - sig;
        if (fabs(den) < fl) den = (den < 0.0) ? -fl : fl;
        const double t = r / den;
        if (act) w.T[e] = t;
        acc[KB] += r * r;
        acc[KB + 1] += t * t;
        if (!restart) {
#pragma unroll
            for (int j = 0; j < KB; ++j) acc[j] += v[j] * t;
        }
    }
    if (!act) return;
    block_reduce<KB + 2>(acc, KB + 2, lds);
    if (threadIdx.x == 0)
        for (int j = 0; j < KB + 2; ++j) w.part[(size_t)c * (KM + 2) + j] = acc[j];
    // note: columns KB, KB+1 of the partial row hold ||r||^2 and ||t||^2
    const int c0 = w.nprob == 1 ? 0 : w.member_chunk[member];
    const int c1 = w.nprob == 1 ? w.nchunk : w.member_chunk[member + 1];
    if (!last_arrival(w.counter, member, c - c0, c1 - c0)) return;
    DavState &Sm = w.st[member];
    member_sums(w.part, c0, c1, KB + 2, scratch, sums);
    const double rr = sums[KB];
    const double tt = sums[KB + 1];
    double ss = 0.0;
    if (!restart) {
        if ((int)threadIdx.x < i) Sm.s[threadIdx.x] = sums[threadIdx.x];
        for (int j = 0; j < i; ++j) ss += sums[j] * sums[j];
    }
    if (threadIdx.x == 0) {
        Sm.rnorm = sqrt(rr);
        Sm.tn0 = sqrt(tt);
        if (!(Sm.rnorm == Sm.rnorm) || isinf(Sm.rnorm)) {
            w.active[member] = 0;
            Sm.bad_start = 2;  // non-finite iterate
            atomicSub(w.nactive, 1);
        } else if (Sm.rnorm <= Sm.tol) {
            Sm.converged = 1;
            w.active[member] = 0;
            atomicSub(w.nactive, 1);
        } else if (Sm.iters >= Sm.max_iter) {
            w.active[member] = 0;
            atomicSub(w.nactive, 1);
        } else if (!restart) {
            // ||t - V s||^2 = ||t||^2 - ||s||^2; reliable unless it cancels below half
            Sm.dgks = (tt - ss) < 0.5 * tt;
            if (!(tt > 0.0)) {
                Sm.breakdown = 1;
                w.active[member] = 0;
                atomicSub(w.nactive, 1);
            } else if (!Sm.dgks) {
                Sm.scale = 1.0 / sqrt(tt - ss);
            }
        }
    }
}

// Thick restart: V(:, :kmin) = V(:, :i) Y(:, :kmin), same for W; then s = V^T t, ||t||^2.
template <int KB>
__global__ __launch_bounds__(TPB) void k_restart(DavArgs w, int i, int kmin) {
    __shared__ double lds[4 * (KB + 1)];
    __shared__ double Ys[KB * KB];
    __shared__ double scratch[TPB];
    __shared__ double sums[KB + 1];
    const int c = blockIdx.x;
    const Chunk ck = chunk_of(w, c);
    const int member = ck.member;
    const DavState &S = w.st[member];
    if (!w.active[member]) return;
    for (int e = threadIdx.x; e < KB * KB; e += TPB) {
        int r = e / KB, q = e % KB;
        Ys[r * KB + q] = (r < i && q < kmin) ? S.Y[r * KM + q] : 0.0;
    }
    __syncthreads();
    const int64_t n = w.n;
    double acc[KB + 1];
#pragma unroll
    for (int j = 0; j < KB + 1; ++j) acc[j] = 0.0;
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
            acc[q] += a * t;
        }
        acc[KB] += t * t;
    }
    block_reduce<KB + 1>(acc, KB + 1, lds);
    if (threadIdx.x == 0)
        for (int j = 0; j < KB + 1; ++j) w.part[(size_t)c * (KM + 2) + j] = acc[j];
    const int c0 = w.nprob == 1 ? 0 : w.member_chunk[member];
    const int c1 = w.nprob == 1 ? w.nchunk : w.member_chunk[member + 1];
    if (!last_arrival(w.counter, member, c - c0, c1 - c0)) return;
    DavState &Sm = w.st[member];
    member_sums(w.part, c0, c1, KB + 1, scratch, sums);
    const double tt = sums[KB];
    double ss = 0.0;
    if ((int)threadIdx.x < kmin) Sm.s[threadIdx.x] = sums[threadIdx.x];
    for (int j = 0; j < kmin; ++j) ss += sums[j] * sums[j];
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int r = 0; r < kmin; ++r)
            for (int q = 0; q < kmin; ++q) {
                Sm.Bm[r * KM + q] = (r == q) ? Sm.theta[r] : 0.0;
                Sm.Y[r * KM + q] = (r == q) ? 1.0 : 0.0;
            }
        Sm.tn0 = sqrt(tt);
        Sm.dgks = (tt - ss) < 0.5 * tt;
        if (!(tt > 0.0)) {
            Sm.breakdown = 1;
            w.active[member] = 0;
            atomicSub(w.nactive, 1);
        } else if (!Sm.dgks) {
            Sm.scale = 1.0 / sqrt(tt - ss);
        }
        Sm.restarts += 1;
    }
}

// t <- t - V s; partials: ||t||^2 and V^T t (for the DGKS pass).
template <int KB>
__global__ __launch_bounds__(TPB) void k_orth(DavArgs w, int i) {
    __shared__ double lds[4 * (KB + 1)];
    __shared__ double scratch[TPB];
    __shared__ double sums[KB + 1];
    const int c = blockIdx.x;
    const Chunk ck = chunk_of(w, c);
    const int member = ck.member;
    const DavState &S = w.st[member];
    const int act = w.active[member];
    const int dg = S.dgks;         // second Gram-Schmidt pass needed (decided by the previous tail)
    const double sc = S.scale;     // 1/||t - V s|| by Pythagoras when no second pass is needed
    double s[KB];
#pragma unroll
    for (int j = 0; j < KB; ++j) s[j] = (j < i) ? S.s[j] : 0.0;
    const int64_t n = w.n;
    double acc[KB + 1];
#pragma unroll
    for (int j = 0; j < KB + 1; ++j) acc[j] = 0.0;
    for (int64_t e = ck.e0 + threadIdx.x; e < ck.e1; e += TPB) {
        double v[KB];
        double t = w.T[e];
#pragma unroll
        for (int j = 0; j < KB; ++j) v[j] = w.V[(int64_t)min(j, i - 1) * n + e];
#pragma unroll
        for (int j = 0; j < KB; ++j) {
            v[j] = (j < i) ? v[j] : 0.0;
            t -= v[j] * s[j];
        }
        if (!dg) {
            if (act) w.V[(int64_t)i * n + e] = t * sc;  // line 14: normalize and append
            continue;
        }
        if (act) w.T[e] = t;
#pragma unroll
        for (int j = 0; j < KB; ++j) acc[j] += v[j] * t;
        acc[KB] += t * t;
    }
    if (!act || !dg) return;
    block_reduce<KB + 1>(acc, KB + 1, lds);
    if (threadIdx.x == 0)
        for (int j = 0; j < KB + 1; ++j) w.part[(size_t)c * (KM + 2) + j] = acc[j];
    const int c0 = w.nprob == 1 ? 0 : w.member_chunk[member];
    const int c1 = w.nprob == 1 ? w.nchunk : w.member_chunk[member + 1];
    if (!last_arrival(w.counter, member, c - c0, c1 - c0)) return;
    DavState &Sm = w.st[member];
    member_sums(w.part, c0, c1, KB + 1, scratch, sums);
    const double tt = sums[KB];
    double ss = 0.0;
    if ((int)threadIdx.x < i) Sm.s2[threadIdx.x] = sums[threadIdx.x];
    for (int j = 0; j < i; ++j) ss += sums[j] * sums[j];
    if (threadIdx.x == 0) {
        const double nrm = sqrt(fmax(tt - ss, 0.0));
        if (!(nrm > 1e-13 * Sm.tn0)) {
            Sm.breakdown = 1;
            w.active[member] = 0;
            atomicSub(w.nactive, 1);
        } else {
            Sm.scale = 1.0 / nrm;
        }
    }
}

// Second Gram-Schmidt pass: V(:, i) = (t - V s2) * scale; no-op unless needed.
template <int KB>
__global__ __launch_bounds__(TPB) void k_append(DavArgs w, int i) {
    const int c = blockIdx.x;
    const Chunk ck = chunk_of(w, c);
    const int member = ck.member;
    const DavState &S = w.st[member];
    if (!S.dgks || !w.active[member]) return;
    double s2[KB];
#pragma unroll
    for (int j = 0; j < KB; ++j) s2[j] = (j < i) ? S.s2[j] : 0.0;
    const double sc = S.scale;
    const int64_t n = w.n;
    for (int64_t e = ck.e0 + threadIdx.x; e < ck.e1; e += TPB) {
        double t = w.T[e];
        double v[KB];
#pragma unroll
        for (int j = 0; j < KB; ++j) v[j] = w.V[(int64_t)min(j, i - 1) * n + e];
#pragma unroll
        for (int j = 0; j < KB; ++j) t -= v[j] * s2[j];
        w.V[(int64_t)i * n + e] = t * sc;
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
    for (int j = 0; j < KB; ++j) y[j] = (j < nv) ? S.Y[j * KM] : 0.0;
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

__global__ void k_set_state(DavArgs w, double tol, double floor_, int max_iter) {
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= w.nprob) return;
    DavState &S = w.st[m];
    S.tol = tol;
    S.floor_ = floor_;
    S.max_iter = max_iter;
    w.active[m] = 1;
    S.converged = 0;
    S.breakdown = 0;
    S.bad_start = 0;
    S.dgks = 0;
    S.nvec = 1;
    S.iters = 0;  // counts are per phase; the host adds the phases
    S.nproj = 0;
    S.restarts = 0;
    S.Y[0] = 1.0;  // (arrival counters are zeroed at allocation and by every completed reduction)
    if (m == 0) *w.nactive = w.nprob;
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

static dmrg_status work_alloc(dmrg_plan *plan, int kmax, int kmin, hipStream_t s) {
    DavidsonWork *w = plan->dav;
    if (w && w->kmax == kmax && w->kmin == kmin) return DMRG_OK;
    davidson_free(plan);
    w = new DavidsonWork();
    plan->dav = w;
    w->kmax = kmax;
    w->kmin = kmin;
    DavArgs &A = w->a;
    A.n = plan->n;
    A.nprob = plan->nprob;
    // chunks: at most 2048 elements, never crossing a member boundary
    std::vector<int32_t> cm;
    std::vector<int64_t> cb;
    std::vector<int32_t> mc(1, 0);
    const int64_t CH = TPB;  // one element per thread: many blocks, every column load in flight
    for (int p = 0; p < plan->nprob; ++p) {
        int64_t b = plan->member_off[p], e = plan->member_off[p + 1];
        if (e == b) {  // empty member: one empty chunk keeps the bookkeeping uniform
            cm.push_back(p);
            cb.push_back(b);
        }
        for (int64_t x = b; x < e; x += CH) {
            cm.push_back(p);
            cb.push_back(x);
        }
        mc.push_back((int32_t)cm.size());
    }
    cb.push_back(plan->n);
    A.nchunk = (int)cm.size();
    // two-level arrival counters bound the chunks (and output tiles) of one member
    const int64_t max_arrivals = (int64_t)ARRIVE_G * (CTR_STRIDE - 1);
    for (int p = 0; p < plan->nprob; ++p)
        if (mc[p + 1] - mc[p] > max_arrivals)
            return set_error(DMRG_E_UNSUPPORTED, "member %d: target sector larger than %lld elements", p,
                             (long long)(max_arrivals * CH));
    for (int q = 0; q < 2; ++q)
        if (plan->fwd[q].stageB.ntask > max_arrivals)
            return set_error(DMRG_E_UNSUPPORTED, "more than %lld output tiles", (long long)max_arrivals);
    auto alloc = [&](void **p, size_t bytes) -> dmrg_status {
        DMRG_HIP(hipMalloc(p, std::max<size_t>(bytes, 8)));
        w->owned.push_back(*p);
        return DMRG_OK;
    };
    const size_t n = (size_t)plan->n;
    DMRG_TRY(alloc((void **)&A.V, (kmax + 1) * n * 8));
    DMRG_TRY(alloc((void **)&A.W, (kmax + 1) * n * 8));
    DMRG_TRY(alloc((void **)&A.T, n * 8));
    DMRG_TRY(alloc((void **)&A.D, n * 8));
    DMRG_TRY(alloc((void **)&A.dfold, n * 8));
    DMRG_TRY(alloc((void **)&A.coef, std::max(plan->nterm_total, 1) * 8));
    // partial rows: one per chunk, or one per output tile when the projection runs the Rayleigh step
    const int rows = std::max({A.nchunk, plan->fwd[0].stageB.ntask, plan->fwd[1].stageB.ntask});
    DMRG_TRY(alloc((void **)&A.part, (size_t)rows * (KM + 2) * 8));
    DMRG_TRY(alloc((void **)&A.chunk_member, cm.size() * 4));
    DMRG_TRY(alloc((void **)&A.chunk_begin, cb.size() * 8));
    DMRG_TRY(alloc((void **)&A.member_chunk, mc.size() * 4));
    DMRG_TRY(alloc((void **)&A.counter, (size_t)plan->nprob * CTR_STRIDE * 4));
    DMRG_TRY(alloc((void **)&A.nactive, 4));
    DMRG_TRY(alloc((void **)&A.st, plan->nprob * sizeof(DavState)));
    DMRG_TRY(alloc((void **)&A.active, plan->nprob * 4));
    DMRG_HIP(hipHostMalloc((void **)&w->h_nactive, 4, hipHostMallocDefault));
    DMRG_HIP(hipMemcpyAsync(A.chunk_member, cm.data(), cm.size() * 4, hipMemcpyHostToDevice, s));
    DMRG_HIP(hipMemcpyAsync(A.chunk_begin, cb.data(), cb.size() * 8, hipMemcpyHostToDevice, s));
    DMRG_HIP(hipMemcpyAsync(A.member_chunk, mc.data(), mc.size() * 4, hipMemcpyHostToDevice, s));
    DMRG_HIP(hipMemsetAsync(A.st, 0, plan->nprob * sizeof(DavState), s));
    DMRG_HIP(hipMemsetAsync(A.counter, 0, (size_t)plan->nprob * CTR_STRIDE * 4, s));
    DMRG_HIP(hipStreamSynchronize(s));
    return DMRG_OK;
}

dmrg_status davidson_free(dmrg_plan *plan) {
    DavidsonWork *w = plan->dav;
    if (!w) return DMRG_OK;
    for (auto &kv : w->graphs) (void)hipGraphExecDestroy(kv.second);
    for (void *p : w->owned) (void)hipFree(p);
    if (w->h_nactive) (void)hipHostFree(w->h_nactive);
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
    r.part = A.part;
    r.counter = A.counter;
    r.st = A.st;
    return r;  // slot_begin is filled per pass by the launcher
}

// Enqueue `count` iterations starting at subspace size i; returns the next i.
static dmrg_status enqueue_iters(dmrg_plan *plan, int slot, int i, int count, int *i_next, hipStream_t s) {
    DavidsonWork *w = plan->dav;
    const DavArgs &A = w->a;
    const int kmax = w->kmax, kmin = w->kmin;
    const dim3 grid(A.nchunk), block(TPB);
    for (int it = 0; it < count; ++it) {
        const bool restart = (i == kmax);
        // the Rayleigh step of this iteration ran in the tail of the previous projection
        set_kb(i, [&](auto kb) {
            constexpr int KB = decltype(kb)::value;
            hipLaunchKernelGGL(k_ritz<KB>, grid, block, 0, s, A, i, restart ? 1 : 0);
        });
        int ie = i;
        if (restart) {
            set_kb(i, [&](auto kb) {
                constexpr int KB = decltype(kb)::value;
                hipLaunchKernelGGL(k_restart<KB>, grid, block, 0, s, A, i, kmin);
            });
            ie = kmin;
        }
        set_kb(ie, [&](auto kb) {
            constexpr int KB = decltype(kb)::value;
            hipLaunchKernelGGL(k_orth<KB>, grid, block, 0, s, A, ie);
            hipLaunchKernelGGL(k_append<KB>, grid, block, 0, s, A, ie);
        });
        DMRG_HIP(hipGetLastError());
        const RayArgs ray = ray_args(A, ie + 1);
        DMRG_TRY(launch_project(plan, slot, A.coef, A.V + (int64_t)ie * A.n, A.W + (int64_t)ie * A.n, s, A.active,
                                A.dfold, &ray));
        i = ie + 1;
    }
    *i_next = i;
    return DMRG_OK;
}

static dmrg_status run_phase(dmrg_plan *plan, int slot, const double *psi_in, double tol, double floor_,
                             int max_iter, bool use_graph, int chunk, hipStream_t s, int *iters_out) {
    DavidsonWork *w = plan->dav;
    const DavArgs &A = w->a;
    const dim3 grid(A.nchunk), block(TPB);
    hipLaunchKernelGGL(k_set_state, dim3((A.nprob + 63) / 64), dim3(64), 0, s, A, tol, floor_, max_iter);
    hipLaunchKernelGGL(k_init_norm, grid, block, 0, s, psi_in, A);
    hipLaunchKernelGGL(k_init_vec, grid, block, 0, s, psi_in, A);
    DMRG_HIP(hipGetLastError());
    DMRG_TRY(launch_diag_fold(plan, slot, A.coef, A.dfold, s));  // coefficients are fixed for the phase
    const RayArgs ray = ray_args(A, 1);  // W(:, 0) and the first Rayleigh step
    DMRG_TRY(launch_project(plan, slot, A.coef, A.V, A.W, s, A.active, A.dfold, &ray));
    int i = 1;
    int done = 0;
    while (done < max_iter) {
        int cnt = std::min(chunk, max_iter - done);
        int inext = i;
        if (use_graph) {
            auto key = std::make_tuple(slot, i, cnt, w->kmax);
            auto it = w->graphs.find(key);
            if (it == w->graphs.end()) {
                hipStream_t cs;
                DMRG_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
                hipGraph_t g;
                DMRG_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
                dmrg_status st = enqueue_iters(plan, slot, i, cnt, &inext, cs);
                hipError_t ce = hipStreamEndCapture(cs, &g);
                (void)hipStreamDestroy(cs);
                if (st < 0) return st;
                if (ce != hipSuccess) return set_error(DMRG_E_HIP, "graph capture failed: %s", hipGetErrorString(ce));
                hipGraphExec_t ge;
                hipError_t ie = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
                (void)hipGraphDestroy(g);
                if (ie != hipSuccess)
                    return set_error(DMRG_E_HIP, "graph instantiate failed: %s", hipGetErrorString(ie));
                it = w->graphs.emplace(key, ge).first;
            } else {
                // the subspace sequence is deterministic: recompute the next i
                int ii = i;
                for (int q = 0; q < cnt; ++q) ii = (ii == w->kmax ? w->kmin : ii) + 1;
                inext = ii;
            }
            DMRG_HIP(hipGraphLaunch(it->second, s));
        } else {
            DMRG_TRY(enqueue_iters(plan, slot, i, cnt, &inext, s));
        }
        i = inext;
        done += cnt;
        DMRG_HIP(hipMemcpyAsync(w->h_nactive, A.nactive, 4, hipMemcpyDeviceToHost, s));
        DMRG_HIP(hipStreamSynchronize(s));
        if (*w->h_nactive <= 0) break;
    }
    *iters_out = done;
    return DMRG_OK;
}

}  // namespace dmrg

// ================================================================== ABI

using namespace dmrg;

template <int KB>
__global__ __launch_bounds__(TPB) void k_gemv_t_part(int64_t n, int k, const double *__restrict__ V, int64_t ldv,
                                                     const double *__restrict__ x, double *__restrict__ part) {
    __shared__ double lds[4 * KB];
    double acc[KB];
#pragma unroll
    for (int j = 0; j < KB; ++j) acc[j] = 0.0;
    for (int64_t e = (int64_t)blockIdx.x * TPB + threadIdx.x; e < n; e += (int64_t)gridDim.x * TPB) {
        const double xv = x[e];
#pragma unroll
        for (int j = 0; j < KB; ++j)
            if (j < k) acc[j] += V[(int64_t)j * ldv + e] * xv;
    }
    block_reduce<KB>(acc, k, lds);
    if (threadIdx.x == 0)
        for (int j = 0; j < k; ++j) part[(size_t)blockIdx.x * KB + j] = acc[j];
}

// second stage: all k columns at once, thread t owns column t % k and every
// (TPB / k)-th block from t / k; slots are then added in order (deterministic)
template <int KB>
__global__ __launch_bounds__(TPB) void k_gemv_t_final(int nblk, int k, const double *__restrict__ part,
                                                      double *__restrict__ s) {
    __shared__ double scratch[TPB];
    const int t = threadIdx.x, per = TPB / k, j = t % k, slot = t / k;
    double v = 0.0;
    if (slot < per) {
#pragma unroll 4
        for (int b = slot; b < nblk; b += per) v += part[(size_t)b * KB + j];
    }
    scratch[t] = v;
    __syncthreads();
    if (t < k) {
        double acc = 0.0;
        for (int q = 0; q < per; ++q) acc += scratch[t + q * k];
        s[t] = acc;
    }
}

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

// per-device partials of dmrg_gemv_t (kept until the process ends)
struct GemvScratch {
    double *p = nullptr;
    size_t bytes = 0;
};
static std::map<int, GemvScratch> g_gemv_scratch;

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
    const DavArgs &A = w->a;
    if (plan->nterm_total)
        DMRG_HIP(hipMemcpyAsync(A.coef, coef, plan->nterm_total * 8, hipMemcpyDeviceToDevice, s));
    DMRG_TRY(launch_diagonal(plan, A.coef, A.D, s));

    std::vector<DavState> hs(plan->nprob);
    std::vector<int> low_iters(plan->nprob, 0);
    int done = 0;
    const bool two_phase = o.prec != DMRG_F64;
    if (two_phase) {
        double tl = o.tol_lowprec > 0 ? o.tol_lowprec : (o.prec == DMRG_F32 ? 1e-5 : 1e-3);
        tl = std::max(tl, o.tol);
        DMRG_TRY(run_phase(plan, 1, psi, tl, o.precond_floor, o.max_iter, o.use_graph != 0, o.graph_chunk, s,
                           &done));
        set_kb(kmax, [&](auto kb) {  // nvec <= kmax
            constexpr int KB = decltype(kb)::value;
            hipLaunchKernelGGL(k_finalize<KB>, dim3(A.nchunk), dim3(TPB), 0, s, A, psi);
        });
        DMRG_HIP(hipGetLastError());
        DMRG_HIP(hipMemcpyAsync(hs.data(), A.st, plan->nprob * sizeof(DavState), hipMemcpyDeviceToHost, s));
        DMRG_HIP(hipStreamSynchronize(s));
        for (int p = 0; p < plan->nprob; ++p) {
            if (hs[p].bad_start == 1) return set_error(DMRG_E_NONFINITE, "member %d: zero or non-finite start", p);
            low_iters[p] = hs[p].iters;
        }
    }
    std::vector<DavState> low = hs;
    if (!two_phase || o.refine) {
        DMRG_TRY(run_phase(plan, 0, psi, o.tol, o.precond_floor, o.max_iter, o.use_graph != 0, o.graph_chunk, s,
                           &done));
        set_kb(kmax, [&](auto kb) {  // nvec <= kmax
            constexpr int KB = decltype(kb)::value;
            hipLaunchKernelGGL(k_finalize<KB>, dim3(A.nchunk), dim3(TPB), 0, s, A, psi);
        });
        DMRG_HIP(hipGetLastError());
        DMRG_HIP(hipMemcpyAsync(hs.data(), A.st, plan->nprob * sizeof(DavState), hipMemcpyDeviceToHost, s));
        DMRG_HIP(hipStreamSynchronize(s));
    }
    dmrg_status ret = DMRG_OK;
    for (int p = 0; p < plan->nprob; ++p) {
        const DavState &S = hs[p];
        if (S.bad_start == 1) return set_error(DMRG_E_NONFINITE, "member %d: zero or non-finite start vector", p);
        if (S.bad_start == 2) ret = set_error(DMRG_E_NONFINITE, "member %d: non-finite iterate", p);
        if (energy) energy[p] = S.lambda;
        if (info) {
            dmrg_davidson_info &I = info[p];
            I.energy = S.lambda;
            I.residual = S.rnorm;
            I.iterations = S.iters + (two_phase && o.refine ? low_iters[p] : 0);
            I.iterations_low = two_phase ? low_iters[p] : 0;
            I.projections = S.nproj + (two_phase && o.refine ? low[p].nproj : 0);
            I.restarts = S.restarts + (two_phase && o.refine ? low[p].restarts : 0);
            I.converged = S.converged;
            I.breakdown = S.breakdown;
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
    int nblk = (int)std::min<int64_t>((n + TPB - 1) / TPB, 1024);
    size_t need = (size_t)nblk * 64 * 8;
    int dev = 0;
    DMRG_HIP(hipGetDevice(&dev));
    GemvScratch &gs = g_gemv_scratch[dev];
    if (need > gs.bytes) {
        // the stream may still use the old buffer: let it finish before freeing
        DMRG_HIP(hipStreamSynchronize((hipStream_t)stream));
        if (gs.p) (void)hipFree(gs.p);
        gs.p = nullptr;
        gs.bytes = 0;
        DMRG_HIP(hipMalloc((void **)&gs.p, need));
        gs.bytes = need;
    }
    double *part = gs.p;
    hipStream_t st = (hipStream_t)stream;
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
