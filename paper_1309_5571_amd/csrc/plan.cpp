// Host side of the library: validation, sector pairs, operation records, tile
// task lists, low-precision operator copies, and the plan/ABI bookkeeping.
//
// The operation records follow the paper's host algorithm for the projection
// (Sec. "Accelerating projection operation", Alg. 5 step 1): A and B do not
// change during the Davidson iterations, so the list of (A X) B^T jobs with
// their input and output segments of psi is built once per plan.  Instead of
// the paper's CPU/GPU partition and stream scheduling (Alg. 5 steps 2-4,
// Alg. 6-7), every record of every output segment becomes part of one task
// list that a single kernel launch consumes (one owner per output tile, so
// no atomics and a deterministic summation order).
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <numeric>
#include <set>
#include <tuple>

#include "enlarge.h"
#include "internal.h"

namespace dmrg {

// ------------------------------------------------------------------ errors

static thread_local std::string g_last_error;

dmrg_status set_error(dmrg_status st, const char *fmt, ...) {
    char buf[1024];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return st;
}

void clear_error() { g_last_error.clear(); }

// ------------------------------------------------------------------ tile table

static int g_ncls = 0;
static int32_t g_bound[8];
static int32_t g_tile[8];

int tile_for(int64_t rows, int64_t cols) {
    int64_t d = std::max(rows, cols);
    if (g_ncls > 0) {
        for (int c = 0; c < g_ncls; ++c)
            if (d <= g_bound[c]) return g_tile[c];
        return g_tile[g_ncls - 1];
    }
    return d <= 16 ? 16 : 32;
}

// ------------------------------------------------------------------ validation

static int cmp_label(const int32_t *a, const int32_t *b, int rank) {
    for (int c = 0; c < rank; ++c) {
        if (a[c] < b[c]) return -1;
        if (a[c] > b[c]) return 1;
    }
    return 0;
}

// index of the sector with the given label, -1 if absent (labels ascending)
static int find_sector(const dmrg_space &s, const int32_t *lab) {
    int lo = 0, hi = s.nsec - 1;
    while (lo <= hi) {
        int mid = (lo + hi) / 2;
        int c = cmp_label(s.label + (size_t)mid * s.rank, lab, s.rank);
        if (c == 0) return mid;
        if (c < 0)
            lo = mid + 1;
        else
            hi = mid - 1;
    }
    return -1;
}

static dmrg_status check_space(const dmrg_space &s, const char *side) {
    if (s.nsec < 1 || s.rank < 1 || s.rank > 2 || !s.label || !s.dim)
        return set_error(DMRG_E_INVALID_ARG, "%s space: need nsec >= 1, rank 1 or 2, label and dim arrays",
                         side);
    for (int i = 0; i < s.nsec; ++i) {
        if (s.dim[i] < 0) return set_error(DMRG_E_INVALID_ARG, "%s space: negative dim at sector %d", side, i);
        if (s.dim[i] > (int64_t)1 << 30)
            return set_error(DMRG_E_UNSUPPORTED, "%s space: sector %d dimension too large", side, i);
        if (i > 0 && cmp_label(s.label + (size_t)(i - 1) * s.rank, s.label + (size_t)i * s.rank, s.rank) >= 0)
            return set_error(DMRG_E_LAYOUT, "%s space: labels not strictly ascending at sector %d", side, i);
    }
    return DMRG_OK;
}

static dmrg_status check_op(const dmrg_space &s, const dmrg_op &op, const char *side, int idx) {
    if (op.kind == DMRG_OP_IDENTITY) return DMRG_OK;
    if (op.kind == DMRG_OP_DIAG) {
        if (!op.data) return set_error(DMRG_E_INVALID_ARG, "%s op %d: diagonal operator without data", side, idx);
        return DMRG_OK;
    }
    if (op.kind != DMRG_OP_DENSE) return set_error(DMRG_E_INVALID_ARG, "%s op %d: unknown kind %d", side, idx, op.kind);
    if (op.nblk < 0) return set_error(DMRG_E_INVALID_ARG, "%s op %d: negative nblk", side, idx);
    if (op.nblk > 0 && (!op.src || !op.dst || !op.off || !op.data))
        return set_error(DMRG_E_INVALID_ARG, "%s op %d: missing block arrays", side, idx);
    std::vector<std::pair<int, int>> seen;
    seen.reserve(op.nblk);
    for (int b = 0; b < op.nblk; ++b) {
        if (op.src[b] < 0 || op.src[b] >= s.nsec || op.dst[b] < 0 || op.dst[b] >= s.nsec)
            return set_error(DMRG_E_INVALID_ARG, "%s op %d block %d: sector index out of range", side, idx, b);
        if (op.off[b] < 0) return set_error(DMRG_E_INVALID_ARG, "%s op %d block %d: negative offset", side, idx, b);
        seen.emplace_back(op.src[b], op.dst[b]);
    }
    std::sort(seen.begin(), seen.end());
    for (size_t i = 1; i < seen.size(); ++i)
        if (seen[i] == seen[i - 1])
            return set_error(DMRG_E_LAYOUT, "%s op %d: duplicate block %d -> %d", side, idx, seen[i].first,
                             seen[i].second);
    return DMRG_OK;
}

// resolved blocks of an operator grouped by source sector
using BySrc = std::vector<std::vector<OpBlock>>;

static BySrc resolve(const dmrg_space &s, const dmrg_op &op, int gop) {
    BySrc out(s.nsec);
    std::vector<int64_t> off(s.nsec + 1, 0);
    for (int i = 0; i < s.nsec; ++i) off[i + 1] = off[i] + s.dim[i];
    if (op.kind == DMRG_OP_IDENTITY || op.kind == DMRG_OP_DIAG) {
        for (int i = 0; i < s.nsec; ++i) {
            OpBlock b{i, i, op.kind, s.dim[i], s.dim[i],
                      op.kind == DMRG_OP_DIAG ? op.data + off[i] : nullptr, gop, -1};
            out[i].push_back(b);
        }
        return out;
    }
    for (int k = 0; k < op.nblk; ++k) {
        OpBlock b{op.src[k], op.dst[k], DMRG_OP_DENSE, s.dim[op.dst[k]], s.dim[op.src[k]],
                  op.data + op.off[k], gop, k};
        out[op.src[k]].push_back(b);
    }
    return out;
}

struct MemberPairs {
    std::vector<Pair> pairs;
    std::vector<int> by_left;  // left sector -> local pair index or -1
};

static MemberPairs make_pairs(const dmrg_problem &p) {
    MemberPairs mp;
    mp.by_left.assign(p.left.nsec, -1);
    int rank = p.left.rank;
    int64_t off = 0;
    std::vector<int32_t> want(rank);
    for (int sl = 0; sl < p.left.nsec; ++sl) {
        for (int c = 0; c < rank; ++c) want[c] = p.target[c] - p.left.label[(size_t)sl * rank + c];
        int sr = find_sector(p.right, want.data());
        if (sr < 0) continue;
        int64_t dl = p.left.dim[sl], dr = p.right.dim[sr];
        if (dl == 0 || dr == 0) continue;
        mp.by_left[sl] = (int)mp.pairs.size();
        mp.pairs.push_back(Pair{sl, sr, dl, dr, off});
        off += dl * dr;
    }
    return mp;
}

// Full host-side check of one problem; optionally returns pairs and records.
static dmrg_status analyse(const dmrg_problem *p, MemberPairs *mp_out, std::vector<Record> *recs_out,
                           int gop_base, int gterm_base) {
    if (!p) return set_error(DMRG_E_INVALID_ARG, "null problem");
    DMRG_TRY(check_space(p->left, "left"));
    DMRG_TRY(check_space(p->right, "right"));
    if (p->left.rank != p->right.rank)
        return set_error(DMRG_E_INVALID_ARG, "left and right label ranks differ");
    if (!p->target) return set_error(DMRG_E_INVALID_ARG, "null target label");
    if (p->nop_left < 0 || p->nop_right < 0 || p->nterm < 0)
        return set_error(DMRG_E_INVALID_ARG, "negative operator or term count");
    if ((p->nop_left && !p->ops_left) || (p->nop_right && !p->ops_right) || (p->nterm && !p->terms))
        return set_error(DMRG_E_INVALID_ARG, "missing operator or term array");
    for (int i = 0; i < p->nop_left; ++i) DMRG_TRY(check_op(p->left, p->ops_left[i], "left", i));
    for (int i = 0; i < p->nop_right; ++i) DMRG_TRY(check_op(p->right, p->ops_right[i], "right", i));
    for (int k = 0; k < p->nterm; ++k) {
        if (p->terms[k].a < 0 || p->terms[k].a >= p->nop_left || p->terms[k].b < 0 ||
            p->terms[k].b >= p->nop_right)
            return set_error(DMRG_E_INVALID_ARG, "term %d: operator index out of range", k);
    }
    MemberPairs mp = make_pairs(*p);
    std::vector<BySrc> L(p->nop_left), R(p->nop_right);
    for (int i = 0; i < p->nop_left; ++i) L[i] = resolve(p->left, p->ops_left[i], gop_base + i);
    for (int i = 0; i < p->nop_right; ++i)
        R[i] = resolve(p->right, p->ops_right[i], gop_base + p->nop_left + i);
    int rank = p->left.rank;
    std::vector<Record> recs;
    for (int k = 0; k < p->nterm; ++k) {
        const BySrc &A = L[p->terms[k].a];
        const BySrc &B = R[p->terms[k].b];
        for (int pi = 0; pi < (int)mp.pairs.size(); ++pi) {
            const Pair &in = mp.pairs[pi];
            for (const OpBlock &a : A[in.sl]) {
                for (const OpBlock &b : B[in.sr]) {
                    bool ok = true;
                    for (int c = 0; c < rank; ++c)
                        ok &= p->left.label[(size_t)a.dst * rank + c] + p->right.label[(size_t)b.dst * rank + c] ==
                              p->target[c];
                    if (!ok)
                        return set_error(DMRG_E_SECTOR,
                                         "term %d: block %d->%d (x) %d->%d leaves the target sector", k, a.src,
                                         a.dst, b.src, b.dst);
                    int po = mp.by_left[a.dst];
                    if (po < 0 || mp.pairs[po].sr != b.dst) continue;  // empty output segment
                    Record r{};
                    r.term = k;
                    r.gterm = gterm_base + k;
                    r.pin = pi;
                    r.pout = po;
                    r.a = a;
                    r.b = b;
                    r.gin = Geo{in.off, in.dl, in.dr, in.dr};
                    r.gout = Geo{mp.pairs[po].off, mp.pairs[po].dl, mp.pairs[po].dr, mp.pairs[po].dr};
                    r.oin = pi;
                    r.oout = po;
                    r.w = 1.0;
                    bool da = a.kind == DMRG_OP_DENSE, db = b.kind == DMRG_OP_DENSE;
                    if (da && db) {
                        int64_t di = in.dl, dk = in.dr, dj = mp.pairs[po].dl, dl = mp.pairs[po].dr;
                        int64_t cl = dj * di * dk + dj * dk * dl, cr = di * dk * dl + dj * di * dl;
                        r.order = cr < cl ? 1 : 0;
                    } else {
                        r.order = 2;
                    }
                    recs.push_back(r);
                }
            }
        }
    }
    if (mp_out) *mp_out = std::move(mp);
    if (recs_out) *recs_out = std::move(recs);
    return DMRG_OK;
}

// ------------------------------------------------------------------ pass building

struct HostPass {
    std::vector<Task> A, B;
    std::vector<Seg> segs;
    std::vector<DiagTerm> diags;
    int64_t tmp = 0;
};

static uint64_t U(const void *p) { return (uint64_t)(uintptr_t)p; }

// Largest intermediate width a fused two-sided segment keeps in LDS (16 rows x 64).
constexpr int64_t FUSE_MAX_K2 = 64;

static void add_tiles(std::vector<Task> &out, int64_t rows, int64_t cols, int64_t c_off, int64_t x_off, int64_t ld,
                      int32_t seg_b, int32_t seg_e, int32_t d_b, int32_t d_e, int member) {
    int ts = tile_for(rows, cols);
    for (int64_t r0 = 0; r0 < rows; r0 += ts)
        for (int64_t c0 = 0; c0 < cols; c0 += ts) {
            Task t{};
            t.seg_begin = seg_b;
            t.seg_end = seg_e;
            t.diag_begin = d_b;
            t.diag_end = d_e;
            t.c_off = c_off;
            t.x_off = x_off;
            t.ldc = (int32_t)ld;
            t.row0 = (int32_t)r0;
            t.col0 = (int32_t)c0;
            t.m = (int32_t)std::min<int64_t>(ts, rows - r0);
            t.n = (int32_t)std::min<int64_t>(ts, cols - c0);
            t.member = member;
            out.push_back(t);
        }
}

static double task_cost(const Task &t, const std::vector<Seg> &segs) {
    double sub = std::ceil(t.m / 16.0) * std::ceil(t.n / 16.0);
    double c = 8.0 * (t.diag_end - t.diag_begin) + 1.0;
    for (int s = t.seg_begin; s < t.seg_end; ++s) {
        const Seg &g = segs[s];
        if (g.fused)
            c += (g.K + 16) * std::ceil(g.K2 / 16.0) + sub * (g.K2 + 16);
        else
            c += sub * (g.K + 16);
    }
    return c;
}

static void sort_tasks(std::vector<Task> &v, const std::vector<Seg> &segs) {
    std::vector<std::pair<double, int>> key(v.size());
    for (size_t i = 0; i < v.size(); ++i) key[i] = {-task_cost(v[i], segs), (int)i};
    std::stable_sort(key.begin(), key.end());
    std::vector<Task> o(v.size());
    for (size_t i = 0; i < v.size(); ++i) o[i] = v[key[i].second];
    v.swap(o);
}

// Low-precision copies of operator blocks: (op, blk, variant) -> device address.
struct LowStore {
    struct Job {
        const double *src;
        int64_t rows, cols;
        int offdiag;  // 1: diagonal zeroed
        size_t off;   // byte offset in the arena
        int diag;     // 1: this job extracts the FP64 diagonal instead
    };
    std::map<std::tuple<int, int, int>, size_t> where;
    std::vector<Job> jobs;
    size_t bytes = 0;
    int esize = 4;
    size_t add(const OpBlock &b, int variant) {  // variant 0 full, 1 off-diagonal, 2 FP64 diagonal
        auto key = std::make_tuple(b.op, b.blk, variant);
        auto it = where.find(key);
        if (it != where.end()) return it->second;
        size_t sz = variant == 2 ? (size_t)b.rows * 8 : (size_t)(b.rows * b.cols) * esize;
        size_t off = bytes;
        bytes += (sz + 255) & ~(size_t)255;
        where[key] = off;
        jobs.push_back(Job{b.data, b.rows, b.cols, variant == 1, off, variant == 2});
        return off;
    }
};

// Builds the forward (adjoint = false) or adjoint pass of one precision slot.
// With `low` set, dense operator blocks are taken from low-precision copies and
// the diagonals of square blocks in one-sided records are split off in FP64.
static void build_pass(const dmrg_plan *plan, bool adjoint, LowStore *low, uint64_t low_base, HostPass &hp) {
    const int nout = (int)plan->out_geo.size();
    std::vector<std::vector<int>> by_out(nout);
    for (int r = 0; r < (int)plan->records.size(); ++r) {
        const Record &rc = plan->records[r];
        by_out[adjoint ? rc.oin : rc.oout].push_back(r);
    }
    auto blk_addr = [&](const OpBlock &b, int variant) -> uint64_t {
        if (!low) return U(b.data);
        return low_base + low->add(b, variant);
    };
    auto diag_addr = [&](const OpBlock &b) -> uint64_t {  // identity -> 0, diag -> slice
        return b.kind == DMRG_OP_DIAG ? U(b.data) : 0;
    };
    struct TMat {
        int64_t rows, cols, off;
        int seg;
        int member;
    };
    std::vector<TMat> tmats;
    std::vector<Seg> segsA;  // stage-A (intermediate) segments, appended after the output lists
    for (int q = 0; q < nout; ++q) {
        const Geo &go = plan->out_geo[q];
        int member = plan->out_member[q];
        int seg_b = (int)hp.segs.size(), d_b = (int)hp.diags.size();
        for (int ri : by_out[q]) {
            const Record &rc = plan->records[ri];
            const Geo &gi = adjoint ? rc.gout : rc.gin;  // where the input sub-matrix lives
            bool da = rc.a.kind == DMRG_OP_DENSE, db = rc.b.kind == DMRG_OP_DENSE;
            int gt = rc.gterm;
            if (!da && !db) {
                if (gi.off == go.off && gi.ld == go.ld) {  // same place: an epilogue term
                    DiagTerm dt{diag_addr(rc.a), diag_addr(rc.b), gt, gt, 1, 1};
                    dt.w = rc.w;
                    hp.diags.push_back(dt);
                } else {  // the input lies elsewhere: a copy segment
                    Seg c{};
                    c.fused = 2;
                    c.q = (uint64_t)gi.off;
                    c.qkind = OPD_IN;
                    c.ldq = (int32_t)gi.ld;
                    c.pscale = diag_addr(rc.a);
                    c.qscale = diag_addr(rc.b);
                    c.coef = gt;
                    c.term = gt;
                    c.w = rc.w;
                    hp.segs.push_back(c);
                }
                continue;
            }
            Seg s{};
            s.coef = gt;
            s.term = gt;
            s.w = rc.w;
            if (!adjoint) {
                // X = input [di x dk] (rows gi.ld apart); output [dj x dl]; A [dj x di], B [dl x dk]
                int64_t di = gi.rows, dk = gi.cols;
                if (da && !db) {
                    bool split = low && rc.a.src == rc.a.dst;
                    s.p = blk_addr(rc.a, split ? 1 : 0);
                    s.pkind = OPD_ABS;
                    s.ldp = (int32_t)di;
                    s.q = (uint64_t)gi.off;
                    s.qkind = OPD_IN;
                    s.ldq = (int32_t)gi.ld;
                    s.qscale = diag_addr(rc.b);
                    s.K = (int32_t)di;
                    hp.segs.push_back(s);
                    if (split) {
                        DiagTerm dt{blk_addr(rc.a, 2), diag_addr(rc.b), gt, -1, 1, 1};
                        dt.w = rc.w;
                        hp.diags.push_back(dt);
                    }
                } else if (!da && db) {
                    bool split = low && rc.b.src == rc.b.dst;
                    s.p = (uint64_t)gi.off;
                    s.pkind = OPD_IN;
                    s.ldp = (int32_t)gi.ld;
                    s.pscale = diag_addr(rc.a);
                    s.q = blk_addr(rc.b, split ? 1 : 0);
                    s.qkind = OPD_ABS;
                    s.qtrans = 1;
                    s.ldq = (int32_t)dk;
                    s.K = (int32_t)dk;
                    hp.segs.push_back(s);
                    if (split) {
                        DiagTerm dt{diag_addr(rc.a), blk_addr(rc.b, 2), gt, -1, 1, 1};
                        dt.w = rc.w;
                        hp.diags.push_back(dt);
                    }
                } else if (tile_for(go.rows, go.cols) == 16 && dk <= FUSE_MAX_K2) {
                    // small intermediate: fused in the output tile (no stage-A task)
                    s.fused = 1;
                    s.p = blk_addr(rc.a, 0);
                    s.pkind = OPD_ABS;
                    s.ldp = (int32_t)di;
                    s.q = (uint64_t)gi.off;
                    s.qkind = OPD_IN;
                    s.ldq = (int32_t)gi.ld;
                    s.K = (int32_t)di;
                    s.r = blk_addr(rc.b, 0);
                    s.ldr = (int32_t)dk;
                    s.K2 = (int32_t)dk;
                    hp.segs.push_back(s);
                } else {
                    int64_t dj = go.rows, dl = go.cols;
                    Seg a{};
                    a.coef = -1;
                    a.term = -1;
                    TMat tm{};
                    if (rc.order == 0) {  // T = A X  [dj x dk];  Y += c T B^T
                        a.p = blk_addr(rc.a, 0);
                        a.pkind = OPD_ABS;
                        a.ldp = (int32_t)di;
                        a.q = (uint64_t)gi.off;
                        a.qkind = OPD_IN;
                        a.ldq = (int32_t)gi.ld;
                        a.K = (int32_t)di;
                        tm = TMat{dj, dk, hp.tmp, 0, member};
                        s.p = (uint64_t)hp.tmp;
                        s.pkind = OPD_TMP;
                        s.ldp = (int32_t)dk;
                        s.q = blk_addr(rc.b, 0);
                        s.qkind = OPD_ABS;
                        s.qtrans = 1;
                        s.ldq = (int32_t)dk;
                        s.K = (int32_t)dk;
                    } else {  // T = X B^T  [di x dl];  Y += c A T
                        a.p = (uint64_t)gi.off;
                        a.pkind = OPD_IN;
                        a.ldp = (int32_t)gi.ld;
                        a.q = blk_addr(rc.b, 0);
                        a.qkind = OPD_ABS;
                        a.qtrans = 1;
                        a.ldq = (int32_t)dk;
                        a.K = (int32_t)dk;
                        tm = TMat{di, dl, hp.tmp, 0, member};
                        s.p = blk_addr(rc.a, 0);
                        s.pkind = OPD_ABS;
                        s.ldp = (int32_t)di;
                        s.q = (uint64_t)hp.tmp;
                        s.qkind = OPD_TMP;
                        s.ldq = (int32_t)dl;
                        s.K = (int32_t)di;
                    }
                    hp.tmp += (tm.rows * tm.cols + 31) & ~(int64_t)31;
                    tm.seg = (int)segsA.size();
                    tmats.push_back(tm);
                    segsA.push_back(a);
                    hp.segs.push_back(s);
                }
            } else {
                // adjoint: output = gpsi [di x dk] at the record's input sub-matrix,
                // input G = gbar [dj x dl] at its output sub-matrix (rows gi.ld apart)
                int64_t di = go.rows, dk = go.cols, dj = gi.rows, dl = gi.cols;
                if (da && !db) {  // gpsi += c A^T (G * v)
                    s.p = U(rc.a.data);
                    s.pkind = OPD_ABS;
                    s.ptrans = 1;
                    s.ldp = (int32_t)di;
                    s.q = (uint64_t)gi.off;
                    s.qkind = OPD_IN;
                    s.ldq = (int32_t)gi.ld;
                    s.qscale = diag_addr(rc.b);
                    s.K = (int32_t)dj;
                    hp.segs.push_back(s);
                } else if (!da && db) {  // gpsi += c (v * G) B
                    s.p = (uint64_t)gi.off;
                    s.pkind = OPD_IN;
                    s.ldp = (int32_t)gi.ld;
                    s.pscale = diag_addr(rc.a);
                    s.q = U(rc.b.data);
                    s.qkind = OPD_ABS;
                    s.qtrans = 0;
                    s.ldq = (int32_t)dk;
                    s.K = (int32_t)dl;
                    hp.segs.push_back(s);
                } else {
                    Seg a{};
                    a.coef = -1;
                    a.term = -1;
                    TMat tm{};
                    int64_t cA = di * dj * dl + di * dl * dk, cB = dj * dl * dk + di * dj * dk;
                    if (cA <= cB) {  // T = A^T G [di x dl];  gpsi += c T B
                        a.p = U(rc.a.data);
                        a.pkind = OPD_ABS;
                        a.ptrans = 1;
                        a.ldp = (int32_t)di;
                        a.q = (uint64_t)gi.off;
                        a.qkind = OPD_IN;
                        a.ldq = (int32_t)gi.ld;
                        a.K = (int32_t)dj;
                        tm = TMat{di, dl, hp.tmp, 0, member};
                        s.p = (uint64_t)hp.tmp;
                        s.pkind = OPD_TMP;
                        s.ldp = (int32_t)dl;
                        s.q = U(rc.b.data);
                        s.qkind = OPD_ABS;
                        s.ldq = (int32_t)dk;
                        s.K = (int32_t)dl;
                    } else {  // T = G B [dj x dk];  gpsi += c A^T T
                        a.p = (uint64_t)gi.off;
                        a.pkind = OPD_IN;
                        a.ldp = (int32_t)gi.ld;
                        a.q = U(rc.b.data);
                        a.qkind = OPD_ABS;
                        a.ldq = (int32_t)dk;
                        a.K = (int32_t)dl;
                        tm = TMat{dj, dk, hp.tmp, 0, member};
                        s.p = U(rc.a.data);
                        s.pkind = OPD_ABS;
                        s.ptrans = 1;
                        s.ldp = (int32_t)di;
                        s.q = (uint64_t)hp.tmp;
                        s.qkind = OPD_TMP;
                        s.ldq = (int32_t)dk;
                        s.K = (int32_t)dj;
                    }
                    hp.tmp += (tm.rows * tm.cols + 31) & ~(int64_t)31;
                    tm.seg = (int)segsA.size();
                    tmats.push_back(tm);
                    segsA.push_back(a);
                    hp.segs.push_back(s);
                }
            }
        }
        int seg_e = (int)hp.segs.size();
        add_tiles(hp.B, go.rows, go.cols, go.off, go.off, go.ld, seg_b, seg_e, d_b, (int)hp.diags.size(), member);
    }
    int baseA = (int)hp.segs.size();
    hp.segs.insert(hp.segs.end(), segsA.begin(), segsA.end());
    for (const TMat &tm : tmats)
        add_tiles(hp.A, tm.rows, tm.cols, tm.off, 0, tm.cols, baseA + tm.seg, baseA + tm.seg + 1, 0, 0, tm.member);
    sort_tasks(hp.A, hp.segs);
    sort_tasks(hp.B, hp.segs);
}

template <class T>
static dmrg_status upload(dmrg_plan *plan, const std::vector<T> &v, T **dst, hipStream_t s) {
    *dst = nullptr;
    if (v.empty()) return DMRG_OK;
    void *p = nullptr;
    DMRG_HIP(hipMalloc(&p, v.size() * sizeof(T)));
    plan->owned.push_back(p);
    DMRG_HIP(hipMemcpyAsync(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, s));
    *dst = (T *)p;
    return DMRG_OK;
}

static dmrg_status upload_pass(dmrg_plan *plan, HostPass &hp, PassSet &ps, hipStream_t s) {
    // member-contiguous rows for the per-tile Rayleigh partials of stage B
    std::vector<int32_t> begin(plan->nprob + 1, 0), next;
    for (const Task &t : hp.B) begin[t.member + 1] += 1;
    for (int m = 0; m < plan->nprob; ++m) begin[m + 1] += begin[m];
    next.assign(begin.begin(), begin.end() - 1);
    for (Task &t : hp.B) t.rslot = next[t.member]++;
    DMRG_TRY(upload(plan, begin, &ps.slot_begin, s));
    DMRG_TRY(upload(plan, hp.segs, &ps.segs, s));
    DMRG_TRY(upload(plan, hp.diags, &ps.diags, s));
    DMRG_TRY(upload(plan, hp.A, &ps.stageA.tasks, s));
    DMRG_TRY(upload(plan, hp.B, &ps.stageB.tasks, s));
    ps.stageA.ntask = (int32_t)hp.A.size();
    ps.stageB.ntask = (int32_t)hp.B.size();
    for (const Task &t : hp.A)
        if (t.m > 16 || t.n > 16) ps.stageA.ns = 2;
    for (const Task &t : hp.B)
        if (t.m > 16 || t.n > 16) ps.stageB.ns = 2;
    ps.nseg = (int32_t)hp.segs.size();
    ps.ndiag = (int32_t)hp.diags.size();
    ps.tmp_elems = hp.tmp;
    return DMRG_OK;
}

static dmrg_status finish_plan(dmrg_plan *plan, int32_t prec, hipStream_t stream, const dmrg_problem *probs);

// Preconditioner diagonal of a plan without LR problems: every record whose
// input and output sub-matrices coincide has only square blocks, and adds
// c w diag(A)[r] diag(B)[c] there.
static dmrg_status diag_from_records(dmrg_plan *plan, hipStream_t stream) {
    const int nout = (int)plan->out_geo.size();
    std::vector<std::vector<DiagTerm>> per(nout);
    auto slice = [](const OpBlock &b, uint64_t *addr, int32_t *stride) {
        if (b.kind == DMRG_OP_IDENTITY) {
            *addr = 0;
            *stride = 0;
        } else if (b.kind == DMRG_OP_DIAG) {
            *addr = U(b.data);
            *stride = 1;
        } else {
            *addr = U(b.data);
            *stride = (int32_t)(b.rows + 1);
        }
    };
    for (const Record &rc : plan->records) {
        if (rc.oin != rc.oout) continue;
        DiagTerm dt{};
        dt.coef = rc.gterm;
        dt.term = rc.gterm;
        dt.w = rc.w;
        slice(rc.a, &dt.vl, &dt.sl);
        slice(rc.b, &dt.vr, &dt.sr);
        per[rc.oout].push_back(dt);
    }
    std::vector<Task> tasks;
    std::vector<DiagTerm> terms;
    for (int q = 0; q < nout; ++q) {
        const Geo &g = plan->out_geo[q];
        const int d_b = (int)terms.size();
        terms.insert(terms.end(), per[q].begin(), per[q].end());
        if (g.rows <= 0 || g.cols <= 0) continue;
        const int64_t tn = std::min<int64_t>(g.cols, 1024), tm = std::max<int64_t>(1, 1024 / tn);
        for (int64_t r0 = 0; r0 < g.rows; r0 += tm)
            for (int64_t c0 = 0; c0 < g.cols; c0 += tn) {
                Task t{};
                t.diag_begin = d_b;
                t.diag_end = (int)terms.size();
                t.c_off = g.off;
                t.x_off = g.off;
                t.ldc = (int32_t)g.ld;
                t.row0 = (int32_t)r0;
                t.col0 = (int32_t)c0;
                t.m = (int32_t)std::min<int64_t>(tm, g.rows - r0);
                t.n = (int32_t)std::min<int64_t>(tn, g.cols - c0);
                t.member = plan->out_member[q];
                tasks.push_back(t);
            }
    }
    DMRG_TRY(upload(plan, terms, &plan->d_diag_terms, stream));
    DMRG_TRY(upload(plan, tasks, &plan->d_diag_tasks, stream));
    plan->n_diag_tasks = (int32_t)tasks.size();
    return DMRG_OK;
}

// Host analysis of LR problems: pairs, psi layout, records, FLOP and byte counts.
static dmrg_status analyse_plan(dmrg_plan *plan, int32_t nprob, const dmrg_problem *probs, int32_t prec) {
    plan->nprob = nprob;
    plan->prec = prec;
    plan->member_off.assign(1, 0);
    plan->term_off.assign(1, 0);
    int gop = 0;
    std::set<std::pair<int, int>> used_blocks;  // (global op, block) for the byte count
    std::set<std::pair<int, int>> used_slices;  // (global op, sector)
    int64_t flop = 0, opbytes = 0;
    for (int p = 0; p < nprob; ++p) {
        MemberPairs mp;
        std::vector<Record> recs;
        DMRG_TRY(analyse(&probs[p], &mp, &recs, gop, plan->term_off.back()));
        int pair_base = (int)plan->pairs.size();
        int64_t base = plan->member_off.back();
        for (Pair q : mp.pairs) {
            q.off += base;
            plan->pairs.push_back(q);
            plan->pair_member.push_back(p);
        }
        for (const Pair &q : mp.pairs) {
            plan->out_geo.push_back(Geo{base + q.off, q.dl, q.dr, q.dr});
            plan->out_member.push_back(p);
        }
        for (Record r : recs) {
            r.pin += pair_base;
            r.pout += pair_base;
            r.oin += pair_base;
            r.oout += pair_base;
            r.gin.off += base;
            r.gout.off += base;
            const Pair &in = plan->pairs[r.pin], &out = plan->pairs[r.pout];
            int64_t di = in.dl, dk = in.dr, dj = out.dl, dl = out.dr;
            bool da = r.a.kind == DMRG_OP_DENSE, db = r.b.kind == DMRG_OP_DENSE;
            if (da && db)
                flop += 2 * std::min(dj * di * dk + dj * dk * dl, di * dk * dl + dj * di * dl);
            else if (da)
                flop += 2 * dj * di * dk;
            else if (db)
                flop += 2 * di * dk * dl;
            else
                flop += 2 * dj * dl;
            for (const OpBlock *b : {&r.a, &r.b}) {
                if (b->kind == DMRG_OP_DENSE) {
                    if (used_blocks.insert({b->op, b->blk}).second) opbytes += 8 * b->rows * b->cols;
                } else if (b->kind == DMRG_OP_DIAG) {
                    if (used_slices.insert({b->op, b->src}).second) opbytes += 8 * b->rows;
                }
            }
            plan->records.push_back(r);
        }
        plan->member_off.push_back(base + (mp.pairs.empty() ? 0 : mp.pairs.back().off + mp.pairs.back().dl * mp.pairs.back().dr));
        plan->term_off.push_back(plan->term_off.back() + probs[p].nterm);
        gop += probs[p].nop_left + probs[p].nop_right;
    }
    plan->n = plan->member_off.back();
    plan->nterm_total = plan->term_off.back();
    plan->flop = flop;
    plan->bytes = opbytes + 16 * plan->n;
    return DMRG_OK;
}

dmrg_status build_plan(dmrg_plan *plan, int32_t nprob, const dmrg_problem *probs, int32_t prec,
                       hipStream_t stream) {
    DMRG_TRY(analyse_plan(plan, nprob, probs, prec));
    return finish_plan(plan, prec, stream, probs);
}

// Scratch of an analysed plan: intermediate-buffer elements (largest over the
// passes), coefficient-gradient partial slots (one per segment and diagonal
// term of every forward FP64 stage-B task) and the largest stage-B task count.
static void scratch_sizes(const dmrg_plan *plan, int32_t prec, int64_t *tmp, int32_t *npart, int32_t *tiles) {
    HostPass f64, a64;
    build_pass(plan, false, nullptr, 0, f64);
    build_pass(plan, true, nullptr, 0, a64);
    int64_t t = std::max(f64.tmp, a64.tmp);
    int32_t part = 0;
    for (const Task &k : f64.B) part += (k.seg_end - k.seg_begin) + (k.diag_end - k.diag_begin);
    int32_t tl = std::max<int32_t>(1, (int32_t)f64.B.size());
    if (prec != DMRG_F64) {
        LowStore ls;
        ls.esize = prec == DMRG_F32 ? 4 : 2;
        HostPass lo;
        build_pass(plan, false, &ls, 0, lo);
        t = std::max(t, lo.tmp);
        tl = std::max(tl, (int32_t)lo.B.size());
    }
    *tmp = std::max<int64_t>(t, 1);
    *npart = part;
    *tiles = tl;
}

// Bytes of the caller workspace of LR problems (host only), and the offsets of
// its partial-slot and Davidson regions.
static dmrg_status workspace_need(int32_t nprob, const dmrg_problem *probs, int32_t prec, int32_t kmax,
                                  size_t *bytes, size_t *part_off, size_t *dav_off) {
    dmrg_plan tmp;
    DMRG_TRY(analyse_plan(&tmp, nprob, probs, prec));
    int64_t te;
    int32_t npart, tiles;
    scratch_sizes(&tmp, prec, &te, &npart, &tiles);
    const size_t po = ws_align((size_t)te * 8);
    const size_t dav = po + ws_align((size_t)std::max(npart, 1) * 8);
    if (part_off) *part_off = po;
    if (dav_off) *dav_off = dav;
    *bytes = dav + dav_workspace_bytes(&tmp, kmax, tiles);
    return DMRG_OK;
}

// Everything after the analysis: task lists of both directions, reduced-
// precision copies, intermediate buffer, preconditioner-diagonal tasks (from
// the LR problems when given, else from the records whose input and output
// coincide) and the density tiles.
static dmrg_status finish_plan(dmrg_plan *plan, int32_t prec, hipStream_t stream, const dmrg_problem *probs) {
    // ---- forward and adjoint passes in FP64
    HostPass f64, a64;
    build_pass(plan, false, nullptr, 0, f64);
    build_pass(plan, true, nullptr, 0, a64);
    // coefficient-gradient partial slots (forward FP64 stage B)
    {
        int32_t part = 0;
        std::vector<std::vector<int32_t>> per_term(plan->nterm_total);
        for (Task &t : f64.B) {
            t.part0 = part;
            for (int s = t.seg_begin; s < t.seg_end; ++s) {
                if (f64.segs[s].term >= 0) per_term[f64.segs[s].term].push_back(part);
                ++part;
            }
            for (int d = t.diag_begin; d < t.diag_end; ++d) {
                if (f64.diags[d].term >= 0) per_term[f64.diags[d].term].push_back(part);
                ++part;
            }
        }
        plan->fwd[0].npart = part;
        std::vector<int32_t> ptr(1, 0), ent;
        for (auto &v : per_term) {
            ent.insert(ent.end(), v.begin(), v.end());
            ptr.push_back((int32_t)ent.size());
        }
        DMRG_TRY(upload(plan, ptr, &plan->d_term_ptr, stream));
        DMRG_TRY(upload(plan, ent, &plan->d_term_ent, stream));
        if (part > 0 && plan->ws) {
            if (plan->ws_part + (size_t)part * 8 > plan->ws_dav)
                return set_error(DMRG_E_NOMEM, "workspace layout does not hold the gradient partials");
            plan->d_partials = (double *)(plan->ws + plan->ws_part);
        } else if (part > 0) {
            void *q = nullptr;
            DMRG_HIP(hipMalloc(&q, (size_t)part * sizeof(double)));
            plan->owned.push_back(q);
            plan->d_partials = (double *)q;
        }
    }
    DMRG_TRY(upload_pass(plan, f64, plan->fwd[0], stream));
    DMRG_TRY(upload_pass(plan, a64, plan->adj[0], stream));
    int64_t tmp = std::max(f64.tmp, a64.tmp);

    // ---- low-precision forward pass with converted operator copies
    if (prec != DMRG_F64) {
        LowStore ls;
        ls.esize = prec == DMRG_F32 ? 4 : 2;
        HostPass lo;
        build_pass(plan, false, &ls, 0, lo);  // first pass: collect the copies with base 0
        void *arena = nullptr;
        if (ls.bytes) {
            DMRG_HIP(hipMalloc(&arena, ls.bytes));
            plan->owned.push_back(arena);
        }
        // rebuild with the real base address (same order, so the same offsets)
        HostPass lo2;
        build_pass(plan, false, &ls, U(arena), lo2);
        std::vector<ConvJob> jobs;
        jobs.reserve(ls.jobs.size());
        for (const auto &j : ls.jobs)
            jobs.push_back(ConvJob{j.src, (char *)arena + j.off, j.rows, j.cols, j.diag ? 2 : (j.offdiag ? 1 : 0), 0});
        ConvJob *d_jobs = nullptr;
        DMRG_TRY(upload(plan, jobs, &d_jobs, stream));
        DMRG_TRY(launch_convert_jobs(d_jobs, (int)jobs.size(), prec, stream));
        DMRG_TRY(upload_pass(plan, lo2, plan->fwd[1], stream));
        tmp = std::max(tmp, lo2.tmp);
    }
    plan->tmp_bytes = std::max<int64_t>(tmp, 1) * 8;
    if (plan->ws) {
        if ((size_t)plan->tmp_bytes > plan->ws_part)
            return set_error(DMRG_E_NOMEM, "workspace layout does not hold the intermediate buffer");
        plan->d_tmp = plan->ws;
    } else {
        DMRG_HIP(hipMalloc(&plan->d_tmp, plan->tmp_bytes));
        plan->owned.push_back(plan->d_tmp);
    }

    // ---- preconditioner diagonal: per pair, sum_k c_k diag(A_k)(sl) (x) diag(B_k)(sr)
    if (!probs) {
        DMRG_TRY(diag_from_records(plan, stream));
    } else {
        std::vector<Task> tasks;
        std::vector<DiagTerm> terms;
        for (int q = 0; q < (int)plan->pairs.size(); ++q) {
            const Pair &pr = plan->pairs[q];
            int member = plan->pair_member[q];
            const dmrg_problem &pb = probs[member];
            int d_b = (int)terms.size();
            for (int k = 0; k < pb.nterm; ++k) {
                const dmrg_op &A = pb.ops_left[pb.terms[k].a];
                const dmrg_op &B = pb.ops_right[pb.terms[k].b];
                auto src = [](const dmrg_space &sp, const dmrg_op &op, int s, uint64_t *addr, int32_t *stride) {
                    int64_t off = 0;
                    for (int i = 0; i < s; ++i) off += sp.dim[i];
                    if (op.kind == DMRG_OP_IDENTITY) {
                        *addr = 0;
                        *stride = 0;
                        return true;
                    }
                    if (op.kind == DMRG_OP_DIAG) {
                        *addr = U(op.data + off);
                        *stride = 1;
                        return true;
                    }
                    for (int b = 0; b < op.nblk; ++b)
                        if (op.src[b] == s && op.dst[b] == s) {
                            *addr = U(op.data + op.off[b]);
                            *stride = (int32_t)(sp.dim[s] + 1);
                            return true;
                        }
                    return false;  // no diagonal block: contributes zero
                };
                DiagTerm dt{};
                dt.coef = plan->term_off[member] + k;
                dt.term = dt.coef;
                if (!src(pb.left, A, pr.sl, &dt.vl, &dt.sl)) continue;
                if (!src(pb.right, B, pr.sr, &dt.vr, &dt.sr)) continue;
                terms.push_back(dt);
            }
            // tiles of at most 1024 elements (whole rows when they fit)
            if (pr.dl <= 0 || pr.dr <= 0) continue;
            const int64_t tn = std::min<int64_t>(pr.dr, 1024), tm = std::max<int64_t>(1, 1024 / tn);
            for (int64_t r0 = 0; r0 < pr.dl; r0 += tm)
                for (int64_t c0 = 0; c0 < pr.dr; c0 += tn) {
                    Task t{};
                    t.diag_begin = d_b;
                    t.diag_end = (int)terms.size();
                    t.c_off = pr.off;
                    t.x_off = pr.off;
                    t.ldc = (int32_t)pr.dr;
                    t.row0 = (int32_t)r0;
                    t.col0 = (int32_t)c0;
                    t.m = (int32_t)std::min<int64_t>(tm, pr.dl - r0);
                    t.n = (int32_t)std::min<int64_t>(tn, pr.dr - c0);
                    t.member = member;
                    tasks.push_back(t);
                }
        }
        DMRG_TRY(upload(plan, terms, &plan->d_diag_terms, stream));
        DMRG_TRY(upload(plan, tasks, &plan->d_diag_tasks, stream));
        plan->n_diag_tasks = (int32_t)tasks.size();
    }
    DMRG_TRY(build_density(plan, stream));
    DMRG_HIP(hipStreamSynchronize(stream));
    return DMRG_OK;
}

// ------------------------------------------------------------------ l-1-1-r plans

// One member of an l-1-1-r plan: pairs of the enlarged blocks, output
// sub-matrices and records (offsets member-local).
struct Member4 {
    std::vector<Pair> pairs;
    std::vector<Geo> outs;
    std::vector<Record> recs;
    int64_t n = 0, flop = 0;
};

static const char *SUB_NAME[4] = {"block l", "site 1", "site 2", "block r"};

// Validation, records and sub-matrices of one four-subsystem problem (Eq. 13):
// for every term, every sector quadruple of psi and every combination of the
// four operators' blocks leaving it, one record per pair of non-zero site
// matrix elements, acting on the [d_l x d_r] slice of fixed site indices.
static dmrg_status analyse4(const dmrg_problem4 *p, Member4 *out, int gop_base, int gterm_base) {
    if (!p) return set_error(DMRG_E_INVALID_ARG, "null problem");
    for (int s = 0; s < 4; ++s) DMRG_TRY(check_space(p->space[s], SUB_NAME[s]));
    const int rank = p->space[0].rank;
    for (int s = 1; s < 4; ++s)
        if (p->space[s].rank != rank) return set_error(DMRG_E_INVALID_ARG, "label ranks differ");
    if (!p->target) return set_error(DMRG_E_INVALID_ARG, "null target label");
    if (p->nterm < 0 || (p->nterm && !p->terms)) return set_error(DMRG_E_INVALID_ARG, "missing term array");
    for (int s = 0; s < 4; ++s) {
        if (p->nop[s] < 0 || (p->nop[s] && !p->ops[s]))
            return set_error(DMRG_E_INVALID_ARG, "%s: missing operator array", SUB_NAME[s]);
        for (int i = 0; i < p->nop[s]; ++i) DMRG_TRY(check_op(p->space[s], p->ops[s][i], SUB_NAME[s], i));
    }
    for (int s = 1; s <= 2; ++s)
        for (int i = 0; i < p->space[s].nsec; ++i)
            if (p->space[s].dim[i] > 64)
                return set_error(DMRG_E_UNSUPPORTED, "%s: sector %d has more than 64 states", SUB_NAME[s], i);
    for (int k = 0; k < p->nterm; ++k) {
        const dmrg_term4 &t = p->terms[k];
        const int idx[4] = {t.a, t.b, t.c, t.d};
        for (int s = 0; s < 4; ++s)
            if (idx[s] < 0 || idx[s] >= p->nop[s])
                return set_error(DMRG_E_INVALID_ARG, "term %d: operator index out of range", k);
    }
    const Enlarged EL = enlarged_space(p->space[0], p->space[1]);
    const Enlarged ER = enlarged_space(p->space[2], p->space[3]);
    // pairs of the enlarged blocks (LR layout)
    std::vector<int> by_left(EL.nsec(), -1);
    std::vector<int32_t> want(rank);
    int64_t off = 0;
    for (int i = 0; i < EL.nsec(); ++i) {
        for (int c = 0; c < rank; ++c) want[c] = p->target[c] - EL.label[(size_t)i * rank + c];
        const int j = ER.find(want.data());
        if (j < 0) continue;
        by_left[i] = (int)out->pairs.size();
        out->pairs.push_back(Pair{i, j, EL.dim[i], ER.dim[j], off});
        off += EL.dim[i] * ER.dim[j];
    }
    out->n = off;
    const dmrg_space &sl = p->space[0], &s1 = p->space[1], &s2 = p->space[2], &sr = p->space[3];
    // output sub-matrices: (pair, left combination, right combination, i1, i2)
    std::map<std::tuple<int, int, int, int, int, int>, int> geo_of;  // (s_l, s_1, s_2, s_r, i1, i2)
    std::vector<std::tuple<int, int, int, int>> quads;               // every quadruple of psi, in order
    std::vector<int> quad_pair;
    for (int pi = 0; pi < (int)out->pairs.size(); ++pi) {
        const Pair &pr = out->pairs[pi];
        for (const Combo &cl : EL.combos[pr.sl])
            for (const Combo &cr : ER.combos[pr.sr]) {
                quads.emplace_back(cl.s, cl.f, cr.s, cr.f);
                quad_pair.push_back(pi);
                const int64_t d1 = s1.dim[cl.f], d2 = s2.dim[cr.s], dl = sl.dim[cl.s], dr = sr.dim[cr.f];
                for (int64_t i1 = 0; i1 < d1; ++i1)
                    for (int64_t i2 = 0; i2 < d2; ++i2) {
                        geo_of[{cl.s, cl.f, cr.s, cr.f, (int)i1, (int)i2}] = (int)out->outs.size();
                        out->outs.push_back(Geo{pr.off + (cl.off + i1) * pr.dr + cr.off + i2 * dr, dl, dr, d1 * pr.dr});
                    }
            }
    }
    // operators: blocks l and r resolved on the device data, sites read on the host
    std::vector<BySrc> L(p->nop[0]), R(p->nop[3]);
    for (int i = 0; i < p->nop[0]; ++i) L[i] = resolve(sl, p->ops[0][i], gop_base + i);
    for (int i = 0; i < p->nop[3]; ++i) R[i] = resolve(sr, p->ops[3][i], gop_base + p->nop[0] + i);
    std::vector<std::vector<HostBlock>> S1(p->nop[1]), S2(p->nop[2]);
    for (int i = 0; i < p->nop[1]; ++i) S1[i] = host_blocks(s1, p->ops[1][i]);
    for (int i = 0; i < p->nop[2]; ++i) S2[i] = host_blocks(s2, p->ops[2][i]);
    auto lab = [&](const dmrg_space &sp, int s, int c) { return sp.label[(size_t)s * rank + c]; };
    for (int k = 0; k < p->nterm; ++k) {
        const dmrg_term4 &t = p->terms[k];
        for (size_t qi = 0; qi < quads.size(); ++qi) {
            const int ql = std::get<0>(quads[qi]), q1 = std::get<1>(quads[qi]), q2 = std::get<2>(quads[qi]),
                      qr = std::get<3>(quads[qi]);
            for (const OpBlock &a : L[t.a][ql])
                for (const HostBlock &b1 : S1[t.b]) {
                    if (b1.src != q1) continue;
                    for (const HostBlock &b2 : S2[t.c]) {
                        if (b2.src != q2) continue;
                        for (const OpBlock &b : R[t.d][qr]) {
                            bool ok = true;
                            for (int c = 0; c < rank; ++c)
                                ok &= lab(sl, a.dst, c) + lab(s1, b1.dst, c) + lab(s2, b2.dst, c) + lab(sr, b.dst, c) ==
                                      p->target[c];
                            if (!ok)
                                return set_error(DMRG_E_SECTOR, "term %d leaves the target sector", k);
                            const int eL = EL.where[a.dst][b1.dst], eR = ER.where[b2.dst][b.dst];
                            if (eL < 0 || eR < 0) continue;  // an empty output block
                            const int po = by_left[eL];
                            if (po < 0 || out->pairs[po].sr != eR) continue;
                            for (int64_t o1 = 0; o1 < b1.rows; ++o1)
                                for (int64_t i1 = 0; i1 < b1.cols; ++i1) {
                                    const double w1 = b1.m[(size_t)(o1 * b1.cols + i1)];
                                    if (w1 == 0.0) continue;
                                    for (int64_t o2 = 0; o2 < b2.rows; ++o2)
                                        for (int64_t i2 = 0; i2 < b2.cols; ++i2) {
                                            const double w2 = b2.m[(size_t)(o2 * b2.cols + i2)];
                                            if (w2 == 0.0) continue;
                                            Record r{};
                                            r.term = k;
                                            r.gterm = gterm_base + k;
                                            r.pin = quad_pair[qi];
                                            r.pout = po;
                                            r.a = a;
                                            r.b = b;
                                            r.oin = geo_of.at({ql, q1, q2, qr, (int)i1, (int)i2});
                                            r.oout = geo_of.at({a.dst, b1.dst, b2.dst, b.dst, (int)o1, (int)o2});
                                            r.gin = out->outs[r.oin];
                                            r.gout = out->outs[r.oout];
                                            r.w = w1 * w2;
                                            const bool da = a.kind == DMRG_OP_DENSE, db = b.kind == DMRG_OP_DENSE;
                                            const int64_t di = r.gin.rows, dk = r.gin.cols, dj = r.gout.rows,
                                                          dl = r.gout.cols;
                                            if (da && db) {
                                                const int64_t cl = dj * di * dk + dj * dk * dl,
                                                              cr = di * dk * dl + dj * di * dl;
                                                r.order = cr < cl ? 1 : 0;
                                                out->flop += 2 * std::min(cl, cr);
                                            } else {
                                                r.order = 2;
                                                out->flop += da ? 2 * dj * di * dk : (db ? 2 * di * dk * dl : 2 * dj * dl);
                                            }
                                            out->recs.push_back(r);
                                        }
                                }
                        }
                    }
                }
        }
    }
    return DMRG_OK;
}

static dmrg_status build_plan_l11r(dmrg_plan *plan, int32_t nprob, const dmrg_problem4 *probs, hipStream_t stream) {
    plan->nprob = nprob;
    plan->prec = DMRG_F64;
    plan->member_off.assign(1, 0);
    plan->term_off.assign(1, 0);
    int gop = 0;
    std::set<std::pair<int, int>> used_blocks, used_slices;
    int64_t flop = 0, opbytes = 0;
    for (int p = 0; p < nprob; ++p) {
        Member4 m4;
        DMRG_TRY(analyse4(&probs[p], &m4, gop, plan->term_off.back()));
        const int pair_base = (int)plan->pairs.size(), out_base = (int)plan->out_geo.size();
        const int64_t base = plan->member_off.back();
        for (Pair q : m4.pairs) {
            q.off += base;
            plan->pairs.push_back(q);
            plan->pair_member.push_back(p);
        }
        for (Geo g : m4.outs) {
            g.off += base;
            plan->out_geo.push_back(g);
            plan->out_member.push_back(p);
        }
        for (Record r : m4.recs) {
            r.pin += pair_base;
            r.pout += pair_base;
            r.oin += out_base;
            r.oout += out_base;
            r.gin.off += base;
            r.gout.off += base;
            for (const OpBlock *b : {&r.a, &r.b}) {
                if (b->kind == DMRG_OP_DENSE) {
                    if (used_blocks.insert({b->op, b->blk}).second) opbytes += 8 * b->rows * b->cols;
                } else if (b->kind == DMRG_OP_DIAG) {
                    if (used_slices.insert({b->op, b->src}).second) opbytes += 8 * b->rows;
                }
            }
            plan->records.push_back(r);
        }
        flop += m4.flop;
        plan->member_off.push_back(base + m4.n);
        plan->term_off.push_back(plan->term_off.back() + probs[p].nterm);
        gop += probs[p].nop[0] + probs[p].nop[3];
    }
    plan->n = plan->member_off.back();
    plan->nterm_total = plan->term_off.back();
    plan->flop = flop;
    plan->bytes = opbytes + 16 * plan->n;
    return finish_plan(plan, DMRG_F64, stream, nullptr);
}

dmrg_status plan_free(dmrg_plan *plan) {
    davidson_free(plan);
    block_free(plan);
    for (void *p : plan->owned) (void)hipFree(p);
    plan->owned.clear();
    if (plan->d_multi_tmp) (void)hipFree(plan->d_multi_tmp);
    plan->d_multi_tmp = nullptr;
    return DMRG_OK;
}

}  // namespace dmrg

// ================================================================== ABI

using namespace dmrg;

extern "C" {

const char *dmrg_last_error(void) { return g_last_error.c_str(); }

const char *dmrg_version(void) { return "dmrg-mi355x 0.1 (gfx950)"; }

dmrg_status dmrg_problem_check(const dmrg_problem *prob) {
    clear_error();
    return analyse(prob, nullptr, nullptr, 0, 0);
}

dmrg_status dmrg_set_tile_table(int32_t ncls, const int32_t *bound, const int32_t *tile) {
    clear_error();
    if (ncls < 0 || ncls > 8 || (ncls > 0 && (!bound || !tile)))
        return set_error(DMRG_E_INVALID_ARG, "tile table: 0 <= ncls <= 8 with bound and tile arrays");
    for (int c = 0; c < ncls; ++c) {
        if (tile[c] != 16 && tile[c] != 32) return set_error(DMRG_E_INVALID_ARG, "tile sizes must be 16 or 32");
        if (c > 0 && bound[c] <= bound[c - 1]) return set_error(DMRG_E_INVALID_ARG, "bounds must ascend");
    }
    g_ncls = ncls;
    for (int c = 0; c < ncls; ++c) {
        g_bound[c] = bound[c];
        g_tile[c] = tile[c];
    }
    return DMRG_OK;
}

static dmrg_status validate_problems(int32_t nprob, const dmrg_problem *probs, int32_t prec) {
    if (nprob < 1 || !probs) return set_error(DMRG_E_INVALID_ARG, "need nprob >= 1 problems");
    if (prec != DMRG_F64 && prec != DMRG_F32 && prec != DMRG_BF16)
        return set_error(DMRG_E_INVALID_ARG, "unknown precision %d", prec);
    for (int p = 0; p < nprob; ++p) {
        dmrg_status st = analyse(&probs[p], nullptr, nullptr, 0, 0);
        if (st < 0) {
            std::string m = g_last_error;
            return set_error(st, "problem %d: %s", p, m.c_str());
        }
    }
    return DMRG_OK;
}

dmrg_status dmrg_plan_workspace_size(int32_t nprob, const dmrg_problem *probs, int32_t prec, int32_t kmax,
                                     size_t *bytes) {
    clear_error();
    if (!bytes) return set_error(DMRG_E_INVALID_ARG, "null output pointer");
    *bytes = 0;
    if (kmax < 2 || kmax > KM) return set_error(DMRG_E_INVALID_ARG, "need 2 <= kmax <= %d", KM);
    DMRG_TRY(validate_problems(nprob, probs, prec));
    return workspace_need(nprob, probs, prec, kmax, bytes, nullptr, nullptr);
}

dmrg_status dmrg_plan_create(dmrg_plan **out, int32_t nprob, const dmrg_problem *probs, int32_t prec,
                             int32_t ws_kmax, void *workspace, size_t ws_bytes, void *stream) {
    clear_error();
    if (!out) return set_error(DMRG_E_INVALID_ARG, "null output pointer");
    *out = nullptr;
    // host validation first: no GPU is touched for invalid input or a short workspace
    DMRG_TRY(validate_problems(nprob, probs, prec));
    size_t need = 0, part_off = 0, dav_off = 0;
    if (workspace) {
        if (ws_kmax < 2 || ws_kmax > KM) return set_error(DMRG_E_INVALID_ARG, "need 2 <= ws_kmax <= %d", KM);
        if ((uintptr_t)workspace % WS_ALIGN)
            return set_error(DMRG_E_INVALID_ARG, "workspace must be %d-byte aligned", (int)WS_ALIGN);
        DMRG_TRY(workspace_need(nprob, probs, prec, ws_kmax, &need, &part_off, &dav_off));
        if (ws_bytes < need)
            return set_error(DMRG_E_NOMEM, "workspace of %zu bytes is smaller than the %zu this plan needs", ws_bytes,
                             need);
    }
    dmrg_plan *plan = new (std::nothrow) dmrg_plan();
    if (!plan) return set_error(DMRG_E_NOMEM, "host allocation failed");
    if (workspace) {
        plan->ws = (char *)workspace;
        plan->ws_bytes = ws_bytes;
        plan->ws_kmax = ws_kmax;
        plan->ws_part = part_off;
        plan->ws_dav = dav_off;
    }
    hipError_t e = hipGetDevice(&plan->device);
    if (e != hipSuccess) {
        delete plan;
        return set_error(DMRG_E_HIP, "hipGetDevice failed: %s", hipGetErrorString(e));
    }
    dmrg_status st = build_plan(plan, nprob, probs, prec, (hipStream_t)stream);
    if (st < 0) {
        plan_free(plan);
        delete plan;
        return st;
    }
    *out = plan;
    return DMRG_OK;
}

dmrg_status dmrg_plan_create_l11r(dmrg_plan **out, int32_t nprob, const dmrg_problem4 *probs, void *stream) {
    clear_error();
    if (!out) return set_error(DMRG_E_INVALID_ARG, "null output pointer");
    *out = nullptr;
    if (nprob < 1 || !probs) return set_error(DMRG_E_INVALID_ARG, "need nprob >= 1 problems");
    for (int p = 0; p < nprob; ++p) {  // host validation first: no GPU is touched for invalid input
        Member4 m4;
        dmrg_status st = analyse4(&probs[p], &m4, 0, 0);
        if (st < 0) {
            std::string m = g_last_error;
            return set_error(st, "problem %d: %s", p, m.c_str());
        }
    }
    dmrg_plan *plan = new (std::nothrow) dmrg_plan();
    if (!plan) return set_error(DMRG_E_NOMEM, "host allocation failed");
    hipError_t e = hipGetDevice(&plan->device);
    if (e != hipSuccess) {
        delete plan;
        return set_error(DMRG_E_HIP, "hipGetDevice failed: %s", hipGetErrorString(e));
    }
    dmrg_status st = build_plan_l11r(plan, nprob, probs, (hipStream_t)stream);
    if (st < 0) {
        plan_free(plan);
        delete plan;
        return st;
    }
    *out = plan;
    return DMRG_OK;
}

dmrg_status dmrg_plan_sizes(const dmrg_plan *plan, int64_t *n, int32_t *npair, int32_t *nrec, int64_t *flop,
                            int64_t *bytes) {
    clear_error();
    if (!plan) return set_error(DMRG_E_INVALID_ARG, "null plan");
    if (n) *n = plan->n;
    if (npair) *npair = (int32_t)plan->pairs.size();
    if (nrec) *nrec = (int32_t)plan->records.size();
    if (flop) *flop = plan->flop;
    if (bytes) *bytes = plan->bytes;
    return DMRG_OK;
}

dmrg_status dmrg_plan_layout(const dmrg_plan *plan, int32_t *member, int32_t *pair_left, int32_t *pair_right,
                             int64_t *pair_off, int64_t *member_off) {
    clear_error();
    if (!plan) return set_error(DMRG_E_INVALID_ARG, "null plan");
    size_t np = plan->pairs.size();
    for (size_t i = 0; i < np; ++i) {
        if (member) member[i] = plan->pair_member[i];
        if (pair_left) pair_left[i] = plan->pairs[i].sl;
        if (pair_right) pair_right[i] = plan->pairs[i].sr;
        if (pair_off) pair_off[i] = plan->pairs[i].off;
    }
    if (pair_off) pair_off[np] = plan->n;
    if (member_off)
        for (size_t i = 0; i < plan->member_off.size(); ++i) member_off[i] = plan->member_off[i];
    return DMRG_OK;
}

dmrg_status dmrg_plan_records(const dmrg_plan *plan, int32_t *term, int32_t *pair_in, int32_t *pair_out,
                              int32_t *order) {
    clear_error();
    if (!plan) return set_error(DMRG_E_INVALID_ARG, "null plan");
    for (size_t i = 0; i < plan->records.size(); ++i) {
        const Record &r = plan->records[i];
        if (term) term[i] = r.term;
        if (pair_in) pair_in[i] = r.pin;
        if (pair_out) pair_out[i] = r.pout;
        if (order) order[i] = r.order;
    }
    return DMRG_OK;
}

void dmrg_plan_destroy(dmrg_plan *plan) {
    if (!plan) return;
    int cur = 0;
    bool switched = false;
    if (hipGetDevice(&cur) == hipSuccess && cur != plan->device) switched = hipSetDevice(plan->device) == hipSuccess;
    (void)hipDeviceSynchronize();
    plan_free(plan);
    if (switched) (void)hipSetDevice(cur);
    delete plan;
}

}  // extern "C"
