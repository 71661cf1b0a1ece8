// Enlarged-block basis (enlarge.h) and dmrg_enlarge: an enlarged block's
// operators from the operators of a block and a site (Alg. 1, steps 1-2),
// computed on the host.
#include "enlarge.h"

#include <algorithm>
#include <cstring>
#include <map>
#include <tuple>

#include "internal.h"

namespace dmrg {

static int cmp_lab(const int32_t *a, const int32_t *b, int rank) {
    for (int c = 0; c < rank; ++c) {
        if (a[c] < b[c]) return -1;
        if (a[c] > b[c]) return 1;
    }
    return 0;
}

int Enlarged::find(const int32_t *lab) const {
    int lo = 0, hi = nsec() - 1;
    while (lo <= hi) {
        const int mid = (lo + hi) / 2;
        const int c = cmp_lab(label.data() + (size_t)mid * rank, lab, rank);
        if (c == 0) return mid;
        if (c < 0)
            lo = mid + 1;
        else
            hi = mid - 1;
    }
    return -1;
}

Enlarged enlarged_space(const dmrg_space &slow, const dmrg_space &fast) {
    Enlarged e;
    e.rank = slow.rank;
    const int r = e.rank;
    // label sum -> combinations (s, f, size), s ascending by construction
    std::map<std::vector<int32_t>, std::vector<std::tuple<int32_t, int32_t, int64_t>>> sums;
    for (int s = 0; s < slow.nsec; ++s)
        for (int f = 0; f < fast.nsec; ++f) {
            const int64_t d = slow.dim[s] * fast.dim[f];
            if (d == 0) continue;
            std::vector<int32_t> lab(r);
            for (int c = 0; c < r; ++c) lab[c] = slow.label[(size_t)s * r + c] + fast.label[(size_t)f * r + c];
            sums[lab].emplace_back(s, f, d);
        }
    e.where.assign(slow.nsec, std::vector<int32_t>(fast.nsec, -1));
    e.at.assign(slow.nsec, std::vector<int64_t>(fast.nsec, 0));
    for (auto &kv : sums) {  // std::map: labels ascend lexicographically
        const int q = e.nsec();
        e.label.insert(e.label.end(), kv.first.begin(), kv.first.end());
        int64_t off = 0;
        std::vector<Combo> cs;
        for (auto &t : kv.second) {
            const int32_t s = std::get<0>(t), f = std::get<1>(t);
            cs.push_back(Combo{s, f, off});
            e.where[s][f] = q;
            e.at[s][f] = off;
            off += std::get<2>(t);
        }
        e.combos.push_back(std::move(cs));
        e.dim.push_back(off);
    }
    return e;
}

std::vector<HostBlock> host_blocks(const dmrg_space &sp, const dmrg_op &op) {
    std::vector<HostBlock> out;
    std::vector<int64_t> off(sp.nsec + 1, 0);
    for (int i = 0; i < sp.nsec; ++i) off[i + 1] = off[i] + sp.dim[i];
    if (op.kind == DMRG_OP_IDENTITY || op.kind == DMRG_OP_DIAG) {
        for (int s = 0; s < sp.nsec; ++s) {
            const int64_t d = sp.dim[s];
            HostBlock b{s, s, d, d, std::vector<double>((size_t)(d * d), 0.0)};
            for (int64_t i = 0; i < d; ++i) b.m[(size_t)(i * d + i)] = op.kind == DMRG_OP_DIAG ? op.data[off[s] + i] : 1.0;
            out.push_back(std::move(b));
        }
        return out;
    }
    for (int k = 0; k < op.nblk; ++k) {
        const int64_t rows = sp.dim[op.dst[k]], cols = sp.dim[op.src[k]];
        HostBlock b{op.src[k], op.dst[k], rows, cols, std::vector<double>(op.data + op.off[k], op.data + op.off[k] + rows * cols)};
        out.push_back(std::move(b));
    }
    return out;
}

}  // namespace dmrg

using namespace dmrg;

static dmrg_status check_space_h(const dmrg_space *s, const char *which) {
    if (!s || s->nsec < 1 || s->rank < 1 || s->rank > 2 || !s->label || !s->dim)
        return set_error(DMRG_E_INVALID_ARG, "%s space: need nsec >= 1, rank 1 or 2, label and dim arrays", which);
    for (int i = 0; i < s->nsec; ++i) {
        if (s->dim[i] < 0) return set_error(DMRG_E_INVALID_ARG, "%s space: negative dim at sector %d", which, i);
        if (s->dim[i] > (int64_t)1 << 20)
            return set_error(DMRG_E_UNSUPPORTED, "%s space: sector %d too large for a host enlargement", which, i);
        if (i > 0 && cmp_lab(s->label + (size_t)(i - 1) * s->rank, s->label + (size_t)i * s->rank, s->rank) >= 0)
            return set_error(DMRG_E_LAYOUT, "%s space: labels not strictly ascending at sector %d", which, i);
    }
    return DMRG_OK;
}

static dmrg_status check_op_h(const dmrg_space &s, const dmrg_op &op, const char *which, int idx) {
    if (op.kind == DMRG_OP_IDENTITY) return DMRG_OK;
    if (op.kind == DMRG_OP_DIAG)
        return op.data ? DMRG_OK : set_error(DMRG_E_INVALID_ARG, "%s op %d: diagonal without data", which, idx);
    if (op.kind != DMRG_OP_DENSE) return set_error(DMRG_E_INVALID_ARG, "%s op %d: unknown kind %d", which, idx, op.kind);
    if (op.nblk < 0 || (op.nblk > 0 && (!op.src || !op.dst || !op.off || !op.data)))
        return set_error(DMRG_E_INVALID_ARG, "%s op %d: missing block arrays", which, idx);
    std::vector<std::pair<int, int>> seen;
    for (int b = 0; b < op.nblk; ++b) {
        if (op.src[b] < 0 || op.src[b] >= s.nsec || op.dst[b] < 0 || op.dst[b] >= s.nsec || op.off[b] < 0)
            return set_error(DMRG_E_INVALID_ARG, "%s op %d block %d: sector index or offset out of range", which, idx, b);
        seen.emplace_back(op.src[b], op.dst[b]);
    }
    std::sort(seen.begin(), seen.end());
    for (size_t i = 1; i < seen.size(); ++i)
        if (seen[i] == seen[i - 1]) return set_error(DMRG_E_LAYOUT, "%s op %d: duplicate block", which, idx);
    return DMRG_OK;
}

extern "C" dmrg_status dmrg_enlarge(const dmrg_space *slow, int32_t nop_slow, const dmrg_op *ops_slow,
                                    const dmrg_space *fast, int32_t nop_fast, const dmrg_op *ops_fast,
                                    int32_t nterm, const dmrg_kron_term *terms, int32_t nout,
                                    dmrg_enlarge_sizes *sizes, int32_t *label, int64_t *dim, int32_t *op_kind,
                                    int32_t *op_nblk, int64_t *op_off, int32_t *src, int32_t *dst, int64_t *off,
                                    double *data) {
    clear_error();
    if (!sizes) return set_error(DMRG_E_INVALID_ARG, "null sizes");
    DMRG_TRY(check_space_h(slow, "slow"));
    DMRG_TRY(check_space_h(fast, "fast"));
    if (slow->rank != fast->rank) return set_error(DMRG_E_INVALID_ARG, "slow and fast label ranks differ");
    if (nop_slow < 0 || nop_fast < 0 || nterm < 0 || nout < 0 || (nop_slow && !ops_slow) || (nop_fast && !ops_fast) ||
        (nterm && !terms))
        return set_error(DMRG_E_INVALID_ARG, "negative count or missing operator / term array");
    for (int i = 0; i < nop_slow; ++i) DMRG_TRY(check_op_h(*slow, ops_slow[i], "slow", i));
    for (int i = 0; i < nop_fast; ++i) DMRG_TRY(check_op_h(*fast, ops_fast[i], "fast", i));
    for (int t = 0; t < nterm; ++t)
        if (terms[t].out < 0 || terms[t].out >= nout || terms[t].a < 0 || terms[t].a >= nop_slow || terms[t].b < 0 ||
            terms[t].b >= nop_fast)
            return set_error(DMRG_E_INVALID_ARG, "term %d: index out of range", t);
    const Enlarged E = enlarged_space(*slow, *fast);
    const int rank = E.rank, ns = E.nsec();
    int64_t m = 0;
    for (int64_t d : E.dim) m += d;
    std::vector<int64_t> eoff(ns + 1, 0);
    for (int q = 0; q < ns; ++q) eoff[q + 1] = eoff[q] + E.dim[q];
    // per output: kind and, for dense outputs, its blocks (src, dst) -> dense values
    std::vector<int32_t> kind(nout, DMRG_OP_DENSE);
    std::vector<std::map<std::pair<int, int>, std::vector<double>>> blocks(nout);
    std::vector<std::vector<double>> diag(nout);
    std::vector<std::vector<int>> by_out(nout);
    for (int t = 0; t < nterm; ++t) by_out[terms[t].out].push_back(t);
    for (int o = 0; o < nout; ++o) {
        bool all_id = !by_out[o].empty(), all_diag = !by_out[o].empty();
        for (int t : by_out[o]) {
            const int ka = ops_slow[terms[t].a].kind, kb = ops_fast[terms[t].b].kind;
            all_id = all_id && ka == DMRG_OP_IDENTITY && kb == DMRG_OP_IDENTITY && terms[t].coef == 1.0;
            all_diag = all_diag && ka != DMRG_OP_DENSE && kb != DMRG_OP_DENSE;
        }
        if (all_id && by_out[o].size() == 1) {
            kind[o] = DMRG_OP_IDENTITY;
            continue;
        }
        if (all_diag) {
            kind[o] = DMRG_OP_DIAG;
            diag[o].assign((size_t)m, 0.0);
        }
        for (int t : by_out[o]) {
            const std::vector<HostBlock> A = host_blocks(*slow, ops_slow[terms[t].a]);
            const std::vector<HostBlock> F = host_blocks(*fast, ops_fast[terms[t].b]);
            const double c = terms[t].coef;
            for (const HostBlock &a : A)
                for (const HostBlock &f : F) {
                    const int q = E.where[a.src][f.src], q2 = E.where[a.dst][f.dst];
                    if (q < 0 || q2 < 0) continue;  // an empty source or destination sub-block
                    const int64_t r0 = E.at[a.dst][f.dst], c0 = E.at[a.src][f.src];
                    const int64_t ld = E.dim[q];
                    if (kind[o] == DMRG_OP_DIAG) {
                        for (int64_t i = 0; i < a.rows; ++i)
                            for (int64_t j = 0; j < f.rows; ++j)
                                diag[o][(size_t)(eoff[q2] + r0 + i * f.rows + j)] +=
                                    c * a.m[(size_t)(i * a.cols + i)] * f.m[(size_t)(j * f.cols + j)];
                        continue;
                    }
                    std::vector<double> &B = blocks[o][{q, q2}];
                    if (B.empty()) B.assign((size_t)(E.dim[q2] * ld), 0.0);
                    for (int64_t i = 0; i < a.rows; ++i)
                        for (int64_t k = 0; k < a.cols; ++k) {
                            const double av = a.m[(size_t)(i * a.cols + k)];
                            if (av == 0.0) continue;
                            for (int64_t j = 0; j < f.rows; ++j)
                                for (int64_t l = 0; l < f.cols; ++l)
                                    B[(size_t)((r0 + i * f.rows + j) * ld + c0 + k * f.cols + l)] +=
                                        c * av * f.m[(size_t)(j * f.cols + l)];
                        }
                }
        }
    }
    int64_t nblk_total = 0, data_len = 0;
    for (int o = 0; o < nout; ++o) {
        if (kind[o] == DMRG_OP_DIAG) data_len += m;
        if (kind[o] != DMRG_OP_DENSE) continue;
        nblk_total += (int64_t)blocks[o].size();
        for (auto &kv : blocks[o]) data_len += (int64_t)kv.second.size();
    }
    if (nblk_total > INT32_MAX) return set_error(DMRG_E_UNSUPPORTED, "too many blocks");
    sizes->nsec = ns;
    sizes->m = m;
    sizes->nblk_total = (int32_t)nblk_total;
    sizes->data_len = data_len;
    if (!label) return DMRG_OK;  // size query
    if (!dim || (nout && (!op_kind || !op_nblk || !op_off)) || (nblk_total && (!src || !dst || !off)) ||
        (data_len && !data))
        return set_error(DMRG_E_INVALID_ARG, "output arrays missing (query the sizes with label = NULL first)");
    std::memcpy(label, E.label.data(), sizeof(int32_t) * (size_t)ns * rank);
    std::memcpy(dim, E.dim.data(), sizeof(int64_t) * (size_t)ns);
    int64_t b = 0, d = 0;
    for (int o = 0; o < nout; ++o) {
        op_kind[o] = kind[o];
        op_off[o] = d;
        op_nblk[o] = 0;
        if (kind[o] == DMRG_OP_DIAG) {
            std::memcpy(data + d, diag[o].data(), sizeof(double) * (size_t)m);
            d += m;
        } else if (kind[o] == DMRG_OP_DENSE) {
            op_nblk[o] = (int32_t)blocks[o].size();
            for (auto &kv : blocks[o]) {  // ascending (src, dst)
                src[b] = kv.first.first;
                dst[b] = kv.first.second;
                off[b] = d - op_off[o];
                std::memcpy(data + d, kv.second.data(), sizeof(double) * kv.second.size());
                d += (int64_t)kv.second.size();
                ++b;
            }
        }
    }
    return DMRG_OK;
}
