"""The l-1-1-r strategy (Sec. "l-1-1-r strategy", Eq. 12-13, Alg. 2), FP64.

Test infrastructure (see the package docstring).

A superblock of four subsystems -- block l, site 1, site 2, block r -- has
H_SB = sum_k c_k A_k (x) a_k (x) b_k (x) B_k (Eq. 12); the projection is the
sum over terms of Alg. 2 applied to every sector quadruple (Eq. 13).

Basis order (a reading: the paper fixes none).  The two halves are the
enlarged blocks L = l (x) s1 and R = s2 (x) r.  An enlarged space has one
sector per label sum q = q_slow + q_fast that has states, in ascending
lexicographic order; inside sector q the combinations (s_slow, s_fast) with
q_slow + q_fast = q follow in ascending order of s_slow, each a row-major
[d(s_slow), d(s_fast)] sub-block (slow index first, the order of the
Kronecker product slow (x) fast).  The superblock vector then has the LR
layout of (L, R) (see :mod:`oracle.sectors`): for every left sector in
ascending order, the row-major block [d_L, d_R]; a quadruple (s_l, s_1, s_2,
s_r) occupies the rows of its combination (s_l, s_1) and the columns of its
combination (s_2, s_r), i.e. a [d_l d_1] x [d_2 d_r] sub-block, which
reshapes to the four-index tensor X[i_l, i_1, i_2, i_r] of Alg. 2 (i_r
fastest).  With this order the projection of Eq. 13 equals the LR projection
(Eq. 11) of the same superblock written with enlarged-block operators
A (x) a and b (x) B (:func:`to_lr`).

Functions:
  enlarged_space   the enlarged sectors and their combinations
  enlarge_operator sum_t c_t (X_t (x) F_t) as a sector-form operator on slow (x) fast
  to_lr            the same superblock as an LR problem (enlarged blocks)
  layout           psi layout: pairs, offsets, and each quadruple's sub-block
  project_dense    P_Q (sum_k c_k A_k (x) a_k (x) b_k (x) B_k) P_Q^T psi by Kronecker products
  project_sectors  Eq. 13: Alg. 2 on every sector quadruple and block combination
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import Dict, List, Tuple

import numpy as np

from . import projection, sectors


class _Space:
    """A sector table (labels [nsec, rank], dims [nsec]) built by the oracle."""

    def __init__(self, labels, dims):
        self.labels = np.asarray(labels, dtype=np.int32).reshape(len(dims), -1)
        self.dims = np.asarray(dims, dtype=np.int64)

    @property
    def nsec(self):
        return int(self.dims.shape[0])

    @property
    def m(self):
        return int(self.dims.sum())

    def offsets(self):
        return np.concatenate([[0], np.cumsum(self.dims)]).astype(np.int64)


class _Dense:
    """A sector-form dense operator built by the oracle (blocks [d_dst, d_src])."""

    kind = "dense"
    diag = None

    def __init__(self, src, dst, blocks):
        self.src, self.dst, self.blocks = np.asarray(src), np.asarray(dst), blocks

    @property
    def nblk(self):
        return len(self.blocks)


class _LR:
    """An LR superblock (Eq. 9) built by the oracle from a four-subsystem one."""

    def __init__(self, left, right, target, ops_left, ops_right, terms, coef):
        self.left, self.right, self.target = left, right, np.asarray(target, dtype=np.int32)
        self.ops_left, self.ops_right = ops_left, ops_right
        self.terms = np.asarray(terms, dtype=np.int32).reshape(-1, 2)
        self.coef = np.asarray(coef, dtype=np.float64)


def enlarged_space(slow, fast):
    """Sectors of slow (x) fast: returns (labels [nsec, rank], dims [nsec],
    combos) with combos[q] = [(s_slow, s_fast, offset inside sector q), ...]
    in ascending s_slow (the module's basis order)."""
    sums = {}
    for s in range(slow.nsec):
        for f in range(fast.nsec):
            d = int(slow.dims[s]) * int(fast.dims[f])
            if d == 0:
                continue
            lab = tuple(int(x) for x in (slow.labels[s] + fast.labels[f]))
            sums.setdefault(lab, []).append((s, f, d))
    labels = sorted(sums)
    combos, dims = [], []
    for lab in labels:
        lst = sorted(sums[lab])  # ascending s_slow (s_fast is determined by it)
        off, out = 0, []
        for s, f, d in lst:
            out.append((s, f, off))
            off += d
        combos.append(out)
        dims.append(off)
    rank = slow.labels.shape[1]
    return (np.array(labels, dtype=np.int32).reshape(-1, rank), np.array(dims, dtype=np.int64), combos)


def _dense_full(space, op):
    """The operator as a dense matrix in the sector-grouped basis."""
    return sectors.dense_operator(space, op)


def enlarged_index(slow, fast):
    """For every state (i_slow, i_fast) of the natural Kronecker basis
    (index i_slow * m_fast + i_fast, each factor's basis sector-grouped), its
    index in the enlarged basis (sector-grouped in the module's order)."""
    labels, dims, combos = enlarged_space(slow, fast)
    off_e = np.concatenate([[0], np.cumsum(dims)])
    off_s, off_f = slow.offsets(), fast.offsets()
    mf = int(fast.dims.sum())
    out = np.full(int(slow.dims.sum()) * mf, -1, dtype=np.int64)
    for q, lst in enumerate(combos):
        for s, f, o in lst:
            ds, df = int(slow.dims[s]), int(fast.dims[f])
            for a in range(ds):
                for b in range(df):
                    out[(off_s[s] + a) * mf + off_f[f] + b] = off_e[q] + o + a * df + b
    return out


def enlarge_operator(slow, fast, parts):
    """sum over parts (coef, X, F) of coef * X (x) F, X on ``slow`` and F on
    ``fast`` (Alg. 1, steps 1-2: an enlarged block's operator), returned as a
    sector-form dense operator on the enlarged space (blocks that are exactly
    zero are dropped), together with that space."""
    labels, dims, combos = enlarged_space(slow, fast)
    E = _Space(labels, dims)
    idx = enlarged_index(slow, fast)
    m = int(dims.sum())
    M = np.zeros((m, m))
    for c, X, F in parts:
        K = np.kron(_dense_full(slow, X), _dense_full(fast, F))
        P = np.zeros((m, K.shape[0]))
        keep = idx >= 0
        P[idx[keep], np.flatnonzero(keep)] = 1.0
        M += c * (P @ K @ P.T)
    off = E.offsets()
    src, dst, blocks = [], [], []
    for j in range(E.nsec):
        for i in range(E.nsec):
            blk = M[off[i]:off[i + 1], off[j]:off[j + 1]]
            if np.any(blk):
                src.append(j)
                dst.append(i)
                blocks.append(blk.copy())
    return E, _Dense(src, dst, blocks)


def to_lr(p4):
    """The same superblock as an LR problem (Eq. 9): term k becomes
    c_k (A_k (x) a_k) (x) (b_k (x) B_k) on the enlarged blocks L = l (x) s1 and
    R = s2 (x) r (one enlarged operator pair per term)."""
    l, s1, s2, r = p4.spaces
    opsL, opsR, terms = [], [], []
    L = R = None
    for k, (a, b, c, d) in enumerate(p4.terms):
        L, A = enlarge_operator(l, s1, [(1.0, p4.ops[0][a], p4.ops[1][b])])
        R, B = enlarge_operator(s2, r, [(1.0, p4.ops[2][c], p4.ops[3][d])])
        opsL.append(A)
        opsR.append(B)
        terms.append((k, k))
    return _LR(L, R, p4.target, opsL, opsR, terms, p4.coef.copy())


@dataclass
class Layout4:
    n: int
    pairs: List[Tuple[int, int]]   # (enlarged left sector, enlarged right sector) in psi order
    pair_offset: np.ndarray        # [npair + 1]
    # quadruple (s_l, s_1, s_2, s_r) -> (pair offset, row0, col0, ld): its [d_l d_1, d_2 d_r]
    # sub-block starts at pair_offset + row0 * ld + col0, rows of length ld
    quad: Dict[Tuple[int, int, int, int], Tuple[int, int, int, int]]


def layout(p4) -> Layout4:
    l, s1, s2, r = p4.spaces
    labL, dimL, combL = enlarged_space(l, s1)
    labR, dimR, combR = enlarged_space(s2, r)
    Q = np.asarray(p4.target, dtype=np.int64)
    pairs, offs, quad = [], [0], {}
    for i in range(len(dimL)):
        want = tuple(int(x) for x in (Q - labL[i]))
        hit = [j for j in range(len(dimR)) if tuple(int(x) for x in labR[j]) == want]
        if not hit:
            continue
        j = hit[0]
        if dimL[i] == 0 or dimR[j] == 0:
            continue
        base = offs[-1]
        for (sl, f1, ro) in combL[i]:
            for (f2, sr, co) in combR[j]:
                quad[(sl, f1, f2, sr)] = (base, ro, co, int(dimR[j]))
        pairs.append((i, j))
        offs.append(base + int(dimL[i]) * int(dimR[j]))
    return Layout4(offs[-1], pairs, np.array(offs, dtype=np.int64), quad)


def full_index(p4) -> np.ndarray:
    """For every psi entry, its index in the natural four-fold Kronecker basis
    ((i_l m_1 + i_1) m_2 + i_2) m_r + i_r (each factor sector-grouped)."""
    lay = layout(p4)
    l, s1, s2, r = p4.spaces
    offs = [sp.offsets() for sp in p4.spaces]
    m = [int(sp.dims.sum()) for sp in p4.spaces]
    out = np.full(lay.n, -1, dtype=np.int64)
    for (sl, f1, f2, sr), (base, ro, co, ld) in lay.quad.items():
        d = [int(l.dims[sl]), int(s1.dims[f1]), int(s2.dims[f2]), int(r.dims[sr])]
        for a in range(d[0]):
            for b in range(d[1]):
                for c in range(d[2]):
                    for e in range(d[3]):
                        pos = base + (ro + a * d[1] + b) * ld + co + c * d[3] + e
                        gi = (((offs[0][sl] + a) * m[1] + offs[1][f1] + b) * m[2] + offs[2][f2] + c) * m[3] \
                            + offs[3][sr] + e
                        out[pos] = gi
    return out


def superblock_hamiltonian(p4, coef=None) -> np.ndarray:
    """Dense sum_k c_k A_k (x) a_k (x) b_k (x) B_k (Eq. 12) in the natural basis."""
    coef = p4.coef if coef is None else np.asarray(coef, dtype=np.float64)
    mats = [[_dense_full(sp, op) for op in ops] for sp, ops in zip(p4.spaces, p4.ops)]
    H = 0.0
    for k, (a, b, c, d) in enumerate(p4.terms):
        H = H + coef[k] * np.kron(np.kron(np.kron(mats[0][a], mats[1][b]), mats[2][c]), mats[3][d])
    return H


def projected_hamiltonian(p4, coef=None) -> np.ndarray:
    idx = full_index(p4)
    H = superblock_hamiltonian(p4, coef)
    return H[np.ix_(idx, idx)]


def project_dense(p4, psi, coef=None) -> np.ndarray:
    """The plain definition at tiny sizes: P_Q H_SB P_Q^T psi."""
    return projected_hamiltonian(p4, coef) @ np.asarray(psi, dtype=np.float64)


def _apply(p, X4, axis):
    """Contract one operator block (identity, diagonal or dense [d', d]) with
    index ``axis`` of the four-index tensor."""
    if p is None:
        return X4
    if p.ndim == 1:
        shape = [1, 1, 1, 1]
        shape[axis] = -1
        return X4 * p.reshape(shape)
    return np.moveaxis(np.tensordot(p, X4, axes=([1], [axis])), 0, axis)


def project_sectors(p4, psi, coef=None) -> np.ndarray:
    """Eq. 13: for every term and every sector quadruple of psi, every
    combination of the four operators' blocks leaving that quadruple, Alg. 2 on
    the reshaped block X[i_l, i_1, i_2, i_r]: first the operator of block r on
    the fastest index, then site 2's, then site 1's, then block l's (the
    paper's order D, C, B, A), added into the output quadruple."""
    coef = p4.coef if coef is None else np.asarray(coef, dtype=np.float64)
    psi = np.asarray(psi, dtype=np.float64)
    lay = layout(p4)
    y = np.zeros(lay.n)
    by_src = [[projection._by_src(sp, op) for op in ops] for sp, ops in zip(p4.spaces, p4.ops)]
    dims = [sp.dims for sp in p4.spaces]

    def block(q):
        base, ro, co, ld = lay.quad[q]
        d = [int(dims[s][q[s]]) for s in range(4)]
        rows = np.arange(ro, ro + d[0] * d[1])
        cols = np.arange(co, co + d[2] * d[3])
        return base, rows, cols, ld, d

    for k, t in enumerate(p4.terms):
        for q, _ in lay.quad.items():
            base, rows, cols, ld, d = block(q)
            X = psi[base + rows[:, None] * ld + cols[None, :]].reshape(d)
            for (dl, pl) in by_src[0][t[0]].get(q[0], []):
                for (d1, p1) in by_src[1][t[1]].get(q[1], []):
                    for (d2, p2) in by_src[2][t[2]].get(q[2], []):
                        for (dr, pr) in by_src[3][t[3]].get(q[3], []):
                            out = (dl, d1, d2, dr)
                            if out not in lay.quad:
                                continue  # an empty output block
                            X1 = _apply(pr, X, 3)   # D: block r
                            X1 = _apply(p2, X1, 2)  # C: site 2
                            X1 = _apply(p1, X1, 1)  # B: site 1
                            X1 = _apply(pl, X1, 0)  # A: block l
                            ob, orow, ocol, old, od = block(out)
                            y[ob + orow[:, None] * old + ocol[None, :]] += coef[k] * X1.reshape(len(orow), len(ocol))
    return y


__all__ = ["enlarged_space", "enlarged_index", "enlarge_operator", "to_lr", "layout", "full_index",
           "superblock_hamiltonian", "projected_hamiltonian", "project_dense", "project_sectors"]
