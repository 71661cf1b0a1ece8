"""The superblock projection y = H_SB psi and its adjoint, in FP64.

Test infrastructure (see the package docstring).

Two independent evaluations of the same definition
    y = P_Q ( sum_k c_k A_k (x) B_k ) P_Q^T psi                (Eq. 9-10)
are given:

* :func:`project_dense` forms the Kronecker products explicitly (tiny blocks);
* :func:`project_sectors` follows Eq. 11 literally: for every term and every
  pair of blocks A_{i->j}, B_{k->l} whose input segment (i, k) lies in the
  target sector, X'_{jl} += c (A_{i->j} X_{ik}) B_{k->l}^T, always in that
  order (A X first), with NumPy matmul as the only primitive.

The row-major identity kron(A, B) vec(X) = vec(A X B^T) connects the two; it is
what Eq. 10 states for the column-major reading of the reshape.
"""
from __future__ import annotations

import numpy as np

from . import sectors


# ---------------------------------------------------------------------------
# dense (Kronecker) form, tiny problems only
# ---------------------------------------------------------------------------


def term_matrix(prob, k: int) -> np.ndarray:
    """A_k (x) B_k on the full m_L m_R space (Eq. 9)."""
    a, b = (int(x) for x in prob.terms[k])
    A = sectors.dense_operator(prob.left, prob.ops_left[a])
    B = sectors.dense_operator(prob.right, prob.ops_right[b])
    return np.kron(A, B)


def superblock_hamiltonian(prob, coef=None) -> np.ndarray:
    """H_SB = sum_k c_k A_k (x) B_k (Eq. 9), dense."""
    coef = prob.coef if coef is None else np.asarray(coef, dtype=np.float64)
    mL, mR = prob.left.m, prob.right.m
    H = np.zeros((mL * mR, mL * mR))
    for k in range(prob.terms.shape[0]):
        H += coef[k] * term_matrix(prob, k)
    return H


def projected_hamiltonian(prob, coef=None) -> np.ndarray:
    """H_Q = P_Q H_SB P_Q^T in the psi layout."""
    lay = sectors.layout(prob.left, prob.right, prob.target)
    H = superblock_hamiltonian(prob, coef)
    return H[np.ix_(lay.index_map, lay.index_map)]


def project_dense(prob, psi, coef=None) -> np.ndarray:
    return projected_hamiltonian(prob, coef) @ np.asarray(psi, dtype=np.float64)


def project_adjoint_dense(prob, gbar, coef=None) -> np.ndarray:
    """g_psi = H_Q^T gbar."""
    return projected_hamiltonian(prob, coef).T @ np.asarray(gbar, dtype=np.float64)


# ---------------------------------------------------------------------------
# sector form (Eq. 11)
# ---------------------------------------------------------------------------


def _blocks(space, op):
    """(src sector, dst sector, payload) for every block of an operator.

    payload is None for the identity, a 1-D array for a diagonal operator
    (the diagonal of the s -> s block) and a 2-D array for a dense block.
    """
    if op.kind == "identity":
        return [(s, s, None) for s in range(space.nsec)]
    if op.kind == "diag":
        off = space.offsets()
        return [(s, s, op.diag[off[s]:off[s + 1]]) for s in range(space.nsec)]
    return [(int(s), int(d), blk) for s, d, blk in zip(op.src, op.dst, op.blocks)]


def _by_src(space, op):
    out = {}
    for s, d, p in _blocks(space, op):
        out.setdefault(s, []).append((d, p))
    return out


def _left(p, X):
    """A X for one block (identity, diagonal or dense)."""
    if p is None:
        return X
    if p.ndim == 1:
        return p[:, None] * X
    return p @ X


def _right_t(p, X):
    """X B^T for one block."""
    if p is None:
        return X
    if p.ndim == 1:
        return X * p[None, :]
    return X @ p.T


def _left_t(p, X):
    """A^T X for one block."""
    if p is None:
        return X
    if p.ndim == 1:
        return p[:, None] * X
    return p.T @ X


def _right(p, X):
    """X B for one block."""
    if p is None:
        return X
    if p.ndim == 1:
        return X * p[None, :]
    return X @ p


def records(prob):
    """Every (term, input pair, output pair, A block, B block) the projection
    touches -- the operation records of Alg. 5, step 1."""
    table, n = sectors.pair_table(prob.left, prob.right, prob.target)
    Q = prob.target.astype(np.int64)
    out = []
    for k, (a, b) in enumerate(prob.terms):
        A = _by_src(prob.left, prob.ops_left[int(a)])
        B = _by_src(prob.right, prob.ops_right[int(b)])
        for (i, kk), _ in table.items():
            for j, pa in A.get(i, []):
                for l, pb in B.get(kk, []):
                    lab = prob.left.labels[j].astype(np.int64) + prob.right.labels[l].astype(np.int64)
                    if not np.array_equal(lab, Q):
                        raise ValueError(f"term {k} does not conserve the target label")
                    if (j, l) not in table:
                        continue  # the output segment is empty
                    out.append((k, (i, kk), (j, l), pa, pb))
    return out, table, n


def project_sectors(prob, psi, coef=None) -> np.ndarray:
    """Eq. 11: X'_{jl} += c_k (A_{k,i->j} X_{ik}) B_{k,k->l}^T over all records."""
    coef = prob.coef if coef is None else np.asarray(coef, dtype=np.float64)
    recs, table, n = records(prob)
    psi = np.asarray(psi, dtype=np.float64)
    y = np.zeros(n)
    for k, pin, pout, pa, pb in recs:
        o, dL, dR = table[pin]
        X = psi[o:o + dL * dR].reshape(dL, dR)
        o2, dL2, dR2 = table[pout]
        y[o2:o2 + dL2 * dR2] += (coef[k] * _right_t(pb, _left(pa, X))).reshape(-1)
    return y


def term_apply(prob, psi, k: int) -> np.ndarray:
    """T_k psi = P_Q (A_k (x) B_k) P_Q^T psi for a single term."""
    unit = np.zeros(prob.terms.shape[0])
    unit[k] = 1.0
    return project_sectors(prob, psi, unit)


def project_adjoint_sectors(prob, gbar, coef=None) -> np.ndarray:
    """g_psi = P_Q (sum_k c_k A_k^T (x) B_k^T) P_Q^T gbar: every record of Eq. 11
    run backwards, G_{ik} += c_k A_{k,i->j}^T Gbar_{jl} B_{k,k->l}."""
    coef = prob.coef if coef is None else np.asarray(coef, dtype=np.float64)
    recs, table, n = records(prob)
    g = np.asarray(gbar, dtype=np.float64)
    out = np.zeros(n)
    for k, pin, pout, pa, pb in recs:
        o2, dL2, dR2 = table[pout]
        G = g[o2:o2 + dL2 * dR2].reshape(dL2, dR2)
        o, dL, dR = table[pin]
        out[o:o + dL * dR] += (coef[k] * _right(pb, _left_t(pa, G))).reshape(-1)
    return out


def coef_gradient(prob, psi, gbar) -> np.ndarray:
    """d <gbar, y> / d c_k = <gbar, T_k psi>."""
    g = np.asarray(gbar, dtype=np.float64)
    return np.array([g @ term_apply(prob, psi, k) for k in range(prob.terms.shape[0])])


def diagonal(prob, coef=None) -> np.ndarray:
    """diag(H_Q): diag(A (x) B) = diag(A) (x) diag(B), summed over terms,
    restricted to the target sector (used by the Davidson correction step)."""
    coef = prob.coef if coef is None else np.asarray(coef, dtype=np.float64)
    table, n = sectors.pair_table(prob.left, prob.right, prob.target)
    D = np.zeros(n)

    def op_diag(space, op):
        m = space.m
        if op.kind == "identity":
            return np.ones(m)
        if op.kind == "diag":
            return op.diag.copy()
        d = np.zeros(m)
        off = space.offsets()
        for s, t, blk in zip(op.src, op.dst, op.blocks):
            if s == t:
                d[off[s]:off[s + 1]] += np.diag(blk)
        return d

    for k, (a, b) in enumerate(prob.terms):
        dA = op_diag(prob.left, prob.ops_left[int(a)])
        dB = op_diag(prob.right, prob.ops_right[int(b)])
        offL, offR = prob.left.offsets(), prob.right.offsets()
        for (sL, sR), (o, dL, dR) in table.items():
            D[o:o + dL * dR] += coef[k] * np.outer(dA[offL[sL]:offL[sL + 1]],
                                                   dB[offR[sR]:offR[sR + 1]]).reshape(-1)
    return D


def flop_count(prob) -> int:
    """Algorithmic FLOP of one projection: a two-sided record costs
    2 min(dj di dk + dj dk dl, di dk dl + dj di dl); a one-sided (identity)
    record 2 x its single product; a record with a diagonal factor counts
    that factor as an elementwise scaling; purely diagonal records 2 per
    element (multiply-add)."""
    recs, table, n = records(prob)
    total = 0
    for k, pin, pout, pa, pb in recs:
        _, di, dk = table[pin]
        _, dj, dl = table[pout]
        da = pa is not None and pa.ndim == 2
        db = pb is not None and pb.ndim == 2
        if da and db:
            total += 2 * min(dj * di * dk + dj * dk * dl, di * dk * dl + dj * di * dl)
        elif da:
            total += 2 * dj * di * dk
        elif db:
            total += 2 * di * dk * dl
        else:
            total += 2 * dj * dl
    return int(total)
