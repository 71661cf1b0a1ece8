"""Reduced density matrices of the two blocks, in FP64 (Alg. 1, step 5).

Test infrastructure (see the package docstring).

After the lowest eigenstate psi of the superblock is found, each block's
density matrix is the partial trace of |psi><psi| over the other block
(Sec. "The DMRG algorithm").  Two independent evaluations are given:

* :func:`density_dense` scatters psi into the full m_L m_R space through the
  brute-force index map and forms rho_L = Psi Psi^T and rho_R = Psi^T Psi
  from the dense [m_L, m_R] coefficient matrix (tiny blocks only);
* :func:`density_sectors` works pair by pair: a left (right) sector meets
  exactly one right (left) sector inside the target Q, so its block of rho_L
  (rho_R) is Psi_p Psi_p^T (Psi_p^T Psi_p) of that pair's row-major block.
"""
from __future__ import annotations

from typing import List, Tuple

import numpy as np

from . import sectors


def density_dense(prob, psi) -> Tuple[np.ndarray, np.ndarray]:
    """Dense rho_L [m_L, m_L] and rho_R [m_R, m_R] of the state psi (psi layout)."""
    lay = sectors.layout(prob.left, prob.right, prob.target)
    mL, mR = prob.left.m, prob.right.m
    full = np.zeros(mL * mR)
    full[lay.index_map] = np.asarray(psi, dtype=np.float64)
    Psi = full.reshape(mL, mR)
    return Psi @ Psi.T, Psi.T @ Psi


def density_sectors(prob, psi) -> Tuple[List[np.ndarray], List[np.ndarray]]:
    """Per pair p of the psi layout: (rho_L block [d_L, d_L], rho_R block [d_R, d_R])."""
    psi = np.asarray(psi, dtype=np.float64)
    table, _ = sectors.pair_table(prob.left, prob.right, prob.target)
    left, right = [], []
    for off, dL, dR in table.values():
        X = psi[off:off + dL * dR].reshape(dL, dR)
        left.append(X @ X.T)
        right.append(X.T @ X)
    return left, right


def eigh_blocks(blocks) -> Tuple[List[np.ndarray], List[np.ndarray]]:
    """Alg. 1, step 6: the eigenvalues (and eigenvectors) of each density-matrix
    block, by LAPACK, in descending order; each eigenvector's first entry of
    largest magnitude is made positive.  Returns (values, vectors) with
    vectors[b][:, j] the eigenvector of values[b][j]."""
    vals, vecs = [], []
    for B in blocks:
        w, U = np.linalg.eigh(np.asarray(B, dtype=np.float64))
        w, U = w[::-1].copy(), U[:, ::-1].copy()
        for j in range(U.shape[1]):
            k = int(np.argmax(np.abs(U[:, j])))
            if U[k, j] < 0:
                U[:, j] = -U[:, j]
        vals.append(w)
        vecs.append(U)
    return vals, vecs


def truncate(values, m: int) -> Tuple[np.ndarray, float]:
    """Alg. 1, step 7: keep the m states of largest density-matrix eigenvalue
    over all sector blocks of one block.  values: per block, the eigenvalues in
    descending order.  Equal values are taken in block order, then in index
    order.  Returns (kept count per block, discarded weight = sum of the
    eigenvalues not kept)."""
    flat = np.concatenate([np.asarray(v, dtype=np.float64) for v in values]) if values else np.zeros(0)
    owner = np.concatenate([np.full(len(v), b) for b, v in enumerate(values)]) if values else np.zeros(0, int)
    order = np.argsort(-flat, kind="stable")
    kept = np.zeros(flat.size, dtype=bool)
    kept[order[:max(0, min(m, flat.size))]] = True
    counts = np.array([int(kept[owner == b].sum()) for b in range(len(values))], dtype=np.int64)
    return counts, float(flat[~kept].sum())


def renormalize_block(O, U_dst, U_src, k_dst: int, k_src: int) -> np.ndarray:
    """Alg. 1, step 7: one operator block in the kept basis,
    U_dst[:, :k_dst]^T O U_src[:, :k_src].  O is a dense [rows, cols] block,
    or a 1-D diagonal (then rows = cols and O stands for diag(O))."""
    O = np.asarray(O, dtype=np.float64)
    if O.ndim == 1:
        O = np.diag(O)
    return U_dst[:, :k_dst].T @ O @ U_src[:, :k_src]


def density_flat(prob, psi) -> Tuple[np.ndarray, np.ndarray]:
    """The blocks of :func:`density_sectors` concatenated in pair order, each
    row-major: the layout of the library's output."""
    left, right = density_sectors(prob, psi)
    cat = lambda bl: np.concatenate([b.reshape(-1) for b in bl]) if bl else np.zeros(0)
    return cat(left), cat(right)
