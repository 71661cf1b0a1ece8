"""Sector bookkeeping for the oracle, done by brute force.

Test infrastructure (see the package docstring).

The target-sector state psi is laid out as follows (the paper leaves the order
open; Eq. 10-11 only fix that each segment X_ik is a row-major reshaped block):
left sectors ascend lexicographically by label, each block basis is grouped by
sector in that order, and psi is the concatenation, over left sectors in
ascending order, of the row-major blocks [d_L(q_L), d_R(Q - q_L)] whose two
dimensions are both non-zero.  With that layout the full-space index
(off_L + a) * m_R + off_R + b of consecutive psi entries is strictly
increasing, so the layout is exactly "all full-space basis pairs whose labels
add up to Q, in increasing order" -- which is what :func:`layout` enumerates.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import Dict, List, Tuple

import numpy as np


def basis_labels(space) -> np.ndarray:
    """Label of every basis state of a block, ``[m, rank]`` (sector-grouped basis)."""
    return np.repeat(space.labels, space.dims, axis=0)


def basis_sector(space) -> np.ndarray:
    """Sector index of every basis state."""
    return np.repeat(np.arange(space.nsec), space.dims)


@dataclass
class Layout:
    index_map: np.ndarray  # int64 [n] full-space index a * m_R + b of each psi entry
    pairs: List[Tuple[int, int]]  # (left sector, right sector), in psi order
    pair_offset: np.ndarray  # int64 [npair + 1]
    n: int


def layout(L, R, Q) -> Layout:
    """Brute force over all m_L * m_R basis pairs (Sec. "Symmetries", Eq. 11)."""
    Q = np.asarray(Q, dtype=np.int64).reshape(-1)
    labL = basis_labels(L).astype(np.int64)
    labR = basis_labels(R).astype(np.int64)
    mL, mR = labL.shape[0], labR.shape[0]
    hit = np.ones((mL, mR), dtype=bool)
    for c in range(Q.shape[0]):
        hit &= (labL[:, c][:, None] + labR[:, c][None, :]) == Q[c]
    idx = np.flatnonzero(hit.reshape(-1)).astype(np.int64)
    secL = basis_sector(L)[idx // mR] if mR else np.zeros(0, dtype=np.int64)
    secR = basis_sector(R)[idx % mR] if mR else np.zeros(0, dtype=np.int64)
    pairs: List[Tuple[int, int]] = []
    starts = []
    for pos in range(idx.shape[0]):
        key = (int(secL[pos]), int(secR[pos]))
        if not pairs or pairs[-1] != key:
            if key in pairs:
                raise AssertionError("pair blocks are not contiguous")
            pairs.append(key)
            starts.append(pos)
    off = np.array(starts + [idx.shape[0]], dtype=np.int64)
    return Layout(idx, pairs, off, int(idx.shape[0]))


def pair_table(L, R, Q) -> Tuple[Dict[Tuple[int, int], Tuple[int, int, int]], int]:
    """(left sector, right sector) -> (offset, d_L, d_R), built the direct way:
    for every left sector in ascending order, the right sector whose label
    completes Q, both non-empty."""
    Q = np.asarray(Q, dtype=np.int64).reshape(-1)
    table = {}
    off = 0
    for sL in range(L.nsec):
        want = Q - L.labels[sL].astype(np.int64)
        sR = -1
        for r in range(R.nsec):
            if np.array_equal(R.labels[r].astype(np.int64), want):
                sR = r
                break
        if sR < 0:
            continue
        dL, dR = int(L.dims[sL]), int(R.dims[sR])
        if dL == 0 or dR == 0:
            continue
        table[(sL, sR)] = (off, dL, dR)
        off += dL * dR
    return table, off


def dense_operator(space, op) -> np.ndarray:
    """Assemble a sector-form operator into its dense m x m matrix (Eq. 11's
    A_{q_i -> q_j} blocks placed at rows of q_j and columns of q_i)."""
    m = space.m
    if op.kind == "identity":
        return np.eye(m)
    if op.kind == "diag":
        return np.diag(op.diag)
    off = space.offsets()
    M = np.zeros((m, m))
    seen = set()
    for s, d, blk in zip(op.src, op.dst, op.blocks):
        key = (int(s), int(d))
        if key in seen:
            raise ValueError("duplicate block")
        seen.add(key)
        M[off[d]:off[d + 1], off[s]:off[s + 1]] = blk
    return M
