"""Exact spin-1/2 XXZ chains assembled by the library's block enlargement.

Alg. 1, steps 1-2: a block grows by one site at a time, its operators being
sums of Kronecker products of the block's and the site's operators
(dmrg_enlarge, on the host, in the enlarged basis the library defines).  A
left block grows to the right (block (x) site) and keeps its last site's
spin operators as coupling operators; a right block grows to the left
(site (x) block) and keeps its first site's.  Eq. 1 with J and Delta:
H = J sum_i [ (S+_i S-_{i+1} + S-_i S+_{i+1}) / 2 + Delta Sz_i Sz_{i+1} ].

Operator order of every block: I, H, S+, S-, Sz (edge site).
"""
from __future__ import annotations

import numpy as np

from . import EnlargedOp, EnlargedSpace, enlarge


class Superblock:
    """An LR superblock (Eq. 9) in the layout every problem description uses."""

    def __init__(self, left, right, target, ops_left, ops_right, terms, coef, name=""):
        self.left, self.right = left, right
        self.target = np.asarray(target, dtype=np.int32)
        self.ops_left, self.ops_right = ops_left, ops_right
        self.terms = np.asarray(terms, dtype=np.int32).reshape(-1, 2)
        self.coef = np.asarray(coef, dtype=np.float64)
        self.name = name


def spin_site():
    """One spin-1/2 site, labels 2 S^z = -1, +1: I, H = 0, S+, S-, Sz (Eq. 3)."""
    space = EnlargedSpace(np.array([[-1], [1]]), np.array([1, 1]))
    one = np.ones((1, 1))
    ops = [EnlargedOp("identity"),
           EnlargedOp("dense", src=np.zeros(0, np.int32), dst=np.zeros(0, np.int32), blocks=[]),
           EnlargedOp("dense", src=np.array([0], np.int32), dst=np.array([1], np.int32), blocks=[one]),
           EnlargedOp("dense", src=np.array([1], np.int32), dst=np.array([0], np.int32), blocks=[one]),
           EnlargedOp("diag", diag=np.array([-0.5, 0.5]))]
    return space, ops


I, H, SP, SM, SZ = range(5)


def grow(block, site, left: bool, J: float = 1.0, delta: float = 1.0):
    """The block enlarged by one site: block (x) site for a left block,
    site (x) block for a right block."""
    (bs, bo), (ss, so) = block, site
    h, z = 0.5 * J, J * delta
    if left:  # slow = block, fast = site; the new edge is the site
        terms = [(0, I, I, 1.0),
                 (1, H, I, 1.0), (1, I, H, 1.0), (1, SP, SM, h), (1, SM, SP, h), (1, SZ, SZ, z),
                 (2, I, SP, 1.0), (3, I, SM, 1.0), (4, I, SZ, 1.0)]
        return enlarge(bs, bo, ss, so, terms, 5)
    # slow = site, fast = block; the new edge is the site
    terms = [(0, I, I, 1.0),
             (1, I, H, 1.0), (1, H, I, 1.0), (1, SP, SM, h), (1, SM, SP, h), (1, SZ, SZ, z),
             (2, SP, I, 1.0), (3, SM, I, 1.0), (4, SZ, I, 1.0)]
    return enlarge(ss, so, bs, bo, terms, 5)


def block(nsites: int, left: bool, J: float = 1.0, delta: float = 1.0):
    """Exact block of `nsites` spins grown one site at a time from a single site."""
    site = spin_site()
    b = site
    for _ in range(nsites - 1):
        b = grow(b, site, left, J, delta)
    return b


def xxz_superblock(n_left: int = 5, n_right: int = 5, J: float = 1.0, delta: float = 1.0) -> Superblock:
    """The open chain of n_left + n_right sites as the superblock of two exact
    blocks (S^z_total = 0): H_L (x) I + I (x) H_R + J/2 (S+ (x) S- + S- (x) S+)
    + J Delta Sz (x) Sz across the cut."""
    L, oL = block(n_left, True, J, delta)
    R, oR = block(n_right, False, J, delta)
    terms = [(H, I), (I, H), (SP, SM), (SM, SP), (SZ, SZ)]
    coef = [1.0, 1.0, 0.5 * J, 0.5 * J, J * delta]
    return Superblock(L, R, [0], oL, oR, terms, coef, name=f"xxz_{n_left}+{n_right}")
