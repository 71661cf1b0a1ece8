"""Seeded synthetic workloads for the superblock projection and Davidson solver.

This package only *draws inputs*: symmetry-sector tables, block operators in
sector form, term lists, coefficients and random start vectors.  It contains
none of the projection or eigensolver arithmetic and imports neither the HIP
library nor the oracle; both sides receive the same plain NumPy arrays from it.

Conventions (the paper's LR strategy, Eq. 9-11):

* A *space* is a block basis grouped by U(1) symmetry sectors.  ``labels`` is an
  int32 array ``[nsec, rank]`` in strictly ascending lexicographic order and
  ``dims`` an int64 array ``[nsec]`` (zero-dimension sectors are allowed).
* An *operator* is block-sparse in that basis (Sec. "Symmetries to be
  exploited" and Eq. 11: dense matrices A_{q_i -> q_j}).  Kinds:

  - ``identity``: the identity on the whole block;
  - ``diag``: a diagonal operator given as one length-m vector in sector order;
  - ``dense``: a list of blocks ``(src, dst, M)`` with ``M`` row-major of shape
    ``[dims[dst], dims[src]]``.

* A *term* ``(c, a, b)`` stands for ``c * A_a (x) B_b`` with ``A_a`` from the
  left operator list and ``B_b`` from the right one (Eq. 9).
* A four-subsystem superblock (Sec. "l-1-1-r strategy", :class:`Problem4`)
  has one space and operator list per subsystem (block l, site 1, site 2,
  block r) and terms ``(c, a, b, c', d)`` for c * A_a (x) a_b (x) b_c' (x) B_d.
"""
from .workloads import (  # noqa: F401
    Space,
    Operator,
    Problem,
    Problem4,
    largest_remainder,
    heisenberg_exact,
    hubbard_exact,
    heisenberg_synthetic,
    hubbard_synthetic,
    j1j2_synthetic,
    batched_heisenberg,
    random_problem,
    random_problem4,
    spin_site,
    hubbard_site,
    heisenberg_l11r,
    hubbard_l11r_exact,
    hubbard_l11r_synthetic,
    start_vector,
    config,
    CONFIG_NAMES,
)
