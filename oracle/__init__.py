"""FP64 CPU oracle for the superblock projection and the Davidson ground state.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
baseline leg of the benchmark may import this package.  The product path (the
HIP library and its Python binding) never calls it, and this package shares no
code with that path: it reads the plain arrays produced by ``gen`` and nothing
else.

Modules
-------
models      dense Hamiltonians of whole chains (Eq. 1-8), conserved charges
sectors     brute-force sector bookkeeping: psi layout, dense assembly
projection  y = P_Q (sum_k c_k A_k (x) B_k) P_Q^T psi, by Kronecker products
            (tiny) and by the sector-by-sector form of Eq. 11; the adjoint
davidson    the Davidson iteration of Alg. 3 with the readings listed in the
            design notes; LAPACK/ARPACK ground states for pinning
precision   emulated FP32/BF16 operator rounding with the FP64 diagonal split
density     reduced density matrices of both blocks (Alg. 1, step 5), by pair
            blocks and by the dense partial trace
l11r        the l-1-1-r strategy (Eq. 12-13, Alg. 2): enlarged-basis order,
            four-fold Kronecker definition, sector-wise evaluation, LR form

Every function states the passage of the paper it follows.  Nothing here is
"parity unpinned": each function has at least one independent pin in
``tests/test_oracle_*.py`` (closed forms, brute force, library routines).
"""
from . import models, sectors, projection, davidson, precision, density, l11r  # noqa: F401
