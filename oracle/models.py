"""Dense Hamiltonians of whole chains, written straight from Eq. 1-8.

Test infrastructure (see the package docstring).  These build the full
2^N (spin) or 4^N (Hubbard) matrices, so they are for N <= ~12 sites.
"""
from __future__ import annotations

import numpy as np

# Eq. 3 — spin-1/2 operators; basis index 0 is S^z = +1/2.
SP = np.array([[0.0, 1.0], [0.0, 0.0]])
SM = np.array([[0.0, 0.0], [1.0, 0.0]])
SZ = np.array([[0.5, 0.0], [0.0, -0.5]])
# Eq. 7-8 — fermionic phase factor and one-mode ladder operators; [1;0] is empty.
PHI = np.array([[1.0, 0.0], [0.0, -1.0]])
CDAG = np.array([[0.0, 0.0], [1.0, 0.0]])
C = np.array([[0.0, 1.0], [0.0, 0.0]])


def site_op(op: np.ndarray, j: int, n: int) -> np.ndarray:
    """Eq. 2: ``op`` on site j (1-based) of an n-site chain, identity elsewhere."""
    left = np.eye(2 ** (j - 1))
    right = np.eye(2 ** (n - j))
    return np.kron(np.kron(left, op), right)


def heisenberg_chain(n: int, delta: float = 1.0, J1=1.0, J2=0.0,
                     end_factor: float = 1.0) -> np.ndarray:
    """Open spin-1/2 chain, Eq. 1, with optional next-nearest S.S couplings.

    H = sum_j J1_j [1/2 (S+_j S-_{j+1} + S-_j S+_{j+1}) + delta S^z_j S^z_{j+1}]
      + sum_j J2   [1/2 (S+_j S-_{j+2} + h.c.) + delta S^z_j S^z_{j+2}]
    ``end_factor`` scales the first and last nearest-neighbour bonds (used for
    the Majumdar-Ghosh point).
    """
    dim = 2 ** n
    H = np.zeros((dim, dim))
    sp = [site_op(SP, j, n) for j in range(1, n + 1)]
    sm = [site_op(SM, j, n) for j in range(1, n + 1)]
    sz = [site_op(SZ, j, n) for j in range(1, n + 1)]

    def bond(i, k, J):
        return J * (0.5 * (sp[i] @ sm[k] + sm[i] @ sp[k]) + delta * (sz[i] @ sz[k]))

    for j in range(n - 1):
        f = end_factor if j in (0, n - 2) else 1.0
        H += bond(j, j + 1, J1 * f)
    if J2:
        for j in range(n - 2):
            H += bond(j, j + 2, J2)
    return H


def total_sz(n: int) -> np.ndarray:
    """Symmetry operator S_z = sum_j S^z_j (Sec. "Symmetries to be exploited")."""
    return sum(site_op(SZ, j, n) for j in range(1, n + 1))


def spin_labels(n: int) -> np.ndarray:
    """2 S^z_total of every product basis state (site 1 is the leading factor)."""
    return np.rint(2 * np.diag(total_sz(n))).astype(np.int64)


def mode_op(op: np.ndarray, k: int, nmodes: int) -> np.ndarray:
    """Eq. 5-6 flattened: phase string Phi on modes before k, ``op`` on mode k."""
    out = np.ones((1, 1))
    for i in range(nmodes):
        out = np.kron(out, PHI if i < k else (op if i == k else np.eye(2)))
    return out


def hubbard_chain(n: int, t: float = 1.0, U: float = 4.0):
    """Spin-1/2 Hubbard chain, Eq. 4 with F = 1/2 (U/2 sum_{s!=s'} n n = U n_up n_dn).

    Mode order follows Eq. 5-6: site by site, within a site polarization
    sigma = -1/2 ("down") before sigma = +1/2 ("up").
    Returns (H, N_up, N_dn) with the number operators of Sec. "Symmetries".
    """
    nm = 2 * n
    cd = [mode_op(CDAG, k, nm) for k in range(nm)]
    cc = [mode_op(C, k, nm) for k in range(nm)]
    dim = 2 ** nm
    H = np.zeros((dim, dim))
    for j in range(n - 1):
        for s in (0, 1):
            a, b = 2 * j + s, 2 * (j + 1) + s
            hop = cd[a] @ cc[b]
            H += -t * (hop + hop.T)
    for j in range(n):
        H += U * (cd[2 * j + 1] @ cc[2 * j + 1]) @ (cd[2 * j] @ cc[2 * j])
    Nup = sum(cd[2 * j + 1] @ cc[2 * j + 1] for j in range(n))
    Ndn = sum(cd[2 * j] @ cc[2 * j] for j in range(n))
    return H, Nup, Ndn


# ---------------------------------------------------------------------------
# closed forms used as pins
# ---------------------------------------------------------------------------


def xx_chain_energy(n: int) -> float:
    """Delta = 0 open chain = free fermions with hopping 1/2: fill the negative
    single-particle levels cos(k pi / (n+1))."""
    k = np.arange(1, n + 1)
    eps = np.cos(k * np.pi / (n + 1))
    return float(eps[eps < 0].sum())


def free_hubbard_energy(n: int, n_up: int, n_dn: int, t: float = 1.0) -> float:
    """U = 0 open Hubbard chain: levels -2t cos(k pi/(n+1)), filled per spin."""
    k = np.arange(1, n + 1)
    eps = np.sort(-2 * t * np.cos(k * np.pi / (n + 1)))
    return float(eps[:n_up].sum() + eps[:n_dn].sum())


def hubbard_dimer_energy(t: float, U: float) -> float:
    """Two-site Hubbard model at half filling: (U - sqrt(U^2 + 16 t^2)) / 2."""
    return 0.5 * (U - np.sqrt(U * U + 16 * t * t))


def chain_ground_energy(n: int, delta: float = 1.0) -> float:
    """Lowest energy of the open Heisenberg chain of Eq. 1 in the S^z = 0 sector,
    by LAPACK on the dense sector block (n <= 14)."""
    H = heisenberg_chain(n, delta)
    idx = np.flatnonzero(spin_labels(n) == 0)
    return float(np.linalg.eigvalsh(H[np.ix_(idx, idx)])[0])


def hulthen_energy_per_site() -> float:
    """Ground-state energy per site of the infinite spin-1/2 Heisenberg chain
    (J = 1, Delta = 1), Hulthen's Bethe-ansatz result 1/4 - ln 2."""
    return 0.25 - float(np.log(2.0))


def majumdar_ghosh_energy(n: int, J1: float = 1.0) -> float:
    """J2 = J1/2 open chain with halved end bonds: sum of triangle projectors,
    ground energy -3 J1 (n - 2) / 8 (dimer states)."""
    return -3.0 * J1 * (n - 2) / 8.0
