"""Davidson iteration (Alg. 3) and reference ground states, FP64.

Test infrastructure (see the package docstring).

Davidson's method as the paper states it (Alg. 3): the basis V grows by one
vector per iteration; its projections W = H V and the Rayleigh matrix
B = V^T W give the smallest Ritz pair (lambda, y), the Ritz vector x = V y and
the residual r = W y - lambda x; the run stops once r is small, otherwise the
corrected residual is orthogonalized against V, normalized and appended.  The
paper leaves several points open; this oracle takes these readings (the HIP
solver takes the same):

* "correct r": shifted diagonal (Davidson) preconditioner
  t_i = r_i / (D_ii - sigma) with D = diag(H_Q) and sigma = min(lambda, min_i D_ii),
  so the preconditioner stays positive definite while lambda lies inside the
  range of the diagonal; where |D_ii - sigma| < floor (default 1e-3) the
  denominator is +-floor with its sign (zero counts as positive).  Without the
  shift a random start on a nearly diagonal H can lose the ground state across
  restarts; without the floor, once lambda sits just below an isolated
  diagonal entry the corrected vector is nearly parallel to x and the
  iteration stagnates after orthogonalization;
* Gram-Schmidt: classical, repeated once more (DGKS) when the norm drops
  below 1/sqrt(2) of its value before the pass; breakdown when the norm
  falls below 1e-13 of the pre-orthogonalization norm;
* "norm(r) ~ 0": ||r||_2 <= tol with ||x||_2 = 1;
* subspace limit k_max (the paper's runs use 20; default 32 here) with a
  thick restart to the k_min lowest Ritz vectors: V <- V Y, W <- W Y,
  B <- diag(theta), before the correction vector is appended;
* the small eigenproblem is solved by LAPACK (``numpy.linalg.eigh``).

An "iteration" is one Ritz evaluation (Rayleigh matrix column, small
eigenproblem, Ritz vector, residual, stop test); the number of projections is
one more than the number of appended vectors.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Callable, List

import numpy as np

from . import projection


@dataclass
class DavidsonResult:
    energy: float
    x: np.ndarray
    iterations: int
    projections: int
    residual: float
    converged: bool
    breakdown: bool = False
    restarts: int = 0
    history: List[float] = field(default_factory=list)


def davidson(matvec: Callable[[np.ndarray], np.ndarray], D: np.ndarray, x0: np.ndarray,
             tol: float = 1e-10, kmax: int = 32, kmin: int = 8, max_iter: int = 500,
             floor: float = 1e-3) -> DavidsonResult:
    n = x0.shape[0]
    kmax = max(2, min(kmax, n))
    kmin = max(1, min(kmin, kmax - 1))
    V = np.zeros((n, kmax))
    W = np.zeros((n, kmax))
    Bm = np.zeros((kmax, kmax))
    V[:, 0] = x0 / np.linalg.norm(x0)
    W[:, 0] = matvec(V[:, 0])
    nproj = 1
    i = 1  # current subspace size
    Bm[0, 0] = V[:, 0] @ W[:, 0]
    hist = []
    restarts = 0
    dmin = float(D.min())
    for it in range(1, max_iter + 1):
        # Rayleigh-Ritz: smallest eigenpair of B restricted to the current basis
        theta, Y = np.linalg.eigh(Bm[:i, :i])
        lam, y = theta[0], Y[:, 0]
        # Ritz vector and its residual
        x = V[:, :i] @ y
        r = W[:, :i] @ y - lam * x
        rn = float(np.linalg.norm(r))
        hist.append(rn)
        if rn <= tol:  # converged
            return DavidsonResult(lam, x, it, nproj, rn, True, restarts=restarts, history=hist)
        if i == n:
            return DavidsonResult(lam, x, it, nproj, rn, False, restarts=restarts, history=hist)
        # preconditioned correction of the residual
        den = D - min(lam, dmin)
        small = np.abs(den) < floor
        den[small] = np.where(den[small] < 0, -floor, floor)
        t = r / den
        # thick restart before appending
        if i == kmax:
            keep = kmin
            V[:, :keep] = V[:, :i] @ Y[:, :keep]
            W[:, :keep] = W[:, :i] @ Y[:, :keep]
            Bm[:, :] = 0.0
            Bm[:keep, :keep] = np.diag(theta[:keep])
            i = keep
            restarts += 1
        # orthonormalize the correction against V (CGS, DGKS repeat) and append it
        n0 = np.linalg.norm(t)
        s = V[:, :i].T @ t
        t = t - V[:, :i] @ s
        n1 = np.linalg.norm(t)
        if n1 < n0 / np.sqrt(2.0):
            s = V[:, :i].T @ t
            t = t - V[:, :i] @ s
            n1 = np.linalg.norm(t)
        if n1 <= 1e-13 * n0:
            return DavidsonResult(lam, x, it, nproj, rn, False, breakdown=True,
                                  restarts=restarts, history=hist)
        V[:, i] = t / n1
        # project the new basis vector and extend B by its column
        W[:, i] = matvec(V[:, i])
        nproj += 1
        col = V[:, :i + 1].T @ W[:, i]
        Bm[:i + 1, i] = col
        Bm[i, :i + 1] = col
        i += 1
    return DavidsonResult(lam, x, max_iter, nproj, rn, False, restarts=restarts, history=hist)


def ground_state_davidson(prob, x0, coef=None, **kw) -> DavidsonResult:
    coef = prob.coef if coef is None else np.asarray(coef, dtype=np.float64)
    D = projection.diagonal(prob, coef)
    return davidson(lambda v: projection.project_sectors(prob, v, coef), D,
                    np.asarray(x0, dtype=np.float64), **kw)


def ground_state_dense(prob, coef=None):
    """Lowest eigenpair of the dense H_Q by LAPACK (tiny problems)."""
    w, U = np.linalg.eigh(projection.projected_hamiltonian(prob, coef))
    return float(w[0]), U[:, 0], w


def ground_state_arpack(prob, coef=None, tol: float = 1e-13, v0=None):
    """Lowest eigenpair of H_Q by ARPACK's implicitly restarted Lanczos, with the
    sector-form projection as the only access to H (no Davidson code)."""
    from scipy.sparse.linalg import LinearOperator, eigsh

    coef = prob.coef if coef is None else np.asarray(coef, dtype=np.float64)
    _, n = projection.sectors.pair_table(prob.left, prob.right, prob.target)
    op = LinearOperator((n, n), matvec=lambda v: projection.project_sectors(prob, v, coef),
                        dtype=np.float64)
    w, U = eigsh(op, k=1, which="SA", tol=tol, v0=v0, ncv=40, maxiter=20000)
    return float(w[0]), U[:, 0]


def fix_sign(x: np.ndarray) -> np.ndarray:
    """Eigenvector sign convention: the first largest-magnitude entry is positive."""
    k = int(np.argmax(np.abs(x)))
    return x if x[k] >= 0 else -x
