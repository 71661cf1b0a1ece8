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


@dataclass
class BlockResult:
    energies: np.ndarray      # [nroots] ascending
    X: np.ndarray             # [n, nroots] Ritz vectors (orthonormal)
    iterations: int
    projections: int
    residuals: np.ndarray     # [nroots]
    converged: bool
    restarts: int = 0


def block_davidson(matvec: Callable[[np.ndarray], np.ndarray], D: np.ndarray, X0: np.ndarray,
                   tol: float = 1e-10, kmax: int = 32, kmin: int = 0, max_iter: int = 500,
                   floor: float = 1e-3, drop: float = 1e-8) -> BlockResult:
    """Block Davidson-Liu iteration for the b = X0.shape[1] lowest eigenpairs
    (the block version named in Sec. "Runtime & Parallelism"; Liu's method adds
    one corrected residual per unconverged root per iteration, so the products
    with H and the Gram-Schmidt steps act on blocks of vectors).

    Readings (the paper gives only the name): the b start columns are
    orthonormalized; each iteration takes the b lowest Ritz pairs (theta_j,
    x_j) of B = V^T H V (LAPACK eigh) and their residuals r_j = H x_j -
    theta_j x_j; the run stops when every ||r_j|| <= tol; otherwise every root
    with ||r_j|| > tol contributes t_j = r_j / (D - sigma_j), sigma_j =
    min(theta_j, min D) for the lowest root (the single-vector reading) and
    theta_j for the others, |D - sigma_j| floored at ``floor`` with its sign;
    the corrections are orthogonalized against V by two classical passes and
    among themselves in order (modified Gram-Schmidt, a second pass, a vector
    keeping less than ``drop`` of its norm is discarded), and appended with
    their products H t.  Thick restart: when they would not fit in kmax, V
    and HV are replaced by the kkeep = max(kmin, 2 b) lowest Ritz vectors
    first.  ``matvec`` takes and returns an [n, p] block."""
    n, b = X0.shape
    kmax = max(2 * b, min(kmax, n))
    kkeep = min(max(kmin, 2 * b), kmax - b)
    V = np.zeros((n, kmax))
    W = np.zeros((n, kmax))
    Q, _ = np.linalg.qr(np.asarray(X0, dtype=np.float64))
    V[:, :b] = Q
    W[:, :b] = matvec(Q)
    nproj = b
    k = b
    restarts = 0
    dmin = float(D.min())
    for it in range(1, max_iter + 1):
        Bm = V[:, :k].T @ W[:, :k]
        Bm = 0.5 * (Bm + Bm.T)
        theta, Y = np.linalg.eigh(Bm)
        X = V[:, :k] @ Y[:, :b]
        R = W[:, :k] @ Y[:, :b] - X * theta[:b]
        rn = np.linalg.norm(R, axis=0)
        if np.all(rn <= tol) or k == n:
            return BlockResult(theta[:b].copy(), X, it, nproj, rn, bool(np.all(rn <= tol)), restarts)
        T = []
        for j in range(b):
            if rn[j] <= tol:
                continue
            sig = min(theta[j], dmin) if j == 0 else theta[j]
            den = D - sig
            small = np.abs(den) < floor
            den[small] = np.where(den[small] < 0, -floor, floor)
            T.append(R[:, j] / den)
        T = np.array(T).T
        if k + T.shape[1] > kmax:
            V[:, :kkeep] = V[:, :k] @ Y[:, :kkeep]
            W[:, :kkeep] = W[:, :k] @ Y[:, :kkeep]
            k = kkeep
            restarts += 1
        for _ in range(2):  # against the basis, two classical passes
            T = T - V[:, :k] @ (V[:, :k].T @ T)
        new = []
        for j in range(T.shape[1]):  # among themselves, in order
            t = T[:, j].copy()
            n0 = np.linalg.norm(t)
            for _ in range(2):
                for q in new:
                    t -= (q @ t) * q
            n1 = np.linalg.norm(t)
            if n1 > drop * n0 and n0 > 0:
                new.append(t / n1)
        if not new:
            return BlockResult(theta[:b].copy(), X, it, nproj, rn, False, restarts)
        Tn = np.array(new).T
        V[:, k:k + Tn.shape[1]] = Tn
        W[:, k:k + Tn.shape[1]] = matvec(Tn)
        nproj += Tn.shape[1]
        k += Tn.shape[1]
    return BlockResult(theta[:b].copy(), X, max_iter, nproj, rn, False, restarts)


def lowest_block_davidson(prob, X0, coef=None, **kw) -> BlockResult:
    """block_davidson on a superblock through the sector-form projection."""
    coef = prob.coef if coef is None else np.asarray(coef, dtype=np.float64)
    D = projection.diagonal(prob, coef)

    def mv(X):
        return np.stack([projection.project_sectors(prob, X[:, j], coef) for j in range(X.shape[1])], axis=1)

    return block_davidson(mv, D, np.asarray(X0, dtype=np.float64), **kw)


def lowest_arpack(prob, k: int, coef=None, tol: float = 1e-13):
    """The k lowest eigenvalues of H_Q by ARPACK (no Davidson code)."""
    from scipy.sparse.linalg import LinearOperator, eigsh

    coef = prob.coef if coef is None else np.asarray(coef, dtype=np.float64)
    _, n = projection.sectors.pair_table(prob.left, prob.right, prob.target)
    op = LinearOperator((n, n), matvec=lambda v: projection.project_sectors(prob, v, coef), dtype=np.float64)
    w = eigsh(op, k=k, which="SA", tol=tol, ncv=max(40, 4 * k), maxiter=20000, return_eigenvectors=False)
    return np.sort(w)


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
