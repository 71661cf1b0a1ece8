"""Pins of the oracle's Davidson solver (Alg. 3) and its energy gradients."""
import json
import os

import numpy as np
import pytest

import gen
from oracle import davidson, models, projection, sectors

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "exact_energies.json")))["energies"]
ARPACK = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "arpack_energies.json")))["energies"]


def _n(p):
    return sectors.pair_table(p.left, p.right, p.target)[1]


def test_exact_ten_site_chain_random_start():
    """Config 1: Davidson from a seeded random start reaches the exact energy."""
    p = gen.config(1)
    r = davidson.ground_state_davidson(p, gen.start_vector(_n(p), 3), tol=1e-12)
    assert r.converged
    assert r.energy == pytest.approx(GOLDEN["heisenberg_open_N10_Sz0"], abs=1e-10)
    E, x, _ = davidson.ground_state_dense(p)
    assert abs(abs(r.x @ x) - 1.0) <= 1e-10


def test_xx_chain_through_lr_blocks():
    p = gen.heisenberg_exact(5, 5, delta=0.0)
    r = davidson.ground_state_davidson(p, gen.start_vector(_n(p), 4), tol=1e-11)
    assert r.converged
    assert r.energy == pytest.approx(models.xx_chain_energy(10), abs=1e-10)


def test_hubbard_lr_blocks_dimer_and_free_limit():
    p = gen.hubbard_exact(1, 1, t=1.0, U=4.0)
    r = davidson.ground_state_davidson(p, gen.start_vector(_n(p), 5), tol=1e-11)
    assert r.energy == pytest.approx(models.hubbard_dimer_energy(1.0, 4.0), abs=1e-10)
    q = gen.hubbard_exact(2, 2, t=1.0, U=0.0)
    r = davidson.ground_state_davidson(q, gen.start_vector(_n(q), 6), tol=1e-11)
    assert r.energy == pytest.approx(models.free_hubbard_energy(4, 2, 2), abs=1e-10)


@pytest.mark.parametrize("maker,m,seed", [(gen.heisenberg_synthetic, 64, 11), (gen.heisenberg_synthetic, 96, 5),
                                          (gen.hubbard_synthetic, 64, 2), (gen.j1j2_synthetic, 64, 8)])
def test_synthetic_matches_lapack(maker, m, seed):
    p = maker(m, seed=seed)
    E, x, w = davidson.ground_state_dense(p)
    r = davidson.ground_state_davidson(p, gen.start_vector(_n(p), seed + 2), tol=1e-10)
    assert r.converged
    assert abs(r.energy - E) <= 1e-10
    if w[1] - w[0] > 1e-6:
        assert abs(abs(r.x @ x) - 1.0) <= 1e-10


def test_restart_path():
    """A tiny subspace limit forces many thick restarts; the result is unchanged."""
    p = gen.config(1)
    x0 = gen.start_vector(_n(p), 3)
    r = davidson.ground_state_davidson(p, x0, tol=1e-11, kmax=5, kmin=2, max_iter=2000)
    assert r.converged and r.restarts > 0
    assert r.energy == pytest.approx(GOLDEN["heisenberg_open_N10_Sz0"], abs=1e-10)


def test_not_converged_flag():
    p = gen.config(1)
    r = davidson.ground_state_davidson(p, gen.start_vector(_n(p), 3), tol=1e-12, max_iter=1)
    assert not r.converged and r.iterations == 1


def test_exact_eigenvector_start_converges_immediately():
    p = gen.config(1)
    E, x, _ = davidson.ground_state_dense(p)
    r = davidson.ground_state_davidson(p, x, tol=1e-12)
    assert r.converged and r.iterations == 1 and r.energy == pytest.approx(E, abs=1e-13)


def test_degenerate_majumdar_ghosh_energy_only():
    """J1-J2 at J2 = J1/2 with halved end bonds: degenerate dimer ground states;
    only the energy is unique."""
    n = 8
    H = models.heisenberg_chain(n, J1=1.0, J2=0.5, end_factor=0.5)
    idx = np.flatnonzero(models.spin_labels(n) == 0)
    HQ = H[np.ix_(idx, idx)]
    x0 = gen.start_vector(len(idx), 1)
    r = davidson.davidson(lambda v: HQ @ v, np.diag(HQ).copy(), x0, tol=1e-11)
    assert r.converged
    assert r.energy == pytest.approx(models.majumdar_ghosh_energy(n), abs=1e-10)
    assert np.linalg.norm(HQ @ r.x - r.energy * r.x) <= 1e-10


@pytest.mark.slow
def test_hubbard_m2048_matches_arpack():
    """The Hubbard m=2048 workload: Davidson vs ARPACK Lanczos (no shared code)."""
    p = gen.config(3)
    r = davidson.ground_state_davidson(p, gen.start_vector(_n(p), 7), tol=1e-10)
    E, _ = davidson.ground_state_arpack(p, tol=1e-15)
    assert r.converged
    assert abs(r.energy - E) <= 1e-10
    assert abs(ARPACK[gen.CONFIG_NAMES[3]] - E) <= 1e-10


@pytest.mark.parametrize("cfg", [2, 5])
def test_synthetic_m1024_matches_arpack(cfg):
    """Heisenberg m=1024 and J1-J2 m=1024: the oracle's Davidson vs ARPACK
    Lanczos run live on the oracle projection (no shared solver code), and
    both vs the stored ARPACK energy the GPU tests compare with."""
    p = gen.config(cfg)
    r = davidson.ground_state_davidson(p, gen.start_vector(_n(p), 7), tol=1e-10)
    E, x = davidson.ground_state_arpack(p, tol=1e-15)
    assert r.converged
    assert abs(r.energy - E) <= 1e-10
    assert abs(abs(r.x @ x) - 1.0) <= 1e-10
    assert abs(ARPACK[gen.CONFIG_NAMES[cfg]] - E) <= 1e-10


def test_hellmann_feynman_two_site():
    # H = J S1.S2 -> E = -3J/4, dE/dJ = -3/4 = <psi| dH/dJ |psi>
    p = gen.heisenberg_exact(1, 1, J=1.3)
    E, x, _ = davidson.ground_state_dense(p)
    assert E == pytest.approx(-0.75 * 1.3, abs=1e-14)
    dc = projection.coef_gradient(p, x, x)  # dE/dc_k for normalized x
    dcdJ = np.array([0.0, 0.0, 0.5, 0.5, 1.0])  # coef = (1, 1, J/2, J/2, J Delta)
    assert dc @ dcdJ == pytest.approx(-0.75, abs=1e-13)


def test_hellmann_feynman_matches_finite_differences_j1j2():
    p = gen.j1j2_synthetic(64, seed=3)
    basis = p.meta["coef_basis"]
    E, x, _ = davidson.ground_state_dense(p)
    dc = projection.coef_gradient(p, x, x)
    g = basis.T @ dc  # (d/dconst, dE/dJ1, dE/dJ2)
    h = 1e-5
    for j in (1, 2):
        e = np.zeros(3)
        e[j] = h
        Ep = davidson.ground_state_dense(p, basis @ (np.array([1.0, 1.0, 0.5]) + e))[0]
        Em = davidson.ground_state_dense(p, basis @ (np.array([1.0, 1.0, 0.5]) - e))[0]
        assert g[j] == pytest.approx((Ep - Em) / (2 * h), rel=1e-7, abs=1e-9)


# ------------------------------------------------------------------ block Davidson-Liu


@pytest.mark.parametrize("b", [1, 2, 4])
def test_block_davidson_ten_site_chain_lapack(b):
    """The b lowest eigenpairs of the exact 10-site chain: LAPACK's eigenvalues,
    orthonormal Ritz vectors, residuals measured by the projection."""
    p = gen.config(1)
    n = _n(p)
    X0 = np.random.default_rng(b).standard_normal((n, b))
    r = davidson.lowest_block_davidson(p, X0, tol=1e-10)
    assert r.converged
    w = np.linalg.eigvalsh(projection.projected_hamiltonian(p))[:b]
    assert np.max(np.abs(r.energies - w)) <= 1e-10
    assert np.allclose(r.X.T @ r.X, np.eye(b), atol=1e-12)
    for j in range(b):
        res = projection.project_sectors(p, r.X[:, j]) - r.energies[j] * r.X[:, j]
        assert np.linalg.norm(res) <= 2e-10


def test_block_davidson_small_synthetic_lapack():
    p = gen.heisenberg_synthetic(96, seed=3)
    n = _n(p)
    r = davidson.lowest_block_davidson(p, np.random.default_rng(0).standard_normal((n, 3)), tol=1e-10, kmax=18)
    assert r.converged and r.restarts >= 1
    w = np.linalg.eigvalsh(projection.projected_hamiltonian(p))[:3]
    assert np.max(np.abs(r.energies - w)) <= 1e-10


def test_block_of_one_is_the_single_vector_method():
    p = gen.config(1)
    x0 = gen.start_vector(_n(p), 3)
    a = davidson.ground_state_davidson(p, x0, tol=1e-11)
    b = davidson.lowest_block_davidson(p, x0[:, None], tol=1e-11)
    assert a.converged and b.converged
    assert abs(a.energy - b.energies[0]) <= 1e-12


@pytest.mark.slow
def test_block_davidson_hubbard_m2048_arpack():
    """The four lowest energies of the Hubbard m=2048 workload: block
    Davidson-Liu vs the stored ARPACK values (tests/golden/make_golden.py)."""
    p = gen.config(3)
    n = _n(p)
    r = davidson.lowest_block_davidson(p, np.random.default_rng(1).standard_normal((n, 4)), tol=1e-10)
    assert r.converged
    ref = np.array(ARPACK["hubbard_m2048_lowest4"])
    assert np.max(np.abs(r.energies - ref)) <= 1e-10
