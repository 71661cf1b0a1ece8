"""The infinite-lattice DMRG iteration (Alg. 1) on the device, every step
through the C ABI, against exact diagonalization and closed forms.

* Without truncation (m above the block dimension) the enlarged block is the
  exact chain in a rotated basis: its Hamiltonian has the chain's spectrum
  (LAPACK on the dense chain of Eq. 1), and the superblock energies equal the
  exact ground energies.
* The XX chain (Delta = 0) has the free-fermion ground energy.
* With truncation the energy per site from the last two growth steps
  approaches Hulthen's 1/4 - ln 2.
"""
import numpy as np
import pytest

from oracle import models

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _inf():
    from paper_1309_5571_amd import infinite

    return infinite


def _dense_h(E):
    """The enlarged block's Hamiltonian assembled on the host from its device blocks."""
    off = np.concatenate([[0], np.cumsum(E.dims)])
    m = int(off[-1])
    H = np.zeros((m, m))
    op = E.ops["H"]
    data = op.device_data.cpu().numpy()
    for a, b, o in zip(op.src, op.dst, op.off):
        r, c = int(E.dims[b]), int(E.dims[a])
        H[off[b]:off[b] + r, off[a]:off[a] + c] = data[o:o + r * c].reshape(r, c)
    return H


def test_enlarged_block_spectrum_matches_exact_chain():
    inf = _inf()
    from paper_1309_5571_amd import Plan

    dev = torch.device("cuda", 0)
    B = inf.site_block(dev)
    for _ in range(5):
        E = inf.enlarge(B)
        H = _dense_h(E)
        np.testing.assert_allclose(H, H.T, atol=1e-13)
        want = np.linalg.eigvalsh(models.heisenberg_chain(E.nsites))
        np.testing.assert_allclose(np.linalg.eigvalsh(H), want, atol=1e-10)
        plan = Plan(inf.superblock(E), device=dev, tiles=None)
        x0 = torch.from_numpy(np.random.default_rng(1).standard_normal(plan.n)).to(dev)
        psi, _, infos, st = plan.davidson(x0, tol=1e-11, kmax=min(32, plan.n), kmin=min(8, plan.n - 1))
        assert infos[0]["converged"]
        B, disc, kept = inf.renormalize_block(E, plan, psi, 1 << 20)  # keep everything
        assert kept == int(E.dims.sum()) and abs(disc) < 1e-12
        plan.close()


def test_infinite_dmrg_is_exact_without_truncation():
    res = _inf().run(12, m=64, tol=1e-11)
    assert [r.nsites for r in res] == [4, 6, 8, 10, 12]
    for r in res:
        assert r.energy == pytest.approx(models.chain_ground_energy(r.nsites), abs=1e-9)


def test_infinite_dmrg_xx_chain_free_fermions():
    res = _inf().run(24, m=64, delta=0.0, tol=1e-11)
    for r in res:
        assert r.energy == pytest.approx(models.xx_chain_energy(r.nsites), abs=1e-5)


def test_infinite_dmrg_approaches_hulthen():
    res = _inf().run(100, m=32, tol=1e-10)
    e = [r.energy for r in res]
    assert res[-1].nsites == 100
    per_site = (e[-1] - e[-2]) / 2
    assert abs(per_site - models.hulthen_energy_per_site()) < 2e-3
    # the discarded weight stays small and every step keeps m states once the block is larger
    assert max(r.discarded for r in res) < 1e-3
    assert all(r.kept == 32 for r in res[5:])


@pytest.mark.parametrize("delta", [0.5, 2.0])
def test_infinite_dmrg_anisotropic_chain_is_exact(delta):
    """The Sz Sz coupling enters through its own placement call: XXZ chains
    without truncation equal their exact ground energies."""
    res = _inf().run(10, m=64, delta=delta, tol=1e-11)
    for r in res:
        assert r.energy == pytest.approx(models.chain_ground_energy(r.nsites, delta), abs=1e-9)


def test_infinite_dmrg_energy_scales_with_coupling():
    """H is linear in J: the same growth with J = 2 doubles every energy."""
    a = _inf().run(16, m=16, tol=1e-11)
    b = _inf().run(16, m=16, J=2.0, tol=1e-11)
    for x, y in zip(a, b):
        assert y.energy == pytest.approx(2.0 * x.energy, abs=1e-8)
        assert y.discarded == pytest.approx(x.discarded, abs=1e-9)


def test_finite_sweeps_exact_without_truncation():
    """Finite-lattice sweeps (right blocks renormalized from rho_R) keep the
    exact ground energy when nothing is truncated."""
    grow, mid = _inf().run_finite(10, m=64, sweeps=1, tol=1e-11)
    assert grow[-1].nsites == 10
    exact = models.chain_ground_energy(10)
    assert grow[-1].energy == pytest.approx(exact, abs=1e-9)
    assert mid[-1] == pytest.approx(exact, abs=1e-9)


def test_finite_sweeps_improve_the_truncated_xx_chain():
    """With truncation the sweeps lower the energy towards the exact
    free-fermion value and never below it (variational); consecutive sweeps
    agree to the truncation level (with m fixed they need not decrease)."""
    grow, mid = _inf().run_finite(20, m=10, sweeps=2, delta=0.0, tol=1e-11)
    exact = models.xx_chain_energy(20)
    e_inf = grow[-1].energy
    assert grow[-1].nsites == 20
    assert all(e >= exact - 1e-9 for e in [e_inf] + mid)
    assert abs(mid[-1] - exact) < abs(e_inf - exact)
    assert abs(mid[-1] - mid[0]) < 1e-5
