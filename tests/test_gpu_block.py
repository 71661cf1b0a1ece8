"""Block Davidson-Liu on the device (dmrg_block_davidson): the b lowest
eigenpairs against LAPACK, the stored ARPACK energies and the oracle's block
solver."""
import json
import os

import numpy as np
import pytest

import gen
from oracle import davidson as odav
from oracle import l11r, projection, sectors

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

ARPACK = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "arpack_energies.json")))["energies"]


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _n(p):
    return sectors.pair_table(p.left, p.right, p.target)[1]


def _start(b, n, seed):
    return np.random.default_rng(seed).standard_normal((b, n))


def _check_vectors(p, X, E, tol):
    b = X.shape[0]
    assert np.allclose(X @ X.T, np.eye(b), atol=1e-10)
    for j in range(b):
        r = projection.project_sectors(p, X[j]) - E[j] * X[j]
        assert np.linalg.norm(r) <= tol


@pytest.mark.parametrize("b", [1, 2, 4])
def test_ten_site_chain_lapack(b):
    import paper_1309_5571_amd as dm

    p = gen.config(1)
    pl = dm.Plan(p)
    print(f"block davidson ten-site b={b}", flush=True)
    X, E, R, info, st = pl.block_davidson(torch.from_numpy(_start(b, pl.n, b)).cuda(), tol=1e-10)
    assert st == 0 and info["converged"] == 1, info
    w = np.linalg.eigvalsh(projection.projected_hamiltonian(p))[:b]
    assert np.max(np.abs(E - w)) <= 1e-10
    assert np.all(R <= 1e-10)
    _check_vectors(p, X.cpu().numpy(), E, 2e-10)
    pl.close()


def test_restarts_small_basis():
    import paper_1309_5571_amd as dm

    p = gen.heisenberg_synthetic(96, seed=3)
    pl = dm.Plan(p)
    X, E, R, info, st = pl.block_davidson(torch.from_numpy(_start(3, pl.n, 0)).cuda(), tol=1e-10, kmax=9)
    assert st == 0 and info["restarts"] >= 1, info
    w = np.linalg.eigvalsh(projection.projected_hamiltonian(p))[:3]
    assert np.max(np.abs(E - w)) <= 1e-10
    _check_vectors(p, X.cpu().numpy(), E, 2e-10)
    pl.close()


@pytest.mark.parametrize("cfg", [2, 3])
def test_workloads_match_arpack(cfg):
    """The four lowest energies of the Heisenberg m=1024 and Hubbard m=2048
    workloads against ARPACK (stored), and the Ritz vectors' residuals."""
    import paper_1309_5571_amd as dm

    p = gen.config(cfg)
    pl = dm.Plan(p)
    print(f"block davidson cfg={cfg}", flush=True)
    X, E, R, info, st = pl.block_davidson(torch.from_numpy(_start(4, pl.n, 1)).cuda(), tol=1e-10)
    assert st == 0, info
    ref = np.array(ARPACK[gen.CONFIG_NAMES[cfg] + "_lowest4"])
    assert np.max(np.abs(E - ref)) <= 1e-10, (E, ref)
    _check_vectors(p, X.cpu().numpy(), E, 3e-10)
    pl.close()


def test_j1j2_matches_oracle_block_solver():
    import paper_1309_5571_amd as dm

    p = gen.config(5)
    pl = dm.Plan(p)
    X0 = _start(4, pl.n, 2)
    X, E, R, info, st = pl.block_davidson(torch.from_numpy(X0).cuda(), tol=1e-10)
    assert st == 0, info
    ref = odav.lowest_block_davidson(p, X0.T, tol=1e-10)
    assert ref.converged
    assert np.max(np.abs(E - ref.energies)) <= 1e-10
    assert abs(E[0] - ARPACK[gen.CONFIG_NAMES[5]]) <= 1e-10
    pl.close()


def test_l11r_plan_block_solver():
    """Block Davidson on an l-1-1-r plan: the three lowest levels of the
    4 + 1 + 1 + 4 Heisenberg chain (S^z = 0)."""
    import paper_1309_5571_amd as dm

    p = gen.heisenberg_l11r(4, 4)
    pl = dm.Plan(p)
    X, E, R, info, st = pl.block_davidson(torch.from_numpy(_start(3, pl.n, 5)).cuda(), tol=1e-10)
    assert st == 0, info
    w = np.linalg.eigvalsh(l11r.projected_hamiltonian(p))[:3]
    assert np.max(np.abs(E - w)) <= 1e-10
    pl.close()


def test_argument_errors():
    import paper_1309_5571_amd as dm

    pl = dm.Plan([gen.config(1), gen.config(1)])
    with pytest.raises(dm.DmrgError) as e:
        pl.block_davidson(torch.zeros(2, pl.n, dtype=torch.float64, device="cuda"))
    assert e.value.status == -8  # batched plans: unsupported
    pl.close()
    pl = dm.Plan(gen.config(1))
    with pytest.raises(dm.DmrgError) as e:
        pl.block_davidson(torch.zeros(9, pl.n, dtype=torch.float64, device="cuda"))
    assert e.value.status == -1
    pl.close()
