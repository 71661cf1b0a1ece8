"""GPU parity of the l-1-1-r strategy (Eq. 12-13, Alg. 2): projection,
adjoint, preconditioner diagonal and Davidson of plans built from the four
subsystems' operators, against oracle.l11r, the whole chains' exact energies
and the LR projection of the same superblock's enlarged blocks."""
import json
import os

import numpy as np
import pytest

import gen
from oracle import davidson as odav
from oracle import l11r, models, projection

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "exact_energies.json")))["energies"]


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _dev(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).cuda()


def _relerr(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


TILES = {"auto": "auto", "t16": ((1 << 30,), (16,)), "t32": ((1 << 30,), (32,))}
RANDOM = [(s, r) for s in range(8) for r in (1, 2)]


@pytest.mark.parametrize("tiles", ["t16", "t32"])
@pytest.mark.parametrize("seed,rank", RANDOM)
def test_projection_random_structures(seed, rank, tiles):
    import paper_1309_5571_amd as dm

    p = gen.random_problem4(seed, rank=rank, dmax=20 if seed % 3 == 0 else 7, site_dmax=2)
    pl = dm.Plan(p, tiles=TILES[tiles])
    lay = l11r.layout(p)
    assert pl.n == lay.n
    assert np.array_equal(pl.layout()["pair_off"], lay.pair_offset)
    psi = np.random.default_rng(seed).standard_normal(pl.n)
    y = pl.project_raw(_dev(psi)).cpu().numpy()
    assert _relerr(y, l11r.project_sectors(p, psi)) <= 1e-12
    pl.close()


@pytest.mark.parametrize("name", ["heis_4_4", "hub_2_2", "hub_synth_256"])
def test_projection_workloads(name):
    import paper_1309_5571_amd as dm

    p = {"heis_4_4": lambda: gen.heisenberg_l11r(4, 4), "hub_2_2": lambda: gen.hubbard_l11r_exact(2, 2),
         "hub_synth_256": lambda: gen.hubbard_l11r_synthetic(256)}[name]()
    pl = dm.Plan(p)
    psi = gen.start_vector(pl.n, 5)
    y = pl.project_raw(_dev(psi)).cpu().numpy()
    assert _relerr(y, l11r.project_sectors(p, psi)) <= 1e-12
    pl.close()


def test_same_vector_as_lr_plan_of_enlarged_blocks():
    """The l-1-1-r plan and an LR plan whose enlarged operators come from
    dmrg_enlarge share the psi layout and give the same projection."""
    import paper_1309_5571_amd as dm

    p = gen.hubbard_l11r_synthetic(128, seed=5)
    l, s1, s2, r = p.spaces
    # enlarged operators, one pair per term
    nt = len(p.coef)
    EL, oL = dm.enlarge(l, p.ops[0], s1, p.ops[1], [(k, int(t[0]), int(t[1]), 1.0) for k, t in enumerate(p.terms)], nt)
    ER, oR = dm.enlarge(s2, p.ops[2], r, p.ops[3], [(k, int(t[2]), int(t[3]), 1.0) for k, t in enumerate(p.terms)], nt)
    from paper_1309_5571_amd.chains import Superblock

    lr = Superblock(EL, ER, p.target, oL, oR, [(k, k) for k in range(nt)], p.coef)
    a, b = dm.Plan(p), dm.Plan(lr)
    assert a.n == b.n and np.array_equal(a.layout()["pair_off"], b.layout()["pair_off"])
    psi = _dev(gen.start_vector(a.n, 9))
    ya, yb = a.project_raw(psi).cpu().numpy(), b.project_raw(psi).cpu().numpy()
    assert _relerr(ya, yb) <= 1e-12
    a.close()
    b.close()


@pytest.mark.parametrize("seed,rank", RANDOM[:8])
def test_adjoint_and_coefficient_gradient(seed, rank):
    import paper_1309_5571_amd as dm

    p = gen.random_problem4(seed, rank=rank, site_dmax=2)
    pl = dm.Plan(p, tiles=TILES["t16" if seed % 2 else "t32"])
    rng = np.random.default_rng(seed + 3)
    psi, g = rng.standard_normal(pl.n), rng.standard_normal(pl.n)
    gpsi, gcoef = pl.backward_raw(_dev(psi), _dev(g))
    Hq = l11r.projected_hamiltonian(p)
    assert _relerr(gpsi.cpu().numpy(), Hq.T @ g) <= 1e-12
    K = len(p.coef)
    ref = np.array([g @ l11r.project_sectors(p, psi, coef=np.eye(K)[k]) for k in range(K)])
    got = gcoef.cpu().numpy()[:K]
    assert np.all(np.abs(got - ref) <= 1e-12 * np.maximum(np.abs(ref), np.abs(ref).max()))
    pl.close()


@pytest.mark.parametrize("name", ["heis_4_4", "random"])
def test_preconditioner_diagonal(name):
    import paper_1309_5571_amd as dm

    p = gen.heisenberg_l11r(4, 4) if name == "heis_4_4" else gen.random_problem4(7, rank=2, site_dmax=2)
    pl = dm.Plan(p)
    d = pl.diagonal().cpu().numpy()
    ref = np.diag(l11r.projected_hamiltonian(p))
    assert np.max(np.abs(d - ref)) <= 1e-13 * max(1.0, np.abs(ref).max())
    pl.close()


def test_davidson_ten_site_chain():
    """4 + 1 + 1 + 4 Heisenberg sites: the device Davidson on the l-1-1-r plan
    reaches the exact 10-site ground energy."""
    import paper_1309_5571_amd as dm

    p = gen.heisenberg_l11r(4, 4)
    pl = dm.Plan(p)
    psi, E, info, st = pl.davidson(_dev(gen.start_vector(pl.n, 3)), tol=1e-12)
    assert st == 0 and info[0]["converged"] == 1
    assert abs(E[0] - GOLDEN["heisenberg_open_N10_Sz0"]) <= 1e-10
    pl.close()


def test_davidson_hubbard_six_sites():
    """2 + 1 + 1 + 2 Hubbard sites at half filling: the whole chain's exact
    ground energy (dense ED of Eq. 4-8)."""
    import paper_1309_5571_amd as dm

    p = gen.hubbard_l11r_exact(2, 2)
    pl = dm.Plan(p)
    _, E, info, st = pl.davidson(_dev(gen.start_vector(pl.n, 4)), tol=1e-11)
    assert st == 0
    H, Nup, Ndn = models.hubbard_chain(6)
    idx = np.flatnonzero((np.rint(np.diag(Nup)) == 3) & (np.rint(np.diag(Ndn)) == 3))
    E0 = np.linalg.eigvalsh(H[np.ix_(idx, idx)])[0]
    assert abs(E[0] - E0) <= 1e-10
    pl.close()


def test_davidson_synthetic_hubbard_matches_oracle():
    import paper_1309_5571_amd as dm

    p = gen.hubbard_l11r_synthetic(256)
    pl = dm.Plan(p)
    x0 = gen.start_vector(pl.n, 7)
    psi, E, info, st = pl.davidson(_dev(x0), tol=1e-10)
    assert st == 0, info
    lr = l11r.to_lr(p)  # the same superblock through its enlarged blocks (pinned equal on the CPU)
    ref = odav.ground_state_davidson(lr, x0, tol=1e-10)
    assert ref.converged
    assert abs(E[0] - ref.energy) <= 1e-10
    pl.close()


def test_ten_site_chain_built_by_enlargement_on_gpu():
    """Config 1 assembled from single sites by dmrg_enlarge (host), solved by
    the device Davidson: the exact ground energy."""
    import paper_1309_5571_amd as dm
    from paper_1309_5571_amd import chains

    p = chains.xxz_superblock(5, 5)
    pl = dm.Plan(p, tiles=None)
    _, E, info, st = pl.davidson(_dev(gen.start_vector(pl.n, 3)), tol=1e-12)
    assert st == 0 and info[0]["converged"] == 1
    assert abs(E[0] - GOLDEN["heisenberg_open_N10_Sz0"]) <= 1e-10
    pl.close()
