"""GPU Davidson (device-resident Alg. 3) against the oracle's ground states,
plus the energy gradient through the adjoint kernel."""
import json
import os

import numpy as np
import pytest

import gen
from oracle import davidson as odav
from oracle import models, projection, sectors

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "exact_energies.json")))["energies"]
ARPACK = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "arpack_energies.json")))["energies"]


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _dev(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).cuda()


def _plan(p, prec="f64"):
    import paper_1309_5571_amd as dm

    return dm.Plan(p, prec=prec)


def test_exact_ten_site_chain():
    p = gen.config(1)
    pl = _plan(p)
    psi, E, info, st = pl.davidson(_dev(gen.start_vector(pl.n, 3)), tol=1e-12)
    assert st == 0 and info[0]["converged"] == 1
    assert abs(E[0] - GOLDEN["heisenberg_open_N10_Sz0"]) <= 1e-10
    Ed, xd, _ = odav.ground_state_dense(p)
    x = psi.cpu().numpy()
    assert abs(np.linalg.norm(x) - 1) <= 1e-12
    assert abs(abs(x @ xd) - 1.0) <= 1e-10


def test_xx_chain_closed_form():
    p = gen.heisenberg_exact(5, 5, delta=0.0)
    pl = _plan(p)
    _, E, info, st = pl.davidson(_dev(gen.start_vector(pl.n, 4)), tol=1e-11)
    assert st == 0
    assert abs(E[0] - models.xx_chain_energy(10)) <= 1e-10


@pytest.mark.parametrize("cfg", [2, 3, 5])
def test_synthetic_configs_match_oracle(cfg):
    p = gen.config(cfg)
    pl = _plan(p)
    x0 = gen.start_vector(pl.n, 7)
    psi, E, info, st = pl.davidson(_dev(x0), tol=1e-10)
    assert st == 0, info
    ref = odav.ground_state_davidson(p, x0, tol=1e-10)
    assert ref.converged
    assert abs(E[0] - ref.energy) <= 1e-10
    x = psi.cpu().numpy()
    assert abs(abs(x @ ref.x) - 1.0) <= 1e-10
    # the residual of the returned vector, measured by the oracle
    r = projection.project_sectors(p, x) - E[0] * x
    assert np.linalg.norm(r) <= 2e-10


@pytest.mark.parametrize("solver", ["arrowhead", "jacobi"])
def test_restart_path_matches(solver):
    p = gen.config(1)
    pl = _plan(p)
    psi, E, info, st = pl.davidson(_dev(gen.start_vector(pl.n, 3)), tol=1e-11, kmax=5, kmin=2, max_iter=3000,
                                   eig_solver=solver)
    assert st == 0 and info[0]["restarts"] > 0
    assert abs(E[0] - GOLDEN["heisenberg_open_N10_Sz0"]) <= 1e-10


@pytest.mark.parametrize("cfg", [1, 2, 3, 5])
def test_small_eigensolvers_agree(cfg):
    """The arrowhead solve of the Rayleigh step and the Jacobi sweeps give the
    same Davidson run up to rounding (same iterations, energy, vector)."""
    p = gen.config(cfg)
    pl = _plan(p)
    x0 = _dev(gen.start_vector(pl.n, 7))
    a, Ea, ia, sa = pl.davidson(x0, tol=1e-10, kmax=12, kmin=4, eig_solver="arrowhead")
    b, Eb, ib, sb = pl.davidson(x0, tol=1e-10, kmax=12, kmin=4, eig_solver="jacobi")
    assert sa == 0 and sb == 0
    assert abs(Ea[0] - Eb[0]) <= 1e-11 * max(1.0, abs(Eb[0]))
    assert abs(ia[0]["iterations"] - ib[0]["iterations"]) <= 1
    assert abs(abs(float(a @ b)) - 1.0) <= 1e-10


def test_graph_replay_bit_identical_to_eager():
    p = gen.config(3)
    pl = _plan(p)
    x0 = _dev(gen.start_vector(pl.n, 7))
    a, Ea, ia, _ = pl.davidson(x0, tol=1e-10, use_graph=False)
    b, Eb, ib, _ = pl.davidson(x0, tol=1e-10, use_graph=True)
    c, Ec, ic, _ = pl.davidson(x0, tol=1e-10, use_graph=True)  # replay of cached graphs
    assert np.array_equal(a.cpu().numpy(), b.cpu().numpy())
    assert np.array_equal(b.cpu().numpy(), c.cpu().numpy())
    assert Ea[0] == Eb[0] == Ec[0]
    assert ia[0]["iterations"] == ib[0]["iterations"] == ic[0]["iterations"]


@pytest.mark.parametrize("prec", ["f32", "bf16"])
def test_mixed_precision_refinement(prec):
    p = gen.config(3)
    pl = _plan(p, prec=prec)
    x0 = gen.start_vector(pl.n, 7)
    psi, E, info, st = pl.davidson(_dev(x0), tol=1e-10, prec=prec)
    assert st == 0, info
    ref = odav.ground_state_davidson(p, x0, tol=1e-10)
    assert abs(E[0] - ref.energy) <= 1e-8
    assert info[0]["iterations_low"] > 0


def test_queued_fp64_phase_matches_sequential():
    """A repeated mixed-precision solve queues the FP64 phase right behind the
    first launch of the reduced-precision phase, gated on device.  Whether the
    gate opens (phase 1 finished in that launch) or stays shut (phase 1 needs
    more iterations than last time, so it continues and phase 2 restarts), the
    outcome is bit-identical to the sequential run of a fresh plan."""
    p = gen.config(3)
    x0 = gen.start_vector(_plan(p, "f32").n, 7)

    def solve(pl, x):
        psi, E, info, st = pl.davidson(_dev(x), tol=1e-10, prec="f32")
        assert st == 0, info
        return psi.cpu().numpy(), E[0], info[0]

    ref = solve(_plan(p, "f32"), x0)  # first solve of a plan: no queued phase
    pl = _plan(p, "f32")
    solve(pl, x0)
    opened = solve(pl, x0)  # same start: phase 1 ends within its first launch
    solve(pl, ref[0])  # converged start: both phases record one-iteration launch sizes
    shut = solve(pl, x0)  # phase 1 outlasts its first launch: the queued phase idles
    for got in (opened, shut):
        assert np.array_equal(got[0], ref[0])
        assert got[1] == ref[1]
        for key in ("iterations", "iterations_low", "projections", "restarts", "converged"):
            assert got[2][key] == ref[2][key], key


@pytest.mark.parametrize("prec", ["f32", "bf16"])
def test_reduced_precision_phase_exits_on_stagnation(prec):
    """A phase-1 tolerance below what the reduced-precision projection can reach:
    the phase ends when its residual stops halving (5 iterations), long before
    max_iter, and the FP64 phase still converges to the oracle energy."""
    p = gen.config(3)
    pl = _plan(p, prec=prec)
    x0 = gen.start_vector(pl.n, 7)
    psi, E, info, st = pl.davidson(_dev(x0), tol=1e-10, prec=prec, tol_lowprec=1e-10, max_iter=200)
    assert st == 0, info
    assert 0 < info[0]["iterations_low"] < 60
    assert info[0]["converged"] == 1
    ref = odav.ground_state_davidson(p, x0, tol=1e-10)
    assert abs(E[0] - ref.energy) <= 1e-8


def test_batched_members_converge_independently():
    probs = [gen.heisenberg_synthetic(m, seed=s) for m, s in ((128, 1), (256, 2), (64, 3))] + [gen.config(1)]
    pl = _plan(probs)
    rng = np.random.default_rng(0)
    x0 = rng.standard_normal(pl.n)
    psi, E, info, st = pl.davidson(_dev(x0), tol=1e-10)
    assert st == 0
    mo = pl.member_off
    for i, p in enumerate(probs):
        ref = odav.ground_state_davidson(p, x0[mo[i]:mo[i + 1]], tol=1e-10)
        assert abs(E[i] - ref.energy) <= 1e-10, i
        assert info[i]["converged"] == 1


def test_not_converged_and_bad_start():
    import paper_1309_5571_amd as dm

    p = gen.config(1)
    pl = _plan(p)
    _, _, info, st = pl.davidson(_dev(gen.start_vector(pl.n, 3)), tol=1e-12, max_iter=1)
    assert st == 1 and info[0]["converged"] == 0 and info[0]["iterations"] == 1
    with pytest.raises(dm.DmrgError) as e:
        pl.davidson(_dev(np.zeros(pl.n)))
    assert e.value.status == -6


def test_exact_eigenvector_start():
    p = gen.config(1)
    pl = _plan(p)
    E0, x, _ = odav.ground_state_dense(p)
    _, E, info, st = pl.davidson(_dev(x), tol=1e-12)
    assert st == 0 and info[0]["iterations"] == 1 and abs(E[0] - E0) <= 1e-12


def test_energy_gradient_hellmann_feynman_j1j2():
    """dE/dJ through the adjoint kernel vs central finite differences of the
    GPU ground energy and vs the oracle's <psi|dH/dJ|psi>."""
    import paper_1309_5571_amd as dm

    p = gen.j1j2_synthetic(256, seed=5)
    pl = _plan(p)
    basis = torch.from_numpy(p.meta["coef_basis"]).cuda()
    J = torch.tensor([1.0, 1.0, 0.5], dtype=torch.float64, device="cuda", requires_grad=True)
    x0 = _dev(gen.start_vector(pl.n, 2))
    E = dm.ground_energy(pl, basis @ J, x0, tol=1e-11)
    E.sum().backward()
    g = J.grad.cpu().numpy()
    h = 1e-5
    for j in (1, 2):
        e = np.zeros(3)
        e[j] = h
        Ep = pl.davidson(x0, coef=basis @ torch.from_numpy(np.array([1.0, 1.0, 0.5]) + e).cuda(), tol=1e-11)[1][0]
        Em = pl.davidson(x0, coef=basis @ torch.from_numpy(np.array([1.0, 1.0, 0.5]) - e).cuda(), tol=1e-11)[1][0]
        fd = (Ep - Em) / (2 * h)
        assert abs(g[j] - fd) <= 1e-7 * abs(fd) + 1e-9
    ref = odav.ground_state_davidson(p, gen.start_vector(pl.n, 2), tol=1e-11)
    dc = projection.coef_gradient(p, ref.x, ref.x)
    gref = p.meta["coef_basis"].T @ dc
    assert np.all(np.abs(g[1:] - gref[1:]) <= 1e-7 * np.abs(gref[1:]))


def test_subspace_filling_the_space_is_reproducible_across_plans():
    """A superblock of dimension n <= kmax: the subspace fills the whole space.
    Plans created one after another (device memory reused) must reach the same
    converged result from the same start vector (the workspace starts at zero;
    stale memory once made the second plan break down)."""
    import paper_1309_5571_amd as dm

    p = gen.heisenberg_exact(2, 2)  # n = 6
    x0 = gen.start_vector(6, 3)
    out = []
    for _ in range(3):
        pl = dm.Plan(p)
        big = torch.full((1 << 20,), 1e300, dtype=torch.float64, device="cuda")  # dirty memory between plans
        del big
        psi, E, infos, st = pl.davidson(torch.from_numpy(x0).cuda(), tol=1e-11, kmax=6, kmin=5)
        assert st == 0 and infos[0]["converged"]
        out.append(float(E[0]))
        pl.close()
        del pl
    assert out[0] == pytest.approx(-1.6160254037844386, abs=1e-12)
    assert out[0] == out[1] == out[2]


@pytest.mark.parametrize("cfg", [2, 3, 5])
def test_synthetic_configs_match_arpack(cfg):
    """GPU ground energies of the m=1024 / m=2048 workloads against ARPACK
    Lanczos on the oracle projection (stored by tests/golden/make_golden.py),
    FP64 and mixed precision with refinement."""
    p = gen.config(cfg)
    E_ref = ARPACK[gen.CONFIG_NAMES[cfg]]
    x0 = gen.start_vector(_plan(p).n, 7)
    for prec, tol in (("f64", 1e-10), ("f32", 1e-8)):
        pl = _plan(p, prec=prec)
        _, E, info, st = pl.davidson(_dev(x0), tol=1e-10, prec=prec)
        assert st == 0 and info[0]["converged"] == 1, info
        assert abs(E[0] - E_ref) <= tol, (prec, E[0], E_ref)
        pl.close()


def test_forced_restart_heisenberg_m1024_matches_oracle():
    """kmax = 4, kmin = 2 on the Heisenberg m=1024 workload (it converges in 7
    iterations, so only a small subspace forces restarts): the thick restart
    runs twice at full size; the device and the oracle (same subspace
    bounds, same start) agree on the energy and the vector, and both on ARPACK."""
    p = gen.config(2)
    pl = _plan(p)
    x0 = gen.start_vector(pl.n, 7)
    psi, E, info, st = pl.davidson(_dev(x0), tol=1e-10, kmax=4, kmin=2)
    assert st == 0, info
    assert info[0]["restarts"] >= 2, info
    ref = odav.ground_state_davidson(p, x0, tol=1e-10, kmax=4, kmin=2)
    assert ref.converged and ref.restarts >= 2
    assert abs(E[0] - ref.energy) <= 1e-10
    assert abs(E[0] - ARPACK[gen.CONFIG_NAMES[2]]) <= 1e-10
    x = psi.cpu().numpy()
    assert abs(abs(x @ ref.x) - 1.0) <= 1e-10
    assert abs(info[0]["iterations"] - ref.iterations) <= 2


def test_energy_gradient_j1j2_m1024():
    """The J1-J2 m=1024 workload: dE/dJ1 and dE/dJ2 through the adjoint kernel
    against central finite differences (h = 1e-5) of the GPU ground energy and
    against Hellmann-Feynman <psi|dH/dJ|psi> from the oracle's ground state,
    relative error <= 1e-7 each."""
    import paper_1309_5571_amd as dm

    p = gen.config(5)
    pl = _plan(p)
    basis = torch.from_numpy(p.meta["coef_basis"]).cuda()
    J0 = np.array([1.0, 1.0, 0.5])
    J = torch.tensor(J0, dtype=torch.float64, device="cuda", requires_grad=True)
    x0 = _dev(gen.start_vector(pl.n, 2))
    E = dm.ground_energy(pl, basis @ J, x0, tol=1e-11)
    E.sum().backward()
    g = J.grad.cpu().numpy()
    h = 1e-5
    for j in (1, 2):
        e = np.zeros(3)
        e[j] = h
        Ep = pl.davidson(x0, coef=basis @ torch.from_numpy(J0 + e).cuda(), tol=1e-11)[1][0]
        Em = pl.davidson(x0, coef=basis @ torch.from_numpy(J0 - e).cuda(), tol=1e-11)[1][0]
        fd = (Ep - Em) / (2 * h)
        assert abs(g[j] - fd) <= 1e-7 * abs(fd), (j, g[j], fd)
    ref = odav.ground_state_davidson(p, gen.start_vector(pl.n, 2), tol=1e-11)
    assert abs(ref.energy - ARPACK[gen.CONFIG_NAMES[5]]) <= 1e-10
    dc = projection.coef_gradient(p, ref.x, ref.x)
    gref = p.meta["coef_basis"].T @ dc
    assert np.all(np.abs(g[1:] - gref[1:]) <= 1e-7 * np.abs(gref[1:])), (g, gref)


def test_same_plan_recovers_after_a_non_finite_solve():
    """A solve whose iterate turns non-finite (NaN coefficients) leaves its
    NaNs in the plan's workspace; the next solve on the same plan clears it and
    reaches the exact result (also with a subspace that fills the space)."""
    import paper_1309_5571_amd as dm

    for p, kw, E_ref in ((gen.heisenberg_exact(2, 2), dict(kmax=6, kmin=5), -1.6160254037844386),
                         (gen.config(1), dict(kmax=32, kmin=8), GOLDEN["heisenberg_open_N10_Sz0"])):
        pl = _plan(p)
        x0 = _dev(gen.start_vector(pl.n, 3))
        bad = torch.full((len(p.coef),), float("nan"), dtype=torch.float64, device="cuda")
        with pytest.raises(dm.DmrgError) as e:
            pl.davidson(x0, coef=bad, tol=1e-11, **kw)
        assert e.value.status == -6  # non-finite iterate
        psi, E, info, st = pl.davidson(x0, tol=1e-11, **kw)
        assert st == 0 and info[0]["converged"] == 1
        assert abs(E[0] - E_ref) <= 1e-10
        assert np.all(np.isfinite(psi.cpu().numpy()))
        pl.close()
