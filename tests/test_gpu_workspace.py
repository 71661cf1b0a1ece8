"""Plans built on a caller workspace (dmrg_plan_workspace_size + the workspace
arguments of dmrg_plan_create): every result equals the one of a plan that
allocates its own scratch, bit for bit, and a solve that needs more Davidson
vectors than the workspace holds fails with DMRG_E_NOMEM."""
import numpy as np
import pytest

import gen

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _dev(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).cuda()


@pytest.mark.parametrize("cfg,prec", [(2, "f64"), (3, "f32"), (5, "bf16")])
def test_workspace_plan_matches_own_scratch(cfg, prec):
    import paper_1309_5571_amd as dm

    p = gen.config(cfg)
    ref = dm.Plan(p, prec=prec)
    nb = dm.Plan.workspace_size(p, prec, 32)
    # dirty memory: every array the plan reads before writing would show
    ws = torch.full((nb,), 0x7F, dtype=torch.uint8, device="cuda")
    pl = dm.Plan(p, prec=prec, workspace=ws, ws_kmax=32)
    assert pl.n == ref.n and pl.workspace is ws
    x0 = _dev(gen.start_vector(pl.n, 11))
    psi = x0 / x0.norm()
    for pr in ("f64", prec):
        assert torch.equal(pl.project_raw(psi, prec=pr), ref.project_raw(psi, prec=pr))
    a = ref.davidson(x0, tol=1e-10, prec=prec)
    b = pl.davidson(x0, tol=1e-10, prec=prec)
    assert a[3] == 0 and b[3] == 0
    assert np.array_equal(a[1], b[1]), (a[1], b[1])
    assert torch.equal(a[0], b[0])
    assert [i["iterations"] for i in a[2]] == [i["iterations"] for i in b[2]]
    _, ga = ref.backward_raw(a[0], a[0], want_psi=False, want_coef=True)
    _, gb = pl.backward_raw(b[0], b[0], want_psi=False, want_coef=True)
    assert torch.equal(ga, gb)
    # a second solve on the same workspace (its contents left by the first)
    c = pl.davidson(x0, tol=1e-10, prec=prec)
    assert np.array_equal(c[1], b[1]) and torch.equal(c[0], b[0])
    ref.close()
    pl.close()


def test_workspace_kmax_limit_and_smaller_subspace():
    import paper_1309_5571_amd as dm
    from paper_1309_5571_amd import _native as N

    p = gen.config(2)
    pl = dm.Plan(p, workspace=True, ws_kmax=16)
    ref = dm.Plan(p)
    x0 = _dev(gen.start_vector(pl.n, 5))
    with pytest.raises(RuntimeError, match="workspace"):
        pl.davidson(x0, tol=1e-10, kmax=32, kmin=8, raise_on_warning=True)
    assert N.last_error() and "16" in N.last_error()
    # kmax below the workspace's limit (small enough to restart): same result
    # as the plan's own scratch
    a = ref.davidson(x0, tol=1e-10, kmax=4, kmin=2)
    b = pl.davidson(x0, tol=1e-10, kmax=4, kmin=2)
    assert a[3] == 0 and b[3] == 0 and np.array_equal(a[1], b[1]) and torch.equal(a[0], b[0])
    assert b[2][0]["restarts"] >= 1
    pl.close()
    ref.close()


def test_workspace_plan_allocates_no_davidson_arrays():
    """The first solve on a workspace plan takes no new device memory of the
    size of the Davidson basis (a plan without one does)."""
    import paper_1309_5571_amd as dm

    p = gen.config(2)
    warm = dm.Plan(p)
    x0 = _dev(gen.start_vector(warm.n, 5))
    warm.davidson(x0, tol=1e-10)  # torch's own temporaries exist from here on
    basis = 2 * 33 * warm.n * 8
    torch.cuda.synchronize()
    pl = dm.Plan(p, workspace=True, ws_kmax=32)
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    r = pl.davidson(x0, tol=1e-10)
    torch.cuda.synchronize()
    free1 = torch.cuda.mem_get_info()[0]
    assert r[3] == 0
    assert free0 - free1 < basis // 4, (free0 - free1, basis)
    fresh = dm.Plan(p)
    torch.cuda.synchronize()
    free2 = torch.cuda.mem_get_info()[0]
    fresh.davidson(x0, tol=1e-10)
    torch.cuda.synchronize()
    free3 = torch.cuda.mem_get_info()[0]
    assert free2 - free3 >= basis // 2, (free2 - free3, basis)
    for q in (warm, pl, fresh):
        q.close()
