"""The batched workload: 64 independent Heisenberg superblocks (m drawn from
256..2048) in one plan -- one launch per projection stage over every output
tile of every member, and one lock-step Davidson over all members."""
import numpy as np
import pytest

import gen
from oracle import davidson as odav
from oracle import precision, projection

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.fixture(scope="module")
def batch():
    return gen.config(4)


def _dev(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).cuda()


def _relerr(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _sample(batch):
    ms = np.array([p.meta["m"] for p in batch])
    return sorted({int(np.argmin(ms)), int(np.argmax(ms)), 5, 17, 40})


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_batched_equals_single_plans(batch, prec):
    """Same tiles and segment order per member, so the batched launch is
    bit-identical to one plan per member."""
    import paper_1309_5571_amd as dm

    tiles = ((1 << 30,), (32,))
    big = dm.Plan(batch, prec=prec, tiles=tiles)
    psi = np.random.default_rng(0).standard_normal(big.n)
    y = big.project_raw(_dev(psi), prec=prec).cpu().numpy()
    mo = big.member_off
    for i in _sample(batch):
        one = dm.Plan(batch[i], prec=prec, tiles=tiles)
        yi = one.project_raw(_dev(psi[mo[i]:mo[i + 1]]), prec=prec).cpu().numpy()
        assert np.array_equal(y[mo[i]:mo[i + 1]], yi), i
        one.close()


def test_batched_projection_vs_oracle(batch):
    import paper_1309_5571_amd as dm

    pl = dm.Plan(batch)
    psi = np.random.default_rng(1).standard_normal(pl.n)
    y = pl.project_raw(_dev(psi)).cpu().numpy()
    mo = pl.member_off
    assert pl.flop == sum(projection.flop_count(p) for p in batch)
    for i in range(len(batch)):  # every member
        ref = projection.project_sectors(batch[i], psi[mo[i]:mo[i + 1]])
        assert _relerr(y[mo[i]:mo[i + 1]], ref) <= 1e-12, i


def test_batched_fp32_projection_elementwise(batch):
    """FP32 projection of all 64 members: every output entry inside its own
    rounding envelope around the emulated oracle (oracle.precision), plus the
    FP64 rounding of the per-record sums."""
    import paper_1309_5571_amd as dm

    pl = dm.Plan(batch, prec="f32")
    psi = np.random.default_rng(3).standard_normal(pl.n)
    y = pl.project_raw(_dev(psi), prec="f32").cpu().numpy()
    mo = pl.member_off
    for i, p in enumerate(batch):
        x = psi[mo[i]:mo[i + 1]]
        emul = precision.project_emulated(p, x, "fp32")
        env = precision.project_envelope(p, x, "fp32") + 8 * 2.0 ** -53 * precision.project_magnitude(p, x)
        assert np.all(np.abs(y[mo[i]:mo[i + 1]] - emul) <= env), i


def test_batched_davidson_mixed_precision(batch):
    """FP32 projection + FP64 refinement for all 64 members at once; sampled
    members against the oracle's FP64 Davidson from the same start."""
    import paper_1309_5571_amd as dm

    pl = dm.Plan(batch, prec="f32")
    x0 = np.random.default_rng(2).standard_normal(pl.n)
    psi, E, info, st = pl.davidson(_dev(x0), tol=1e-10, prec="f32")
    assert st == 0, [i for i in info if not i["converged"]]
    assert all(i["converged"] for i in info)
    mo = pl.member_off
    ms = np.array([p.meta["m"] for p in batch])
    order = np.argsort(ms, kind="stable")
    for i in sorted({int(order[j]) for j in (0, 1, 9, 20, 31, 42, 53, 63)}):  # smallest to largest m
        ref = odav.ground_state_davidson(batch[i], x0[mo[i]:mo[i + 1]], tol=1e-10)
        assert ref.converged
        assert abs(E[i] - ref.energy) <= 1e-8, (i, E[i], ref.energy)
    # graph chunk length and eager execution give identical results
    psi2, E2, _, _ = pl.davidson(_dev(x0), tol=1e-10, prec="f32", graph_chunk=32)
    psi3, E3, _, _ = pl.davidson(_dev(x0), tol=1e-10, prec="f32", use_graph=False)
    assert np.array_equal(E, E2) and np.array_equal(E, E3)
    assert torch.equal(psi, psi2) and torch.equal(psi, psi3)
