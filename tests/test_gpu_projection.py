"""GPU parity of the projection, its adjoint and the preconditioner diagonal
against the FP64 oracle (called through the C ABI)."""
import numpy as np
import pytest

import gen
from oracle import precision, projection, sectors

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _plan(p, prec="f64"):
    import paper_1309_5571_amd as dm

    return dm.Plan(p, prec=prec)


def _dev(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).cuda()


def _relerr(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _n(p):
    return sectors.pair_table(p.left, p.right, p.target)[1]


RANDOM = [(s, r) for s in range(10) for r in (1, 2)]


# ------------------------------------------------------------------ layout and records (exact)


@pytest.mark.parametrize("cfg", [1, 2, 3, 5])
def test_layout_bit_exact(cfg):
    p = gen.config(cfg)
    pl = _plan(p)
    lay = pl.layout()
    ref = sectors.layout(p.left, p.right, p.target)
    assert pl.n == ref.n
    assert [(int(a), int(b)) for a, b in zip(lay["pair_left"], lay["pair_right"])] == ref.pairs
    assert np.array_equal(lay["pair_off"], ref.pair_offset)


@pytest.mark.parametrize("seed,rank", RANDOM[:8])
def test_records_match_oracle(seed, rank):
    p = gen.random_problem(seed, rank=rank)
    pl = _plan(p)
    recs, table, n = projection.records(p)
    keys = list(table.keys())
    ref = sorted((k, keys.index(pin), keys.index(pout)) for k, pin, pout, _, _ in recs)
    got = pl.records()
    mine = sorted(zip(got["term"].tolist(), got["pair_in"].tolist(), got["pair_out"].tolist()))
    assert mine == ref
    assert pl.flop == projection.flop_count(p)


# ------------------------------------------------------------------ FP64 projection


@pytest.mark.parametrize("cfg", [1, 2, 3, 5])
def test_projection_fp64_configs(cfg):
    p = gen.config(cfg)
    pl = _plan(p)
    psi = gen.start_vector(pl.n, 11)
    y = pl.project_raw(_dev(psi)).cpu().numpy()
    ref = projection.project_sectors(p, psi)
    assert _relerr(y, ref) <= 1e-12, _relerr(y, ref)


TILES = {"auto": "auto", "t16": ((1 << 30,), (16,)), "t32": ((1 << 30,), (32,))}


@pytest.mark.parametrize("tiles", ["auto", "t16", "t32"])
@pytest.mark.parametrize("seed,rank", RANDOM)
def test_projection_fp64_random_structures(seed, rank, tiles):
    """Ragged, empty and 1x1 sectors, missing blocks, diagonal factors on either
    side; 16-row tiles take the fused two-sided path, 32-row tiles the two-stage one."""
    import paper_1309_5571_amd as dm

    p = gen.random_problem(seed, rank=rank, dmax=40 if seed % 3 == 0 else 12)
    pl = dm.Plan(p, tiles=TILES[tiles])
    psi = np.random.default_rng(seed).standard_normal(pl.n)
    y = pl.project_raw(_dev(psi)).cpu().numpy()
    ref = projection.project_sectors(p, psi)
    assert _relerr(y, ref) <= 1e-12


def test_projection_coefficients_are_read_at_call_time():
    p = gen.config(2)
    pl = _plan(p)
    psi = gen.start_vector(pl.n, 3)
    c = np.random.default_rng(0).standard_normal(len(p.coef))
    y = pl.project_raw(_dev(psi), coef=_dev(c)).cpu().numpy()
    assert _relerr(y, projection.project_sectors(p, psi, c)) <= 1e-12


def test_projection_zero_coefficients_and_zero_input():
    p = gen.config(3)
    pl = _plan(p)
    y = pl.project_raw(_dev(gen.start_vector(pl.n, 1)), coef=_dev(np.zeros(len(p.coef)))).cpu().numpy()
    assert not np.any(y)
    y = pl.project_raw(_dev(np.zeros(pl.n))).cpu().numpy()
    assert not np.any(y)


def test_projection_deterministic():
    p = gen.config(2)
    pl = _plan(p)
    psi = _dev(gen.start_vector(pl.n, 5))
    a = pl.project_raw(psi).cpu().numpy()
    b = pl.project_raw(psi).cpu().numpy()
    assert np.array_equal(a, b)


def test_batched_plan_equals_members():
    probs = [gen.random_problem(s, rank=1 + s % 2, dmax=20) for s in range(5)] + [gen.heisenberg_synthetic(256, seed=9)]
    pl = _plan(probs)
    psi = np.random.default_rng(1).standard_normal(pl.n)
    y = pl.project_raw(_dev(psi)).cpu().numpy()
    mo = pl.member_off
    for i, p in enumerate(probs):
        ref = projection.project_sectors(p, psi[mo[i]:mo[i + 1]])
        assert _relerr(y[mo[i]:mo[i + 1]], ref) <= 1e-12


# ------------------------------------------------------------------ adjoint and coefficient gradient


@pytest.mark.parametrize("tiles", ["t16", "t32"])
@pytest.mark.parametrize("seed,rank", RANDOM[:10])
def test_adjoint_random(seed, rank, tiles):
    import paper_1309_5571_amd as dm

    p = gen.random_problem(seed, rank=rank, dmax=24)
    pl = dm.Plan(p, tiles=TILES[tiles])
    rng = np.random.default_rng(seed + 7)
    psi, g = rng.standard_normal(pl.n), rng.standard_normal(pl.n)
    gpsi, gcoef = pl.backward_raw(_dev(psi), _dev(g))
    gpsi, gcoef = gpsi.cpu().numpy(), gcoef.cpu().numpy()[: len(p.coef)]
    assert _relerr(gpsi, projection.project_adjoint_sectors(p, g)) <= 1e-12
    ref = projection.coef_gradient(p, psi, g)
    assert np.all(np.abs(gcoef - ref) <= 1e-12 * np.maximum(np.abs(ref), np.abs(ref).max()))


@pytest.mark.parametrize("cfg", [2, 5])
def test_adjoint_configs(cfg):
    p = gen.config(cfg)
    pl = _plan(p)
    rng = np.random.default_rng(cfg)
    psi, g = rng.standard_normal(pl.n), rng.standard_normal(pl.n)
    gpsi, gcoef = pl.backward_raw(_dev(psi), _dev(g))
    assert _relerr(gpsi.cpu().numpy(), projection.project_adjoint_sectors(p, g)) <= 1e-12
    ref = projection.coef_gradient(p, psi, g)
    assert np.max(np.abs(gcoef.cpu().numpy()[: len(ref)] - ref) / np.abs(ref)) <= 1e-12


def test_autograd_gradcheck_tiny():
    import paper_1309_5571_amd as dm

    p = gen.random_problem(3, rank=1, dmax=5)
    pl = _plan(p)
    psi = torch.randn(pl.n, dtype=torch.float64, device="cuda", requires_grad=True)
    coef = pl.coef.clone().requires_grad_(True)
    assert torch.autograd.gradcheck(lambda a, c: dm.project(pl, a, c), (psi, coef), eps=1e-6, atol=1e-8)


# ------------------------------------------------------------------ preconditioner diagonal


@pytest.mark.parametrize("cfg", [1, 3, 5])
def test_diagonal(cfg):
    p = gen.config(cfg)
    pl = _plan(p)
    d = pl.diagonal().cpu().numpy()
    ref = projection.diagonal(p)
    assert np.max(np.abs(d - ref)) <= 1e-13 * max(1.0, np.abs(ref).max())


# ------------------------------------------------------------------ reduced precision


@pytest.mark.parametrize("prec,u", [("f32", 2.0 ** -24), ("bf16", 2.0 ** -8)])
@pytest.mark.parametrize("cfg", [2, 3])
def test_lowprec_projection_envelope(cfg, prec, u):
    """The device result lies in an accumulation envelope around the emulated
    rounding of the oracle, and within the operand-rounding envelope of the
    exact FP64 projection."""
    p = gen.config(cfg)
    pl = _plan(p, prec=prec)
    psi = gen.start_vector(pl.n, 4)
    y = pl.project_raw(_dev(psi), prec=prec).cpu().numpy()
    emul = precision.project_emulated(p, psi, "fp32" if prec == "f32" else "bf16")
    mag = precision.project_magnitude(p, psi)
    K = precision.max_contraction(p)
    # FP32 accumulation (and, for BF16, the re-rounded intermediate) around the emulation
    env = (K * 2.0 ** -24 + (4 * u if prec == "bf16" else 0.0)) * np.linalg.norm(mag)
    assert np.linalg.norm(y - emul) <= env
    exact = projection.project_sectors(p, psi)
    assert np.linalg.norm(y - exact) <= (K * 2.0 ** -24 + 6 * u) * np.linalg.norm(mag)
    # and FP64 through the same plan is still exact
    y64 = pl.project_raw(_dev(psi)).cpu().numpy()
    assert _relerr(y64, exact) <= 1e-12


@pytest.mark.parametrize("tiles", ["t16", "t32"])
def test_lowprec_random_structures(tiles):
    import paper_1309_5571_amd as dm

    for seed in range(6):
        p = gen.random_problem(seed, rank=1 + seed % 2, dmax=30)
        for prec in ("f32", "bf16"):
            pl = dm.Plan(p, prec=prec, tiles=TILES[tiles])
            psi = np.random.default_rng(seed).standard_normal(pl.n)
            y = pl.project_raw(_dev(psi), prec=prec).cpu().numpy()
            emul = precision.project_emulated(p, psi, "fp32" if prec == "f32" else "bf16")
            mag = precision.project_magnitude(p, psi)
            K = max(precision.max_contraction(p), 1)
            u = 2.0 ** -24 if prec == "f32" else 2.0 ** -8
            env = (K * 2.0 ** -24 + (4 * u if prec == "bf16" else 0.0)) * np.linalg.norm(mag)
            assert np.linalg.norm(y - emul) <= env + 1e-300, (seed, prec)


def _elementwise_ok(y, p, psi, prec):
    """|device - emulation| <= the per-entry envelope of oracle.precision (the
    FP32 sums and the rounded intermediate of that entry's own records), plus
    the FP64 rounding of the per-record and diagonal-term sums (a few units of
    2^-53 of the entry's magnitude, which the envelope leaves out)."""
    key = "fp32" if prec == "f32" else "bf16"
    emul = precision.project_emulated(p, psi, key)
    env = precision.project_envelope(p, psi, key) + 8 * 2.0 ** -53 * precision.project_magnitude(p, psi)
    bad = np.abs(y - emul) > env
    return int(bad.sum()), float(np.max(np.abs(y - emul) / np.maximum(env, 1e-300)))


@pytest.mark.parametrize("prec", ["f32", "bf16"])
@pytest.mark.parametrize("cfg", [2, 3, 5])
def test_lowprec_projection_elementwise(cfg, prec):
    """Every output entry of the FP32/BF16 projection lies inside its own
    rounding envelope around the emulated oracle (no global norm)."""
    p = gen.config(cfg)
    pl = _plan(p, prec=prec)
    psi = gen.start_vector(pl.n, 4)
    y = pl.project_raw(_dev(psi), prec=prec).cpu().numpy()
    nbad, worst = _elementwise_ok(y, p, psi, prec)
    assert nbad == 0, (nbad, worst)


@pytest.mark.parametrize("tiles", ["t16", "t32"])
@pytest.mark.parametrize("prec", ["f32", "bf16"])
def test_lowprec_random_structures_elementwise(tiles, prec):
    import paper_1309_5571_amd as dm

    for seed in range(6):
        p = gen.random_problem(seed, rank=1 + seed % 2, dmax=30)
        pl = dm.Plan(p, prec=prec, tiles=TILES[tiles])
        psi = np.random.default_rng(seed).standard_normal(pl.n)
        y = pl.project_raw(_dev(psi), prec=prec).cpu().numpy()
        nbad, worst = _elementwise_ok(y, p, psi, prec)
        assert nbad == 0, (seed, nbad, worst)
        pl.close()


# ------------------------------------------------------------------ several vectors per call


@pytest.mark.parametrize("name", ["cfg3", "cfg2", "random_t16", "l11r"])
@pytest.mark.parametrize("nvec", [1, 4, 9])
def test_project_block_matches_oracle(name, nvec):
    """dmrg_project_block: groups of four vectors share every operator load in
    one launch (16 x 16 tiles) or fall back to one launch per vector; each
    result matches the oracle to 1e-12 and the single-vector call to 1e-13."""
    import paper_1309_5571_amd as dm

    from oracle import l11r

    if name == "cfg3":
        p, ref = gen.config(3), projection.project_sectors
        pl = _plan(p)
    elif name == "cfg2":
        p, ref = gen.config(2), projection.project_sectors
        pl = _plan(p)
    elif name == "random_t16":
        p, ref = gen.random_problem(3, rank=2, dmax=40), projection.project_sectors
        pl = dm.Plan(p, tiles=TILES["t16"])
    else:
        p, ref = gen.hubbard_l11r_synthetic(128, seed=2), l11r.project_sectors
        pl = dm.Plan(p)
    X = np.random.default_rng(nvec).standard_normal((nvec, pl.n))
    Y = pl.project_block(_dev(X)).cpu().numpy()
    for v in range(nvec):
        assert _relerr(Y[v], ref(p, X[v])) <= 1e-12, v
        one = pl.project_raw(_dev(X[v])).cpu().numpy()
        assert _relerr(Y[v], one) <= 1e-13, v
    pl.close()
