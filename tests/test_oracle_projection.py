"""Pins of the oracle's sector layout and projection (Eq. 9-11)."""
import numpy as np
import pytest

import gen
from oracle import models, precision, projection, sectors

RANDOM_CASES = [(s, r) for s in range(6) for r in (1, 2)]


def _rand(seed, rank, **kw):
    return gen.random_problem(seed, rank=rank, **kw)


# --------------------------------------------------------------------------- layout


@pytest.mark.parametrize("seed,rank", RANDOM_CASES)
def test_pair_table_matches_brute_force(seed, rank):
    p = _rand(seed, rank)
    lay = sectors.layout(p.left, p.right, p.target)
    table, n = sectors.pair_table(p.left, p.right, p.target)
    assert n == lay.n
    assert list(table.keys()) == lay.pairs
    assert [v[0] for v in table.values()] == list(lay.pair_offset[:-1])
    assert np.all(np.diff(lay.index_map) > 0)


def test_layout_counts_configs():
    # the Heisenberg S^z = 0 sector of 10 spins has binomial(10, 5) states
    p = gen.config(1)
    lay = sectors.layout(p.left, p.right, p.target)
    assert lay.n == 252 and len(lay.pairs) == 6
    q = gen.config(3)
    assert sectors.pair_table(q.left, q.right, q.target)[1] == 37668


def test_lr_split_reproduces_full_heisenberg_chain():
    """Config 1: H_L (x) I + I (x) H_R + cross terms equals Eq. 1 on 10 sites."""
    p = gen.heisenberg_exact(5, 5)
    HQ = projection.projected_hamiltonian(p)
    # map psi positions to product states of the full chain, independently of gen
    labs = models.spin_labels(5)
    permL = np.argsort(labs, kind="stable")
    lay = sectors.layout(p.left, p.right, p.target)
    a, b = lay.index_map // 32, lay.index_map % 32
    full = permL[a] * 32 + permL[b]
    Hfull = models.heisenberg_chain(10)
    assert np.array_equal(HQ, Hfull[np.ix_(full, full)])


def test_lr_split_reproduces_full_hubbard_chain():
    """Cross-cut hopping with the left parity on the source sector equals the
    Jordan-Wigner Hamiltonian of Eq. 4-6 (4 sites, N_up = N_dn = 2)."""
    p = gen.hubbard_exact(2, 2, t=1.0, U=4.0)
    HQ = projection.projected_hamiltonian(p)
    nm = 4
    st = np.arange(16)
    nup = sum(((st >> (nm - 1 - k)) & 1) for k in (1, 3))
    ndn = sum(((st >> (nm - 1 - k)) & 1) for k in (0, 2))
    permL = np.lexsort((st, ndn, nup))  # sector-grouped: labels (N_up, N_dn) ascending
    lay = sectors.layout(p.left, p.right, p.target)
    a, b = lay.index_map // 16, lay.index_map % 16
    full = permL[a] * 16 + permL[b]
    H, _, _ = models.hubbard_chain(4, t=1.0, U=4.0)
    assert np.abs(HQ - H[np.ix_(full, full)]).max() == 0.0
    w = np.linalg.eigvalsh(HQ)[0]
    assert w == pytest.approx(-1.95314530868455, abs=1e-12)


# --------------------------------------------------------------------------- projection


@pytest.mark.parametrize("seed,rank", RANDOM_CASES)
def test_sector_form_equals_kronecker_form(seed, rank):
    p = _rand(seed, rank)
    n = sectors.pair_table(p.left, p.right, p.target)[1]
    psi = np.random.default_rng(seed).standard_normal(n)
    y1 = projection.project_sectors(p, psi)
    y2 = projection.project_dense(p, psi)
    assert np.linalg.norm(y1 - y2) <= 1e-14 * max(1.0, np.linalg.norm(y2))


def test_kron_reshape_identity():
    # Eq. 10 in row-major form: kron(A, B) vec(X) = vec(A X B^T)
    rng = np.random.default_rng(3)
    A, B, X = rng.standard_normal((4, 3)), rng.standard_normal((5, 6)), rng.standard_normal((3, 6))
    assert np.allclose(np.kron(A, B) @ X.reshape(-1), (A @ X @ B.T).reshape(-1), atol=1e-14, rtol=0)


@pytest.mark.parametrize("cfg", [2, 3])
def test_hermitian_term_sets_are_symmetric(cfg):
    p = gen.config(cfg)
    n = sectors.pair_table(p.left, p.right, p.target)[1]
    rng = np.random.default_rng(cfg)
    u, v = rng.standard_normal(n), rng.standard_normal(n)
    a = u @ projection.project_sectors(p, v)
    b = v @ projection.project_sectors(p, u)
    assert abs(a - b) <= 1e-13 * abs(a)


def test_linear_in_coefficients():
    p = _rand(11, 2)
    n = sectors.pair_table(p.left, p.right, p.target)[1]
    rng = np.random.default_rng(0)
    psi = rng.standard_normal(n)
    c1, c2 = rng.standard_normal(len(p.coef)), rng.standard_normal(len(p.coef))
    y = projection.project_sectors(p, psi, 2.0 * c1 - c2)
    z = 2.0 * projection.project_sectors(p, psi, c1) - projection.project_sectors(p, psi, c2)
    assert np.linalg.norm(y - z) <= 1e-13 * np.linalg.norm(y)


def test_one_sided_term_is_a_plain_matmul():
    """With A = I the projection of every block is X B^T (a library matmul)."""
    p = gen.heisenberg_synthetic(128, seed=5)
    p.terms = np.array([[0, 1]], dtype=np.int32)  # I (x) H_R
    p.coef = np.array([1.0])
    table, n = sectors.pair_table(p.left, p.right, p.target)
    psi = np.random.default_rng(1).standard_normal(n)
    y = projection.project_sectors(p, psi)
    H = p.ops_right[1]
    for (sL, sR), (o, dL, dR) in table.items():
        k = list(H.src).index(sR)
        ref = psi[o:o + dL * dR].reshape(dL, dR) @ H.blocks[k].T
        assert np.array_equal(y[o:o + dL * dR], ref.reshape(-1))


def test_non_conserving_term_is_rejected():
    p = gen.heisenberg_synthetic(64, seed=1)
    p.terms = np.array([[3, 3]], dtype=np.int32)  # S+ (x) S+ changes S^z by 2
    p.coef = np.array([1.0])
    with pytest.raises(ValueError):
        projection.records(p)


@pytest.mark.parametrize("seed,rank", RANDOM_CASES[:6])
def test_diagonal_matches_dense(seed, rank):
    p = _rand(seed, rank)
    D = projection.diagonal(p)
    assert np.abs(D - np.diag(projection.projected_hamiltonian(p))).max() <= 1e-14 * max(1, np.abs(D).max())


# --------------------------------------------------------------------------- adjoint


@pytest.mark.parametrize("seed,rank", RANDOM_CASES)
def test_adjoint_dot_product(seed, rank):
    p = _rand(seed, rank)
    n = sectors.pair_table(p.left, p.right, p.target)[1]
    rng = np.random.default_rng(seed + 100)
    psi, g = rng.standard_normal(n), rng.standard_normal(n)
    lhs = g @ projection.project_sectors(p, psi)
    gpsi = projection.project_adjoint_sectors(p, g)
    assert abs(lhs - gpsi @ psi) <= 1e-13 * max(1.0, abs(lhs))
    assert np.linalg.norm(gpsi - projection.project_adjoint_dense(p, g)) <= 1e-13 * max(1.0, np.linalg.norm(gpsi))


def test_coef_gradient_finite_difference():
    p = _rand(4, 1)
    n = sectors.pair_table(p.left, p.right, p.target)[1]
    rng = np.random.default_rng(9)
    psi, g = rng.standard_normal(n), rng.standard_normal(n)
    gc = projection.coef_gradient(p, psi, g)
    h = 1e-3  # the map is linear in c, so central differences are exact up to rounding
    for k in range(len(p.coef)):
        cp, cm = p.coef.copy(), p.coef.copy()
        cp[k] += h
        cm[k] -= h
        fd = (g @ projection.project_sectors(p, psi, cp) - g @ projection.project_sectors(p, psi, cm)) / (2 * h)
        assert gc[k] == pytest.approx(fd, rel=1e-9, abs=1e-9)
    idx = sectors.layout(p.left, p.right, p.target).index_map
    for k in range(len(p.coef)):
        Tk = projection.term_matrix(p, k)[np.ix_(idx, idx)]
        assert gc[k] == pytest.approx(g @ Tk @ psi, rel=1e-12, abs=1e-12)


# --------------------------------------------------------------------------- FLOP rule


def test_flop_count_hand_case():
    # one two-sided record: A 3x2 block, X 2x4, B 5x4  ->  2 min(3*2*4 + 3*4*5, 2*4*5 + 3*2*5)
    L = gen.Space([[0], [1]], [2, 3])
    R = gen.Space([[-1], [0]], [5, 4])
    A = gen.Operator("dense", src=[0], dst=[1], blocks=[np.ones((3, 2))])
    B = gen.Operator("dense", src=[1], dst=[0], blocks=[np.ones((5, 4))])
    p = gen.Problem(L, R, [0], [A], [B], [(0, 0)], [1.0])
    assert projection.flop_count(p) == 2 * min(3 * 2 * 4 + 3 * 4 * 5, 2 * 4 * 5 + 3 * 2 * 5)


def test_flop_count_configs():
    assert projection.flop_count(gen.config(2)) == 223067808
    assert projection.flop_count(gen.config(3)) == 18194816


# --------------------------------------------------------------------------- precision emulation


def test_bf16_rounding_pins():
    x = np.array([1.0, 1 + 2.0 ** -8, 1 + 3 * 2.0 ** -8, -2.5, 1e-3, 3.0e38])
    r = precision.round_bf16(x)
    assert r[0] == 1.0
    assert r[1] == 1.0  # tie goes to even
    assert r[2] == 1 + 2.0 ** -6  # tie goes to even (upwards here)
    assert r[3] == -2.5
    torch = pytest.importorskip("torch")
    v = np.random.default_rng(0).standard_normal(10000) * 10.0 ** np.random.default_rng(1).integers(-20, 20, 10000)
    ref = torch.tensor(v.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(precision.round_bf16(v), ref)


def test_fp32_rounding_matches_struct():
    import struct
    v = np.random.default_rng(2).standard_normal(500) * 1e3
    ref = np.array([struct.unpack("f", struct.pack("f", float(x)))[0] for x in v])
    assert np.array_equal(precision.round_fp32(v), ref)


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_emulation_is_exact_for_representable_inputs(prec):
    """Small-integer operators and inputs are exact in BF16, so the emulated
    projection must equal the FP64 one."""
    p = gen.random_problem(21, rank=1, dmax=6)
    rng = np.random.default_rng(0)
    for op in p.ops_left + p.ops_right:
        if op.kind == "dense":
            op.blocks = [np.round(rng.uniform(-4, 4, b.shape)) for b in op.blocks]
        elif op.kind == "diag":
            op.diag = np.round(rng.uniform(-4, 4, op.diag.shape))
    p.coef = np.round(rng.uniform(-3, 3, p.coef.shape))
    n = sectors.pair_table(p.left, p.right, p.target)[1]
    psi = np.round(rng.uniform(-4, 4, n))
    assert np.array_equal(precision.project_emulated(p, psi, prec), projection.project_sectors(p, psi))


def test_magnitude_bounds_result():
    p = _rand(3, 2)
    n = sectors.pair_table(p.left, p.right, p.target)[1]
    psi = np.random.default_rng(3).standard_normal(n)
    assert np.all(np.abs(projection.project_sectors(p, psi)) <= precision.project_magnitude(p, psi) * (1 + 1e-12))


def _float32_projection(p, psi, prec, order_flip):
    """Eq. 11 evaluated with FP32 sums (NumPy float32 matmul), the operands
    rounded like the device's (FP64 diagonal split, rounded input, rounded
    intermediate), and the intermediate formed as X B^T instead of A X for
    every record where order_flip(i) is true: a second, independent reduced-
    precision evaluation for pinning the elementwise envelope."""
    rnd = precision.ROUND[prec]
    f32 = lambda a: rnd(a).astype(np.float32)
    recs, table, n = projection.records(p)
    y = np.zeros(n)
    for i, (k, pin, pout, pa, pb) in enumerate(recs):
        o, dL, dR = table[pin]
        X = np.asarray(psi[o:o + dL * dR], dtype=np.float64).reshape(dL, dR)
        o2, dL2, dR2 = table[pout]
        da = pa is not None and pa.ndim == 2
        db = pb is not None and pb.ndim == 2
        if not da and not db:
            Z = projection._right_t(pb, projection._left(pa, X))
        elif da and not db:
            Xs = projection._right_t(pb, X)
            R, dpart = pa, 0.0
            if pin[0] == pout[0]:
                R = pa - np.diag(np.diag(pa))
                dpart = np.diag(pa)[:, None] * Xs
            Z = dpart + (f32(R) @ f32(Xs)).astype(np.float64)
        elif db and not da:
            Xs = projection._left(pa, X)
            R, dpart = pb, 0.0
            if pin[1] == pout[1]:
                R = pb - np.diag(np.diag(pb))
                dpart = Xs * np.diag(pb)[None, :]
            Z = dpart + (f32(Xs) @ f32(R).T).astype(np.float64)
        elif order_flip(i):
            T = f32((f32(X) @ f32(pb).T).astype(np.float64))
            Z = (f32(pa) @ T).astype(np.float64)
        else:
            T = f32((f32(pa) @ f32(X)).astype(np.float64))
            Z = (T @ f32(pb).T).astype(np.float64)
        y[o2:o2 + dL2 * dR2] += (p.coef[k] * Z).reshape(-1)
    return y


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
@pytest.mark.parametrize("seed", range(6))
def test_envelope_holds_for_an_independent_fp32_evaluation(prec, seed):
    """The elementwise envelope contains an FP32-accumulated evaluation with
    either order of the two-sided products (what the device may do)."""
    p = gen.random_problem(40 + seed, rank=1 + seed % 2, dmax=40)
    n = sectors.pair_table(p.left, p.right, p.target)[1]
    psi = np.random.default_rng(seed).standard_normal(n)
    emul = precision.project_emulated(p, psi, prec)
    env = precision.project_envelope(p, psi, prec)
    for flip in (lambda i: False, lambda i: True, lambda i: i % 2 == 1):
        y = _float32_projection(p, psi, prec, flip)
        assert np.all(np.abs(y - emul) <= env), prec


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_envelope_catches_a_missing_or_transposed_contribution(prec):
    """Tight enough to fail on a plausible device bug.  The envelope is an
    elementwise fraction of the magnitude (about 1e-5 for FP32, 1 % for BF16:
    the operand rounding itself), so in FP32 any single record left out, or
    one block applied transposed, breaks the bound somewhere; in BF16 every
    record that carries more than 1.2 % of an entry's magnitude does."""
    p = gen.random_problem(7, rank=1, dmax=9, square=True)
    n = sectors.pair_table(p.left, p.right, p.target)[1]
    psi = np.random.default_rng(1).standard_normal(n)
    emul = precision.project_emulated(p, psi, prec)
    env = precision.project_envelope(p, psi, prec)
    mag = precision.project_magnitude(p, psi)
    K = precision.max_contraction(p)
    width = 1.25 * (K * 2.0 ** -24 + 2 * precision.UNIT[prec])
    assert np.all(env <= width * mag)
    recs, table, _ = projection.records(p)
    checked = 0
    for k, pin, pout, pa, pb in recs:
        o, dL, dR = table[pin]
        X = psi[o:o + dL * dR].reshape(dL, dR)
        o2, dL2, dR2 = table[pout]
        Z = p.coef[k] * projection._right_t(pb, projection._left(pa, X))
        if prec == "fp32" and np.abs(Z).max() < 1e-6:
            continue
        if prec == "bf16" and not np.any(np.abs(Z).reshape(-1) > 1.2 * width * mag[o2:o2 + dL2 * dR2]):
            continue
        bad = emul.copy()
        bad[o2:o2 + dL2 * dR2] -= Z.reshape(-1)  # the record is missing
        assert np.any(np.abs(bad - emul) > env)
        if pa is not None and pa.ndim == 2 and pa.shape[0] == pa.shape[1] and not np.allclose(pa, pa.T):
            Zt = p.coef[k] * projection._right_t(pb, pa.T @ X)
            bad = emul.copy()
            bad[o2:o2 + dL2 * dR2] += (Zt - Z).reshape(-1)  # A applied transposed
            if prec == "fp32":
                assert np.any(np.abs(bad - emul) > env)
        checked += 1
    assert checked >= 5
