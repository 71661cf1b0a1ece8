"""GPU parity of the blockwise eigen-decomposition (Alg. 1, step 6) against
the oracle (LAPACK through NumPy), called through the C ABI.

Tolerances follow the backward error of the device methods (Jacobi up to
order 8, Householder tridiagonalization + divide and conquer or implicit QL
above), a small
multiple of d u |A|_F per block (u = 2^-53, d the block order): eigenvalues and the
reconstruction U diag(w) U^T within 16 d u |A|_F, U^T U within 16 d u of
the identity, and each eigenvector within 16 d u |A|_F / gap of the oracle's
(up to sign) where its eigenvalue is separated by `gap` from the others.
"""
import numpy as np
import pytest

import gen
from oracle import davidson, density

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

U64 = 2.0 ** -53


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _dm():
    import paper_1309_5571_amd as dm

    return dm


def _run(blocks):
    dims = [b.shape[0] for b in blocks]
    flat = np.concatenate([b.reshape(-1) for b in blocks])
    w, u, info = _dm().eigh_blocks(torch.from_numpy(flat).cuda(), dims, return_info=True)
    w, u, info = w.cpu().numpy(), u.cpu().numpy(), info.cpu().numpy()
    out, o, ow = [], 0, 0
    for d in dims:
        out.append((w[ow:ow + d], u[o:o + d * d].reshape(d, d)))
        o += d * d
        ow += d
    return out, info


def _check(blocks, res):
    vals, vecs = density.eigh_blocks(blocks)
    for B, (w, U), wr, Ur in zip(blocks, res, vals, vecs):
        d = B.shape[0]
        fro = max(float(np.linalg.norm(B)), 1e-300)
        tol = 16 * d * U64 * fro
        assert np.all(np.diff(w) <= 0)
        assert np.max(np.abs(w - wr)) <= tol
        assert np.max(np.abs(U @ np.diag(w) @ U.T - B)) <= tol
        assert np.max(np.abs(U.T @ U - np.eye(d))) <= 16 * d * U64
        for j in range(d):
            k = int(np.argmax(np.abs(U[:, j])))
            assert U[k, j] > 0
            others = np.delete(wr, j)
            gap = float(np.min(np.abs(others - wr[j]))) if d > 1 else np.inf
            if gap > 1e-8 * fro:
                sgn = 1.0 if U[:, j] @ Ur[:, j] >= 0 else -1.0
                assert np.max(np.abs(sgn * U[:, j] - Ur[:, j])) <= tol / gap + 1e-14


def _sym(rng, d):
    G = rng.standard_normal((d, d))
    return (G + G.T) / 2


def _psd(rng, d, r):
    X = rng.standard_normal((d, r))
    return X @ X.T


@pytest.mark.parametrize("seed", range(3))
def test_eigh_random_blocks_small_and_large(seed):
    rng = np.random.default_rng(seed)
    dims = [1, 2, 3, 17, 47, 48, 49, 64, 100, 181]
    blocks = []
    for d in dims:
        blocks.append(_sym(rng, d))
        blocks.append(_psd(rng, d, max(1, d // 2)))  # rank-deficient, like rho_L when d_L > d_R
    res, info = _run(blocks)
    assert np.all(info >= 1)
    _check(blocks, res)


def test_eigh_kernel_boundary_orders():
    """Orders at the edges of each kernel's range: the register reduction's row
    counts (4, 16, 36 rows per thread up to 64, 128, 180), the global-memory
    reduction above 180, the last divide-and-conquer order (512: 32 panels of
    the reflector back-transformation) and the first QL one; random, rank-
    deficient, already tridiagonal (every reflector the identity) and block
    diagonal (some columns already reduced) blocks."""
    rng = np.random.default_rng(9)
    blocks = []
    for d in (9, 16, 64, 65, 128, 129, 180, 181, 512, 513):
        blocks.append(_sym(rng, d))
        blocks.append(_psd(rng, d, max(1, d // 3)))
    d = 130
    T = np.diag(rng.standard_normal(d)) + np.diag(rng.standard_normal(d - 1), 1)
    blocks.append(T + np.triu(T, 1).T)
    B = np.zeros((90, 90))
    X = rng.standard_normal((40, 40))
    B[:40, :40] = X + X.T
    B[50:, 50:] = 3.0 * np.eye(40)
    blocks.append(B)
    res, info = _run(blocks)
    assert np.all(info >= 1)
    _check(blocks, res)


def test_eigh_large_orders():
    """The tridiagonal path at the orders of the 64-member batch (361) and up
    to the largest supported one, random and density-like (rank-deficient,
    exponentially decaying spectrum) blocks."""
    rng = np.random.default_rng(21)
    blocks = [_sym(rng, 361), _psd(rng, 700, 350), _sym(rng, 2048)]
    X = rng.standard_normal((400, 1200)) * np.exp(-np.arange(400) / 6.0)[:, None]
    rho = X @ X.T
    blocks.append(rho / np.trace(rho))
    res, info = _run(blocks)
    assert np.all(info >= 1)
    _check(blocks, res)


def test_eigh_degenerate_and_special_blocks():
    rng = np.random.default_rng(5)
    D = np.diag(rng.standard_normal(20))
    D2 = np.diag(rng.standard_normal(80))
    blocks = [np.zeros((3, 3)), np.eye(7), 2.5 * np.eye(60), D, np.array([[0.0, 1.0], [1.0, 0.0]]), D2,
              np.zeros((50, 50))]
    res, info = _run(blocks)
    assert np.all(info >= 1)
    # already diagonal: no rotation, eigenvalues are the diagonal sorted, exactly
    w, U = res[3]
    assert np.array_equal(w, np.sort(np.diag(D))[::-1])
    assert np.array_equal(np.abs(U), np.abs(U).round())
    w, U = res[5]  # the same on the tridiagonal path (no reflection, no QL step)
    assert np.array_equal(w, np.sort(np.diag(D2))[::-1])
    assert np.array_equal(np.abs(U), np.abs(U).round())
    for (w, U), B in zip(res[:3] + res[6:], blocks[:3] + blocks[6:]):
        assert np.array_equal(w, np.diag(B)) and np.array_equal(U, np.eye(B.shape[0]))
    w, U = res[4]
    np.testing.assert_allclose(w, [1.0, -1.0], atol=1e-15)
    _check(blocks, res)


@pytest.mark.parametrize("cfg", [2, 3])
def test_eigh_of_density_blocks(cfg):
    """Alg. 1, steps 5 and 6 on the device: density matrices of both blocks of
    a full-size workload, then their eigen-decomposition."""
    p = gen.config(cfg)
    pl = _dm().Plan(p)
    psi = gen.start_vector(pl.n, 13)
    psi /= np.linalg.norm(psi)
    rl, rr = pl.density(torch.from_numpy(psi).cuda())
    lo, ro = pl.density_layout()
    dl = np.sqrt(np.diff(lo)).round().astype(int)
    dr = np.sqrt(np.diff(ro)).round().astype(int)
    for rho, dims in ((rl, dl), (rr, dr)):
        # the device's density blocks are the input of both sides (step 5 has its own parity tests)
        host = rho.cpu().numpy()
        ref, o = [], 0
        for d in dims:
            ref.append(host[o:o + d * d].reshape(d, d))
            o += d * d
        w, u, info = _dm().eigh_blocks(rho, dims, return_info=True)
        assert np.all(info.cpu().numpy() >= 1)
        w, u = w.cpu().numpy(), u.cpu().numpy()
        res, o, ow = [], 0, 0
        for d in dims:
            res.append((w[ow:ow + d], u[o:o + d * d].reshape(d, d)))
            o += d * d
            ow += d
        _check(ref, res)
        # eigenvalues of a density matrix of a unit state: non-negative, sum 1
        assert w.min() > -1e-12 and abs(w.sum() - 1.0) < 1e-12


def test_xx_chain_step_5_and_6_on_gpu():
    """Davidson ground state, density matrix and its spectrum, all on the
    device, against the free-fermion-pinned oracle spectrum."""
    p = gen.heisenberg_exact(4, 4, delta=0.0)
    pl = _dm().Plan(p)
    psi, _, infos, st = pl.davidson(torch.from_numpy(gen.start_vector(pl.n, 2)).cuda(), tol=1e-12)
    assert st == 0
    rl, _ = pl.density(psi)
    lo, _ = pl.density_layout()
    dims = np.sqrt(np.diff(lo)).round().astype(int)
    w, _ = _dm().eigh_blocks(rl, dims)
    _, psi_ref, _ = davidson.ground_state_dense(p)
    vals, _ = density.eigh_blocks(density.density_sectors(p, psi_ref)[0])
    np.testing.assert_allclose(w.cpu().numpy(), np.concatenate(vals), atol=1e-10)


def test_eigh_rejects_unsupported_order_on_device():
    """A block order beyond 2048 is reported in info and the block untouched."""
    from paper_1309_5571_amd import _native as N

    a = torch.arange(4, dtype=torch.float64).cuda()
    w = torch.full((2,), 7.0, dtype=torch.float64).cuda()
    u = torch.full((4,), 7.0, dtype=torch.float64).cuda()
    off = torch.tensor([0], dtype=torch.int64).cuda()
    dim = torch.tensor([4096], dtype=torch.int32).cuda()
    woff = torch.tensor([0], dtype=torch.int64).cuda()
    info = torch.zeros(1, dtype=torch.int32).cuda()
    st = N.lib().dmrg_eigh_blocks(1, off.data_ptr(), dim.data_ptr(), woff.data_ptr(), a.data_ptr(), w.data_ptr(),
                                  u.data_ptr(), info.data_ptr(), None)
    torch.cuda.synchronize()
    assert st == N.OK and int(info[0]) == -1
    assert torch.all(u == 7.0) and torch.all(w == 7.0)
    assert N.lib().dmrg_eigh_blocks(1, off.data_ptr(), dim.data_ptr(), woff.data_ptr(), a.data_ptr(), w.data_ptr(),
                                    a.data_ptr(), None, None) == N.E_INVALID_ARG
    with pytest.raises(ValueError):
        _dm().eigh_blocks(a, [3000])


# ------------------------------------------------------------------ step 7: state selection


def _desc_blocks(rng, dims, ties=True):
    vals = []
    for d in dims:
        v = rng.choice([0.5, 0.25, 0.125, 0.0], size=d) if ties else rng.random(d)
        vals.append(np.sort(v)[::-1].copy())
    return vals


@pytest.mark.parametrize("ties", [True, False])
def test_truncate_matches_oracle_exactly(ties):
    rng = np.random.default_rng(11 if ties else 12)
    dims = [3, 1, 7, 40, 2, 33]
    vals = _desc_blocks(rng, dims, ties)
    w = torch.from_numpy(np.concatenate(vals)).cuda()
    total = sum(dims)
    for m in (0, 1, 5, total // 2, total - 1, total, total + 9):
        keep, disc = _dm().truncate(w, dims, m)
        counts, ref = density.truncate(vals, m)
        assert keep.tolist() == counts.tolist()
        assert abs(disc[0] - ref) <= 1e-14 * total


def test_truncate_groups_are_independent():
    rng = np.random.default_rng(3)
    dims = [4, 9, 2, 6, 6, 1, 30]
    groups = [3, 0, 2, 2]
    ms = [5, 2, 3, 10]
    vals = _desc_blocks(rng, dims)
    keep, disc = _dm().truncate(torch.from_numpy(np.concatenate(vals)).cuda(), dims, ms, groups=groups)
    b = 0
    for g, (cnt, m) in enumerate(zip(groups, ms)):
        counts, ref = density.truncate(vals[b:b + cnt], m)
        assert keep[b:b + cnt].tolist() == counts.tolist()
        assert abs(disc[g] - ref) <= 1e-13
        b += cnt


@pytest.mark.parametrize("cfg,m", [(3, 256), (2, 128)])
def test_steps_5_to_7_on_full_size_workloads(cfg, m):
    """Density matrices, their eigenvalues and the kept states, all on the
    device; the selection matches the oracle's on the device's eigenvalues and
    the kept weight is within rounding of the oracle's full FP64 chain."""
    p = gen.config(cfg)
    pl = _dm().Plan(p)
    psi = gen.start_vector(pl.n, 21)
    psi /= np.linalg.norm(psi)
    rl, _ = pl.density(torch.from_numpy(psi).cuda())
    lo, _ = pl.density_layout()
    dims = np.sqrt(np.diff(lo)).round().astype(int)
    w, _ = _dm().eigh_blocks(rl, dims)
    keep, disc = _dm().truncate(w, dims, m)
    wh, o, vals = w.cpu().numpy(), 0, []
    for d in dims:
        vals.append(wh[o:o + d])
        o += d
    counts, ref = density.truncate(vals, m)
    assert keep.tolist() == counts.tolist() and keep.sum() == min(m, dims.sum())
    assert abs(disc[0] - ref) <= 1e-13
    ovals, _ = density.eigh_blocks(density.density_sectors(p, psi)[0])
    _, ref64 = density.truncate(ovals, m)
    assert abs(disc[0] - ref64) <= 1e-12


def test_truncate_batched_members():
    probs = gen.config(4)
    pl = _dm().Plan(probs)
    psi = gen.start_vector(pl.n, 5)
    rl, _ = pl.density(torch.from_numpy(psi).cuda())
    lo, _ = pl.density_layout()
    dims = np.sqrt(np.diff(lo)).round().astype(int)
    lay = pl.layout()
    groups = np.bincount(lay["member"], minlength=len(probs))
    w, _ = _dm().eigh_blocks(rl, dims)
    keep, disc = _dm().truncate(w, dims, 100, groups=groups)
    wh, o, vals = w.cpu().numpy(), 0, []
    for d in dims:
        vals.append(wh[o:o + d])
        o += d
    b = 0
    for g, cnt in enumerate(groups):
        counts, ref = density.truncate(vals[b:b + cnt], 100)
        assert keep[b:b + cnt].tolist() == counts.tolist()
        assert abs(disc[g] - ref) <= 1e-12 * max(1.0, abs(ref))
        b += cnt


def test_truncate_reports_oversized_group():
    from paper_1309_5571_amd import _native as N

    w = torch.zeros(4, dtype=torch.float64).cuda()
    gblk = torch.tensor([0, 1], dtype=torch.int32).cuda()
    dim = torch.tensor([20000], dtype=torch.int32).cuda()
    woff = torch.tensor([0], dtype=torch.int64).cuda()
    m = torch.tensor([5], dtype=torch.int32).cuda()
    keep = torch.zeros(1, dtype=torch.int32).cuda()
    disc = torch.zeros(1, dtype=torch.float64).cuda()
    st = N.lib().dmrg_truncate(1, gblk.data_ptr(), dim.data_ptr(), woff.data_ptr(), w.data_ptr(), m.data_ptr(),
                               keep.data_ptr(), disc.data_ptr(), None)
    torch.cuda.synchronize()
    assert st == N.OK and int(keep[0]) == -1 and torch.isnan(disc[0])
    with pytest.raises(ValueError):
        _dm().truncate(w, [20000], 5)


def test_truncate_signed_zero_ties_like_equal_values():
    """-0 and +0 are equal values: their order is the storage order."""
    vals = [np.array([0.5, 0.0, -0.0]), np.array([0.0, -0.0]), np.array([-0.0, -1.0])]
    dims = [3, 2, 2]
    w = torch.from_numpy(np.concatenate(vals)).cuda()
    for m in range(0, 8):
        keep, disc = _dm().truncate(w, dims, m)
        counts, ref = density.truncate(vals, m)
        assert keep.tolist() == counts.tolist() and disc[0] == ref
