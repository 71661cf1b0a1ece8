"""GPU parity of the operator transform to the kept basis (Alg. 1, step 7)
against the oracle, called through the C ABI.

The device's own density-matrix eigenvectors and kept counts are the input
of both sides, so the comparison isolates this step.  Tolerance: each entry
is a sum of products over two contractions of lengths cols and rows, so the
error is at most 2 (rows + cols) u (|U_dst|^T |O| |U_src|) entrywise
(u = 2^-53); the bound matrix is the oracle's transform of the absolute
values.
"""
import numpy as np
import pytest

import gen
from oracle import density, sectors

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


def _left_basis(p, pl, psi, m):
    """rho_L, its eigenvectors and the kept counts, on the device."""
    rl, _ = pl.density(torch.from_numpy(psi).cuda(), right=False)
    lo, _ = pl.density_layout()
    dims = np.sqrt(np.diff(lo)).round().astype(int)
    w, u = _dm().eigh_blocks(rl, dims)
    keep, _ = _dm().truncate(w, dims, m)
    lay = pl.layout()
    sec = {int(s): k for k, s in enumerate(lay["pair_left"])}  # left sector -> pair index
    return u, lo, dims, keep, sec


def _blocks_of(p, sec, lo, keep):
    """Renormalization requests for every block of every non-identity left
    operator between sectors that have a pair, and the host data they read."""
    data, reqs, meta = [], [], []
    pos = 0
    out = 0
    offs = p.left.offsets()
    for op in p.ops_left:
        if op.kind == "identity":
            continue
        if op.kind == "diag":
            items = [(s, s, op.diag[offs[s]:offs[s + 1]]) for s in range(p.left.nsec)]
        else:
            items = [(int(s), int(d), blk) for s, d, blk in zip(op.src, op.dst, op.blocks)]
        for s, t, blk in items:
            if s not in sec or t not in sec:
                continue
            ps, pt = sec[s], sec[t]
            rows, cols = int(p.left.dims[t]), int(p.left.dims[s])
            kd, ks = int(keep[pt]), int(keep[ps])
            diag = 1 if np.ndim(blk) == 1 else 0
            reqs.append((pos, int(lo[pt]), int(lo[ps]), out, rows, cols, kd, ks, diag))
            meta.append((blk, pt, ps, rows, cols, kd, ks))
            data.append(np.asarray(blk, dtype=np.float64).reshape(-1))
            pos += data[-1].size
            out += kd * ks
    return np.concatenate(data), reqs, meta, out


def _check(u, meta, reqs, got):
    uh = u.cpu().numpy()
    g = got.cpu().numpy()
    for (blk, pt, ps, rows, cols, kd, ks), r in zip(meta, reqs):
        Ut = uh[r[1]:r[1] + rows * rows].reshape(rows, rows)
        Us = uh[r[2]:r[2] + cols * cols].reshape(cols, cols)
        want = density.renormalize_block(blk, Ut, Us, kd, ks)
        bound = density.renormalize_block(np.abs(blk), np.abs(Ut), np.abs(Us), kd, ks)
        have = g[r[3]:r[3] + kd * ks].reshape(kd, ks)
        assert np.all(np.abs(have - want) <= 2 * (rows + cols) * U64 * bound + 1e-300)


@pytest.mark.parametrize("seed,rank,m", [(s, r, m) for s in range(4) for r in (1, 2) for m in (5, 40)])
def test_renormalize_random_problems(seed, rank, m):
    p = gen.random_problem(seed, rank=rank, dmax=60)
    pl = _dm().Plan(p)
    psi = gen.start_vector(pl.n, seed + 1)
    u, lo, dims, keep, sec = _left_basis(p, pl, psi, m)
    data, reqs, meta, nout = _blocks_of(p, sec, lo, keep)
    got = _dm().renormalize(torch.from_numpy(data).cuda(), u, reqs, nout)
    _check(u, meta, reqs, got)


@pytest.mark.parametrize("cfg,m", [(3, 512), (2, 256)])
def test_renormalize_full_size_workloads(cfg, m):
    """Every left operator of the Hubbard m = 2048 and Heisenberg m = 1024
    workloads, after steps 5 and 6 on the device and keeping m states."""
    p = gen.config(cfg)
    pl = _dm().Plan(p)
    psi = gen.start_vector(pl.n, 9)
    psi /= np.linalg.norm(psi)
    u, lo, dims, keep, sec = _left_basis(p, pl, psi, m)
    assert keep.sum() == m
    data, reqs, meta, nout = _blocks_of(p, sec, lo, keep)
    got = _dm().renormalize(torch.from_numpy(data).cuda(), u, reqs, nout)
    _check(u, meta, reqs, got)


def test_renormalize_identity_and_edge_counts():
    """Keeping everything of a diagonal block of ones gives the identity
    (orthonormal eigenvectors); zero kept states give empty results."""
    p = gen.random_problem(2, rank=1, dmax=40)
    pl = _dm().Plan(p)
    psi = gen.start_vector(pl.n, 4)
    u, lo, dims, keep, sec = _left_basis(p, pl, psi, 10 ** 6)  # keep all
    reqs, pos, out = [], 0, 0
    for k, d in enumerate(dims):
        reqs.append((pos, int(lo[k]), int(lo[k]), out, int(d), int(d), int(d), int(d), 1))
        pos += int(d)
        out += int(d) * int(d)
    ones = torch.ones(pos, dtype=torch.float64).cuda()
    got = _dm().renormalize(ones, u, reqs, out).cpu().numpy()
    o = 0
    for d in dims:
        np.testing.assert_allclose(got[o:o + d * d].reshape(d, d), np.eye(d), atol=8 * d * U64)
        o += d * d
    d0 = int(dims[0])
    empty = _dm().renormalize(ones, u, [(0, int(lo[0]), int(lo[0]), 0, d0, d0, 0, d0, 1)], 1)
    assert empty.numel() == 1


def test_renormalize_rejects_bad_requests():
    from paper_1309_5571_amd import _native as N

    x = torch.zeros(16, dtype=torch.float64).cuda()
    with pytest.raises(N.DmrgError):
        _dm().renormalize(x, x.clone(), [(0, 0, 0, 0, 4, 4, 5, 4, 0)], 16)  # k_dst > rows
    with pytest.raises(N.DmrgError):
        _dm().renormalize(x, x.clone(), [(0, 0, 0, 0, 2, 3, 1, 1, 1)], 16)  # diagonal, not square
