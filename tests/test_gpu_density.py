"""GPU parity of the reduced density matrices (Alg. 1, step 5) against the
FP64 oracle, called through the C ABI.

Tolerance: each entry is an FP64 dot product of length K (the pair's other
dimension), so |rho_gpu - rho| <= 2 K u (|Psi| |Psi|^T) entrywise with
u = 2^-53; the bound matrix is the oracle's density of |psi|.
"""
import numpy as np
import pytest

import gen
from oracle import davidson, density, sectors

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

U64 = 2.0 ** -53


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _plan(p, prec="f64"):
    import paper_1309_5571_amd as dm

    return dm.Plan(p, prec=prec)


def _dev(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).cuda()


def _check(problems, psi, rl, rr):
    """Entrywise parity within the FP64 dot-product bound, and exact symmetry."""
    if not isinstance(problems, list):
        problems = [problems]
    refs_l, refs_r, bnd_l, bnd_r, dims = [], [], [], [], []
    off = 0
    for p in problems:
        n = sectors.pair_table(p.left, p.right, p.target)[1]
        x = psi[off:off + n]
        off += n
        fl, fr = density.density_flat(p, x)
        bl, br = density.density_flat(p, np.abs(x))
        refs_l.append(fl), refs_r.append(fr), bnd_l.append(bl), bnd_r.append(br)
        dims += list(sectors.pair_table(p.left, p.right, p.target)[0].values())
    ref_l, ref_r = np.concatenate(refs_l), np.concatenate(refs_r)
    kmax = max(max(d[1], d[2]) for d in dims)
    for got, ref, bnd in ((rl, ref_l, np.concatenate(bnd_l)), (rr, ref_r, np.concatenate(bnd_r))):
        if got is None:
            continue
        g = got.cpu().numpy()
        assert g.shape == ref.shape
        assert np.all(np.abs(g - ref) <= 2 * kmax * U64 * bnd + 1e-300)
    # exact symmetry of every block
    lo, ro = 0, 0
    for (_, dl, dr) in dims:
        for got, o, d in ((rl, lo, dl), (rr, ro, dr)):
            if got is None:
                continue
            B = got[o:o + d * d].cpu().numpy().reshape(d, d)
            assert np.array_equal(B, B.T)
        lo += dl * dl
        ro += dr * dr


@pytest.mark.parametrize("seed,rank,dmax", [(s, r, d) for s in range(6) for r in (1, 2) for d in (12, 70)])
def test_density_random_matches_oracle(seed, rank, dmax):
    p = gen.random_problem(seed, rank=rank, dmax=dmax)
    pl = _plan(p)
    psi = gen.start_vector(pl.n, seed + 11)
    lo, ro = pl.density_layout()
    fl, fr = density.density_flat(p, psi)
    assert lo[-1] == fl.size and ro[-1] == fr.size
    rl, rr = pl.density(_dev(psi))
    _check(p, psi, rl, rr)


@pytest.mark.parametrize("cfg", [2, 3])
def test_density_full_size_configs(cfg):
    """Heisenberg m = 1024 (blocks up to 180) and Hubbard m = 2048 (241 pairs)."""
    p = gen.config(cfg)
    pl = _plan(p)
    psi = gen.start_vector(pl.n, 7)
    rl, rr = pl.density(_dev(psi))
    torch.cuda.synchronize()
    _check(p, psi, rl, rr)
    # both traces equal |psi|^2
    lo, ro = pl.density_layout()
    nrm2 = float(psi @ psi)
    for rho, off in ((rl, lo), (rr, ro)):
        tr = sum(float(torch.trace(rho[off[k]:off[k + 1]].view(int(np.sqrt(off[k + 1] - off[k])), -1)))
                 for k in range(pl.npair))
        assert abs(tr - nrm2) <= 1e-12 * nrm2


def test_density_batched_members():
    probs = gen.config(4)
    pl = _plan(probs)
    psi = gen.start_vector(pl.n, 3)
    rl, rr = pl.density(_dev(psi))
    _check(list(probs), psi, rl, rr)


def test_density_one_side_only():
    p = gen.random_problem(3, rank=2, dmax=40)
    pl = _plan(p)
    psi = gen.start_vector(pl.n, 5)
    rl, _ = pl.density(_dev(psi), right=False)
    _, rr = pl.density(_dev(psi), left=False)
    _check(p, psi, rl, None)
    _check(p, psi, None, rr)


def test_density_tiny_blocks_and_zero_state():
    p = gen.heisenberg_exact(1, 1)  # two 1x1 pairs
    pl = _plan(p)
    rl, rr = pl.density(_dev(np.zeros(pl.n)))
    assert torch.count_nonzero(rl).item() == 0 and torch.count_nonzero(rr).item() == 0
    psi = np.array([0.6, -0.8])
    rl, rr = pl.density(_dev(psi))
    want = [0.6 * 0.6, 0.8 * 0.8]  # one product each, rounded once
    assert rl.cpu().tolist() == want and rr.cpu().tolist() == want


def test_density_rejects_overlap():
    from paper_1309_5571_amd import _native as N

    p = gen.random_problem(1)
    pl = _plan(p)
    psi = _dev(gen.start_vector(pl.n, 1))
    st = N.lib().dmrg_density(pl._h, psi.data_ptr(), psi.data_ptr(), None, None)
    assert st == N.E_INVALID_ARG
    assert "overlap" in N.last_error()
    assert N.lib().dmrg_density(None, psi.data_ptr(), None, None, None) == N.E_INVALID_ARG


def test_xx_ground_state_density_spectrum_on_gpu():
    """Alg. 1, steps 3 and 5 on the device: the Davidson ground state of the
    open XX chain of 8 sites, then the left block's density matrix; its
    spectrum per sector equals the oracle's (free-fermion pinned)."""
    p = gen.heisenberg_exact(4, 4, delta=0.0)
    pl = _plan(p)
    _, psi_ref, _ = davidson.ground_state_dense(p)
    x0 = gen.start_vector(pl.n, 2)
    psi, _, infos, st = pl.davidson(_dev(x0), tol=1e-12)
    assert st == 0 and infos[0]["converged"]
    rl, _ = pl.density(psi)
    got, _ = density.density_sectors(p, psi.cpu().numpy())
    ref, _ = density.density_sectors(p, psi_ref)
    lo, _ = pl.density_layout()
    for k, (g, r) in enumerate(zip(got, ref)):
        d = r.shape[0]
        blk = rl[lo[k]:lo[k + 1]].cpu().numpy().reshape(d, d)
        np.testing.assert_allclose(np.linalg.eigvalsh(blk), np.linalg.eigvalsh(r), atol=1e-10)
