"""Pins of the l-1-1-r oracle (oracle.l11r): the sector-wise evaluation of
Eq. 13 against the four-fold Kronecker definition (Eq. 12) and the LR form
of the same superblock; whole-chain spectra against exact diagonalization
of Eq. 1-8; planted mistakes that the pins must catch."""
import json
import os

import numpy as np
import pytest

import gen
from oracle import l11r, models, projection

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "exact_energies.json")))["energies"]

RANDOM = [(s, r) for s in range(8) for r in (1, 2)]


@pytest.mark.parametrize("seed,rank", RANDOM)
def test_sectorwise_equals_kronecker_definition(seed, rank):
    p = gen.random_problem4(seed, rank=rank)
    n = l11r.layout(p).n
    psi = np.random.default_rng(seed).standard_normal(n)
    y = l11r.project_sectors(p, psi)
    ref = l11r.project_dense(p, psi)
    assert np.linalg.norm(y - ref) <= 1e-14 * max(np.linalg.norm(ref), 1e-300)
    # and the LR form of the same superblock (enlarged blocks) gives the same vector
    ylr = projection.project_sectors(l11r.to_lr(p), psi)
    assert np.linalg.norm(ylr - ref) <= 1e-14 * max(np.linalg.norm(ref), 1e-300)


@pytest.mark.parametrize("seed", range(4))
def test_enlarged_basis_is_a_sector_grouped_permutation(seed):
    p = gen.random_problem4(seed, rank=1 + seed % 2)
    for slow, fast in ((p.spaces[0], p.spaces[1]), (p.spaces[2], p.spaces[3])):
        idx = l11r.enlarged_index(slow, fast)
        assert sorted(idx.tolist()) == list(range(idx.size))  # a bijection
        # labels of the enlarged basis, in its order, ascend lexicographically
        lab_s = np.repeat(slow.labels, slow.dims, axis=0)
        lab_f = np.repeat(fast.labels, fast.dims, axis=0)
        lab = (lab_s[:, None, :] + lab_f[None, :, :]).reshape(-1, slow.labels.shape[1])
        ordered = np.empty_like(lab)
        ordered[idx] = lab
        keys = [tuple(x) for x in ordered]
        assert keys == sorted(keys)


def _sector_spectrum(H, mask):
    idx = np.flatnonzero(mask)
    return np.linalg.eigvalsh(H[np.ix_(idx, idx)])


def test_heisenberg_ten_sites_spectrum():
    """4 + 1 + 1 + 4 sites: the projected H has exactly the spectrum of the
    whole open chain (Eq. 1) in S^z = 0, and its ground energy is the stored
    exact value."""
    p = gen.heisenberg_l11r(4, 4)
    H = l11r.projected_hamiltonian(p)
    assert np.allclose(H, H.T, atol=1e-14)
    w = np.linalg.eigvalsh(H)
    ref = _sector_spectrum(models.heisenberg_chain(10), models.spin_labels(10) == 0)
    assert w.shape == ref.shape == (252,)
    assert np.max(np.abs(w - ref)) <= 1e-12
    assert abs(w[0] - GOLDEN["heisenberg_open_N10_Sz0"]) <= 1e-12


@pytest.mark.parametrize("nl", [1, 2])
def test_hubbard_chain_spectrum(nl):
    """nl + 1 + 1 + nl Hubbard sites at half filling, with Jordan-Wigner signs
    across all three cuts: the spectrum of the whole chain (Eq. 4-8)."""
    p = gen.hubbard_l11r_exact(nl, nl)
    N = 2 * nl + 2
    H = l11r.projected_hamiltonian(p)
    assert np.allclose(H, H.T, atol=1e-13)
    Hc, Nup, Ndn = models.hubbard_chain(N)
    mask = (np.rint(np.diag(Nup)) == N // 2) & (np.rint(np.diag(Ndn)) == N // 2)
    ref = _sector_spectrum(Hc, mask)
    w = np.linalg.eigvalsh(H)
    assert w.shape == ref.shape
    assert np.max(np.abs(w - ref)) <= 1e-11
    if N == 4:
        assert abs(w[0] - GOLDEN["hubbard_open_N4_t1_U4_half"]) <= 1e-12


def test_synthetic_hubbard_is_hermitian_and_linear():
    p = gen.hubbard_l11r_synthetic(64, seed=3)
    n = l11r.layout(p).n
    rng = np.random.default_rng(1)
    u, v = rng.standard_normal(n), rng.standard_normal(n)
    Hu, Hv = l11r.project_sectors(p, u), l11r.project_sectors(p, v)
    assert abs(u @ Hv - Hu @ v) <= 1e-13 * np.linalg.norm(Hu) * np.linalg.norm(v)
    c = rng.standard_normal(len(p.coef))
    lin = sum(c[k] * l11r.project_sectors(p, u, coef=np.eye(len(c))[k]) for k in range(len(c)))
    assert np.allclose(l11r.project_sectors(p, u, coef=c), lin, rtol=0, atol=1e-12 * np.abs(lin).max())


def test_planted_mistakes_are_caught(monkeypatch):
    """Operators applied to the wrong index, or a transposed site block, make
    the sector-wise result differ from the Kronecker definition."""
    p = gen.random_problem4(11, rank=1, site_dmax=2)
    n = l11r.layout(p).n
    psi = np.random.default_rng(2).standard_normal(n)
    ref = l11r.project_dense(p, psi)
    good = l11r._apply

    def wrong_axis(pb, X4, axis):
        return good(pb, X4, {1: 2, 2: 1}.get(axis, axis))

    monkeypatch.setattr(l11r, "_apply", wrong_axis)
    assert np.linalg.norm(l11r.project_sectors(p, psi) - ref) > 1e-6 * np.linalg.norm(ref)

    def transposed(pb, X4, axis):
        if pb is not None and pb.ndim == 2 and axis == 1:
            pb = pb.T if pb.shape[0] == pb.shape[1] else pb
        return good(pb, X4, axis)

    monkeypatch.setattr(l11r, "_apply", transposed)
    assert np.linalg.norm(l11r.project_sectors(p, psi) - ref) > 1e-6 * np.linalg.norm(ref)
