"""Pins of the oracle's dense chain Hamiltonians (Eq. 1-8) against closed forms."""
import json
import os

import numpy as np
import pytest

from oracle import models

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "exact_energies.json")


def sector_min(H, labels, want):
    idx = np.flatnonzero(labels == want)
    return float(np.linalg.eigvalsh(H[np.ix_(idx, idx)])[0])


def test_site_operators_match_eq3():
    # S+ S- - S- S+ = 2 S^z and [S^z, S+] = S+ (spin-1/2 algebra)
    assert np.array_equal(models.SP @ models.SM - models.SM @ models.SP, 2 * models.SZ)
    assert np.array_equal(models.SZ @ models.SP - models.SP @ models.SZ, models.SP)


@pytest.mark.parametrize("n", [2, 3, 6])
def test_heisenberg_hermitian_and_conserves_sz(n):
    H = models.heisenberg_chain(n, delta=0.7)
    Sz = models.total_sz(n)
    assert np.array_equal(H, H.T)
    assert np.abs(H @ Sz - Sz @ H).max() == 0.0


def test_two_site_singlet():
    # H = S1.S2 for Delta = 1: singlet energy -3/4
    assert models.heisenberg_chain(2)[0, 0] == 0.25  # |up up> energy +1/4
    assert np.linalg.eigvalsh(models.heisenberg_chain(2))[0] == pytest.approx(-0.75, abs=1e-15)


def test_four_site_closed_form():
    # open 4-site Heisenberg chain: E0 = -3/4 - sqrt(3)/2
    E = np.linalg.eigvalsh(models.heisenberg_chain(4))[0]
    assert E == pytest.approx(-0.75 - np.sqrt(3) / 2, abs=1e-14)


@pytest.mark.parametrize("n", [6, 8, 10])
def test_xx_chain_free_fermions(n):
    H = models.heisenberg_chain(n, delta=0.0)
    E = sector_min(H, models.spin_labels(n), 0)
    assert E == pytest.approx(models.xx_chain_energy(n), abs=1e-12)


@pytest.mark.parametrize("n", [6, 8])
def test_majumdar_ghosh(n):
    H = models.heisenberg_chain(n, delta=1.0, J1=1.0, J2=0.5, end_factor=0.5)
    w = np.linalg.eigvalsh(H)
    assert w[0] == pytest.approx(models.majumdar_ghosh_energy(n), abs=1e-12)
    # the two dimer coverings (plus end-spin states) make it degenerate
    assert w[1] - w[0] < 1e-10


def test_hubbard_hermitian_and_conserves_particle_numbers():
    H, Nup, Ndn = models.hubbard_chain(3, t=0.8, U=2.5)
    assert np.array_equal(H, H.T)
    assert np.abs(H @ Nup - Nup @ H).max() == 0.0
    assert np.abs(H @ Ndn - Ndn @ H).max() == 0.0


def test_fermion_anticommutation():
    # Jordan-Wigner strings of Eq. 5-6 give {c_i, c_j^dag} = delta_ij
    nm = 4
    c = [models.mode_op(models.C, k, nm) for k in range(nm)]
    cd = [models.mode_op(models.CDAG, k, nm) for k in range(nm)]
    for i in range(nm):
        for j in range(nm):
            ac = c[i] @ cd[j] + cd[j] @ c[i]
            assert np.array_equal(ac, np.eye(2 ** nm) * (i == j))
            assert not np.any(c[i] @ c[j] + c[j] @ c[i])


def _hub_sector(n, U, t=1.0, nup=None, ndn=None):
    H, Nup, Ndn = models.hubbard_chain(n, t=t, U=U)
    nup = n // 2 if nup is None else nup
    ndn = n // 2 if ndn is None else ndn
    lab = np.rint(np.diag(Nup)).astype(int) * 100 + np.rint(np.diag(Ndn)).astype(int)
    return sector_min(H, lab, nup * 100 + ndn)


@pytest.mark.parametrize("U", [0.0, 1.0, 4.0, 10.0])
def test_hubbard_dimer(U):
    assert _hub_sector(2, U) == pytest.approx(models.hubbard_dimer_energy(1.0, U), abs=1e-13)


@pytest.mark.parametrize("n,nup,ndn", [(4, 2, 2), (4, 1, 2), (3, 2, 1)])
def test_free_hubbard(n, nup, ndn):
    assert _hub_sector(n, 0.0, nup=nup, ndn=ndn) == pytest.approx(
        models.free_hubbard_energy(n, nup, ndn), abs=1e-12)


def test_golden_energies_reproduce():
    g = json.load(open(GOLDEN))["energies"]
    assert g["heisenberg_open_N2_Sz0"] == -0.75
    assert g["heisenberg_open_N4_Sz0"] == pytest.approx(-0.75 - np.sqrt(3) / 2, abs=1e-14)
    assert g["xx_open_N10_Sz0"] == pytest.approx(models.xx_chain_energy(10), abs=1e-12)
    assert g["hubbard_open_N2_t1_U4_half"] == pytest.approx(models.hubbard_dimer_energy(1, 4), abs=1e-13)
    H = models.heisenberg_chain(10)
    assert sector_min(H, models.spin_labels(10), 0) == pytest.approx(g["heisenberg_open_N10_Sz0"], abs=1e-12)


def test_chain_ground_energy_matches_closed_forms():
    """The S^z = 0 sector ED of the chain: the dimer -3/4, the XX chain's free
    fermions, and energies per site approaching Hulthen's 1/4 - ln 2 from
    above as the open chain grows (the boundary costs energy)."""
    assert models.chain_ground_energy(2) == pytest.approx(-0.75, abs=1e-14)
    for n in (4, 6, 8):
        assert models.chain_ground_energy(n, delta=0.0) == pytest.approx(models.xx_chain_energy(n), abs=1e-12)
    e = [models.chain_ground_energy(n) for n in (8, 10, 12)]
    d = [(e[1] - e[0]) / 2, (e[2] - e[1]) / 2]
    assert abs(d[1] - models.hulthen_energy_per_site()) < abs(d[0] - models.hulthen_energy_per_site()) < 0.01
