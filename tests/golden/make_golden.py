"""Writes the stored expected values under tests/golden/ using only ``oracle``.

Run from the repository root:  python tests/golden/make_golden.py
exact_energies.json: each value is a full-chain exact diagonalization
(LAPACK) of a Hamiltonian built straight from the paper's Eq. 1-8 by
``oracle.models``.  arpack_energies.json: the ground energies of the
synthetic superblock workloads (Heisenberg m=1024, Hubbard m=2048, J1-J2
m=1024) by ARPACK's implicitly restarted Lanczos (scipy ``eigsh``) with the
oracle's sector-form projection (Eq. 11) as the only access to H, and the
four lowest energies of the Heisenberg and Hubbard workloads the same way.  None comes
from the HIP library.
"""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import gen  # noqa: E402
from oracle import davidson, models  # noqa: E402


def sector_min(H, labels, want):
    idx = np.flatnonzero(labels == want)
    return float(np.linalg.eigvalsh(H[np.ix_(idx, idx)])[0])


def main():
    out = {}
    # Eq. 1-3, open chain, Delta = 1, S^z_total = 0 sector (label 2 S^z = 0)
    for n in (2, 4, 6, 8, 10):
        H = models.heisenberg_chain(n, delta=1.0)
        out[f"heisenberg_open_N{n}_Sz0"] = sector_min(H, models.spin_labels(n), 0)
    # Delta = 0 (XX chain)
    for n in (8, 10):
        H = models.heisenberg_chain(n, delta=0.0)
        out[f"xx_open_N{n}_Sz0"] = sector_min(H, models.spin_labels(n), 0)
    # Eq. 4-8, spin-1/2 Hubbard, t = 1, U = 4, half filling
    for n in (2, 4):
        H, Nup, Ndn = models.hubbard_chain(n, t=1.0, U=4.0)
        lab = np.rint(np.diag(Nup)).astype(int) * 100 + np.rint(np.diag(Ndn)).astype(int)
        out[f"hubbard_open_N{n}_t1_U4_half"] = sector_min(H, lab, (n // 2) * 100 + n // 2)
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "exact_energies.json")
    with open(path, "w") as f:
        json.dump({"source": "oracle.models + numpy.linalg.eigvalsh (LAPACK), FP64",
                   "energies": out}, f, indent=1, sort_keys=True)
    print(json.dumps(out, indent=1))
    arp = {}
    for cfg in (2, 3, 5):
        arp[gen.CONFIG_NAMES[cfg]] = davidson.ground_state_arpack(gen.config(cfg), tol=1e-15)[0]
    for cfg in (2, 3):  # the four lowest, for the block Davidson-Liu solver
        arp[gen.CONFIG_NAMES[cfg] + "_lowest4"] = [float(x) for x in davidson.lowest_arpack(gen.config(cfg), 4,
                                                                                             tol=1e-15)]
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "arpack_energies.json")
    with open(path, "w") as f:
        json.dump({"source": "gen.config + oracle.projection.project_sectors + scipy eigsh (ARPACK, "
                             "which='SA', tol=1e-15, ncv=40), FP64", "energies": arp}, f, indent=1, sort_keys=True)
    print(json.dumps(arp, indent=1))


if __name__ == "__main__":
    main()
