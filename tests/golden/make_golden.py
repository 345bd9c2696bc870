"""Writes tests/golden/ed_energies.json from the oracle only (exact diagonalisation).

Run from the repository root:  python tests/golden/make_golden.py
"""
import json
import os
import sys
from fractions import Fraction

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import ed, model  # noqa: E402


def main():
    out = {"_source": "oracle.ed (bitstring exact diagonalisation of eqs. H_kin + H_int)"}
    cyl = model.Cylinder(4, 8, Fraction(1, 4), 1.0, 1.0)
    mom = model.orbital_momenta(cyl, "mixed")
    sec = {}
    for K in range(4):
        H = ed.hamiltonian(model.mixed_terms(cyl), ed.sector_basis(cyl.n_orb, 4, mom, K, 4))
        sec[str(K)] = [float(e) for e in ed.lowest(H, 2)]
    out["ly4_lx8_flux1_4_V1_N4"] = sec
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "ed_energies.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
