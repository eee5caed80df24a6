"""Writes fock_tiny.json: Fock-space values of E2 = <Psi_T|H2|phi>/<Psi_T|phi>.

The values come from the second-quantised brute force of the CPU reference
(Sec. 2.1.1, Eq. 9) on tiny seeded inputs; the inputs are regenerated from the
recorded seeds by the chain generator.  Run from the repository root:
    python tests/golden/make_golden.py
"""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import fock  # noqa: E402
from tests.golden.cases import CASES, build_case  # noqa: E402


def main():
    out = []
    for case in CASES:
        eri, trial, phi = build_case(case)
        e2, ovlp = fock.mixed_energy_restricted(eri, trial, phi)
        out.append(dict(case, e2=[e2.real, e2.imag], overlap=[ovlp.real, ovlp.imag]))
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "fock_tiny.json")
    with open(path, "w") as f:
        json.dump({"source": "Fock-space expansion of Eq. 9 (Sec. 2.1.1), restricted closed shell",
                   "cases": out}, f, indent=1)
        f.write("\n")


if __name__ == "__main__":
    main()
