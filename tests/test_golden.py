"""The Cholesky route of the CPU reference reproduces stored Fock-space values."""
import json
import os

import numpy as np

from oracle import energy as E
from paper_2202_00832_amd import synth
from tests.golden.cases import CASES, build_case

HERE = os.path.dirname(os.path.abspath(__file__))


def test_cholesky_route_matches_fock_fixtures():
    with open(os.path.join(HERE, "golden", "fock_tiny.json")) as f:
        stored = json.load(f)["cases"]
    assert len(stored) == len(CASES)
    for case, ref in zip(CASES, stored):
        eri, trial, phi = build_case(case)
        chol = synth.chain_cholesky(case["M"], 1e-14)
        theta, logdet, info = E.green_theta(trial, phi)
        assert info == 0
        e2 = sum(E.e2_cholesky(E.half_rotate(chol, trial), theta))
        ref_e2 = complex(*ref["e2"])
        ref_ov = complex(*ref["overlap"])
        assert abs(e2 - ref_e2) < 1e-11 * max(1.0, abs(ref_e2))
        assert abs(np.exp(2 * logdet) - ref_ov) < 1e-11 * abs(ref_ov)
