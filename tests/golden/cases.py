"""Seeded tiny systems for the Fock-space fixtures (inputs only)."""
import numpy as np

from paper_2202_00832_amd import synth

CASES = [
    {"M": 4, "n": 1, "seed": 101, "sigma": 0.3},
    {"M": 5, "n": 2, "seed": 102, "sigma": 0.3},
    {"M": 6, "n": 2, "seed": 103, "sigma": 0.5},
    {"M": 6, "n": 3, "seed": 104, "sigma": 0.2},
]


def build_case(case):
    M, n = case["M"], case["n"]
    rng = np.random.default_rng(case["seed"])
    eri = synth.chain_eri_dense(M)
    trial = synth.lowdin_gaussian_trial(M, n)
    phi = synth.noisy_walkers(trial, 1, case["sigma"], rng)[0]
    return eri, trial, phi
