"""Pins of the reference randomized SVD (randomized subspace iteration, the
approximate decomposition Sec. 2.3.1 mentions) against the exact SVD: with a
test matrix of M columns the projection is exact, and on the localized chain a
sketch a few columns wider than the largest kept rank reproduces the exact
ranks and LO energies."""
import numpy as np

from oracle import energy as E
from paper_2202_00832_amd import synth


def _small():
    s = synth.make_system(synth.CHAIN_SMALL)
    return s, E.half_rotate(s.chol, s.trial)


def test_full_width_sketch_is_the_exact_svd():
    s, lbar = _small()
    M = s.trial.shape[0]
    om = np.random.default_rng(1).standard_normal((M, M))
    exact = E.lo_decompose(lbar, pairs="upper")
    rnd = E.lo_decompose_randomized(lbar, om, 0)
    for key, (U, sv, Vh) in exact.items():
        Ur, sr, Vr = rnd[key]
        assert np.allclose(sr, sv, rtol=0, atol=1e-12 * sv[0])
        k = int(np.count_nonzero(sv > 1e-8 * sv[0]))   # well-separated leading part
        Y = U[:, :k] @ np.diag(sv[:k]) @ Vh[:k]
        assert np.abs(Ur[:, :k] @ np.diag(sr[:k]) @ Vr[:k] - Y).max() <= 1e-11 * sv[0]


def test_narrow_sketch_keeps_exact_ranks_and_energies():
    s, lbar = _small()
    M, n = s.trial.shape
    rng = np.random.default_rng(2)
    for eps in (1e-3, 1e-4, 1e-5):
        exact = E.lo_compress(lbar, eps, pairs="upper")
        kmax = int(E.lo_ranks(exact, n).max())
        om = rng.standard_normal((M, kmax + 6))
        rnd = E.lo_truncate(E.lo_decompose_randomized(lbar, om, 2), eps)
        assert np.array_equal(E.lo_ranks(rnd, n), E.lo_ranks(exact, n))
        for w in range(4):
            th, _, _ = E.green_theta(s.trial, s.walkers[w])
            a = np.array(E.e2_lo(exact, th))
            b = np.array(E.e2_lo(rnd, th))
            assert np.abs(a - b).max() <= 1e-10


def test_too_narrow_sketch_without_power_steps_is_inaccurate():
    """The pins see the difference: a sketch narrower than the kept rank
    cannot reproduce the exact ranks."""
    s, lbar = _small()
    M, n = s.trial.shape
    exact = E.lo_compress(lbar, 1e-5, pairs="upper")
    kmax = int(E.lo_ranks(exact, n).max())
    om = np.random.default_rng(3).standard_normal((M, kmax - 2))
    rnd = E.lo_truncate(E.lo_decompose_randomized(lbar, om, 0), 1e-5)
    assert not np.array_equal(E.lo_ranks(rnd, n), E.lo_ranks(exact, n))
