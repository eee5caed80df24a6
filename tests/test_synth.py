"""Properties of the seeded chain generator (inputs only; no energy arithmetic)."""
import numpy as np

from paper_2202_00832_amd import synth


def test_cholesky_residual_below_tolerance_and_symmetric():
    for M, tol in ((16, 1e-4), (48, 1e-6), (60, 1e-5)):
        L = synth.chain_cholesky(M, tol)
        assert np.abs(L - L.transpose(0, 2, 1)).max() == 0.0
        # residual diagonal of every pair below tol (PSD residual => all entries bounded)
        assert synth.chain_cholesky_residual_max(M, L) < tol
        eri = None
        if M <= 16:
            eri = synth.chain_eri_dense(M)
            rebuilt = np.einsum("gpq,grs->pqrs", L, L)
            assert np.abs(rebuilt - eri).max() < tol


def test_chain_eri_rank_is_two_m_minus_one():
    """(pq|rs) depends on the pair centre c_pq only, which takes 2M-1 values."""
    for M in (12, 48):
        L = synth.chain_cholesky(M, 1e-12)
        assert L.shape[0] <= 2 * M - 1


def test_small_config_shapes():
    s = synth.make_system(synth.CHAIN_SMALL)
    assert s.trial.shape == (48, 8)
    assert s.walkers.shape == (16, 48, 8)
    assert s.n_chol <= 4 * 48
    assert list(synth.gaussian_centres(48, 8)) == [0, 6, 12, 18, 24, 30, 36, 42]
    assert np.abs(s.trial.T @ s.trial - np.eye(8)).max() < 1e-13
    for w in s.walkers:
        assert np.abs(w.conj().T @ w - np.eye(8)).max() < 1e-13


def test_generator_is_deterministic():
    a = synth.make_system(synth.CHAIN_SMALL, nw=2)
    b = synth.make_system(synth.CHAIN_SMALL, nw=2)
    assert np.array_equal(a.chol, b.chol) and np.array_equal(a.walkers, b.walkers)
