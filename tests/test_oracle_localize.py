"""Pins of the CPU reference of the Foster-Boys localization (oracle/localize.py).

On the chain there is one position operator, so the Boys maximum has a
closed form: sum_i x_ii^2 <= ||X||_F^2 for X = C^T x C, with equality exactly
when the rotation diagonalises X.  The Jacobi sweeps must reach the sum of the
squared eigenvalues of X (numpy's eigh, an independent routine), raise the
functional at every sweep, keep the orbitals orthonormal and their span
unchanged, leave the full two-body energy unchanged, and compress the pair
blocks better than the delocalized (canonical-like) orbitals they start from.
"""
import numpy as np
import pytest

from oracle import energy as E
from oracle import localize as B
from paper_2202_00832_amd import synth


@pytest.fixture(scope="module")
def chain():
    s = synth.make_system(synth.CHAIN_SMALL)
    deloc = synth.delocalized_trial(s.trial)
    pos = B.chain_positions(s.config.M)
    loc, hist = B.boys_jacobi(deloc, pos)
    return s, deloc, pos, loc, hist


def test_sweeps_raise_the_functional_to_the_closed_form_maximum(chain):
    s, deloc, pos, loc, hist = chain
    assert all(b >= a - 1e-9 * abs(a) for a, b in zip(hist, hist[1:]))
    X = deloc.T @ (pos[0][:, None] * deloc)
    lam = np.linalg.eigvalsh(X)
    assert abs(hist[-1] - np.sum(lam ** 2)) <= 1e-10 * np.sum(lam ** 2)
    assert abs(B.boys_functional(loc, pos) - hist[-1]) <= 1e-10 * hist[-1]
    Xl = loc.T @ (pos[0][:, None] * loc)
    assert np.abs(Xl - np.diag(np.diag(Xl))).max() <= 1e-6 * np.abs(lam).max()
    # maximising B minimises the summed orbital variances <x^2>_i - <x>_i^2
    # (their <x^2> sum is invariant): the start is far from localized
    var = lambda C: float(np.sum(np.einsum("m,mi->i", pos[0] ** 2, C * C)  # noqa: E731
                                 - np.einsum("m,mi->i", pos[0], C * C) ** 2))
    assert var(loc) < 0.1 * var(deloc)
    assert len(hist) < 40                    # converged well before the sweep limit


def test_orbitals_stay_orthonormal_and_span_the_same_space(chain):
    s, deloc, pos, loc, hist = chain
    n = loc.shape[1]
    assert np.abs(loc.T @ loc - np.eye(n)).max() <= 1e-12
    assert np.abs(loc @ loc.T - deloc @ deloc.T).max() <= 1e-12


def test_full_energy_is_unchanged_by_the_localization(chain):
    s, deloc, pos, loc, hist = chain
    for w in range(4):
        ed = E.e2_cholesky(E.half_rotate(s.chol, deloc), E.green_theta(deloc, s.walkers[w])[0])
        el = E.e2_cholesky(E.half_rotate(s.chol, loc), E.green_theta(loc, s.walkers[w])[0])
        for a, b in zip(ed, el):
            assert abs(a - b) <= 1e-11 * max(1.0, abs(a))


def test_localized_orbitals_compress_better(chain):
    s, deloc, pos, loc, hist = chain
    n = loc.shape[1]
    for eps in (1e-3, 1e-4):
        k_loc = E.lo_ranks(E.lo_compress(E.half_rotate(s.chol, loc), eps, pairs="upper"), n).mean()
        k_del = E.lo_ranks(E.lo_compress(E.half_rotate(s.chol, deloc), eps, pairs="upper"), n).mean()
        assert k_loc < 0.6 * k_del, (eps, k_loc, k_del)


def test_centroids_are_spread_along_the_chain(chain):
    s, deloc, pos, loc, hist = chain
    cent = np.sort(np.einsum("m,mi->i", pos[0], loc * loc))
    # eight orbitals of a 48-site chain: one per stretch of about six sites
    assert np.all(np.diff(cent) > 3.0) and cent[0] < 6 and cent[-1] > 41


def test_three_position_operators_reach_a_stationary_point():
    """With several position operators the Jacobi angle still maximises every
    pair's part: after convergence no single rotation raises B."""
    rng = np.random.default_rng(4)
    M, n = 30, 5
    C = np.linalg.qr(rng.standard_normal((M, n)))[0]
    pos = rng.uniform(-3, 3, (3, M))
    loc, hist = B.boys_jacobi(C, pos, max_sweeps=200, tol=1e-15)
    assert all(b >= a - 1e-9 * abs(a) for a, b in zip(hist, hist[1:]))
    base = B.boys_functional(loc, pos)
    for i in range(n):
        for j in range(i + 1, n):
            for t in (-1e-3, 1e-3):
                R = loc.copy()
                R[:, i], R[:, j] = np.cos(t) * loc[:, i] + np.sin(t) * loc[:, j], \
                    -np.sin(t) * loc[:, i] + np.cos(t) * loc[:, j]
                assert B.boys_functional(R, pos) <= base * (1 + 1e-12)
