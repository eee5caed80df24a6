"""Planted mistakes in the CPU reference must be caught by its pins.

Each mutant is a plausible slip in the Cholesky-route energy or the Green's
function (a dropped factor, a transposed operand, a conjugated walker, a lost
spin sum); the Fock-space value of the same tiny system must reject it.  The
mutants live only here, on the CPU.
"""
import numpy as np
import pytest

from oracle import energy as E
from oracle import fock as F
from paper_2202_00832_amd import synth


def _system(seed=7, M=5, n=2):
    rng = np.random.default_rng(seed)
    chol = synth.random_symmetric_cholesky(M, 3 * M, rng)
    eri = E.eri_from_cholesky(chol)
    trial = np.linalg.qr(rng.standard_normal((M, n)))[0]
    phi = trial + 0.5 * (rng.standard_normal((M, n)) + 1j * rng.standard_normal((M, n)))
    return chol, eri, trial, phi


def _mut_exchange_no_transpose(lbar, theta):
    T = np.matmul(lbar, theta)
    tr = np.einsum("gii->g", T)
    return 2.0 * np.sum(tr * tr), -np.einsum("gij,gij->", T, T)


def _mut_coulomb_factor(lbar, theta):
    ej, ek = E.e2_cholesky(lbar, theta)
    return 2.0 * ej, ek


def _mut_exchange_factor(lbar, theta):
    ej, ek = E.e2_cholesky(lbar, theta)
    return ej, 2.0 * ek


def _mut_conjugated_theta(lbar, theta):
    return E.e2_cholesky(lbar, theta.conj())


def _mut_transposed_lbar(lbar, theta):
    # Lbar_g used as (Psi^T L_g)^T: the r/i roles swapped inside T_g
    M = lbar.shape[2]
    n = lbar.shape[1]
    T = np.einsum("gir,rj->gij", lbar, theta)
    T = T.transpose(0, 2, 1)
    tr = np.einsum("gii->g", T)
    # also drop the factor 2 of the spin sum in the exchange
    return 2.0 * np.sum(tr * tr), -0.5 * np.einsum("gij,gji->", T, T)


MUTANTS = [_mut_exchange_no_transpose, _mut_coulomb_factor, _mut_exchange_factor,
           _mut_conjugated_theta, _mut_transposed_lbar]


def test_reference_route_passes():
    chol, eri, trial, phi = _system()
    theta, _, _ = E.green_theta(trial, phi)
    e_fock, _ = F.mixed_energy_restricted(eri, trial, phi)
    assert abs(sum(E.e2_cholesky(E.half_rotate(chol, trial), theta)) - e_fock) < 1e-11 * abs(e_fock)


@pytest.mark.parametrize("mutant", MUTANTS, ids=lambda f: f.__name__)
def test_mutant_is_rejected(mutant):
    chol, eri, trial, phi = _system()
    theta, _, _ = E.green_theta(trial, phi)
    e_fock, _ = F.mixed_energy_restricted(eri, trial, phi)
    e_mut = sum(mutant(E.half_rotate(chol, trial), theta))
    assert abs(e_mut - e_fock) > 1e-6 * abs(e_fock)


def test_unnormalised_green_function_is_rejected():
    """Eq. 11 divides by the overlap matrix; dropping the inverse changes E2."""
    chol, eri, trial, phi = _system(seed=8)
    G_wrong = (phi @ trial.conj().T).T
    e_fock, _ = F.mixed_energy_restricted(eri, trial, phi)
    e_mut = sum(E.e2_wick(eri, G_wrong, G_wrong))
    assert abs(e_mut - e_fock) > 1e-6 * abs(e_fock)


# ---------------------------------------------------------------------------
# Planted mistakes in the truncation bound (Sec. 2.3.1)
# ---------------------------------------------------------------------------

def _bound_half(factors, theta):
    return 0.5 * E.lo_error_bound(factors, theta)


def _bound_last_kept(factors, theta):
    # sigma_K (the last kept value) in place of the first discarded one
    full = E.expand_upper(factors, theta.shape[1])
    norms = np.linalg.norm(theta, axis=0)
    return float(sum(3.0 * (s[Ub.shape[1] - 1] if Ub.shape[1] else 0.0) * norms[i] * norms[j]
                     for (i, j), (Ub, _, s) in full.items()))


def _bound_row_norms(factors, theta):
    # norms of the rows of theta instead of its orbital columns
    full = E.expand_upper(factors, theta.shape[1])
    norms = np.linalg.norm(theta, axis=1)
    return float(sum(3.0 * (s[Ub.shape[1]] if Ub.shape[1] < s.size else 0.0) * norms[i] * norms[j]
                     for (i, j), (Ub, _, s) in full.items()))


@pytest.mark.parametrize("mutant", [_bound_half, _bound_last_kept, _bound_row_norms], ids=lambda f: f.__name__)
def test_bound_mutant_is_rejected(mutant):
    """A bound must hold (|dE| <= bound) and, on the rank-one Coulomb case,
    be tight to a factor of two (|dE| >= bound / 2)."""
    from tests.test_oracle_pins import bound_case
    fac, exact, theta, _, _, _ = bound_case("coulomb")
    d = abs(sum(E.e2_lo(fac, theta)) - sum(E.e2_lo(exact, theta)))
    b = mutant(fac, theta)
    assert not (d <= b and d >= 0.5 * b)
