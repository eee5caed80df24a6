"""Pins of the multi-determinant reference (Sec. 2.1.1 Eq. 12, Sec. 2.3.2
Eq. 19-23).

The weighted sum over determinants is pinned to the second-quantised Fock
expansion of <psi_T|H2|phi>/<psi_T|phi> for a CI-expanded trial; the SMW
update of Eq. 20 to a fresh inverse of every determinant's overlap matrix and
the overlap ratio to the determinant itself; the paper's SMW ordering of the LO
energy (Eq. 21-23 and the intermediates table) to the plain weighted sum of
single-determinant LO energies; and the special cases (a lone reference is the
single-determinant energy, scaling all c_d changes nothing, LO at T_SVD = 0 is
the Cholesky route, phi -> phi R changes nothing).
"""
import numpy as np
import pytest

from oracle import energy as E
from oracle import fock as F
from oracle import multidet as MD
from paper_2202_00832_amd import synth


def _rel(a, b):
    return abs(a - b) / max(1.0, abs(b))


def _tiny(seed, M=6, n=3, nao=2, nav=2):
    rng = np.random.default_rng(seed)
    chol = synth.random_symmetric_cholesky(M, 2 * M, rng)
    C = np.linalg.qr(rng.standard_normal((M, n + nav)))[0]
    holes, parts, coeffs = synth.cas_expansion(n, nao, nav, 6, 2, rng)   # all 6 up to doubles
    phi = C[:, :n] + 0.4 * (rng.standard_normal((M, n)) + 1j * rng.standard_normal((M, n)))
    return chol, C, holes, parts, coeffs, phi


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_weighted_sum_matches_fock_space(seed):
    chol, C, holes, parts, coeffs, phi = _tiny(seed)
    n = 3
    eri = E.eri_from_cholesky(chol)
    dets = []
    for h, p in zip(holes, parts):
        D = MD.determinant_orbitals(C, n, h, p)
        dets.append((D, D))
    e_fock, ov_fock = F.mixed_energy_multi(eri, dets, coeffs, phi, phi)
    (ej, ek), den = MD.e2_cholesky_plain(E.half_rotate(chol, C), C, n, holes, parts, coeffs, phi)
    assert _rel(ej + ek, e_fock) < 1e-11
    # sum_d c_d det_d^2 is the Fock overlap <psi_T|phi>
    assert _rel(den, ov_fock) < 1e-12


def test_unsquared_weight_fails_the_fock_pin():
    """A plausible slip (open-shell weights c_d det_d instead of c_d det_d^2)
    is caught by the Fock pin."""
    chol, C, holes, parts, coeffs, phi = _tiny(4)
    n = 3
    eri = E.eri_from_cholesky(chol)
    dets = [(MD.determinant_orbitals(C, n, h, p),) * 2 for h, p in zip(holes, parts)]
    e_fock, _ = F.mixed_energy_multi(eri, dets, coeffs, phi, phi)
    lbar = E.half_rotate(chol, C)
    num, den = 0.0, 0.0
    for h, p, c in zip(holes, parts, coeffs):
        Q, det = MD.padded_theta(C, n, h, p, phi)
        num += c * det * sum(E.e2_cholesky(lbar, Q))
        den += c * det
    assert _rel(num / den, e_fock) > 1e-6


def test_smw_update_equals_fresh_inverse():
    rng = np.random.default_rng(7)
    M, n, nao, nav = 30, 6, 3, 3
    C = np.linalg.qr(rng.standard_normal((M, n + nav)))[0]
    phi = C[:, :n] + 0.3 * (rng.standard_normal((M, n)) + 1j * rng.standard_normal((M, n)))
    holes, parts, _ = synth.cas_expansion(n, nao, nav, 20, 3, rng)
    A0 = C[:, :n].T @ phi
    for h, p in zip(holes, parts):
        Q, ratio = MD.smw_theta(C, n, h, p, phi)
        D = MD.determinant_orbitals(C, n, h, p)
        Ad = D.T @ phi
        assert np.abs(Q - phi @ np.linalg.inv(Ad)).max() < 1e-12 * np.abs(Q).max()
        assert _rel(ratio, np.linalg.det(Ad) / np.linalg.det(A0)) < 1e-12
        # Psi_d^T Q^d = I (Eq. 15)
        assert np.abs(D.T @ Q - np.eye(n)).max() < 1e-12


@pytest.mark.parametrize("eps", [0.0, 1e-5, 1e-3])
def test_smw_order_equals_weighted_sum(eps):
    s = synth.make_cas_system(synth.CAS_SMALL, nw=3)
    cfg = s.config
    lbar = E.half_rotate(s.chol, s.orbitals)
    factors = E.lo_compress(lbar, eps, pairs="upper")
    for phi in s.walkers:
        (aj, ak), aden = MD.e2_lo_plain(factors, s.orbitals, cfg.n, s.holes, s.particles, s.coeffs, phi)
        (bj, bk), bden = MD.e2_lo_smw(factors, s.orbitals, cfg.n, cfg.n_act_occ, s.holes, s.particles,
                                      s.coeffs, phi)
        assert abs(aj - bj) < 1e-10 and abs(ak - bk) < 1e-10
        A0 = s.reference.T @ phi
        assert _rel(aden / np.linalg.det(A0) ** 2, bden) < 1e-11


def test_lo_at_zero_threshold_equals_cholesky_route():
    s = synth.make_cas_system(synth.CAS_SMALL, nw=2)
    cfg = s.config
    lbar = E.half_rotate(s.chol, s.orbitals)
    factors = E.lo_compress(lbar, 0.0, pairs="upper")
    for phi in s.walkers:
        (aj, ak), _ = MD.e2_lo_plain(factors, s.orbitals, cfg.n, s.holes, s.particles, s.coeffs, phi)
        (bj, bk), _ = MD.e2_cholesky_plain(lbar, s.orbitals, cfg.n, s.holes, s.particles, s.coeffs, phi)
        assert abs(aj - bj) < 1e-9 and abs(ak - bk) < 1e-9


def test_special_cases():
    s = synth.make_cas_system(synth.CAS_SMALL, nw=2)
    cfg = s.config
    lbar = E.half_rotate(s.chol, s.orbitals)
    factors = E.lo_compress(lbar, 1e-5, pairs="upper")
    ref_factors = E.lo_compress(E.half_rotate(s.chol, s.reference), 1e-5, pairs="upper")
    phi = s.walkers[0]
    # a lone reference determinant is the single-determinant energy
    (aj, ak), _ = MD.e2_lo_smw(factors, s.orbitals, cfg.n, cfg.n_act_occ, [()], [()], [0.7], phi)
    theta, _, _ = E.green_theta(s.reference, phi)
    bj, bk = E.e2_lo(ref_factors, theta)
    assert abs(aj - bj) < 1e-10 and abs(ak - bk) < 1e-10
    # common scaling of the coefficients changes nothing
    (e1j, e1k), _ = MD.e2_lo_smw(factors, s.orbitals, cfg.n, cfg.n_act_occ, s.holes, s.particles, s.coeffs, phi)
    (e2j, e2k), _ = MD.e2_lo_smw(factors, s.orbitals, cfg.n, cfg.n_act_occ, s.holes, s.particles,
                                 -3.0 * s.coeffs, phi)
    assert abs(e1j - e2j) < 1e-10 and abs(e1k - e2k) < 1e-10
    # phi -> phi R (same state) changes nothing
    rng = np.random.default_rng(3)
    R = rng.standard_normal((cfg.n, cfg.n)) + 1j * rng.standard_normal((cfg.n, cfg.n))
    (e3j, e3k), _ = MD.e2_lo_smw(factors, s.orbitals, cfg.n, cfg.n_act_occ, s.holes, s.particles, s.coeffs,
                                 phi @ R)
    assert abs(e1j - e3j) < 1e-9 and abs(e1k - e3k) < 1e-9
    # the excited determinants matter: dropping them moves the energy
    (e4j, e4k), _ = MD.e2_lo_smw(factors, s.orbitals, cfg.n, cfg.n_act_occ, s.holes[:1], s.particles[:1],
                                 s.coeffs[:1], phi)
    assert abs((e4j + e4k) - (e1j + e1k)) > 1e-6
