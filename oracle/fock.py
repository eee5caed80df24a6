"""Second-quantised brute force of the two-body mixed estimator (test infrastructure).

Evaluates E2 = <Psi_T| H2 |phi> / <Psi_T|phi> (Sec. 2.1.1, Eq. 8-9) in the
full N-electron Fock sector of 2M spin orbitals, with

    H2 = 1/2 sum_{pqrs} V_pqrs sum_{sigma tau} c+_{p sigma} c+_{q tau} c_{s tau} c_{r sigma},
    V_pqrs = (pr|qs)  (Sec. 2.1, below Eq. 2).

Nothing here uses Green's functions or Wick's theorem: a Slater determinant is
expanded into occupation-number amplitudes (minors of its orbital matrix) and
the operator acts through explicit fermionic annihilation matrices, so this is
an independent check of every closed-form route.  Only feasible for tiny
spaces (C(2M, N) amplitudes).

Spin orbital P = sigma * M + p (sigma = 0 alpha, 1 beta).  An occupation string
is a bitmask; annihilating orbital k from a string gives the sign
(-1)^(number of occupied orbitals below k).
"""
from __future__ import annotations

import itertools

import numpy as np


def _strings(n_so: int, n_el: int):
    """All occupation strings with n_el electrons in n_so spin orbitals."""
    out = []
    for occ in itertools.combinations(range(n_so), n_el):
        mask = 0
        for k in occ:
            mask |= 1 << k
        out.append(mask)
    return out


def _annihilators(n_so: int, n_el: int):
    """A[k] maps the n_el-electron sector to the (n_el-1) sector: c_k."""
    src = _strings(n_so, n_el)
    dst = _strings(n_so, n_el - 1)
    dst_index = {m: a for a, m in enumerate(dst)}
    mats = []
    for k in range(n_so):
        A = np.zeros((len(dst), len(src)))
        for b, m in enumerate(src):
            if m >> k & 1:
                sign = -1.0 if bin(m & ((1 << k) - 1)).count("1") % 2 else 1.0
                A[dst_index[m & ~(1 << k)], b] = sign
        mats.append(A)
    return src, mats


def determinant_amplitudes(orbitals: np.ndarray, strings) -> np.ndarray:
    """<string|det>: the minor of the (n_so x N) orbital matrix on the string's rows.

    The determinant is c+_{col 1} ... c+_{col N} |0>; expanding each creation
    operator over the spin-orbital basis gives amplitude det(C[rows, :]) with
    rows in increasing order.
    """
    n_so = orbitals.shape[0]
    amps = np.empty(len(strings), dtype=np.complex128)
    for a, m in enumerate(strings):
        rows = [k for k in range(n_so) if m >> k & 1]
        amps[a] = np.linalg.det(orbitals[rows, :])
    return amps


def spin_orbital_matrix(phi_alpha: np.ndarray, phi_beta: np.ndarray) -> np.ndarray:
    """Block-diagonal (2M) x (N_alpha + N_beta) orbital matrix."""
    M = phi_alpha.shape[0]
    na, nb = phi_alpha.shape[1], phi_beta.shape[1]
    C = np.zeros((2 * M, na + nb), dtype=np.complex128)
    C[:M, :na] = phi_alpha
    C[M:, na:] = phi_beta
    return C


def mixed_energy(eri: np.ndarray, trial_alpha, trial_beta, phi_alpha, phi_beta):
    """Returns (E2, <Psi_T|phi>) from the Fock-space expansion."""
    return mixed_energy_multi(eri, [(trial_alpha, trial_beta)], [1.0], phi_alpha, phi_beta)


def mixed_energy_multi(eri: np.ndarray, trial_dets, coeffs, phi_alpha, phi_beta):
    """(E2, <Psi_T|phi>) for the multi-determinant trial
    Psi_T = sum_d c_d |D_d^alpha D_d^beta> (Sec. 2.1.1, Eq. 12), with
    trial_dets a list of (D_alpha, D_beta) orbital matrices: the trial's
    occupation-number amplitudes are the c_d-weighted sum of the determinants'."""
    M = eri.shape[0]
    n_so = 2 * M
    n_el = trial_dets[0][0].shape[1] + trial_dets[0][1].shape[1]
    strings, ann1 = _annihilators(n_so, n_el)
    _, ann2 = _annihilators(n_so, n_el - 1)
    t = np.zeros(len(strings), dtype=np.complex128)
    for (da, db), c in zip(trial_dets, coeffs):
        t += c * determinant_amplitudes(spin_orbital_matrix(da, db), strings)
    f = determinant_amplitudes(spin_orbital_matrix(phi_alpha, phi_beta), strings)
    # u[P,Q] = c_Q c_P |Psi_T>, v[R,S] = c_S c_R |phi>  (vectors in the N-2 sector)
    u = np.empty((n_so, n_so, ann2[0].shape[0]), dtype=np.complex128)
    v = np.empty_like(u)
    for P in range(n_so):
        tp = ann1[P] @ t
        fp = ann1[P] @ f
        for Q in range(n_so):
            u[P, Q] = ann2[Q] @ tp
            v[P, Q] = ann2[Q] @ fp
    # <Psi_T| c+_P c+_Q c_S c_R |phi> = <c_Q c_P Psi_T | c_S c_R phi>
    braket = np.einsum("pqk,rsk->pqrs", u.conj(), v)
    # spin-orbital V'_{PQRS} = V_pqrs delta(s_P, s_R) delta(s_Q, s_S)
    V = eri.transpose(0, 2, 1, 3)
    Vso = np.zeros((n_so,) * 4)
    for sig in (0, 1):
        for tau in (0, 1):
            Vso[sig * M:(sig + 1) * M, tau * M:(tau + 1) * M,
                sig * M:(sig + 1) * M, tau * M:(tau + 1) * M] = V
    ovlp = np.vdot(t, f)
    e2 = 0.5 * np.einsum("pqrs,pqrs->", Vso, braket) / ovlp
    return complex(e2), complex(ovlp)


def mixed_energy_restricted(eri: np.ndarray, trial: np.ndarray, phi: np.ndarray):
    return mixed_energy(eri, trial, trial, phi, phi)
