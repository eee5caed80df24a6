"""Multi-determinant (CAS-type) trials: plain FP64 reference (test infrastructure).

The trial is psi_T = sum_d c_d |Phi_d> (Sec. 2.1.1, below Eq. 11).  Here its
orbitals are the columns of C (M x n_cas): the reference determinant Phi_0
occupies columns 0 .. n-1, the last n_act_occ of which are active, and columns
n .. n_cas-1 are the active virtual orbitals.  Determinant d replaces the
reference columns holes[d] by the orbitals particles[d], hole k by particle k,
in place.  Every determinant is doubly occupied with the same spatial orbitals
for both spins (closed shell), the form of the LO energy expression of
Sec. 2.3.2 (Eq. 19), so <Phi_d|phi> = det(Phi_d^T phi)^2 for a restricted
walker phi.

Two evaluations of the same energy:

* ``e2_plain``: the definition, Eq. 12 (and Eq. 16, 17, 19 for the routes),
  E2 = sum_d c_d <Phi_d|phi> E2^d / sum_d c_d <Phi_d|phi>, with E2^d from
  Q^d = phi (Phi_d^T phi)^{-1} (Eq. 15) formed by a fresh inverse for every
  determinant, its columns placed at the orbitals they belong to in an
  M x n_cas array with zero columns for the orbitals d leaves empty (the
  zero padding of Sec. 2.2 and 2.3.2).
* ``e2_lo_smw``: the paper's order for the LO energy: the reference
  A = Phi_0^T phi and Phi A^{-1}; per determinant the Sherman-Morrison-Woodbury
  update of Eq. 20-21 with U^d the identity columns of the holes and V^dT the
  changed rows; the intermediates of the intermediates table of Sec. 2.3.2
  (projections of the active columns of Phi A^{-1}, S_d); and the four vectors
  of Eq. 22-23, weighted by c_d <Phi_d|phi>.  The overlap ratio
  det(A_d) / det(A) = det(I + V^dT A^{-1} U^d) (matrix determinant lemma).

A determinant whose overlap with the walker is exactly zero has weight zero
and is skipped (its E2^d is undefined).
"""
from __future__ import annotations

import numpy as np

from . import energy as E


def determinant_orbitals(C: np.ndarray, n: int, holes, particles) -> np.ndarray:
    """Phi_d: the reference columns with column holes[k] replaced by C[:, particles[k]]."""
    D = np.array(C[:, :n], copy=True)
    for h, p in zip(holes, particles):
        D[:, h] = C[:, p]
    return D


def occupied_orbitals(n: int, holes, particles) -> list:
    """Orbital (column of C) held by each column of Phi_d."""
    occ = list(range(n))
    for h, p in zip(holes, particles):
        occ[h] = p
    return occ


def padded_theta(C: np.ndarray, n: int, holes, particles, phi: np.ndarray):
    """Q^d = phi (Phi_d^T phi)^{-1} (Eq. 15) as an M x n_cas array (column o is
    the Q column of orbital o, zero if d leaves o empty), and det(Phi_d^T phi)."""
    D = determinant_orbitals(C, n, holes, particles)
    A = D.T @ phi
    det = np.linalg.det(A)
    Q = np.zeros((phi.shape[0], C.shape[1]), dtype=np.complex128)
    if det == 0:
        return Q, det
    Qd = phi @ np.linalg.inv(A)
    for k, o in enumerate(occupied_orbitals(n, holes, particles)):
        Q[:, o] = Qd[:, k]
    return Q, det


def e2_plain(C: np.ndarray, n: int, holes, particles, coeffs, phi: np.ndarray, energy_of_theta):
    """Eq. 12: (E_J, E_K) = sum_d w_d (E_J^d, E_K^d), w_d = c_d det_d^2 / sum c det^2.

    energy_of_theta maps a padded Q^d (M x n_cas) to (E_J^d, E_K^d): the
    Cholesky route (Eq. 16) or the LO route (Eq. 19) over all n_cas orbitals.
    Returns ((E_J, E_K), sum_d c_d det_d^2).
    """
    num_j = 0.0 + 0.0j
    num_k = 0.0 + 0.0j
    den = 0.0 + 0.0j
    for h, p, c in zip(holes, particles, coeffs):
        Q, det = padded_theta(C, n, h, p, phi)
        ov = c * det * det
        den += ov
        if det == 0:
            continue
        ej, ek = energy_of_theta(Q)
        num_j += ov * ej
        num_k += ov * ek
    return (complex(num_j / den), complex(num_k / den)), complex(den)


def e2_cholesky_plain(lbar_cas: np.ndarray, C, n, holes, particles, coeffs, phi):
    """Eq. 12 with the Cholesky route (Eq. 16); lbar_cas half-rotated with all n_cas orbitals."""
    return e2_plain(C, n, holes, particles, coeffs, phi, lambda Q: E.e2_cholesky(lbar_cas, Q))


def e2_lo_plain(factors: dict, C, n, holes, particles, coeffs, phi):
    """Eq. 12 with the LO route (Eq. 19, 22) on factors of all n_cas orbitals."""
    return e2_plain(C, n, holes, particles, coeffs, phi, lambda Q: E.e2_lo(factors, Q))


def smw_theta(C: np.ndarray, n: int, holes, particles, phi: np.ndarray):
    """Q^d by Eq. 20 from the reference inverse, and det(A_d)/det(A).

    A = Phi_0^T phi, U^d = columns holes of the identity (n x eps),
    V^dT = C[:, particles]^T phi - A[holes, :] (the rows the excitation changes),
    Q^d = Phi A^{-1} - Phi A^{-1} U^d (I + V^dT A^{-1} U^d)^{-1} V^dT A^{-1}.
    Columns are in the positions of Phi_d (hole k's column holds particle k).
    """
    A = C[:, :n].T @ phi
    Ainv = np.linalg.inv(A)
    theta = phi @ Ainv
    h = list(holes)
    if not h:
        return theta, 1.0 + 0.0j
    U = np.eye(n)[:, h]
    VT = C[:, list(particles)].T @ phi - A[h, :]
    small = np.eye(len(h)) + VT @ Ainv @ U
    ratio = np.linalg.det(small)
    Q = theta - theta @ U @ np.linalg.solve(small, VT @ Ainv)
    return Q, complex(ratio)


def e2_lo_smw(factors: dict, C: np.ndarray, n: int, n_act_occ: int, holes, particles, coeffs, phi: np.ndarray):
    """Multi-determinant LO energy in the order of Sec. 2.3.2 (Eq. 19-23).

    Per walker: A = Phi_0^T phi, theta = Phi A^{-1}.  Per ordered pair [ij]
    (i, j over all n_cas orbitals) the projections of theta's own columns and
    of its active columns,
        QL_x = Ubar^T theta_x,  QR_x = Vbar theta_x,
        Qint_L = Ubar^T theta[:, act],  Qint_R = Vbar theta[:, act]
    (the first row of the intermediates table).  Per determinant
        S_d = (I + V^dT A^{-1} U^d)^{-1} V^dT A^{-1}     (eps x n, second row)
    and, for the column c of Phi_d that holds orbital i (Eq. 21, 23),
        Qbar_L,i = QL_c - Qint_L[:, holes - act0] S_d[:, c]
    (the third row), the same for R and j, then Eq. 22 with the weight
    c_d det(A_d)^2 / sum, det(A_d) = det(A) det(I + V^dT A^{-1} U^d).
    Returns ((E_J, E_K), sum_d c_d ratio_d^2) with ratio_d = det(A_d)/det(A).
    """
    n_cas = C.shape[1]
    act0 = n - n_act_occ
    A = C[:, :n].T @ phi
    Ainv = np.linalg.inv(A)
    theta = phi @ Ainv
    full = E.expand_upper(factors, n_cas)
    proj = {}
    for (i, j), (Ub, Vb, _) in full.items():
        cols = {}
        for o in (i, j):
            if o < n:
                cols[o] = (Ub.T @ theta[:, o], Vb @ theta[:, o])
        qint = (Ub.T @ theta[:, act0:n], Vb @ theta[:, act0:n])
        proj[(i, j)] = (cols, qint)
    num_j = 0.0 + 0.0j
    num_k = 0.0 + 0.0j
    den = 0.0 + 0.0j
    for hs, ps, c in zip(holes, particles, coeffs):
        h = list(hs)
        if h:
            U = np.eye(n)[:, h]
            VT = C[:, list(ps)].T @ phi - A[h, :]
            small = np.eye(len(h)) + VT @ Ainv @ U
            ratio = np.linalg.det(small)
            S = np.linalg.solve(small, VT @ Ainv) if ratio != 0 else None
        else:
            ratio, S = 1.0, np.zeros((0, n))
        wnum = c * ratio * ratio
        den += wnum
        if ratio == 0:
            continue
        occ = occupied_orbitals(n, hs, ps)
        col_of = {o: k for k, o in enumerate(occ)}
        hl = [x - act0 for x in h]
        e_j = 0.0 + 0.0j
        e_k = 0.0 + 0.0j
        for (i, j) in full:
            if i not in col_of or j not in col_of:
                continue
            cols, (qil, qir) = proj[(i, j)]
            vec = {}
            for o in (i, j):
                c_o = col_of[o]
                if c_o == o:
                    # orbital kept from the reference: its own column of theta
                    base_l, base_r = cols[o]
                else:
                    # particle in a hole's position: the hole column of theta
                    base_l, base_r = qil[:, c_o - act0], qir[:, c_o - act0]
                vec[o] = (base_l - qil[:, hl] @ S[:, c_o], base_r - qir[:, hl] @ S[:, c_o])
            e_j += 2.0 * np.sum(vec[i][0] * vec[j][1])
            e_k -= np.sum(vec[j][0] * vec[i][1])
        num_j += wnum * e_j
        num_k += wnum * e_k
    return (complex(num_j / den), complex(num_k / den)), complex(den)
