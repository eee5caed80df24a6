"""Plain FP64 reference of the walker two-body local energy (test infrastructure).

Conventions (all arrays numpy, float64 / complex128):

* ``eri[p, q, r, s]`` is (pq|rs) in chemists' notation, and the Hamiltonian
  tensor is V_pqrs = (pr|qs) (Sec. 2.1, below Eq. 2).
* ``chol[g, p, r]`` are the Cholesky (auxiliary-field) matrices with
  V_pqrs = sum_g L_g[p][r] L_g[q][s] (Sec. 2.1.1, below Eq. 13).
* ``trial`` is the M x n trial determinant Psi_T (columns are orbitals),
  ``phi`` an M x n walker determinant.  One spatial determinant is used for
  both spins (restricted closed shell) unless a function says otherwise.
* ``lbar[g, i, r]`` is the half-rotated vector Lbar^g_{ri} (Sec. 2.2).
* Energies are returned as (E_J, E_K): the Coulomb (direct) and exchange
  parts of E2, each complex; E2 = E_J + E_K.

Readings of points the paper leaves open (also listed in the design notes):
the half-rotation conjugates the trial (the paper omits the conjugate, which
is immaterial for the real trials used here); products of complex walker
quantities are bilinear (no conjugation of Q); the SVD threshold is an
absolute cut on singular values, keeping sigma >= eps, and eps = 0 keeps every
singular value; Sigma is split evenly, Ubar = U Sigma^(1/2), Vbar =
Sigma^(1/2) V.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg
import scipy.linalg.lapack


# ---------------------------------------------------------------------------
# Green's function and the Q (theta) intermediate
# ---------------------------------------------------------------------------

def overlap_matrix(trial: np.ndarray, phi: np.ndarray) -> np.ndarray:
    """Psi_T^dagger Phi (n x n), the matrix inverted in Eq. 11 and Eq. 15."""
    return trial.conj().T @ phi


def green_theta(trial: np.ndarray, phi: np.ndarray):
    """Q = Phi (Psi_T^dagger Phi)^{-1} (Sec. 2.2, Eq. 15), with LU diagnostics.

    Returns (theta, log_det, info).  ``log_det`` is log det(Psi_T^dagger Phi)
    for one spin (the restricted overlap <Psi_T|phi> is its exponential
    squared).  ``info`` follows the LAPACK getrf convention: 0 on success,
    k > 0 if U(k,k) of the partially pivoted LU is exactly zero, in which case
    theta is None.
    """
    O = overlap_matrix(trial, phi)
    lu, piv, info = scipy.linalg.lapack.zgetrf(np.asarray(O, dtype=np.complex128))
    if info != 0:
        return None, complex("nan"), int(info)
    # theta O = phi  <=>  O^T theta^T = phi^T
    theta = scipy.linalg.lu_solve((lu, piv), phi.T, trans=1).T
    sign, logabs = np.linalg.slogdet(O)
    return theta, complex(np.log(sign) + logabs), 0


def greens_function(trial: np.ndarray, phi: np.ndarray) -> np.ndarray:
    """G_pq = [Phi (Psi_T^dagger Phi)^{-1} Psi_T^dagger]^T_pq (Eq. 11)."""
    O = overlap_matrix(trial, phi)
    return (phi @ np.linalg.inv(O) @ trial.conj().T).T


# ---------------------------------------------------------------------------
# Generalised Wick's theorem with the full ERI tensor (Eq. 10)
# ---------------------------------------------------------------------------

def e2_wick(eri: np.ndarray, G_alpha: np.ndarray, G_beta: np.ndarray):
    """Eq. 10 written out over the spin labels sigma, tau.

    E2 = 1/2 sum_pqrs V_pqrs sum_{sigma tau} (G_{p sigma, r sigma} G_{q tau, s tau}
                                              - G_{p sigma, s tau} G_{q tau, r sigma}),
    with G_{p sigma, q tau} = delta_{sigma tau} G^sigma_pq (Eq. 11).
    Returns (E_J, E_K).
    """
    V = eri.transpose(0, 2, 1, 3)  # V[p,q,r,s] = (pr|qs)
    G = (G_alpha, G_beta)
    direct = 0.0 + 0.0j
    exchange = 0.0 + 0.0j
    for sigma in (0, 1):
        for tau in (0, 1):
            direct += np.einsum("pqrs,pr,qs->", V, G[sigma], G[tau])
            if sigma == tau:  # the Kronecker delta of the exchange term
                exchange += np.einsum("pqrs,ps,qr->", V, G[sigma], G[tau])
    return 0.5 * direct, -0.5 * exchange


def e2_wick_restricted(eri: np.ndarray, trial: np.ndarray, phi: np.ndarray):
    G = greens_function(trial, phi)
    return e2_wick(eri, G, G)


def eri_from_cholesky(chol: np.ndarray) -> np.ndarray:
    """(pr|qs) = sum_g L_g[p][r] L_g[q][s], returned as eri[p,r,q,s]."""
    return np.einsum("gpr,gqs->prqs", chol, chol)


# ---------------------------------------------------------------------------
# Half-rotated Cholesky route (Sec. 2.2, Eq. 16)
# ---------------------------------------------------------------------------

def half_rotate(chol: np.ndarray, trial: np.ndarray) -> np.ndarray:
    """Lbar^g_{ri} = sum_p L^g_{rp} conj(Psi_T)_{pi}, returned as lbar[g, i, r]."""
    return np.einsum("grp,pi->gir", chol, trial.conj())


def e2_cholesky(lbar: np.ndarray, theta: np.ndarray):
    """Eq. 16 for one restricted determinant.

    The spin sums give 4 Q_ri Q_sj for the direct term and 2 Q_si Q_rj for the
    exchange term inside the factor 1/2.  With T_g = Lbar_g Q (n x n):
    E_J = 2 sum_g (Tr T_g)^2 and E_K = -sum_g sum_ij T_g[i,j] T_g[j,i].
    """
    T = np.matmul(lbar, theta)                       # [g, i, j]
    tr = np.einsum("gii->g", T)
    e_j = 2.0 * np.sum(tr * tr)
    e_k = -np.einsum("gij,gji->", T, T)
    return complex(e_j), complex(e_k)


# ---------------------------------------------------------------------------
# HR-ERI route (Eq. 17)
# ---------------------------------------------------------------------------

def pair_block(lbar: np.ndarray, i: int, j: int) -> np.ndarray:
    """Y^{[ij]}_{rs} = sum_g Lbar^g_{ri} Lbar^g_{sj} (Sec. 2.2, above Eq. 17)."""
    return lbar[:, i, :].T @ lbar[:, j, :]


def e2_hr_eri(lbar: np.ndarray, theta: np.ndarray):
    """Eq. 17: E2 = 1/2 sum_ij sum_rs Y^{[ij]}_rs (4 Q_ri Q_sj - 2 Q_si Q_rj)."""
    n = lbar.shape[1]
    e_j = 0.0 + 0.0j
    e_k = 0.0 + 0.0j
    for i in range(n):
        for j in range(n):
            Y = pair_block(lbar, i, j)
            e_j += 2.0 * (theta[:, i] @ Y @ theta[:, j])
            e_k -= theta[:, j] @ Y @ theta[:, i]
    return complex(e_j), complex(e_k)


# ---------------------------------------------------------------------------
# Localized-orbital compression (Sec. 2.3.1, Eq. 18) and LO energy (Eq. 19, 22)
# ---------------------------------------------------------------------------

def lo_decompose(lbar: np.ndarray, pairs: str = "ordered"):
    """Full SVD Y^{[ij]} = U Sigma V of every pair block (Sec. 2.3.1, Eq. 18).

    ``pairs="ordered"`` decomposes all n^2 blocks as the paper lists them;
    ``pairs="upper"`` decomposes only i <= j (Y^{[ji]} is the transpose of
    Y^{[ij]}, whose SVD is V^T Sigma U^T).  Returns dict (i, j) -> (U, sigma, V)
    with sigma in non-increasing order.
    """
    n = lbar.shape[1]
    cols = [np.ascontiguousarray(lbar[:, i, :]) for i in range(n)]  # [g, r] per orbital
    out = {}
    for i in range(n):
        for j in range(n):
            if pairs == "upper" and j < i:
                continue
            out[(i, j)] = np.linalg.svd(cols[i].T @ cols[j])
    return out


def lo_decompose_randomized(lbar: np.ndarray, omega: np.ndarray, power_iters: int):
    """Approximate SVD of every pair block i <= j by randomized subspace
    iteration (Halko, Martinsson and Tropp, SIAM Rev. 53 (2011), Alg. 4.4),
    the cheaper decomposition Sec. 2.3.1 mentions: with the test matrix omega
    (M x l), Z = Y omega; power_iters times Q = orth(Z), Q' = orth(Y^T Q),
    Z = Y Q'; then Q = orth(Z), B = Q^T Y = U_B Sigma V, U = Q U_B.  orth is a
    QR factorisation.  Returns dict (i, j) -> (U [M x l], sigma [l], V [l x M]),
    the input format of lo_truncate.
    """
    n = lbar.shape[1]
    cols = [np.ascontiguousarray(lbar[:, i, :]) for i in range(n)]
    orth = lambda A: np.linalg.qr(A)[0]  # noqa: E731
    out = {}
    for i in range(n):
        for j in range(i, n):
            Y = cols[i].T @ cols[j]
            Z = Y @ omega
            for _ in range(power_iters):
                Q = orth(Z)
                Z = Y @ orth(Y.T @ Q)
            Q = orth(Z)
            Ub, s, Vh = np.linalg.svd(Q.T @ Y, full_matrices=False)
            out[(i, j)] = (Q @ Ub, s, Vh)
    return out


def lo_truncate(decomp: dict, eps: float):
    """Keeps the singular values sigma_K >= eps (all of them when eps == 0).

    Ubar = U Sigma^(1/2) and Vbar = Sigma^(1/2) V.  Returns dict (i, j) ->
    (Ubar [M x K], Vbar [K x M], sigma [M]) where sigma holds all singular
    values of the block (for ranks and error bounds).
    """
    if not (eps >= 0.0):
        raise ValueError("eps must be >= 0")
    out = {}
    for key, (U, s, Vh) in decomp.items():
        K = s.size if eps == 0.0 else int(np.count_nonzero(s >= eps))
        root = np.sqrt(s[:K])
        out[key] = (U[:, :K] * root[None, :], root[:, None] * Vh[:K], s)
    return out


def lo_compress(lbar: np.ndarray, eps: float, pairs: str = "ordered"):
    """Truncated SVD of every pair block (Sec. 2.3.1, Eq. 18): decompose, then
    keep sigma_K >= eps (see lo_decompose and lo_truncate)."""
    if not (eps >= 0.0):
        raise ValueError("eps must be >= 0")
    return lo_truncate(lo_decompose(lbar, pairs), eps)


def expand_upper(factors: dict, n: int) -> dict:
    """Fill (j, i) for j > i from (i, j) using Y^{[ji]} = (Y^{[ij]})^T."""
    full = dict(factors)
    for i in range(n):
        for j in range(i + 1, n):
            if (j, i) not in full:
                Ub, Vb, s = factors[(i, j)]
                full[(j, i)] = (Vb.T, Ub.T, s)
    return full


def lo_ranks(factors: dict, n: int) -> np.ndarray:
    """M_SVD^{[ij]} for every ordered pair."""
    full = expand_upper(factors, n)
    K = np.zeros((n, n), dtype=np.int64)
    for (i, j), (Ub, _, _) in full.items():
        K[i, j] = Ub.shape[1]
    return K


def compression_percent(ranks: np.ndarray, M: int) -> float:
    """(M - <M_SVD>) / M * 100 (Sec. 3, the dodecane discussion)."""
    return float(100.0 * (M - ranks.mean()) / M)


def e2_lo(factors: dict, theta: np.ndarray):
    """Eq. 22 for one determinant, with the four vectors of Eq. 23.

    For each ordered pair [ij]:  QL_i = Ubar^T Q_i, QR_j = Vbar Q_j,
    QL_j = Ubar^T Q_j, QR_i = Vbar Q_i, and
    E2 = 1/2 sum_ij sum_K (4 QL_i QR_j - 2 QL_j QR_i).
    """
    n = theta.shape[1]
    full = expand_upper(factors, n)
    e_j = 0.0 + 0.0j
    e_k = 0.0 + 0.0j
    for i in range(n):
        for j in range(n):
            Ub, Vb, _ = full[(i, j)]
            ql_i = Ub.T @ theta[:, i]
            qr_j = Vb @ theta[:, j]
            ql_j = Ub.T @ theta[:, j]
            qr_i = Vb @ theta[:, i]
            e_j += 2.0 * np.sum(ql_i * qr_j)
            e_k -= np.sum(ql_j * qr_i)
    return complex(e_j), complex(e_k)


def lo_error_bound(factors: dict, theta: np.ndarray) -> float:
    """A-priori bound on |E2_LO - E2_HR-ERI| for one walker.

    With Delta_ij = Y^{[ij]} - Ubar Vbar, ||Delta_ij||_2 is the first discarded
    singular value, and |x^T Delta y| <= ||Delta||_2 ||x|| ||y||, so
    |dE| <= sum_ij (2 + 1) sigma_{K+1}^{[ij]} ||Q_i|| ||Q_j||.
    """
    n = theta.shape[1]
    full = expand_upper(factors, n)
    norms = np.linalg.norm(theta, axis=0)
    bound = 0.0
    for (i, j), (Ub, _, s) in full.items():
        K = Ub.shape[1]
        first_dropped = s[K] if K < s.size else 0.0
        bound += 3.0 * first_dropped * norms[i] * norms[j]
    return float(bound)


# ---------------------------------------------------------------------------
# Batched conveniences (loops over walkers; nothing is fused)
# ---------------------------------------------------------------------------

def green_theta_batch(trial: np.ndarray, walkers: np.ndarray):
    nw, M, n = walkers.shape
    theta = np.full((nw, M, n), np.nan + 0j, dtype=np.complex128)
    logdet = np.zeros(nw, dtype=np.complex128)
    info = np.zeros(nw, dtype=np.int32)
    for w in range(nw):
        t, ld, inf = green_theta(trial, walkers[w])
        info[w] = inf
        logdet[w] = ld
        if inf == 0:
            theta[w] = t
    return theta, logdet, info


def e2_cholesky_batch(lbar: np.ndarray, thetas: np.ndarray) -> np.ndarray:
    """[nw, 2] complex: (E_J, E_K) per walker."""
    return np.array([e2_cholesky(lbar, t) for t in thetas], dtype=np.complex128)


def e2_lo_batch(factors: dict, thetas: np.ndarray) -> np.ndarray:
    return np.array([e2_lo(factors, t) for t in thetas], dtype=np.complex128)
