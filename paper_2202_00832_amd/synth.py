"""Seeded synthetic inputs for the walker local-energy path.

This module only *builds inputs*: a one-dimensional chain Hamiltonian
(electron-repulsion integrals and their pivoted Cholesky factorisation), a
localized single-determinant trial and a population of noisy walkers.  It holds
none of the energy method's arithmetic (no Green's functions, no half-rotation,
no pair compression, no energies), so the CPU reference and the GPU library can
both consume it without sharing any of the method.

Model (the paper's molecules are replaced by this synthetic stand-in):

* M basis functions at x_p = p (unit spacing), treated as orthonormal.
* S_pq = exp(-(x_p - x_q)^2 / 2), set to zero for |p - q| > band (default 8,
  where the dropped values are below 1.3e-14).  Zeroing entries of S is a
  congruence with a diagonal matrix, so the ERI matrix below stays PSD.
* (pq|rs) = S_pq S_rs / sqrt(1 + (c_pq - c_rs)^2) with c_pq = (x_p + x_q)/2.
  1/sqrt(1+d^2) has a positive Fourier transform (2 K_0(|k|)), so the matrix
  over pair indices is positive semidefinite and admits a Cholesky factor.
* The two-electron operator is factorised as V_pqrs = (pr|qs) =
  sum_g L_g[p][r] L_g[q][s] (Sec. 2.1.1, the three-index form below Eq. 13) by
  a diagonal-pivoted ("modified") Cholesky decomposition stopped when the
  largest residual diagonal falls below tol.  Ties pick the lowest flattened
  pair index p*M + q.
* Trial: n Gaussians exp(-(p - c_k)^2/2) centred at c_k = floor(k*M/n),
  Lowdin-orthonormalised, C = G (G^T G)^{-1/2}, with |entries| < 1e-30 set to
  zero (keeps every value in the normal floating-point range).  These orbitals are already
  localized, which is what the compression of Sec. 2.3.1 relies on.
* Walkers: Q factor of the thin QR of Psi_T + sigma (Z1 + i Z2), with Z1, Z2
  independent standard normal matrices.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

DEFAULT_BAND = 8


# ----------------------------------------------------------------------------
# Chain Hamiltonian
# ----------------------------------------------------------------------------

def chain_overlap(M: int, band: int = DEFAULT_BAND) -> np.ndarray:
    """S_pq = exp(-(p-q)^2/2) for |p-q| <= band, zero beyond."""
    p = np.arange(M, dtype=np.float64)
    d = p[:, None] - p[None, :]
    S = np.exp(-0.5 * d * d)
    S[np.abs(d) > band] = 0.0
    return S


def chain_eri_dense(M: int, band: int = DEFAULT_BAND) -> np.ndarray:
    """Dense chemists'-notation tensor eri[p,q,r,s] = (pq|rs) (small M only)."""
    if M > 40:
        raise ValueError("dense ERI is M^4; use the Cholesky factor for M > 40")
    S = chain_overlap(M, band)
    x = np.arange(M, dtype=np.float64)
    c = 0.5 * (x[:, None] + x[None, :])
    d = c[:, :, None, None] - c[None, None, :, :]
    return S[:, :, None, None] * S[None, None, :, :] / np.sqrt(1.0 + d * d)


def _unique_pairs(M: int, band: int):
    """Pairs p <= q with q - p <= band, ordered by flattened index p*M + q."""
    ps, qs = [], []
    for p in range(M):
        for q in range(p, min(M, p + band + 1)):
            ps.append(p)
            qs.append(q)
    return np.asarray(ps, dtype=np.int64), np.asarray(qs, dtype=np.int64)


def chain_cholesky(M: int, tol: float, band: int = DEFAULT_BAND,
                   max_vectors: int | None = None) -> np.ndarray:
    """Pivoted Cholesky factor of the chain ERI, returned as L[g][p][q].

    Each L_g is symmetric (the ERI is symmetric under p<->q), so the
    factorisation runs on the unique pairs p <= q and is mirrored at the end.
    The residual diagonal of every pair stays below ``tol`` on exit.
    """
    ps, qs = _unique_pairs(M, band)
    npair = ps.size
    S = chain_overlap(M, band)
    s_pair = S[ps, qs]
    c_pair = 0.5 * (ps + qs).astype(np.float64)
    diag = s_pair * s_pair  # (pq|pq) = S_pq^2
    cap = max_vectors if max_vectors is not None else min(npair, 12 * M + 64)
    Lp = np.zeros((cap, npair), dtype=np.float64)
    k = 0
    while k < cap:
        piv = int(np.argmax(diag))  # first maximum = lowest flattened index
        dmax = diag[piv]
        if dmax < tol:
            break
        d = c_pair - c_pair[piv]
        col = s_pair * s_pair[piv] / np.sqrt(1.0 + d * d)
        if k:
            col -= Lp[:k].T @ Lp[:k, piv]
        v = col / math.sqrt(dmax)
        Lp[k] = v
        diag = diag - v * v
        diag[piv] = 0.0
        k += 1
    else:
        raise RuntimeError("pivoted Cholesky did not converge within %d vectors" % cap)
    L = np.zeros((k, M, M), dtype=np.float64)
    L[:, ps, qs] = Lp[:k]
    L[:, qs, ps] = Lp[:k]
    return L


def chain_cholesky_residual_max(M: int, L: np.ndarray, band: int = DEFAULT_BAND) -> float:
    """max_pq [(pq|pq) - sum_g L_g[p][q]^2] over all pairs (a check helper)."""
    S = chain_overlap(M, band)
    resid = S * S - np.einsum("gpq,gpq->pq", L, L)
    return float(resid.max())


# ----------------------------------------------------------------------------
# Trial determinant and walkers
# ----------------------------------------------------------------------------

def gaussian_centres(M: int, n: int) -> np.ndarray:
    return np.array([(k * M) // n for k in range(n)], dtype=np.int64)


TRIAL_FLUSH = 1e-30


def lowdin_gaussian_trial(M: int, n: int) -> np.ndarray:
    """Real M x n trial with orthonormal, localized columns.

    Entries below TRIAL_FLUSH in magnitude are set to zero: the Gaussian tails
    otherwise reach the subnormal range, which slows CPU linear algebra by
    orders of magnitude without changing any result above 1e-30.
    """
    p = np.arange(M, dtype=np.float64)[:, None]
    c = gaussian_centres(M, n).astype(np.float64)[None, :]
    G = np.exp(-0.5 * (p - c) ** 2)
    G[G < TRIAL_FLUSH] = 0.0
    w, V = np.linalg.eigh(G.T @ G)
    C = G @ (V * (1.0 / np.sqrt(w))) @ V.T
    C[np.abs(C) < TRIAL_FLUSH] = 0.0
    return C


def noisy_walkers(trial: np.ndarray, nw: int, sigma: float,
                  rng: np.random.Generator) -> np.ndarray:
    """nw walkers [nw][M][n] complex128: Q of QR(trial + sigma (Z1 + i Z2))."""
    M, n = trial.shape
    out = np.empty((nw, M, n), dtype=np.complex128)
    for w in range(nw):
        z = rng.standard_normal((M, n)) + 1j * rng.standard_normal((M, n))
        q, _ = np.linalg.qr(trial + sigma * z)
        out[w] = q
    return out


def random_walks(trial: np.ndarray, n_walks: int, n_steps: int, step: float,
                 rng: np.random.Generator) -> np.ndarray:
    """Walkers along random walks from the trial, [n_steps][n_walks][M][n]
    complex128: phi <- Q of QR(phi + step (Z1 + i Z2)) at every step (a
    stand-in for the propagation, which is not built)."""
    M, n = trial.shape
    out = np.empty((n_steps, n_walks, M, n), dtype=np.complex128)
    phi = np.repeat(trial[None].astype(np.complex128), n_walks, axis=0)
    for k in range(n_steps):
        z = rng.standard_normal(phi.shape) + 1j * rng.standard_normal(phi.shape)
        phi = phi + step * z
        for w in range(n_walks):
            phi[w] = np.linalg.qr(phi[w])[0]
        out[k] = phi
    return out


def delocalized_trial(trial: np.ndarray) -> np.ndarray:
    """Canonical-like orbitals spanning the same space as `trial`: the
    eigenvectors of the chain's nearest-neighbour hopping operator projected
    onto that space (standing waves over the whole chain), C V with
    C^T H C = V diag V^T, H[p][p +- 1] = -1.  Input for the localization
    tests; column signs fixed so that each column's largest entry is
    positive."""
    M = trial.shape[0]
    H = -(np.eye(M, k=1) + np.eye(M, k=-1))
    _, V = np.linalg.eigh(trial.T @ H @ trial)
    C = trial @ V
    big = np.argmax(np.abs(C), axis=0)
    return C * np.sign(C[big, np.arange(C.shape[1])])[None, :]


def random_orthogonal(n: int, rng: np.random.Generator) -> np.ndarray:
    """Haar-ish random real orthogonal n x n matrix (used to delocalize a trial)."""
    q, r = np.linalg.qr(rng.standard_normal((n, n)))
    return q * np.sign(np.diag(r))[None, :]


def random_symmetric_cholesky(M: int, X: int, rng: np.random.Generator) -> np.ndarray:
    """X random symmetric M x M matrices: a generic factorised Hamiltonian."""
    A = rng.standard_normal((X, M, M)) / M
    return 0.5 * (A + A.transpose(0, 2, 1))


# ----------------------------------------------------------------------------
# Named workloads
# ----------------------------------------------------------------------------

@dataclasses.dataclass(frozen=True)
class ChainConfig:
    name: str
    M: int            # basis functions
    n: int            # occupied orbitals per spin
    nw: int           # walkers
    chol_tol: float   # pivoted Cholesky stopping tolerance
    sigma: float      # walker noise
    seed: int
    epsilons: tuple = (1e-3, 1e-4, 1e-5)


# Small case: 48 sites, 8 orbitals per spin (Gaussians on every 6th site),
# Cholesky to 1e-6, 16 walkers with noise 0.1.
CHAIN_SMALL = ChainConfig("chain-M48-n8-w16", 48, 8, 16, 1e-6, 0.1, 1001)
# Polyacene-scale case: 400 sites, 60 orbitals per spin, Cholesky to 1e-5,
# 512 walkers with noise 0.2.
CHAIN_POLYACENE = ChainConfig("chain-M400-n60-w512", 400, 60, 512, 1e-5, 0.2, 1002)
# Mixed-precision study size: 500 sites, 48 orbitals, 1024 walkers.
CHAIN_PRECISION = ChainConfig("chain-M500-n48-w1024", 500, 48, 1024, 1e-5, 0.2, 1003,
                              epsilons=(1e-4,))

# Learned-residual size: 800 sites, 100 orbitals per spin, 2048 walkers, LO at 1e-3.
CHAIN_RESIDUAL = ChainConfig("chain-M800-n100-w2048", 800, 100, 2048, 1e-5, 0.2, 1005, epsilons=(1e-3,))

CONFIGS = {c.name: c for c in (CHAIN_SMALL, CHAIN_POLYACENE, CHAIN_PRECISION, CHAIN_RESIDUAL)}


# ----------------------------------------------------------------------------
# Multi-determinant (CAS-type) trials
# ----------------------------------------------------------------------------

@dataclasses.dataclass(frozen=True)
class CasConfig:
    name: str
    M: int            # basis functions
    n: int            # occupied orbitals per spin in each determinant
    n_act_occ: int    # active orbitals occupied in the reference determinant
    n_act_virt: int   # active orbitals empty in the reference determinant
    n_det: int        # determinants, the reference included
    max_exc: int      # largest excitation level
    nw: int           # walkers
    chol_tol: float
    sigma: float
    seed: int
    epsilon: float = 1e-5

    @property
    def n_cas(self) -> int:
        return self.n + self.n_act_virt


# Small CAS case: 48 sites, 8 occupied + 3 active virtual orbitals, 3 active
# occupied, all 20 determinants up to triples, 16 walkers.
CAS_SMALL = CasConfig("cas-M48-n8-a3x3-d20-w16", 48, 8, 3, 3, 20, 3, 16, 1e-6, 0.1, 2001)
# Polyacene-scale CAS case: 400 sites, 60 occupied + 5 active virtual orbitals,
# 5 active occupied, 200 determinants up to quadruples, 512 walkers.
CAS_POLYACENE = CasConfig("cas-M400-n60-a5x5-d200-w512", 400, 60, 5, 5, 200, 4, 512, 1e-5, 0.2, 2002)


def cas_orbitals(M: int, n: int, n_act_occ: int, n_act_virt: int) -> np.ndarray:
    """M x (n + n_act_virt) orthonormal localized orbitals (Lowdin Gaussians).

    Columns 0 .. n-1 are the reference determinant's orbitals, the last
    n_act_occ of them active; columns n .. are the active virtual orbitals.
    The active orbitals are spread along the chain (evenly spaced centres,
    alternately occupied and virtual) rather than bunched at one end.
    """
    n_cas = n + n_act_virt
    C = lowdin_gaussian_trial(M, n_cas)
    n_act = n_act_occ + n_act_virt
    act = [int(round(x)) for x in np.linspace(0, n_cas - 1, n_act)]
    occ_act, virt_act = [], []
    for k, c in enumerate(act):
        if (k % 2 == 0 and len(occ_act) < n_act_occ) or len(virt_act) == n_act_virt:
            occ_act.append(c)
        else:
            virt_act.append(c)
    inactive = [c for c in range(n_cas) if c not in act]
    order = inactive + occ_act + virt_act
    return np.ascontiguousarray(C[:, order])


def cas_expansion(n: int, n_act_occ: int, n_act_virt: int, n_det: int, max_exc: int,
                  rng: np.random.Generator):
    """Seeded synthetic CI expansion over the active space.

    Determinant d replaces the reference columns holes[d] (among the last
    n_act_occ of the n occupied ones) by the orbitals particles[d] (columns
    n .. n + n_act_virt - 1), hole k by particle k.  The reference comes first,
    then n_det - 1 excitations drawn without replacement from all of those up to
    max_exc, listed by level; coefficients 1 for the reference and
    0.25^level x N(0, 1) otherwise.  Returns (holes, particles, coeffs).
    """
    import itertools
    hole_set = range(n - n_act_occ, n)
    part_set = range(n, n + n_act_virt)
    pool = []
    for k in range(1, max_exc + 1):
        for h in itertools.combinations(hole_set, k):
            for p in itertools.combinations(part_set, k):
                pool.append((h, p))
    if n_det - 1 > len(pool):
        raise ValueError("only %d excitations up to level %d" % (len(pool), max_exc))
    pick = sorted(rng.choice(len(pool), size=n_det - 1, replace=False)) if n_det > 1 else []
    holes, parts, coeffs = [()], [()], [1.0]
    for q in pick:
        h, p = pool[q]
        holes.append(h)
        parts.append(p)
        coeffs.append(0.25 ** len(h) * float(rng.standard_normal()))
    return holes, parts, np.array(coeffs)


@dataclasses.dataclass
class CasSystem:
    config: CasConfig
    chol: np.ndarray      # [X][M][M]
    orbitals: np.ndarray  # [M][n_cas]
    holes: list
    particles: list
    coeffs: np.ndarray    # [n_det]
    walkers: np.ndarray   # [nw][M][n] complex128

    @property
    def reference(self) -> np.ndarray:
        return np.ascontiguousarray(self.orbitals[:, :self.config.n])


def make_cas_system(cfg: CasConfig, nw: int | None = None) -> CasSystem:
    rng = np.random.default_rng(cfg.seed)
    chol = chain_cholesky(cfg.M, cfg.chol_tol)
    C = cas_orbitals(cfg.M, cfg.n, cfg.n_act_occ, cfg.n_act_virt)
    holes, parts, coeffs = cas_expansion(cfg.n, cfg.n_act_occ, cfg.n_act_virt, cfg.n_det, cfg.max_exc, rng)
    walkers = noisy_walkers(np.ascontiguousarray(C[:, :cfg.n]), cfg.nw if nw is None else nw, cfg.sigma, rng)
    return CasSystem(cfg, chol, C, holes, parts, coeffs, walkers)


def batch_configs(count: int = 8, seed: int = 4004, m_range=(100, 600), w_range=(64, 512)) -> list:
    """Ragged set of chain systems: M uniform in m_range, n = M // 7 orbitals
    per spin, Cholesky to 1e-5, walkers uniform in w_range, noise 0.2; one
    seed per system drawn from `seed`."""
    rng = np.random.default_rng(seed)
    out = []
    for k in range(count):
        M = int(rng.integers(m_range[0], m_range[1] + 1))
        nw = int(rng.integers(w_range[0], w_range[1] + 1))
        sd = int(rng.integers(0, 2 ** 31 - 1))
        out.append(ChainConfig("chain-M%d-n%d-w%d" % (M, M // 7, nw), M, M // 7, nw, 1e-5, 0.2, sd, epsilons=()))
    return out


@dataclasses.dataclass
class ChainSystem:
    config: ChainConfig
    chol: np.ndarray      # [X][M][M] float64
    trial: np.ndarray     # [M][n]   float64
    walkers: np.ndarray   # [nw][M][n] complex128

    @property
    def n_chol(self) -> int:
        return self.chol.shape[0]


def make_system(cfg: ChainConfig, nw: int | None = None) -> ChainSystem:
    rng = np.random.default_rng(cfg.seed)
    chol = chain_cholesky(cfg.M, cfg.chol_tol)
    trial = lowdin_gaussian_trial(cfg.M, cfg.n)
    walkers = noisy_walkers(trial, cfg.nw if nw is None else nw, cfg.sigma, rng)
    return ChainSystem(cfg, chol, trial, walkers)
