"""Plain FP64 reference of the Foster-Boys localization of occupied orbitals
(test infrastructure: only tests/, the smoke check and the bench's CPU
baseline use it).

Sec. 3 localizes the occupied trial orbitals by the Foster-Boys criterion
before the pair blocks are compressed; the compression of Sec. 2.3.1 relies on
orbitals of compact support.  The criterion maximises the sum of squared
orbital centroids,
    B(U) = sum_i sum_d (<i|x_d|i>)^2,   orbitals C U with U orthogonal,
over the position operators x_d of the basis.  The chain's basis functions
sit at x = p (one dimension), so x is diag(0, 1, ..., M - 1); the routine takes
any number D of diagonal position operators.

Algorithm (Jacobi sweeps, as in Foster and Boys' and Edmiston and
Ruedenberg's treatments): with X_d = C^T x_d C, for each pair i < j in row
order rotate orbitals i and j by the angle t that maximises the pair's part of
B.  Writing a_d = X_d[i][i], b_d = X_d[j][j], c_d = X_d[i][j], the pair part
after the rotation is const + sum_d (h_d cos 2t + c_d sin 2t)^2 with
h_d = (a_d - b_d) / 2, maximal at
    4t = atan2(2 sum_d c_d h_d, sum_d (h_d^2 - c_d^2)).
Every rotation is applied (no skipping threshold), so the sequence of
rotations is fixed by the input.  Sweeps stop after `max_sweeps` or when B
grows by less than tol * B in a sweep.
"""
from __future__ import annotations

import numpy as np


def boys_functional(C: np.ndarray, positions: np.ndarray) -> float:
    """B = sum_i sum_d (C[:, i]^T diag(positions[d]) C[:, i])^2."""
    cent = np.einsum("dm,mi->di", positions, C * C)
    return float(np.sum(cent * cent))


def boys_jacobi(C: np.ndarray, positions: np.ndarray, max_sweeps: int = 50, tol: float = 1e-14):
    """Localized orbitals C U and the functional after each sweep.

    C: [M][n] orthonormal columns; positions: [D][M] diagonal position
    operators.  Returns (C U, [B before any sweep, B after sweep 1, ...]).
    """
    positions = np.atleast_2d(np.asarray(positions, dtype=np.float64))
    n = C.shape[1]
    X = np.stack([C.T @ (p[:, None] * C) for p in positions])     # [D][n][n]
    U = np.eye(n)
    history = [float(np.sum(np.einsum("dii->di", X) ** 2))]
    for _ in range(max_sweeps):
        for i in range(n):
            for j in range(i + 1, n):
                h = 0.5 * (X[:, i, i] - X[:, j, j])
                c = X[:, i, j]
                t = 0.25 * np.arctan2(2.0 * np.sum(c * h), np.sum(h * h - c * c))
                cs, sn = np.cos(t), np.sin(t)
                # new orbital i = cs i + sn j, new orbital j = -sn i + cs j
                R = np.array([[cs, -sn], [sn, cs]])
                idx = [i, j]
                X[:, :, idx] = X[:, :, idx] @ R
                X[:, idx, :] = np.einsum("ab,dbk->dak", R.T, X[:, idx, :])
                U[:, idx] = U[:, idx] @ R
        history.append(float(np.sum(np.einsum("dii->di", X) ** 2)))
        if history[-1] - history[-2] <= tol * abs(history[-1]):
            break
    return C @ U, history


def chain_positions(M: int) -> np.ndarray:
    """The chain's one position operator, x = diag(0, 1, ..., M - 1), as [1][M]."""
    return np.arange(M, dtype=np.float64)[None, :]
