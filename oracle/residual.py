"""Plain FP64 reference of the learned LO residual (test infrastructure).

Not part of the paper's method: a small network that predicts, per walker,
the part of the two-body energy that the LO truncation drops,
    Re(E_full - E_LO)  ~  sum_i f(x_i),
from cheap per-orbital features x_i of occupied orbital i:
    x_i0 = sum_j K_ij            (retained rank of the pair blocks of orbital i)
    x_i1 = sum_j m_ij            (discarded singular-value mass of those blocks,
                                  m_ij = sum of the singular values of Y^[ij]
                                  below the threshold)
    x_i2 = || theta[:, i] ||_2   (norm of orbital i's column of Q)
    x_i3 = Re(g_i . theta[:, i]) (first-order change of the dropped energy
                                  along orbital i's column; g_i is the
                                  gradient of E_HR - E_LO with respect to
                                  column i of Q at the trial, Q = Psi,
                                  dropped_energy_gradient)
The first three carry no walker-specific information about the sign of the
dropped energy (only column norms vary between walkers), so on their own the
best additive predictor is a constant; x_i3 is the walker-dependent part.
f is a 3-layer perceptron 4 -> 128 -> 128 -> 1 with tanh activations on
standardised inputs z = (x - shift) * scale.  The walker loss is the mean
squared error over walkers of sum_i f(x_i) against the target.

Parameters are one flat float vector, in this order:
    W1 [128][4], b1 [128], W2 [128][128], b2 [128], w3 [128], b3 [1],
    shift [4], scale [4]          (shift and scale are not trained)
Everything here is float64 numpy; the backward pass is written out by hand.
"""
from __future__ import annotations

import numpy as np

WIDTH = 128
NFEAT = 4
SIZES = [("W1", (WIDTH, NFEAT)), ("b1", (WIDTH,)), ("W2", (WIDTH, WIDTH)), ("b2", (WIDTH,)),
         ("w3", (WIDTH,)), ("b3", (1,)), ("shift", (NFEAT,)), ("scale", (NFEAT,))]
NPARAM = sum(int(np.prod(s)) for _, s in SIZES)
TRAINED = ("W1", "b1", "W2", "b2", "w3", "b3")


def unpack(p: np.ndarray) -> dict:
    out, at = {}, 0
    for name, shape in SIZES:
        k = int(np.prod(shape))
        out[name] = p[at:at + k].reshape(shape)
        at += k
    return out


def pack(d: dict) -> np.ndarray:
    return np.concatenate([np.asarray(d[name], dtype=np.float64).reshape(-1) for name, _ in SIZES])


def features(ranks: np.ndarray, discarded: np.ndarray, theta: np.ndarray, grad: np.ndarray) -> np.ndarray:
    """x[i] = (sum_j K_ij, sum_j m_ij, ||theta[:, i]||, Re(grad[i] . theta[:, i]))
    for one walker; grad is dropped_energy_gradient's [n][M]; returns [n][4]."""
    n = theta.shape[1]
    x = np.empty((n, NFEAT))
    x[:, 0] = ranks.sum(axis=1)
    x[:, 1] = discarded.sum(axis=1)
    x[:, 2] = np.sqrt(np.sum(np.abs(theta) ** 2, axis=0))
    x[:, 3] = np.array([np.real(grad[i] @ theta[:, i]) for i in range(n)])
    return x


def dropped_energy_gradient(lbar: np.ndarray, factors: dict, trial: np.ndarray) -> np.ndarray:
    """g[i] = d(E_HR - E_LO)/d theta[:, i] at theta = trial; [n][M].

    Both energies are the same quadratic form of Q (Eq. 17 and Eq. 22) with
    pair matrices A^[ij] = Y^[ij] (exact, oracle.energy.pair_block) or
    Ubar^[ij] Vbar^[ij] (LO, every ordered pair):
        E(Q) = sum_ij 2 Q_i^T A^[ij] Q_j - Q_j^T A^[ij] Q_i,
    whose gradient with respect to column i is
        sum_j 2 (A^[ij] + A^[ji]^T) Q_j - (A^[ji] + A^[ij]^T) Q_j.
    The dropped matrices D^[ij] = Y^[ij] - Ubar Vbar take the place of A.
    lbar is oracle.energy.half_rotate's [X][n][M]; factors from lo_compress.
    """
    from oracle import energy as E
    n = lbar.shape[1]
    full = E.expand_upper(factors, n)
    D = {}
    for (i, j), (Ub, Vb, _) in full.items():
        D[(i, j)] = E.pair_block(lbar, i, j) - Ub @ Vb
    M = trial.shape[0]
    g = np.zeros((n, M))
    for i in range(n):
        for j in range(n):
            psi_j = trial[:, j]
            g[i] += 2.0 * (D[(i, j)] + D[(j, i)].T) @ psi_j - (D[(j, i)] + D[(i, j)].T) @ psi_j
    return g


def forward(p: np.ndarray, x: np.ndarray):
    """Per-orbital outputs for rows x [N][3]; returns (y [N], cache)."""
    q = unpack(p)
    z = (x - q["shift"]) * q["scale"]
    h1 = np.tanh(z @ q["W1"].T + q["b1"])
    h2 = np.tanh(h1 @ q["W2"].T + q["b2"])
    y = h2 @ q["w3"] + q["b3"][0]
    return y, (z, h1, h2)


def walker_predictions(p: np.ndarray, x: np.ndarray) -> np.ndarray:
    """x [nw][n][3] -> sum over orbitals of the network output, [nw]."""
    nw, n, _ = x.shape
    y, _ = forward(p, x.reshape(nw * n, NFEAT))
    return y.reshape(nw, n).sum(axis=1)


def loss_and_grad(p: np.ndarray, x: np.ndarray, target: np.ndarray):
    """L = mean_w (sum_i f(x_wi) - t_w)^2 and dL/dp (zero for shift and scale)."""
    nw, n, _ = x.shape
    q = unpack(p)
    y, (z, h1, h2) = forward(p, x.reshape(nw * n, NFEAT))
    pred = y.reshape(nw, n).sum(axis=1)
    r = pred - target
    loss = float(np.mean(r * r))
    g_row = np.repeat(2.0 * r / nw, n)            # dL/dy for every (walker, orbital) row
    g = {name: np.zeros(shape) for name, shape in SIZES}
    g["w3"] = h2.T @ g_row
    g["b3"] = np.array([g_row.sum()])
    dz2 = np.outer(g_row, q["w3"]) * (1.0 - h2 * h2)
    g["W2"] = dz2.T @ h1
    g["b2"] = dz2.sum(axis=0)
    dz1 = (dz2 @ q["W2"]) * (1.0 - h1 * h1)
    g["W1"] = dz1.T @ z
    g["b1"] = dz1.sum(axis=0)
    return loss, pack(g)


def adam_step(p, g, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba) of the trained parameters; returns (p, m, v)."""
    mask = np.zeros(NPARAM)
    q = unpack(mask)
    for name in TRAINED:
        q[name][...] = 1.0
    mask = pack(q)
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mh = m / (1.0 - beta1 ** t)
    vh = v / (1.0 - beta2 ** t)
    p = p - mask * lr * mh / (np.sqrt(vh) + eps)
    return p, m, v


def init_params(x_train: np.ndarray, seed: int = 0) -> np.ndarray:
    """Glorot-uniform weights, zero biases, inputs standardised by the
    training features' mean and standard deviation."""
    rng = np.random.default_rng(seed)
    flat = x_train.reshape(-1, NFEAT)
    sd = flat.std(axis=0)
    q = {
        "W1": rng.uniform(-1, 1, (WIDTH, NFEAT)) * np.sqrt(6.0 / (WIDTH + NFEAT)),
        "b1": np.zeros(WIDTH),
        "W2": rng.uniform(-1, 1, (WIDTH, WIDTH)) * np.sqrt(6.0 / (2 * WIDTH)),
        "b2": np.zeros(WIDTH),
        "w3": rng.uniform(-1, 1, WIDTH) * np.sqrt(6.0 / (WIDTH + 1)),
        "b3": np.zeros(1),
        "shift": flat.mean(axis=0),
        "scale": np.where(sd > 0, 1.0 / np.where(sd > 0, sd, 1.0), 1.0),
    }
    return pack(q)
