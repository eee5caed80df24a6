"""Pins of the CPU reference of the learned LO residual (oracle/residual.py).

The gradient is pinned by central finite differences, the forward pass by
networks whose output has a closed form, and the optimiser by the known first
step of Adam (bias-corrected, the update is -lr * sign(g) up to eps).
"""
import numpy as np
import pytest

from oracle import residual as R


def _rand_case(seed, nw=5, n=4):
    rng = np.random.default_rng(seed)
    x = np.stack([rng.integers(1, 9, (nw, n)).astype(float), rng.uniform(0, 1e-3, (nw, n)),
                  rng.uniform(0.5, 2.0, (nw, n))], axis=-1)
    p = R.init_params(x, seed=seed)
    q = R.unpack(p)
    q["b1"][...] = rng.normal(0, 0.1, R.WIDTH)
    q["b2"][...] = rng.normal(0, 0.1, R.WIDTH)
    q["b3"][...] = 0.3
    t = rng.normal(0, 1, nw)
    return R.pack(q), x, t


def test_parameter_count_and_packing():
    assert R.NPARAM == 128 * 3 + 128 + 128 * 128 + 128 + 128 + 1 + 3 + 3
    p = np.arange(R.NPARAM, dtype=float)
    assert np.array_equal(R.pack(R.unpack(p)), p)


@pytest.mark.parametrize("seed", [0, 1])
def test_gradient_matches_finite_differences(seed):
    p, x, t = _rand_case(seed)
    loss, g = R.loss_and_grad(p, x, t)
    rng = np.random.default_rng(100 + seed)
    q = R.unpack(np.arange(R.NPARAM, dtype=float))
    idx = []
    for name in R.TRAINED:
        flat = q[name].reshape(-1).astype(int)
        idx.extend(rng.choice(flat, size=min(6, flat.size), replace=False))
    for k in idx:
        h = 1e-6 * max(1.0, abs(p[k]))
        pp, pm = p.copy(), p.copy()
        pp[k] += h
        pm[k] -= h
        fd = (R.loss_and_grad(pp, x, t)[0] - R.loss_and_grad(pm, x, t)[0]) / (2 * h)
        assert abs(fd - g[k]) <= 1e-6 * max(1.0, abs(fd)), (k, fd, g[k])
    # shift and scale are not trained
    gq = R.unpack(g)
    assert not gq["shift"].any() and not gq["scale"].any()


def test_forward_closed_forms():
    p, x, _ = _rand_case(3)
    q = R.unpack(p)
    # second layer switched off: h2 = 0, every orbital contributes b3
    q["W2"][...] = 0.0
    q["b2"][...] = 0.0
    pred = R.walker_predictions(R.pack(q), x)
    assert np.allclose(pred, x.shape[1] * q["b3"][0], rtol=0, atol=1e-15)
    # constant first layer: h1 = tanh(b1), h2 = tanh(W2 tanh(b1) + b2), no input dependence
    q = R.unpack(p.copy())
    q["W1"][...] = 0.0
    h2 = np.tanh(q["W2"] @ np.tanh(q["b1"]) + q["b2"])
    pred = R.walker_predictions(R.pack(q), x)
    assert np.allclose(pred, x.shape[1] * (h2 @ q["w3"] + q["b3"][0]), rtol=1e-14, atol=1e-14)


def test_adam_first_step_is_signed_learning_rate():
    p, x, t = _rand_case(4)
    _, g = R.loss_and_grad(p, x, t)
    m = np.zeros_like(p)
    v = np.zeros_like(p)
    p1, _, _ = R.adam_step(p, g, m, v, 1, 1e-3)
    q0, q1, qg = R.unpack(p), R.unpack(p1), R.unpack(g)
    for name in R.TRAINED:
        big = np.abs(qg[name]) > 1e-4
        assert np.allclose((q0[name] - q1[name])[big], 1e-3 * np.sign(qg[name][big]), rtol=1e-3, atol=0)
    assert np.array_equal(q0["shift"], q1["shift"]) and np.array_equal(q0["scale"], q1["scale"])


def test_features_of_unit_columns():
    n, M = 3, 7
    theta = np.zeros((M, n), dtype=complex)
    theta[0, 0] = 3.0
    theta[1, 0] = 4.0j
    theta[2, 1] = 1.0
    theta[:, 2] = 0.5 + 0.5j
    ranks = np.array([[1, 2, 0], [2, 3, 1], [0, 1, 4]])
    disc = np.array([[0.1, 0.0, 0.2], [0.0, 0.3, 0.0], [0.2, 0.0, 0.0]])
    x = R.features(ranks, disc, theta)
    assert np.allclose(x[:, 0], [3, 6, 5])
    assert np.allclose(x[:, 1], [0.3, 0.3, 0.2])
    assert np.allclose(x[:, 2], [5.0, 1.0, np.sqrt(M * 0.5)])


def test_training_reduces_the_loss():
    p, x, _ = _rand_case(5, nw=40, n=6)
    t = 0.5 * x[:, :, 2].sum(axis=1) - 0.1 * x[:, :, 0].sum(axis=1)
    m = np.zeros_like(p)
    v = np.zeros_like(p)
    l0 = R.loss_and_grad(p, x, t)[0]
    for k in range(1, 301):
        _, g = R.loss_and_grad(p, x, t)
        p, m, v = R.adam_step(p, g, m, v, k, 3e-3)
    assert R.loss_and_grad(p, x, t)[0] < 0.05 * l0
