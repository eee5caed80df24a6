"""Pins of the CPU reference of the learned LO residual (oracle/residual.py).

The gradient is pinned by central finite differences, the forward pass by
networks whose output has a closed form, and the optimiser by the known first
step of Adam (bias-corrected, the update is -lr * sign(g) up to eps).  The
fourth feature's gradient of the dropped energy is pinned by central
differences of the half-rotated ERI and LO energies themselves (both are
quadratic in Q, so the difference quotient is exact up to rounding), and by
the first-order prediction of the dropped energy of walkers near the trial.
"""
import numpy as np
import pytest

from oracle import energy as E
from oracle import residual as R
from paper_2202_00832_amd import synth


def _rand_case(seed, nw=5, n=4):
    rng = np.random.default_rng(seed)
    x = np.stack([rng.integers(1, 9, (nw, n)).astype(float), rng.uniform(0, 1e-3, (nw, n)),
                  rng.uniform(0.5, 2.0, (nw, n)), rng.normal(0, 1e-3, (nw, n))], axis=-1)
    p = R.init_params(x, seed=seed)
    q = R.unpack(p)
    q["b1"][...] = rng.normal(0, 0.1, R.WIDTH)
    q["b2"][...] = rng.normal(0, 0.1, R.WIDTH)
    q["b3"][...] = 0.3
    t = rng.normal(0, 1, nw)
    return R.pack(q), x, t


def test_parameter_count_and_packing():
    assert R.NPARAM == 128 * 4 + 128 + 128 * 128 + 128 + 128 + 1 + 4 + 4
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
    grad = np.zeros((n, M))
    grad[0, 0], grad[0, 1] = 2.0, 5.0     # Re(2 * 3 + 5 * 4i) = 6
    grad[1, 2] = -1.5
    grad[2, :] = 1.0                      # Re(sum (0.5 + 0.5i)) = M / 2
    x = R.features(ranks, disc, theta, grad)
    assert np.allclose(x[:, 0], [3, 6, 5])
    assert np.allclose(x[:, 1], [0.3, 0.3, 0.2])
    assert np.allclose(x[:, 2], [5.0, 1.0, np.sqrt(M * 0.5)])
    assert np.allclose(x[:, 3], [6.0, -1.5, M * 0.5])


def _dropped(lbar, fac, theta):
    return sum(E.e2_hr_eri(lbar, theta)) - sum(E.e2_lo(fac, theta))


@pytest.fixture(scope="module")
def chain_case():
    s = synth.make_system(synth.CHAIN_SMALL, nw=1)
    lbar = E.half_rotate(s.chol, s.trial)
    fac = E.lo_compress(lbar, 1e-3, pairs="upper")
    return s, lbar, fac, R.dropped_energy_gradient(lbar, fac, s.trial)


def test_dropped_energy_gradient_matches_central_differences(chain_case):
    s, lbar, fac, g = chain_case
    M, n = s.trial.shape
    rng = np.random.default_rng(11)
    base = s.trial.astype(complex)
    for i in (0, 3, n - 1):
        for direction in (rng.standard_normal(M), 1j * rng.standard_normal(M)):
            h = 1e-3
            tp, tm = base.copy(), base.copy()
            tp[:, i] += h * direction
            tm[:, i] -= h * direction
            fd = (_dropped(lbar, fac, tp) - _dropped(lbar, fac, tm)) / (2 * h)
            want = g[i] @ direction
            assert abs(fd - want) <= 1e-9 * max(1.0, np.abs(g[i]).sum()), (i, fd, want)
    # the gradient of the dropped part is small but not zero at eps = 1e-3
    assert 0 < np.abs(g).max() < 1e-1


def test_dropped_energy_first_order_prediction(chain_case):
    """sum_i Re(g_i . (theta_i - psi_i)) predicts the change of the dropped
    energy from the trial to a nearby walker, with a remainder quadratic in
    the distance (halving the noise quarters it)."""
    s, lbar, fac, g = chain_case
    M, n = s.trial.shape
    d0 = _dropped(lbar, fac, s.trial.astype(complex)).real
    rem = []
    for sigma in (1e-3, 5e-4):
        rng = np.random.default_rng(5)
        w = synth.noisy_walkers(s.trial, 1, sigma, rng)[0]
        th = E.green_theta(s.trial, w)[0]
        first = sum(np.real(g[i] @ (th[:, i] - s.trial[:, i])) for i in range(n))
        change = _dropped(lbar, fac, th).real - d0
        assert abs(first) > 5 * abs(change - first)
        rem.append(abs(change - first))
    assert 0.15 < rem[1] / rem[0] < 0.35


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
