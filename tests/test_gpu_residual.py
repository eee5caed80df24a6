"""Learned LO residual on the GPU: features, forward, backward, Adam, BF16
inference and training, against the CPU FP64 reference (oracle/residual.py).

Tolerances follow from FP32 arithmetic (unit roundoff u = 2^-24):
* forward: first-order error propagation through the two tanh layers, with
  dot products of k terms carrying at most (k + 2) u sum |a b|;
* gradients: each entry is a sum over N rows of FP32 products, accumulated in
  FP32 within row splits of 4096 rows and in FP64 across them, so its error is
  at most (4096 + 64) u times the sum of the absolute values of its terms plus
  the propagated activation error (bounded by the same factor);
* BF16 inference: activations and W2 rounded to BF16 (unit roundoff 2^-8 each).
"""
import numpy as np
import pytest

from oracle import energy as E
from oracle import residual as R
from paper_2202_00832_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2202_00832_amd import lofqmc  # noqa: E402
from paper_2202_00832_amd import residual as RES  # noqa: E402

U = 2.0 ** -24


@pytest.fixture(scope="module")
def ctx():
    c = lofqmc.Context()
    yield c
    c.close()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def rand_problem(seed, nw=37, n=9):
    rng = np.random.default_rng(seed)
    x = np.stack([rng.integers(1, 12, (nw, n)).astype(float), rng.uniform(0, 2e-3, (nw, n)),
                  rng.uniform(0.5, 2.0, (nw, n))], axis=-1).astype(np.float32)
    p = R.init_params(x.astype(np.float64), seed=seed)
    q = R.unpack(p)
    q["b1"][...] = rng.normal(0, 0.2, R.WIDTH)
    q["b2"][...] = rng.normal(0, 0.2, R.WIDTH)
    q["b3"][...] = 0.05
    p = R.pack(q).astype(np.float32).astype(np.float64)   # exactly representable in FP32
    t = rng.normal(0, 1, nw)
    return x, p, t


def forward_bound(p, x):
    """Per-walker bound on |pred_fp32 - pred_exact| (first order)."""
    q = R.unpack(p)
    nw, n, _ = x.shape
    xr = x.reshape(-1, 3).astype(np.float64)
    z = (xr - q["shift"]) * q["scale"]
    a1 = np.abs(z) @ np.abs(q["W1"]).T + np.abs(q["b1"])
    e_h1 = 8 * U * (a1 + 1.0)                      # input scaling, 3-term dot, tanh
    h1 = np.tanh(z @ q["W1"].T + q["b1"])
    a2 = np.abs(h1) @ np.abs(q["W2"]).T + np.abs(q["b2"])
    e_h2 = e_h1 @ np.abs(q["W2"]).T + (R.WIDTH + 4) * U * a2 + 4 * U
    h2 = np.tanh(h1 @ q["W2"].T + q["b2"])
    e_y = e_h2 @ np.abs(q["w3"]) + (R.WIDTH + 4) * U * (np.abs(h2) @ np.abs(q["w3"]) + abs(q["b3"][0]))
    return e_y.reshape(nw, n).sum(axis=1) + 1e-12


def test_features_match_reference(ctx):
    s = synth.make_system(synth.CHAIN_SMALL)
    lbar = ctx.build_half_rotated_chol(dev(s.chol), dev(s.trial))
    f = ctx.build_lo_factors(lbar, 1e-3)
    theta, _, info = ctx.green_theta(dev(s.trial), dev(s.walkers))
    x = host(ctx.residual_features(f, theta))
    ranks, disc = f.info()["ranks"], f.discarded()
    # discarded mass against the oracle's own SVD (ranks equal, masses to rounding)
    ref_f = E.lo_compress(E.half_rotate(s.chol, s.trial), 1e-3, pairs="upper")
    assert np.array_equal(ranks, E.lo_ranks(ref_f, s.config.n))
    for (i, j), (Ub, _, sv) in ref_f.items():
        assert abs(disc[i, j] - sv[Ub.shape[1]:].sum()) <= 1e-12 * max(1.0, sv[0])
    thetas, _, _ = E.green_theta_batch(s.trial, s.walkers)
    for w in range(s.walkers.shape[0]):
        ref = R.features(ranks, disc, thetas[w])
        assert np.allclose(x[w], ref, rtol=4 * U, atol=1e-30)


@pytest.mark.parametrize("seed,nw,n", [(0, 37, 9), (1, 5, 64), (2, 130, 1)])
def test_forward_fp32_matches_reference(ctx, seed, nw, n):
    x, p, _ = rand_problem(seed, nw, n)
    got = host(ctx.residual_predict(dev(p.astype(np.float32)), dev(x), lofqmc.LO_FP32))
    ref = R.walker_predictions(p, x.astype(np.float64))
    assert np.all(np.abs(got - ref) <= forward_bound(p, x)), np.abs(got - ref).max()


def test_bf16_inference_within_rounding_bound(ctx):
    x, p, _ = rand_problem(3, 64, 12)
    got = host(ctx.residual_predict(dev(p.astype(np.float32)), dev(x), lofqmc.LO_BF16))
    ref = R.walker_predictions(p, x.astype(np.float64))
    q = R.unpack(p)
    z = (x.reshape(-1, 3).astype(np.float64) - q["shift"]) * q["scale"]
    h1 = np.tanh(z @ q["W1"].T + q["b1"])
    # BF16 rounding of h1 and W2 (2^-8 relative each, products exact, FP32 sums)
    e_pre = (2 * 2.0 ** -8 + 2.0 ** -16 + (R.WIDTH + 4) * U) * (np.abs(h1) @ np.abs(q["W2"]).T) + 8 * U
    bound = (e_pre @ np.abs(q["w3"]) + 200 * U * (np.abs(q["w3"]).sum() + 1)).reshape(64, 12).sum(axis=1)
    err = np.abs(got - ref)
    assert np.all(err <= bound), (err.max(), bound.min())
    assert err.max() > 0.0   # it really ran in reduced precision


def test_gradient_and_loss_match_reference(ctx):
    x, p, t = rand_problem(4, 300, 20)
    npar = ctx.residual_nparam()
    assert npar == R.NPARAM
    grad = torch.zeros(npar, dtype=torch.float32, device="cuda")
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    pred = torch.zeros(300, dtype=torch.float64, device="cuda")
    pd = dev(p.astype(np.float32))
    ctx.residual_train_step(pd, None, None, 0, 0.0, dev(x), dev(t), grad=grad, loss=loss, pred=pred)
    g = host(grad).astype(np.float64)
    l_ref, g_ref = R.loss_and_grad(p, x.astype(np.float64), t)
    assert abs(host(loss)[0] - l_ref) <= 1e-4 * l_ref
    # scale of each gradient entry: the same sums over rows with absolute values
    q = R.unpack(p)
    nw, n, _ = x.shape
    _, (z, h1, h2) = R.forward(p, x.reshape(-1, 3).astype(np.float64))
    r = R.walker_predictions(p, x.astype(np.float64)) - t
    grow = np.abs(np.repeat(2.0 * r / nw, n))
    dz2 = np.outer(grow, np.abs(q["w3"])) * (1.0 - h2 * h2)
    dz1 = (dz2 @ np.abs(q["W2"])) * (1.0 - h1 * h1)
    S = {"W2": dz2.T @ np.abs(h1), "b2": dz2.sum(0), "w3": np.abs(h2).T @ grow, "b3": np.array([grow.sum()]),
         "W1": dz1.T @ np.abs(z), "b1": dz1.sum(0)}
    gq, gr = R.unpack(g), R.unpack(g_ref)
    fac = (4096 + 64) * U * 4
    for name, scale in S.items():
        assert np.all(np.abs(gq[name] - gr[name]) <= fac * scale + 1e-12), name
    assert not gq["shift"].any() and not gq["scale"].any()


def test_adam_update_matches_reference(ctx):
    x, p, t = rand_problem(5, 64, 7)
    npar = ctx.residual_nparam()
    pd = dev(p.astype(np.float32))
    m = torch.zeros(npar, dtype=torch.float32, device="cuda")
    v = torch.zeros(npar, dtype=torch.float32, device="cuda")
    grad = torch.zeros(npar, dtype=torch.float32, device="cuda")
    for step in (1, 2, 3):
        p_before = host(pd).astype(np.float64)
        m_before, v_before = host(m).astype(np.float64), host(v).astype(np.float64)
        ctx.residual_train_step(pd, m, v, step, 1e-2, dev(x), dev(t), grad=grad)
        g = host(grad).astype(np.float64)
        p_ref, m_ref, v_ref = R.adam_step(p_before, g, m_before, v_before, step, 1e-2)
        # FP32 moments: each is a two-term sum, error <= 4 u (|b m| + |a g|)
        dm = 4 * U * (0.9 * np.abs(m_before) + 0.1 * np.abs(g)) + 1e-38
        dv = 4 * U * (0.999 * v_before + 0.001 * g * g) + 1e-38
        assert np.all(np.abs(host(m) - m_ref) <= dm)
        assert np.all(np.abs(host(v) - v_ref) <= dv)
        # update lr * mh / (sqrt(vh) + eps): propagate dm, dv, plus rounding of the
        # quotient and of p itself
        c1, c2 = 1 - 0.9 ** step, 1 - 0.999 ** step
        mh, vh = np.abs(m_ref) / c1, v_ref / c2
        den = np.sqrt(vh) + 1e-8
        dq = (dm / c1) / den + (mh / den) * (dv / c2) / (2 * np.maximum(vh, 1e-300)) * np.sqrt(vh) / den
        bound = 1e-2 * (dq + 8 * U * mh / den) + 4 * U * np.abs(p_ref) + 1e-12
        q = R.unpack(np.ones(R.NPARAM))
        q["shift"][...] = 0
        q["scale"][...] = 0
        trained = R.pack(q) > 0
        assert np.all((np.abs(host(pd) - p_ref) <= bound)[trained])
        assert np.array_equal(host(pd)[~trained], p_before[~trained].astype(np.float32))


def _chain_pairs(ctx, nw, eps, seed):
    """(features, target in mHa, E_full, E_LO) for noisy walkers of the 48-site chain."""
    s = synth.make_system(synth.CHAIN_SMALL, nw=1)
    rng = np.random.default_rng(seed)
    walkers = synth.noisy_walkers(s.trial, nw, 0.1, rng)
    lbar = ctx.build_half_rotated_chol(dev(s.chol), dev(s.trial))
    f = ctx.build_lo_factors(lbar, eps)
    theta, _, info = ctx.green_theta(dev(s.trial), dev(walkers))
    ef = ctx.local_energy_full(lbar, theta, info).sum(dim=1)
    el = ctx.local_energy_lo(f, theta, info).sum(dim=1)
    x = ctx.residual_features(f, theta)
    target = ((ef - el).real * RES.MHA).contiguous()
    return s, f, lbar, theta, info, x, target


def test_training_on_method_pairs_reduces_heldout_error(ctx):
    """Trained on 2000 walkers, the network's correction lowers the held-out RMS
    of E_full - E_LO (mostly by removing its mean; the features hold little
    walker-specific information)."""
    s, f, lbar, theta, info, x, target = _chain_pairs(ctx, 3000, 1e-3, seed=5)
    xh = host(x)
    model = RES.ResidualModel(ctx, RES.init_params(xh[:2000], ctx.residual_nparam(), seed=0))
    losses = model.train(x[:2000].contiguous(), target[:2000].contiguous(), steps=1500, lr=1e-3, batch=256)
    # the loss is on standardised targets: it starts near 1 (their variance)
    # and falls by the part of the walker-to-walker variation the features explain
    assert np.mean(losses[-100:]) < np.mean(losses[:10])
    te = slice(2000, 3000)
    y = host(target)[te]
    pred = host(model.predict_mha(x[te].contiguous(), lofqmc.LO_BF16))
    before, after = np.sqrt(np.mean(y ** 2)), np.sqrt(np.mean((y - pred) ** 2))
    print("held-out RMS of E_full - E_LO: %.4f mHa plain, %.4f mHa corrected" % (before, after))
    assert after < 0.6 * before
    # the FP32 and BF16 predictions of the trained network agree closely
    p32 = host(model.predict_mha(x[te].contiguous(), lofqmc.LO_FP32))
    assert np.abs(p32 - pred).max() < 0.05 * np.abs(y).max()


def test_monitor_falls_back_for_a_corrupted_network(ctx):
    s, f, lbar, theta, info, x, target = _chain_pairs(ctx, 256, 1e-3, seed=6)
    xh = host(x)
    p = RES.init_params(xh, ctx.residual_nparam(), seed=1)
    corrupt = p.copy()
    corrupt[128 * 3 + 128 + 128 * 128 + 128:128 * 3 + 128 + 128 * 128 + 256] *= 1e4   # w3
    model = RES.ResidualModel(ctx, corrupt)
    est = RES.CorrectedLO(ctx, f, lbar, model, bound_mha=0.2, check_every=10, check_walkers=64)
    e = est(theta, info)
    assert est.mode in ("lo", "full") and est.last_check["max_err_corrected_mHa"] > 0.2
    e_lo = ctx.local_energy_lo(f, theta, info).sum(dim=1)
    e_full = ctx.local_energy_full(lbar, theta, info).sum(dim=1)
    expect = e_lo if est.mode == "lo" else e_full
    assert torch.equal(e, expect)
