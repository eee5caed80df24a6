"""Learned correction of the LO energy, with a periodic check against the full route.

Not part of the paper's method.  The LO route drops the part of the two-body
energy carried by the discarded singular values of the pair blocks.  A small
network f (4 -> 128 -> 128 -> 1, see include/lofqmc.h) predicts that part per
walker from per-orbital features, sum_i f(x_i), in mHa.  It is trained on the
GPU by the library's own forward and backward kernels on pairs (E_full, E_LO)
that the two routes produce for the same walkers, and it is applied only
while a periodic full evaluation of a walker sample confirms that the
corrected energies stay within a stated bound; otherwise the energies fall
back to plain LO (or to the full route when plain LO also misses its gate).

Host code here sequences library calls and compares a handful of numbers;
the network's forward, backward and update, the training targets and the
corrected energies are the library's kernels (lo_residual_*).  torch only
holds the device arrays and gathers minibatch rows; the mean and standard
deviation of the training targets, which set the standardisation, are taken
on the host.
"""
from __future__ import annotations

import numpy as np

from . import lofqmc

MHA = 1e3   # the network works in mHa


def init_params(x_host: np.ndarray, nparam: int, seed: int = 0) -> np.ndarray:
    """Glorot-uniform weights, zero biases, and the input standardisation
    (shift = mean, scale = 1 / standard deviation of the training features)."""
    rng = np.random.default_rng(seed)
    F = lofqmc.RESIDUAL_NFEAT
    flat = x_host.reshape(-1, F).astype(np.float64)
    sd = flat.std(axis=0)
    W = 128
    parts = [rng.uniform(-1, 1, W * F) * np.sqrt(6.0 / (W + F)), np.zeros(W),
             rng.uniform(-1, 1, W * W) * np.sqrt(6.0 / (2 * W)), np.zeros(W),
             rng.uniform(-1, 1, W) * np.sqrt(6.0 / (W + 1)), np.zeros(1),
             flat.mean(axis=0), np.where(sd > 0, 1.0 / np.where(sd > 0, sd, 1.0), 1.0)]
    p = np.concatenate(parts).astype(np.float32)
    assert p.size == nparam
    return p


class ResidualModel:
    """Parameters and Adam state of the network, on the device.

    The network is trained on standardised targets (t - mean) / scale, with the
    mean and scale of the training targets in mHa; lo_residual_apply maps its
    predictions back, so the model works in mHa at any size of the dropped
    energy.
    """

    def __init__(self, ctx: lofqmc.Context, params_host: np.ndarray):
        import torch
        self.ctx = ctx
        self.params = torch.from_numpy(np.ascontiguousarray(params_host, dtype=np.float32)).cuda()
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.t = 0
        self.t_mean = 0.0
        self.t_scale = 1.0

    def train(self, x, e_exact, e_lo, steps: int, lr: float = 1e-3, batch: int = 256, seed: int = 0):
        """Adam on minibatches of walkers; x [nw][n][4] features, e_exact and
        e_lo [nw][2] energies of the same walkers.  Returns the loss of every
        step (mean squared error of the standardised target)."""
        import torch
        nw = x.shape[0]
        if self.t == 0:
            th = self.ctx.residual_target(e_exact, e_lo).cpu().numpy()
            self.t_mean = float(th.mean())
            self.t_scale = float(th.std()) if th.std() > 0 else 1.0
        tstd = self.ctx.residual_target(e_exact, e_lo, self.t_mean, self.t_scale)
        g = torch.Generator(device="cpu").manual_seed(seed)
        loss = torch.zeros(1, dtype=torch.float64, device=x.device)
        losses = torch.zeros(steps, dtype=torch.float64, device=x.device)
        for k in range(steps):
            idx = torch.randperm(nw, generator=g)[:min(batch, nw)].to(x.device)
            xb = x.index_select(0, idx).contiguous()
            tb = tstd.index_select(0, idx).contiguous()
            self.t += 1
            self.ctx.residual_train_step(self.params, self.m, self.v, self.t, lr, xb, tb, loss=loss)
            losses[k:k + 1].copy_(loss)
        return losses.cpu().numpy()

    def predict(self, x, precision=lofqmc.LO_BF16):
        """Network output in standardised units (double [nw], device)."""
        return self.ctx.residual_predict(self.params, x, precision)

    def corrected(self, e_lo, x, precision=lofqmc.LO_BF16):
        """E_J + E_K of e_lo plus the predicted dropped energy, complex [nw]."""
        return self.ctx.residual_apply(e_lo, self.predict(x, precision), self.t_scale, self.t_mean)


class CorrectedLO:
    """E = E_LO + sum_i f(x_i), checked every `check_every` evaluations against
    an exact route on `check_walkers` sampled walkers.

    The exact route is the Cholesky route with `lbar`, or any callable
    `reference(theta, info) -> energies [nw][2]`, e.g. the half-rotated ERI
    route.  After a check, `mode` is "corrected" if the largest
    |Re(E_exact - E)| of the sample is at most `bound_mha`; otherwise "lo" if
    plain LO's largest error is at most `lo_gate_mha`, else "full".  The
    returned energies follow the mode (the exact route is then evaluated for
    every walker).
    """

    def __init__(self, ctx, factors, lbar, model: ResidualModel, bound_mha=0.2, lo_gate_mha=1.0, check_every=10,
                 check_walkers=64, seed=0, reference=None):
        self.ctx, self.factors, self.lbar, self.model = ctx, factors, lbar, model
        self.reference = reference if reference is not None else \
            (lambda theta, info: ctx.local_energy_full(lbar, theta, info))
        self.bound, self.lo_gate = bound_mha, lo_gate_mha
        self.check_every, self.check_walkers = check_every, check_walkers
        self.rng = np.random.default_rng(seed)
        self.calls = 0
        self.mode = "corrected"
        self.last_check = None

    def check(self, theta, info, e_lo, pred):
        import torch
        nw = theta.shape[0]
        k = min(self.check_walkers, nw)
        idx = torch.from_numpy(np.sort(self.rng.choice(nw, k, replace=False))).to(theta.device)
        th = theta.index_select(0, idx).contiguous()
        inf = info.index_select(0, idx).contiguous() if info is not None else None
        el = e_lo.index_select(0, idx).contiguous()
        ef = self.ctx.residual_apply(self.reference(th, inf)).real.cpu().numpy()
        ec = self.ctx.residual_apply(el, pred.index_select(0, idx).contiguous(), self.model.t_scale,
                                     self.model.t_mean).real.cpu().numpy()
        ep = self.ctx.residual_apply(el).real.cpu().numpy()
        err_c = float(np.max(np.abs(ef - ec)) * MHA)
        err_lo = float(np.max(np.abs(ef - ep)) * MHA)
        if err_c <= self.bound:
            self.mode = "corrected"
        elif err_lo <= self.lo_gate:
            self.mode = "lo"
        else:
            self.mode = "full"
        self.last_check = {"max_err_corrected_mHa": err_c, "max_err_lo_mHa": err_lo, "mode": self.mode}
        return self.last_check

    def __call__(self, theta, info=None):
        """Energies [nw] (complex128: E_J + E_K, plus the correction on the real part)."""
        e_lo = self.ctx.local_energy_lo(self.factors, theta, info)
        x = self.ctx.residual_features(self.factors, theta)
        pred = self.model.predict(x)
        if self.calls % self.check_every == 0:
            self.check(theta, info, e_lo, pred)
        self.calls += 1
        if self.mode == "corrected":
            return self.ctx.residual_apply(e_lo, pred, self.model.t_scale, self.model.t_mean)
        if self.mode == "lo":
            return self.ctx.residual_apply(e_lo)
        return self.ctx.residual_apply(self.reference(theta, info))
