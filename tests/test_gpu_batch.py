"""Several systems in one persistent launch (lo_batch_*), FP32 exchange.

* With the chunk lengths of the single-system call, every work item and every
  partial sum is the same as in local_energy_full(precision=LO_FP32), so the
  batch must reproduce it bit for bit, for plans whose largest orbital-block
  count is 6, 4, 3 and 1.
* With the planner's default chunks, each system must lie within the FP32
  rounding bound of the CPU FP64 reference (the bound of the reduced-precision
  tests) and the Coulomb part within 1e-9.
* A captured graph of several evaluations, replayed with eager work and
  synchronisations in between, must give the eager result bit for bit after
  every replay.
* Systems given their trial and walkers: every evaluation forms theta by
  green_theta first; a graph replay from the walkers must reproduce
  green_theta + local_energy_full(LO_FP32) per system bit for bit.
Shapes: uneven M, n (one to six 16-orbital blocks), n_chol and walkers.
"""
import numpy as np
import pytest

from oracle import energy as E
from paper_2202_00832_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2202_00832_amd import autotune, lofqmc  # noqa: E402

U = 2.0 ** -24
SHAPES = [(37, 5, 11, 3), (131, 81, 23, 6), (70, 33, 30, 9), (20, 1, 7, 2), (100, 60, 40, 5), (96, 70, 17, 4),
          (50, 24, 13, 3)]


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


@pytest.fixture(scope="module")
def systems():
    out = []
    for k, (M, n, X, nw) in enumerate(SHAPES):
        rng = np.random.default_rng(100 + k)
        chol = synth.random_symmetric_cholesky(M, X, rng)
        trial = np.linalg.qr(rng.standard_normal((M, n)))[0]
        walkers = synth.noisy_walkers(trial, nw, 0.3, rng)
        lbar_ref = E.half_rotate(chol, trial)
        thetas, _, info = E.green_theta_batch(trial, walkers)
        assert (info == 0).all()
        out.append({"M": M, "n": n, "X": X, "nw": nw, "lbar_ref": lbar_ref, "thetas": thetas,
                    "lbar": dev(lbar_ref.transpose(0, 2, 1)), "theta": dev(thetas), "trial": trial,
                    "walkers": walkers})
    return out


def _desc(systems):
    return [{"lbar": s["lbar"], "theta": s["theta"]} for s in systems]


def test_green_theta_wide_orbital_blocks(ctx, systems):
    """green_theta for 65-96 orbitals (five and six 16-orbital blocks)."""
    for k, (M, n, X, nw) in enumerate(SHAPES):
        if n <= 64:
            continue
        rng = np.random.default_rng(100 + k)
        synth.random_symmetric_cholesky(M, X, rng)
        trial = np.linalg.qr(rng.standard_normal((M, n)))[0]
        walkers = synth.noisy_walkers(trial, nw, 0.3, rng)
        theta, logov, info = ctx.green_theta(dev(trial), dev(walkers))
        ref = systems[k]["thetas"]
        assert (host(info) == 0).all()
        assert np.abs(host(theta) - ref).max() <= 1e-12 * np.abs(ref).max()
        ld_ref = np.array([E.green_theta(trial, w)[1] for w in walkers])
        lg = host(logov)
        assert np.abs(lg.real - ld_ref.real).max() <= 1e-10
        assert np.abs(np.angle(np.exp(1j * (lg.imag - ld_ref.imag)))).max() <= 1e-10


# subsets whose largest orbital-block count is 6, 5, 4, 3, 2 and 1: the
# persistent kernel is instantiated for the largest block count of the plan
@pytest.mark.parametrize("pick", [None, [0, 2, 5], [0, 2, 3, 4], [0, 2, 3], [6, 0], [3]])
def test_batch_matches_single_system_bitwise(ctx, systems, pick):
    systems = systems if pick is None else [systems[k] for k in pick]
    print("batch bitwise: n = %s" % [s["n"] for s in systems], flush=True)
    singles = [host(ctx.local_energy_full(s["lbar"], s["theta"], precision=lofqmc.LO_FP32)) for s in systems]
    # chunk of the single-system call: ceil(X / nchunk) with the same chunk count
    chunk = []
    for s in systems:
        nw, X = s["nw"], s["X"]
        ngrp, c = (nw + 3) // 4, 1
        while c < 4096 and ngrp * c < 256 and c < X:
            c *= 2
        chunk.append((X + c - 1) // c)
    b = lofqmc.Batch(ctx, _desc(systems), chunk)
    b.execute()
    for s, got, ref in zip(systems, b.energies, singles):
        assert np.array_equal(host(got).view(np.float64), ref.view(np.float64)), (s["M"], s["n"])
    b.close()


def test_batch_default_chunks_within_fp32_bound(ctx, systems):
    b = lofqmc.Batch(ctx, _desc(systems))
    info = b.info()
    assert info["items"] > 0 and (info["chunk"] >= 1).all()
    b.execute()
    for s, got in zip(systems, b.energies):
        e = host(got)
        ref = np.asarray(E.e2_cholesky_batch(s["lbar_ref"], s["thetas"]))
        assert np.abs(e[:, 0] - ref[:, 0]).max() <= 1e-9
        eps = (2.0 + s["M"]) * U
        for w in range(s["nw"]):
            th = s["thetas"][w]
            A = np.einsum("gir,rj->gij", np.abs(s["lbar_ref"]), np.abs(th.real) + np.abs(th.imag))
            bound = (2 * eps + eps * eps) * np.einsum("gij,gji->", A, A)
            assert abs(e[w, 1] - ref[w, 1]) <= bound + 1e-9
    b.close()


def test_graph_replays_match_eager(ctx, systems):
    b = lofqmc.Batch(ctx, _desc(systems))
    b.execute()
    eager = [host(e).copy() for e in b.energies]
    b.capture(3)
    for rep in range(4):
        for e in b.energies:
            e.zero_()
        # eager work of the program between replays
        ctx.local_energy_full(systems[0]["lbar"], systems[0]["theta"], precision=lofqmc.LO_FP32)
        torch.cuda.synchronize()
        b.replay()
        for got, ref in zip(b.energies, eager):
            assert np.array_equal(host(got).view(np.float64), ref.view(np.float64)), rep
    b.close()


def _single_chunks(systems):
    chunk = []
    for s in systems:
        nw, X = s["nw"], s["X"]
        ngrp, c = (nw + 3) // 4, 1
        while c < 4096 and ngrp * c < 256 and c < X:
            c *= 2
        chunk.append((X + c - 1) // c)
    return chunk


def test_graph_from_walkers_matches_per_system_calls(ctx, systems):
    desc = []
    for s in systems:
        desc.append({"lbar": s["lbar"], "theta": torch.zeros_like(s["theta"]),
                     "info": torch.full((s["nw"],), -7, dtype=torch.int32, device="cuda"),
                     "trial": dev(s["trial"]), "phi": dev(s["walkers"])})
    expect = []
    for s, d in zip(systems, desc):
        th, _, inf = ctx.green_theta(d["trial"], d["phi"])
        expect.append((host(th), host(ctx.local_energy_full(s["lbar"], th, inf, precision=lofqmc.LO_FP32))))
    b = lofqmc.Batch(ctx, desc, _single_chunks(systems))
    b.capture(2)
    for rep in range(3):
        for d, e in zip(desc, b.energies):
            d["theta"].zero_()
            d["info"].fill_(-7)
            e.zero_()
        ctx.local_energy_full(systems[0]["lbar"], systems[0]["theta"], precision=lofqmc.LO_FP32)
        torch.cuda.synchronize()
        b.replay()
        for s, d, got, (th_ref, e_ref) in zip(systems, desc, b.energies, expect):
            assert (host(d["info"]) == 0).all()
            assert np.array_equal(host(d["theta"]).view(np.float64), th_ref.view(np.float64)), (s["M"], s["n"])
            assert np.array_equal(host(got).view(np.float64), e_ref.view(np.float64)), (rep, s["M"], s["n"])
    # and the Coulomb part against the CPU reference
    for s, got in zip(systems, b.energies):
        ref = np.asarray(E.e2_cholesky_batch(s["lbar_ref"], s["thetas"]))
        assert np.abs(host(got)[:, 0] - ref[:, 0]).max() <= 1e-9
    b.close()


def test_autotuner_returns_a_valid_table(ctx, systems):
    res = autotune.tune(ctx, _desc(systems), factors=(0.5, 2.0), reps=1)
    assert res["ms"] <= res["default_ms"]
    chunk = autotune.chunks_from_table(_desc(systems), res["table"])
    assert all(1 <= c <= s["X"] for c, s in zip(chunk, systems))
    b = lofqmc.Batch(ctx, _desc(systems), chunk)
    b.execute()
    for s, got in zip(systems, b.energies):
        ref = np.asarray(E.e2_cholesky_batch(s["lbar_ref"], s["thetas"]))
        assert np.abs(host(got)[:, 0] - ref[:, 0]).max() <= 1e-9
    b.close()
