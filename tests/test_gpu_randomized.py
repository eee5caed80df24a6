"""GPU parity of the randomized-SVD LO set-up (build_lo_factors_randomized)
against the CPU reference's randomized subspace iteration with the same test
matrix, and against the exact decomposition: equal ranks, LO energies within
1e-9 Ha per walker, and the error return for a sketch that is too narrow."""
import numpy as np
import pytest

from oracle import energy as E
from paper_2202_00832_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2202_00832_amd import lofqmc  # noqa: E402

TOL_E = 1e-9


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


@pytest.mark.parametrize("eps,width", [(1e-3, 12), (1e-4, 16), (1e-5, 24)])
def test_randomized_factors_match_reference(ctx, eps, width):
    s = synth.make_system(synth.CHAIN_SMALL)
    M, n = s.trial.shape
    print("randomized eps=%g sketch=%d" % (eps, width), flush=True)
    omega = np.random.default_rng(7).standard_normal((M, width))
    lbar_ref = E.half_rotate(s.chol, s.trial)
    ref = E.lo_truncate(E.lo_decompose_randomized(lbar_ref, omega, 2), eps)
    exact = E.lo_compress(lbar_ref, eps, pairs="upper")
    lbar = ctx.build_half_rotated_chol(dev(s.chol), dev(s.trial))
    f = ctx.build_lo_factors_randomized(lbar, eps, dev(omega), power_iters=2)
    assert np.array_equal(f.info()["ranks"], E.lo_ranks(ref, n))
    assert np.array_equal(f.info()["ranks"], E.lo_ranks(exact, n))
    theta, _, info = ctx.green_theta(dev(s.trial), dev(s.walkers))
    got = host(ctx.local_energy_lo(f, theta, info))
    thetas, _, _ = E.green_theta_batch(s.trial, s.walkers)
    want = np.array([E.e2_lo(ref, t) for t in thetas])
    assert np.abs(got - want).max() <= TOL_E
    f_exact = ctx.build_lo_factors(lbar, eps)
    assert np.abs(got - host(ctx.local_energy_lo(f_exact, theta, info))).max() <= TOL_E
    f.close()
    f_exact.close()


def test_randomized_mid_size_against_exact_gpu_factors(ctx):
    """A random Cholesky set (slow singular-value decay) at M = 120: with a
    sketch wide enough for the kept ranks the energies match the exact set-up."""
    rng = np.random.default_rng(11)
    M, n, X, nw = 120, 12, 30, 40
    chol = synth.random_symmetric_cholesky(M, X, rng)
    trial = np.linalg.qr(rng.standard_normal((M, n)))[0]
    walkers = synth.noisy_walkers(trial, nw, 0.3, rng)
    lbar = ctx.build_half_rotated_chol(dev(chol), dev(trial))
    eps = 2e-3
    f_exact = ctx.build_lo_factors(lbar, eps)
    kmax = int(f_exact.info()["ranks"].max())
    omega = rng.standard_normal((M, min(M, 64, kmax + 16)))
    f = ctx.build_lo_factors_randomized(lbar, eps, dev(omega), power_iters=3)
    assert np.array_equal(f.info()["ranks"], f_exact.info()["ranks"])
    theta, _, info = ctx.green_theta(dev(trial), dev(walkers))
    a = host(ctx.local_energy_lo(f, theta, info))
    b = host(ctx.local_energy_lo(f_exact, theta, info))
    assert np.abs(a - b).max() <= 1e-8 * max(1.0, np.abs(b).max())
    f.close()
    f_exact.close()


def test_too_narrow_sketch_is_reported(ctx):
    s = synth.make_system(synth.CHAIN_SMALL)
    M = s.trial.shape[0]
    lbar = ctx.build_half_rotated_chol(dev(s.chol), dev(s.trial))
    omega = dev(np.random.default_rng(5).standard_normal((M, 2)))
    with pytest.raises(lofqmc.LoError) as e:
        ctx.build_lo_factors_randomized(lbar, 1e-5, omega)
    assert e.value.code == lofqmc.LO_EUNSUPPORTED
