"""GPU parity at the benchmark size, in the benchmark's launch configuration.

400-site chain, 60 orbitals per spin, 799 Cholesky vectors, 512 walkers: the
whole batch is evaluated on the GPU exactly as bench.py does (walker-major theta
for the full route, transposed theta [w][j][r] for the LO route at the headline
threshold; orbital-major at eps = 1e-5); the CPU reference
recomputes a sample of walkers one by one from the same inputs (its own
half-rotation, overlap inverse and SVD factors).  Properties that hold at any
size are checked on every walker.
"""
import numpy as np
import pytest

from oracle import energy as E
from paper_2202_00832_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2202_00832_amd import lofqmc  # noqa: E402

SAMPLE = [0, 1, 173, 300, 511]
EPS = 1e-5
EPS_TIGHT = 1e-7


@pytest.fixture(scope="module")
def run():
    cfg = synth.CHAIN_POLYACENE
    s = synth.make_system(cfg)
    print("full-size: M=%d n=%d X=%d walkers=%d" % (cfg.M, cfg.n, s.n_chol, cfg.nw), flush=True)
    ctx = lofqmc.Context()
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()  # noqa: E731
    trial, phi = d(s.trial), d(s.walkers)
    lbar = ctx.build_half_rotated_chol(d(s.chol), trial)
    theta, logov, info = ctx.green_theta(trial, phi)
    e_full = ctx.local_energy_full(lbar, theta, info)
    fac = ctx.build_lo_factors(lbar, EPS)
    theta_om, _, info_om = ctx.green_theta(trial, phi, orbital_major=True)
    e_lo = ctx.local_energy_lo(fac, theta_om, info_om, orbital_major=True)
    # the headline threshold: orbitals touch more than 192 factor rows, so
    # pass 1 cuts each into two tiles; transposed theta as in the bench
    fac7 = ctx.build_lo_factors(lbar, EPS_TIGHT)
    theta_tr, _, info_tr = ctx.green_theta(trial, phi, transposed=True)
    e_lo7 = ctx.local_energy_lo(fac7, theta_tr, info_tr, transposed=True)
    e_lo7_wm = ctx.local_energy_lo(fac7, theta, info)
    torch.cuda.synchronize()
    out = dict(system=s, theta=theta.cpu().numpy(), logov=logov.cpu().numpy(), info=info.cpu().numpy(),
               e_full=e_full.cpu().numpy(), e_lo=e_lo.cpu().numpy(), ranks=fac.info()["ranks"],
               theta_om=theta_om.cpu().numpy(), e_lo7=e_lo7.cpu().numpy(), ranks7=fac7.info()["ranks"],
               theta_tr=theta_tr.cpu().numpy(), info_tr=info_tr.cpu().numpy(), e_lo7_wm=e_lo7_wm.cpu().numpy())
    fac.close()
    fac7.close()
    ctx.close()
    return out


@pytest.fixture(scope="module")
def ref(run):
    s = run["system"]
    lbar = E.half_rotate(s.chol, s.trial)
    thetas, logdets = [], []
    for w in SAMPLE:
        t, ld, info = E.green_theta(s.trial, s.walkers[w])
        assert info == 0
        thetas.append(t)
        logdets.append(ld)
    return dict(lbar=lbar, thetas=thetas, logdets=logdets)


def test_theta_sampled_walkers(run, ref):
    assert (run["info"] == 0).all() and (run["info_tr"] == 0).all()
    for k, w in enumerate(SAMPLE):
        t = ref["thetas"][k]
        scale = np.abs(t).max()
        assert np.abs(run["theta"][w] - t).max() <= 1e-12 * scale
        assert np.abs(run["theta_om"][:, :, w].T - t).max() <= 1e-12 * scale
        assert np.abs(run["theta_tr"][w].T - t).max() <= 1e-12 * scale
        assert abs(run["logov"][w].real - ref["logdets"][k].real) <= 1e-10
        assert abs(np.angle(np.exp(1j * (run["logov"][w].imag - ref["logdets"][k].imag)))) <= 1e-10


def test_full_energy_sampled_walkers(run, ref):
    for k, w in enumerate(SAMPLE):
        e = np.array(E.e2_cholesky(ref["lbar"], ref["thetas"][k]))
        assert np.abs(run["e_full"][w] - e).max() <= 1e-9, (w, run["e_full"][w], e)


@pytest.fixture(scope="module")
def ref_svd(ref, run):
    print("reference SVD of the 1830 pair blocks", flush=True)
    return E.lo_decompose(ref["lbar"], pairs="upper")


@pytest.fixture(scope="module")
def ref_lo(ref_svd):
    return E.lo_truncate(ref_svd, EPS)


def _check_lo(run_ranks, run_e, ref_f, ref, eps):
    ranks = E.lo_ranks(ref_f, run_ranks.shape[0])
    # integer decisions taken in FP64 on both sides; a mismatch is only allowed
    # for a singular value within rounding of the threshold
    for i, j in np.argwhere(ranks != run_ranks):
        s = ref_f[(min(i, j), max(i, j))][2]
        K = min(ranks[i, j], run_ranks[i, j])
        assert abs(s[K] - eps) <= 1e-12 * s[0], (i, j)
    for k, w in enumerate(SAMPLE):
        e = np.array(E.e2_lo(ref_f, ref["thetas"][k]))
        assert np.abs(run_e[w] - e).max() <= 1e-9, (w, run_e[w], e)


def test_lo_energy_at_the_headline_threshold(run, ref, ref_svd):
    """eps = 1e-7 (the largest threshold whose per-walker error stays within
    1 mHa on this workload): orbitals touch more than 192 rows, so pass 1 runs
    two tiles per orbital."""
    assert 2 * run["ranks7"].sum() - np.trace(run["ranks7"]) > 192 * run["ranks7"].shape[0]
    _check_lo(run["ranks7"], run["e_lo7"], E.lo_truncate(ref_svd, EPS_TIGHT), ref, EPS_TIGHT)
    # every walker: the transposed layout gives the walker-major energies bit for bit
    assert np.array_equal(run["e_lo7"].view(np.float64), run["e_lo7_wm"].view(np.float64))


def test_lo_energy_sampled_walkers_and_ranks(run, ref, ref_lo):
    ranks = E.lo_ranks(ref_lo, run["system"].config.n)
    # integer decisions taken in FP64 on both sides; a mismatch is only allowed
    # for a singular value within rounding of the threshold
    for i, j in np.argwhere(ranks != run["ranks"]):
        s = ref_lo[(min(i, j), max(i, j))][2]
        K = min(ranks[i, j], run["ranks"][i, j])
        assert abs(s[K] - EPS) <= 1e-12 * s[0], (i, j)
    for k, w in enumerate(SAMPLE):
        e = np.array(E.e2_lo(ref_lo, ref["thetas"][k]))
        assert np.abs(run["e_lo"][w] - e).max() <= 1e-9, (w, run["e_lo"][w], e)


def test_lo_error_within_a_priori_bound(run, ref, ref_lo):
    """|E_LO - E_full| <= 3 sum_ij sigma_{K+1} ||Q_i|| ||Q_j|| (sampled walkers)."""
    for k, w in enumerate(SAMPLE):
        bound = E.lo_error_bound(ref_lo, ref["thetas"][k])
        d = abs(run["e_lo"][w].sum() - run["e_full"][w].sum())
        assert d <= bound * (1 + 1e-9) + 1e-9, (w, d, bound)
    assert np.isfinite(run["e_lo"]).all() and np.isfinite(run["e_full"]).all()
