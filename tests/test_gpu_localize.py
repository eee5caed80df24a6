"""Foster-Boys localization on the GPU (lo_localize_boys) against the CPU
reference's Jacobi sweeps (oracle/localize.py), and the LO route run from a
delocalized trial localized on the device against the reference run from the
trial it localizes.

The localized orbitals are unique up to column order and sign, which change
neither the pair-block ranks (up to the same permutation) nor any energy, so
orbitals are matched column by column by their overlap and the energies are
compared directly, at the FP64 bar of 1e-9 Ha per walker.
"""
import numpy as np
import pytest

from oracle import energy as E
from oracle import localize as B
from paper_2202_00832_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2202_00832_amd import lofqmc  # noqa: E402


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


def match_columns(got, ref):
    """Permutation and signs taking ref's columns to got's; asserts a one-to-one match."""
    ov = got.T @ ref
    perm = np.argmax(np.abs(ov), axis=1)
    assert sorted(perm.tolist()) == list(range(ref.shape[1]))
    signs = np.sign(ov[np.arange(ov.shape[0]), perm])
    return perm, signs


def test_chain_localization_matches_reference(ctx):
    s = synth.make_system(synth.CHAIN_SMALL, nw=1)
    deloc = synth.delocalized_trial(s.trial)
    pos = B.chain_positions(s.config.M)
    ref, hist = B.boys_jacobi(deloc, pos)
    C = dev(deloc)
    b0, b1, sweeps = ctx.localize_boys(dev(pos), C)
    got = host(C)
    assert abs(b0 - hist[0]) <= 1e-12 * hist[0]
    assert abs(b1 - hist[-1]) <= 1e-11 * hist[-1]
    assert abs(sweeps - (len(hist) - 1)) <= 1
    perm, signs = match_columns(got, ref)
    assert np.abs(got - ref[:, perm] * signs[None, :]).max() <= 1e-9
    assert np.abs(got.T @ got - np.eye(got.shape[1])).max() <= 1e-12


def test_three_position_operators_match_reference(ctx):
    rng = np.random.default_rng(12)
    M, n = 40, 9
    C0 = np.linalg.qr(rng.standard_normal((M, n)))[0]
    pos = rng.uniform(-3, 3, (3, M))
    ref, hist = B.boys_jacobi(C0, pos, max_sweeps=100, tol=1e-14)
    C = dev(C0)
    b0, b1, sweeps = ctx.localize_boys(dev(pos), C, max_sweeps=100, tol=1e-14)
    got = host(C)
    assert abs(b1 - hist[-1]) <= 1e-10 * hist[-1]
    perm, signs = match_columns(got, ref)
    assert np.abs(got - ref[:, perm] * signs[None, :]).max() <= 1e-8


@pytest.mark.parametrize("eps", [1e-4, 1e-3])
def test_lo_route_from_a_delocalized_trial(ctx, eps):
    """Delocalized trial -> lo_localize_boys -> half-rotation -> LO factors ->
    green_theta -> LO energy, all on the device; the reference localizes the
    same trial with its own sweeps and runs its own LO route."""
    s = synth.make_system(synth.CHAIN_SMALL)
    deloc = synth.delocalized_trial(s.trial)
    pos = B.chain_positions(s.config.M)
    C = dev(deloc)
    ctx.localize_boys(dev(pos), C)
    chol_d, phi_d = dev(s.chol), dev(s.walkers)
    lbar = ctx.build_half_rotated_chol(chol_d, C)
    f = ctx.build_lo_factors(lbar, eps)
    theta, _, info = ctx.green_theta(C, phi_d)
    got = host(ctx.local_energy_lo(f, theta, info))
    ranks = f.info()["ranks"]
    # the delocalized trial on the device, for the compression comparison
    lbar_d = ctx.build_half_rotated_chol(chol_d, dev(deloc))
    ranks_deloc = ctx.build_lo_factors(lbar_d, eps).info()["ranks"]

    ref_C, _ = B.boys_jacobi(deloc, pos)
    perm, _ = match_columns(host(C), ref_C)
    ref_f = E.lo_compress(E.half_rotate(s.chol, ref_C), eps, pairs="upper")
    ref_ranks = E.lo_ranks(ref_f, s.config.n)
    assert np.array_equal(ranks, ref_ranks[np.ix_(perm, perm)])
    thetas, _, oinfo = E.green_theta_batch(ref_C, s.walkers)
    assert (oinfo == 0).all()
    ref = E.e2_lo_batch(ref_f, thetas)
    err = np.abs(got - ref).max()
    assert err <= 1e-9, err
    # localized orbitals compress the pair blocks better than the delocalized ones
    assert ranks.mean() < 0.6 * ranks_deloc.mean()
    # and the full energy does not depend on the rotation of the trial
    e_full_loc = host(ctx.local_energy_full(lbar, theta, info))
    theta_d, _, info_d = ctx.green_theta(dev(deloc), phi_d)
    e_full_del = host(ctx.local_energy_full(lbar_d, theta_d, info_d))
    assert np.abs(e_full_loc - e_full_del).max() <= 1e-9
