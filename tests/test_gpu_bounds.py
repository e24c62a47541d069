"""Upper bounds on unknown amplitudes (Eq. pm_bounds): the device projector
against the oracle's, with FP32 and FP16 storage, on shots with a detector
gap; bounds removed again give the unbounded run bit for bit; a served shot
with bounds equals the population run."""

import numpy as np
import pytest

from oracle import mpr

from gpu_cases import Case, rel

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_2409_07413_amd import binding
    c = binding.Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def B():
    from paper_2409_07413_amd import binding
    return binding


def one_raar(B, ctx):
    return B.sched_ops([B.op(B.OP_RAAR, count=1, beta=0.9, chi=0.5), B.op(B.OP_GET_ERROR)], ctx)


@pytest.mark.parametrize("n,fp16", [(64, False), (256, False), (128, True), (384, False), (1024, True)])
def test_bounded_iteration_matches_oracle(ctx, B, n, fp16):
    c = Case(n, 3, seed=n + 31, photons=1e8, gap=4)
    sh = ctx.shot(c.amp32, c.mask8, fp16=fp16)
    rings = sh.set_bounds(1.5, 0.2)
    assert rings > 0
    M = c.M
    if fp16:
        M, s = mpr.fp16_modulus(c.M, c.known)
    U = mpr.upper_bounds(M, c.known, 1.5, 0.2)
    if fp16:
        U = np.where(np.isfinite(U), (U / s).astype(np.float16).astype(np.float64) * s, np.nan)
    # starts with energy on the unknown pixels: scaled copies of the object plus noise
    rng = np.random.default_rng(n)
    obj = c.obj / max(c.obj.max(), 1e-30)
    scale = np.sqrt(np.sum(c.M ** 2) / max(np.sum(np.abs(mpr.fft2(obj)) ** 2), 1e-30))
    rho32 = np.stack([(3.0 * scale * obj * np.exp(1j * 0.3 * p)
                       + 0.1 * scale * (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))))
                      for p in range(c.P)]).astype(np.complex64)
    rho = rho32.astype(np.complex128)
    pop = sh.population(rho32, c.supp8)
    pop.run(one_raar(B, ctx))
    out, _, err = pop.read()
    clamped = 0
    for p in range(c.P):
        ref = mpr.raar(rho[p], c.S[p], M, c.known, 0.5, 0.9, bound=U)
        assert rel(out[p], ref) <= 1e-5
        X = mpr.fft2(rho[p])
        clamped += int((np.isfinite(U) & (np.abs(X) > np.where(np.isfinite(U), U, np.inf))).sum())
        e = mpr.get_error(ref, c.S[p], M, c.known)
        assert abs(err[p] - e) <= 1e-5 * e
    assert clamped > 0  # the bounds were active
    pop.close()
    sh.close()


def test_bounds_removed_restore_the_plain_projector(ctx, B):
    c = Case(64, 2, seed=5, gap=4)
    s = B.sched_ops([B.op(B.OP_HIO, count=3, beta=0.9, chi=0.5), B.op(B.OP_ER, count=2, chi=0.5)], ctx)
    outs = []
    for eta in (None, 1.5, 0.0):
        sh = ctx.shot(c.amp32, c.mask8)
        if eta is not None:
            sh.set_bounds(eta, 0.2)
        pop = sh.population(c.rho32, c.supp8)
        pop.run(s)
        outs.append(pop.read()[0])
        pop.close()
        sh.close()
    np.testing.assert_array_equal(outs[0], outs[2])
    assert not np.array_equal(outs[0], outs[1])


def test_served_shot_with_bounds_equals_population(ctx, B):
    c = Case(96, 3, seed=17, gap=4)
    s = B.sched_plain(ctx, alg=B.ALG_RAAR, G=2, j=4, j_er=2, j_end=0, beta=0.9, chi=0.5, sigma=2.0,
                      sigma_end=1.0, tau=0.1, tau_end=0.1)
    sh = ctx.shot(c.amp32, c.mask8)
    sh.set_bounds(1.5, 0.2)
    pop = sh.population(None, c.supp8[0], seed=77, P=3)
    pop.run(s)
    rho_a, supp_a, err_a = pop.read()
    pop.close()
    sh.close()
    sv = B.Server(ctx, s, P=3, hbm_budget=1 << 30, max_shots=2, manual=True, all_members=True)
    t = sv.submit(c.amp32, c.mask8, c.supp8[0], seed=77, bound_eta=1.5, bound_max_unknown=0.2)
    assert sv.drain(60.0)
    r = sv.poll(t)
    sv.close()
    np.testing.assert_array_equal(r["rho"], rho_a)
    np.testing.assert_array_equal(r["err"], err_a)


def _saturated_wedges(n, mask8):
    """A thin wedge of saturated pixels at radii 14-20 (about 3 % of each ring)
    and a wide one at radii 26-32 (about 8 %), both made unknown in the mask."""
    yy, xx = np.mgrid[0:n, 0:n] - n // 2
    r = np.floor(np.sqrt(yy ** 2 + xx ** 2) + 0.5)
    ang = np.degrees(np.arctan2(yy, xx))
    sat = ((r >= 14) & (r <= 20) & (ang >= 40) & (ang < 50)) | ((r >= 26) & (r <= 32) & (ang >= 40) & (ang < 70))
    mask = mask8.copy()
    mask[sat] = 0
    return sat.astype(np.uint8), mask


@pytest.mark.parametrize("n,fp16", [(128, False), (128, True)])
def test_saturation_rules_match_oracle(ctx, B, n, fp16):
    c = Case(n, 3, seed=n + 7, photons=1e8, gap=4)
    sat8, mask8 = _saturated_wedges(n, c.mask8)
    known = mpr.to_fft_order(mask8.astype(bool))
    sat = mpr.to_fft_order(sat8.astype(bool))
    sh = ctx.shot(c.amp32, mask8, fp16=fp16)
    rings_plain = sh.set_bounds(1.5, 0.2)
    rings = sh.set_bounds(1.5, 0.2, saturated=sat8, max_saturated=0.05)
    assert 0 < rings < rings_plain  # the wide wedge removed rings
    M = np.where(known, c.M, 0.0)
    if fp16:
        M, s = mpr.fp16_modulus(M, known)
    U = mpr.upper_bounds(M, known, 1.5, 0.2, saturated=sat, max_saturated=0.05)
    U_plain = mpr.upper_bounds(M, known, 1.5, 0.2)
    if fp16:
        U = np.where(np.isfinite(U), (U / s).astype(np.float16).astype(np.float64) * s, np.nan)
    # both rules are exercised: saturated pixels in bounded rings lose their
    # bound, and rings of the wide wedge lose theirs altogether
    bins = mpr.radial_bins(n)
    bounded_q = set(np.unique(bins[np.isfinite(U)]))
    assert any(q in bounded_q for q in np.unique(bins[sat]))
    dropped = [q for q in np.unique(bins[sat]) if q not in bounded_q and np.isfinite(U_plain[bins == q]).any()]
    assert dropped
    assert not np.isfinite(U[sat]).any()
    rng = np.random.default_rng(n)
    obj = c.obj / max(c.obj.max(), 1e-30)
    scale = np.sqrt(np.sum(M ** 2) / max(np.sum(np.abs(mpr.fft2(obj)) ** 2), 1e-30))
    rho32 = np.stack([(3.0 * scale * obj * np.exp(1j * 0.3 * p)
                       + 0.1 * scale * (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))))
                      for p in range(c.P)]).astype(np.complex64)
    rho = rho32.astype(np.complex128)
    pop = sh.population(rho32, c.supp8)
    pop.run(one_raar(B, ctx))
    out, _, err = pop.read()
    for p in range(c.P):
        ref = mpr.raar(rho[p], c.S[p], M, known, 0.5, 0.9, bound=U)
        assert rel(out[p], ref) <= 1e-5
        e = mpr.get_error(ref, c.S[p], M, known)
        assert abs(err[p] - e) <= 1e-5 * e
    pop.close()
    sh.close()


def test_saturated_pixel_marked_measured_is_rejected(ctx, B):
    c = Case(64, 2, seed=3, gap=4)
    sh = ctx.shot(c.amp32, c.mask8)
    sat = np.zeros((64, 64), np.uint8)
    sat[np.argwhere(c.mask8 == 1)[0][0], np.argwhere(c.mask8 == 1)[0][1]] = 1
    with pytest.raises(B.SprError) as e:
        sh.set_bounds(1.5, 0.2, saturated=sat)
    assert e.value.code == -1  # SPR_E_INVALID_ARG
    with pytest.raises(B.SprError):
        sh.set_bounds(1.5, 0.2, saturated=np.zeros((64, 64), np.uint8), max_saturated=1.5)
    sh.close()


def test_served_shot_with_saturation_equals_population(ctx, B):
    n = 96
    c = Case(n, 3, seed=19, gap=4)
    sat8, mask8 = _saturated_wedges(n, c.mask8)
    s = B.sched_plain(ctx, alg=B.ALG_RAAR, G=2, j=4, j_er=2, j_end=0, beta=0.9, chi=0.5, sigma=2.0,
                      sigma_end=1.0, tau=0.1, tau_end=0.1)
    sh = ctx.shot(c.amp32, mask8)
    sh.set_bounds(1.5, 0.2, saturated=sat8, max_saturated=0.05)
    pop = sh.population(None, c.supp8[0], seed=78, P=3)
    pop.run(s)
    rho_a, _, err_a = pop.read()
    pop.close()
    sh.close()
    sv = B.Server(ctx, s, P=3, hbm_budget=1 << 30, max_shots=2, manual=True, all_members=True)
    t = sv.submit(c.amp32, mask8, c.supp8[0], seed=78, bound_eta=1.5, bound_max_unknown=0.2,
                  saturated=sat8, bound_max_saturated=0.05)
    assert sv.drain(60.0)
    r = sv.poll(t)
    sv.close()
    np.testing.assert_array_equal(r["rho"], rho_a)
    np.testing.assert_array_equal(r["err"], err_a)
