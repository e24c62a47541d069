"""Step-chained GPU parity of whole schedules against the FP64 oracle.

Every step of a device trajectory -- each HIO, RAAR or ER iteration, each
shrink-wrap, UpdateSupportSize, GetError, statistics, crossover and select
of the schedule -- is compared with one oracle step taken from the device's
own previous state (tests/chained.py).  Bars: iterations and crossover
children <= 1e-5 relative L2 per step (FP32 against FP64), fitness <= 1e-5
relative; HIO decisions and support thresholds exact outside the FP32 band
(the pixels decided inside it are counted and printed); statistics and
selections exact.
"""

import numpy as np
import pytest

from oracle import mpr
from paper_2409_07413_amd import synth

import chained
from gpu_cases import Case

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


def _report(name, rep):
    chained.REPORTS.append((name, rep))
    print(f"{name}: {rep['steps']} steps, max step rel L2 {rep['max_step_rel']:.2e}, "
          f"max fitness rel {rep['max_err_rel']:.2e}, HIO pixels decided in the FP32 band {rep['hio_band_px']}, "
          f"shrink-wrap band pixels {rep['sw_band_px']}, area band pixels {rep['area_band_px']}, "
          f"crossover children {rep['xover_children']} ({rep['xover_flagged']} near-tie flagged), "
          f"selections {rep['selections']}", flush=True)


def _variants():
    from paper_2409_07413_amd import build
    out = []
    for n in (64, 128, 256, 384, 512, 768, 1024):
        for v in ((0, 1) if n in build.VARIANT_SIZES else (0,)):
            out.append((n, v))
    return out


def _variant_sizes():
    from paper_2409_07413_amd import build
    return build.VARIANT_SIZES


def _run_chain(ctx, B, c, ops, variant=0):
    sh = c.shot(ctx)
    tuned = c.n in _variant_sizes()
    if tuned:
        ctx.set_variant(c.n, variant)
    try:
        traj = chained.Trajectory(ctx, B, lambda: sh.population(c.rho32, c.supp8), ops)
        rep = chained.check_trajectory(traj, c.M, c.known)
    finally:
        if tuned:
            ctx.set_variant(c.n, 0)
        sh.close()
    return rep


# ---------------------------------------------------------------------------
# 20-iteration runs from random-phase starts: IA^16 ER^4 (Eq. sequence), every
# iteration checked, every tuned size on both plans
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("n,variant", _variants())
@pytest.mark.parametrize("alg", ("HIO", "RAAR"))
def test_twenty_iterations_chained(ctx, B, n, variant, alg):
    P = 2 if n <= 512 else 1
    c = Case(n, P, seed=n + 5 + 17 * variant)
    kind = B.OP_HIO if alg == "HIO" else B.OP_RAAR
    ops = [B.op(kind, count=16, beta=0.9, chi=0.5), B.op(B.OP_ER, count=4, chi=0.5)]
    rep = _run_chain(ctx, B, c, ops, variant)
    _report(f"{alg}^16 ER^4 at {n}^2 plan {variant}", rep)
    assert rep["steps"] == 20


@pytest.mark.parametrize("n,variant", [(64, 0), (256, 0), (384, 1), (512, 0), (1024, 1)])
@pytest.mark.parametrize("alg", ("HIO", "RAAR"))
@pytest.mark.parametrize("chi", (0.3, 1.0))
def test_twenty_iterations_chained_phase_constraint(ctx, B, n, variant, alg, chi):
    # the cone constraint (chi = 0.3) and no phase constraint (chi = 1)
    P = 2 if n <= 512 else 1
    c = Case(n, P, seed=n + 7 + 13 * variant, per_member_supp=True)
    kind = B.OP_HIO if alg == "HIO" else B.OP_RAAR
    ops = [B.op(kind, count=16, beta=0.9, chi=chi), B.op(B.OP_ER, count=4, chi=chi)]
    rep = _run_chain(ctx, B, c, ops, variant)
    _report(f"{alg}^16 ER^4 chi {chi} at {n}^2 plan {variant}", rep)
    assert rep["steps"] == 20


@pytest.mark.parametrize("variant", (0, 1))
def test_mixed_chain_at_384(ctx, B, variant):
    # RAAR^2 HIO^2 ER^2 at 384^2 (three members with their own supports): the
    # HIO steps decide pixels near the cone boundary (chi = 0.3), so this run
    # parts from an end-to-end FP64 run; step by step it must not
    c = Case(384, 3, seed=384 + 400, per_member_supp=True)
    ops = [B.op(B.OP_RAAR, count=2, beta=0.9, chi=0.5), B.op(B.OP_HIO, count=2, beta=0.8, chi=0.3),
           B.op(B.OP_ER, count=2, chi=0.5), B.op(B.OP_GET_ERROR)]
    rep = _run_chain(ctx, B, c, ops, variant)
    _report(f"RAAR^2 HIO^2 ER^2 at 384^2 plan {variant}", rep)
    assert rep["steps"] == 7


# ---------------------------------------------------------------------------
# The plain method of the 128^2 benchmark configuration, whole: 10 blocks of
# HIO^j ER^(20-j) (j 16 -> 0, beta 0.9) with shrink-wrap (sigma 2 -> 1,
# tau 0.10) and the final GetError; P = 8 device random-phase starts
# (Alg. randomsearch with normalimprove).
# ---------------------------------------------------------------------------
def test_plain_128_schedule_chained(ctx, B):
    n, P, seed = 128, 8, 2001
    sh0 = synth.shot(n, "ellipses", 1001, 1e6, beamstop=8)
    amp = sh0["amp"].astype(np.float32)
    mask = sh0["mask"].astype(np.uint8)
    S0 = synth.centred_square(n, 48).astype(np.uint8)
    sched = B.sched_plain(ctx, alg=B.ALG_HIO, G=10, j=16, j_er=4, j_end=0, beta=0.9, chi=0.5, sigma=2.0,
                          sigma_end=1.0, tau=0.10, tau_end=0.10)
    ops = sched.ops()
    sched.close()
    shot = ctx.shot(amp, mask)
    M = mpr.to_fft_order(amp.astype(np.float64))
    known = mpr.to_fft_order(sh0["mask"])
    try:
        traj = chained.Trajectory(ctx, B, lambda: shot.population(None, S0, seed=seed, P=P), ops)
        rep = chained.check_trajectory(traj, M, known)
    finally:
        shot.close()
    _report("plain method 128^2, P = 8, 200 iterations", rep)
    assert rep["steps"] == 200 + 10 + 1


# ---------------------------------------------------------------------------
# One MPR generation (Alg. mpr, Alg. improve, Alg. crossover, Alg. select),
# every op checked: at 128^2 with the benchmark's per-generation schedule
# (R = 3 sequences of RAAR^16 ER^4, ER^40 evaluation), and at the benchmark's
# 512^2 shot with shorter sequences.
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("n,j,j_er,j_eval", [(128, 16, 4, 40), (512, 4, 2, 4)])
def test_mpr_generation_chained(ctx, B, n, j, j_er, j_eval):
    P, seed_x = 4, 3002
    c = Case(n, P, seed=n + 2004, kind="spheres", photons=1e8, gap=4, side=int(0.35 * n))
    prm = dict(alg=B.ALG_RAAR, G=2, R=3, j=j, j_er=j_er, j_end=0, j_eval=j_eval, t_min=4, t_max=n // 8,
               gen_first=1, gen_count=1, init_error=1, beta=0.9, chi=0.5, sigma=2.0, sigma_end=0.5,
               tau=0.10, tau_end=0.10 * 2 / 3, c_p=0.6, c_w=0.4)
    sched = B.sched_mpr(ctx, **prm)
    ops = sched.ops()
    sched.close()
    sh = c.shot(ctx)
    try:
        traj = chained.Trajectory(ctx, B, lambda: sh.population(c.rho32, c.supp8, memetic=True, seed=seed_x),
                                  ops, memetic=True)
        rep = chained.check_trajectory(traj, c.M, c.known, seed=seed_x)
    finally:
        sh.close()
    _report(f"MPR generation {n}^2, P = {P}", rep)
    assert rep["selections"] == P and rep["xover_children"] == P
    assert rep["xover_flagged"] <= P // 2


# ---------------------------------------------------------------------------
# The same step by step with the modulus stored in FP16 (the oracle uses the
# stored values, reading of the FP16 storage) and with upper bounds on the
# unknown pixels (Eq. pm_bounds), from starts that put energy on them so that
# the clamp acts in every step.
# ---------------------------------------------------------------------------
def _energetic_starts(c, rng):
    obj = c.obj / max(c.obj.max(), 1e-30)
    scale = np.sqrt(np.sum(c.M ** 2) / max(np.sum(np.abs(mpr.fft2(obj)) ** 2), 1e-30))
    n = c.n
    return np.stack([(3.0 * scale * obj * np.exp(1j * 0.3 * p)
                      + 0.1 * scale * (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))))
                     for p in range(c.P)]).astype(np.complex64)


@pytest.mark.parametrize("n,fp16,bounds,alg", [(512, True, False, "RAAR"), (256, False, True, "HIO"),
                                               (1024, True, True, "RAAR")])
def test_chained_fp16_and_bounds(ctx, B, n, fp16, bounds, alg):
    P = 2 if n <= 512 else 1
    c = Case(n, P, seed=n + 61, photons=1e8, gap=4)
    sh = ctx.shot(c.amp32, c.mask8, fp16=fp16)
    M, s = (mpr.fp16_modulus(c.M, c.known) if fp16 else (c.M, 1.0))
    U = None
    if bounds:
        assert sh.set_bounds(1.5, 0.2) > 0
        U = mpr.upper_bounds(M, c.known, 1.5, 0.2)
        if fp16:
            U = np.where(np.isfinite(U), (U / s).astype(np.float16).astype(np.float64) * s, np.nan)
        rho32 = _energetic_starts(c, np.random.default_rng(n))
    else:
        rho32 = c.rho32
    kind = B.OP_HIO if alg == "HIO" else B.OP_RAAR
    ops = [B.op(kind, count=8, beta=0.9, chi=0.5), B.op(B.OP_ER, count=4, chi=0.5), B.op(B.OP_GET_ERROR)]
    try:
        traj = chained.Trajectory(ctx, B, lambda: sh.population(rho32, c.supp8), ops)
        rep = chained.check_trajectory(traj, M, c.known, bound=U)
    finally:
        sh.close()
    _report(f"{alg}^8 ER^4 at {n}^2, FP16 storage {fp16}, upper bounds {bounds}", rep)
    assert rep["steps"] == 13
