"""Resident Sequence at 128^2 (variant 1: one cooperative launch per
Sequence, the member's workgroups meeting at device-memory barriers between
passes) against the default launch pairs of the same passes (variant 0): the
same bits for whole plain and MPR schedules, several population sizes, and
Sequences longer than one launch carries; the timing of both is printed."""

import time

import numpy as np
import pytest

from gpu_cases import Case

pytestmark = pytest.mark.gpu

N = 128


@pytest.fixture(scope="module")
def ctx():
    from paper_2409_07413_amd import binding
    c = binding.Context(0)
    yield c
    c.set_variant(N, 0)
    c.close()


@pytest.fixture(scope="module")
def B():
    from paper_2409_07413_amd import binding
    return binding


def _run_both(ctx, B, case, make_sched, memetic=False, seed=0, reps=1):
    """Results (and seconds per run) of the same schedule on the resident form
    (variant 1) and on launch pairs (variant 0), from the same inputs."""
    assert B.load().spr_size_variants(N) == 2
    out = []
    for variant in (1, 0):
        ctx.set_variant(N, variant)
        try:
            sh, pop = case.population(ctx, memetic=memetic, seed=seed)
            s = make_sched()
            pop.run(s)
            pop.sync()
            t0 = time.perf_counter()
            for _ in range(reps - 1):
                pop.run(s)
            pop.sync()
            dt = (time.perf_counter() - t0) / max(reps - 1, 1)
            rho, supp, err = pop.read()
            out.append((rho, supp, err, dt))
            s.close()
            pop.close()
            sh.close()
        finally:
            ctx.set_variant(N, 0)
    return out


def _same(a, b):
    for x, y in zip(a[:3], b[:3]):
        assert np.array_equal(np.asarray(x).view(np.uint8), np.asarray(y).view(np.uint8))


@pytest.mark.parametrize("P", [1, 5, 8, 13, 100])
def test_plain_schedule_same_bits(ctx, B, P):
    # 100 members exceed one cooperative launch's resident workgroups (8 per
    # member), so the launcher splits them over several launches
    c = Case(N, P, seed=40 + P)
    make = lambda: B.sched_plain(ctx, alg=B.ALG_HIO, G=3, j=16, j_er=4, j_end=0, beta=0.9, chi=0.5,
                                 sigma=2.0, sigma_end=1.0, tau=0.1, tau_end=0.1)
    r, l = _run_both(ctx, B, c, make)
    _same(r, l)
    assert np.isfinite(r[2]).all()


def test_long_sequence_spans_launches(ctx, B):
    # 60 RAAR + 30 ER iterations: one Sequence over two resident launches
    c = Case(N, 8, seed=77)
    make = lambda: B.sched_ops([B.op(B.OP_RAAR, count=60, beta=0.9, chi=0.5), B.op(B.OP_ER, count=30, chi=0.5),
                                B.op(B.OP_GET_ERROR)], ctx)
    r, l = _run_both(ctx, B, c, make)
    _same(r, l)


def test_mpr_generation_same_bits(ctx, B):
    c = Case(N, 8, seed=91)
    make = lambda: B.sched_mpr(ctx, alg=B.ALG_RAAR, G=2, R=3, j=16, j_er=4, j_end=0, j_eval=20, t_min=4, t_max=16,
                               gen_first=1, gen_count=2, init_error=1, beta=0.9, chi=0.5, sigma=2.0,
                               sigma_end=0.5, tau=0.1, tau_end=0.0667, c_p=0.6, c_w=0.4)
    r, l = _run_both(ctx, B, c, make, memetic=True, seed=5)
    _same(r, l)


def test_plain_128_timing(ctx, B):
    # config-1 shape: P = 8, 200 iterations (10 x [HIO^16 ER^4], shrink-wrap each)
    c = Case(N, 8, seed=3)
    make = lambda: B.sched_plain(ctx, alg=B.ALG_HIO, G=10, j=16, j_er=4, j_end=0, beta=0.9, chi=0.5,
                                 sigma=2.0, sigma_end=1.0, tau=0.1, tau_end=0.1)
    r, l = _run_both(ctx, B, c, make, reps=6)
    _same(r, l)
    print(f"plain 128^2 P=8, 200 iterations: resident {r[3] * 1e3:.3f} ms, launch pairs {l[3] * 1e3:.3f} ms")
