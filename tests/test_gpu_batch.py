"""Batched uneven shots (spr_run_batch): each population's result is the same as
when it runs alone (bit for bit: the per-member arithmetic does not depend on
the batch), and matches the oracle."""

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


def plain_sched(B, ctx):
    return B.sched_plain(ctx, alg=B.ALG_HIO, G=3, j=4, j_er=3, j_end=0, beta=0.9, chi=0.5, sigma=2.0,
                         sigma_end=1.0, tau=0.1, tau_end=0.1)


CASES = [(64, 3, 11), (32, 4, 12), (64, 2, 13), (96, 3, 14), (32, 1, 15), (256, 2, 16), (256, 3, 17)]


def test_batch_of_many_members_equals_alone_bitwise(ctx, B):
    # two shots of each size share every launch (their members reach their
    # own modulus through the slot descriptors): the same bits as alone
    cases = [Case(n, P, seed=sd) for n, P, sd in ((512, 12, 31), (512, 12, 32), (1024, 3, 33), (1024, 3, 34))]
    ctx.set_cache_budget(1 << 30)
    try:
        alone = []
        for c in cases:
            sh, pop = c.population(ctx)
            pop.run(plain_sched(B, ctx))
            alone.append(pop.read())
            pop.close()
            sh.close()
        shots, pops = [], []
        for c in cases:
            sh, pop = c.population(ctx)
            shots.append(sh)
            pops.append(pop)
        ctx.run_batch(pops, [plain_sched(B, ctx) for _ in cases])
        for pop, (rho_a, supp_a, err_a) in zip(pops, alone):
            rho, supp, err = pop.read()
            np.testing.assert_array_equal(rho, rho_a)
            np.testing.assert_array_equal(supp, supp_a)
            np.testing.assert_array_equal(err, err_a)
        for pop in pops:
            pop.close()
        for sh in shots:
            sh.close()
    finally:
        ctx.set_cache_budget(256 << 20)


@pytest.mark.parametrize("alt", (False, True))
def test_batch_equals_alone_bitwise(ctx, B, alt):
    # alt: every size with two plans runs its alternative (as after tuning)
    from paper_2409_07413_amd import build
    sizes = sorted({n for n, _, _ in CASES if n in build.VARIANT_SIZES})
    for n in sizes:
        ctx.set_variant(n, 1 if alt else 0)
    try:
        _batch_equals_alone(ctx, B)
    finally:
        for n in sizes:
            ctx.set_variant(n, 0)


def _batch_equals_alone(ctx, B):
    cases = [Case(n, P, seed=sd) for n, P, sd in CASES]
    # alone
    alone = []
    for c in cases:
        sh, pop = c.population(ctx)
        s = plain_sched(B, ctx)
        pop.run(s)
        alone.append(pop.read())
        pop.close()
        sh.close()
    # batched (two size groups with several shots each)
    shots, pops = [], []
    for c in cases:
        sh, pop = c.population(ctx)
        shots.append(sh)
        pops.append(pop)
    scheds = [plain_sched(B, ctx) for _ in cases]
    ctx.run_batch(pops, scheds)
    for c, pop, (rho_a, supp_a, err_a) in zip(cases, pops, alone):
        rho, supp, err = pop.read()
        np.testing.assert_array_equal(rho, rho_a)
        np.testing.assert_array_equal(supp, supp_a)
        np.testing.assert_array_equal(err, err_a)
    for pop in pops:
        pop.close()
    for sh in shots:
        sh.close()


def test_batch_single_operator_parity(ctx, B):
    cases = [Case(n, P, seed=sd) for n, P, sd in CASES[:3]]
    shots, pops = [], []
    for c in cases:
        sh, pop = c.population(ctx)
        shots.append(sh)
        pops.append(pop)
    ops = [B.op(B.OP_RAAR, count=1, beta=0.9, chi=0.5), B.op(B.OP_GET_ERROR)]
    ctx.run_batch(pops, [B.sched_ops(ops, ctx) for _ in cases])
    for c, pop in zip(cases, pops):
        rho, _, err = pop.read()
        for p in range(c.P):
            ref = mpr.raar(c.rho[p], c.S[p], c.M, c.known, 0.5, 0.9)
            assert rel(rho[p], ref) <= 1e-5
            e = mpr.get_error(ref, c.S[p], c.M, c.known)
            assert abs(err[p] - e) <= 1e-5 * e
    for pop in pops:
        pop.close()
    for sh in shots:
        sh.close()


def test_batch_rejects_unequal_or_memetic_schedules(ctx, B):
    a, b = Case(32, 4, seed=1), Case(32, 4, seed=2)
    sa, pa = a.population(ctx, memetic=True)
    sb, pb = b.population(ctx)
    with pytest.raises(B.SprError):
        ctx.run_batch([pa, pb], [B.sched_ops([B.op(B.OP_ER, count=2)], ctx),
                                 B.sched_ops([B.op(B.OP_ER, count=3)], ctx)])
    with pytest.raises(B.SprError):
        ctx.run_batch([pa, pb], [B.sched_ops([B.op(B.OP_SELECT, gen=1)], ctx)] * 2)
    with pytest.raises(B.SprError):
        ctx.run_batch([pa, pa], [B.sched_ops([B.op(B.OP_ER, count=1)], ctx)] * 2)
    for p in (pa, pb):
        p.close()
    sa.close()
    sb.close()
