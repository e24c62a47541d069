"""Serving engine on the device: a served shot gives the same result as the
same schedule run on a population (bit for bit: same kernels, same per-member
arithmetic), the same result alone and in a mix of shots of other sizes that
arrive while it runs, and matches the oracle."""

import time

import numpy as np
import pytest

from oracle import mpr

from gpu_cases import Case, rel

pytestmark = pytest.mark.gpu

BUDGET = 2 << 30


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


def plain(B, ctx=None, G=3):
    return B.sched_plain(ctx, alg=B.ALG_HIO, G=G, j=5, j_er=3, j_end=0, beta=0.9, chi=0.5, sigma=2.0,
                         sigma_end=1.0, tau=0.1, tau_end=0.1)


def alone_population(ctx, B, c, sched, seed=None):
    """Reference: the schedule on a population (spr_run)."""
    sh = c.shot(ctx)
    if seed is None:
        pop = sh.population(c.rho32, c.supp8)
    else:
        pop = sh.population(None, c.supp8[0], seed=seed, P=c.P)
    pop.run(sched)
    out = pop.read()
    pop.close()
    sh.close()
    return out


def serve(ctx, B, cases, sched, P, seeds=None, manual=True, all_members=True, stagger=0.0, max_shots=8):
    sv = B.Server(ctx, sched, P=P, hbm_budget=BUDGET, max_shots=max_shots, manual=manual,
                  all_members=all_members)
    ts = []
    for i, c in enumerate(cases):
        if seeds is None:
            ts.append(sv.submit(c.amp32, c.mask8, c.supp8, rho0=c.rho32))
        else:
            ts.append(sv.submit(c.amp32, c.mask8, c.supp8[0], seed=seeds[i]))
        if stagger:
            time.sleep(stagger)
    assert sv.drain(120.0)
    res = [sv.poll(t) for t in ts]
    st = sv.stats()
    sv.close()
    return res, st


def test_served_equals_population_run(ctx, B):
    c = Case(64, 4, seed=41)
    s = plain(B, ctx)
    rho_a, supp_a, err_a = alone_population(ctx, B, c, s)
    (r,), st = serve(ctx, B, [c], s, P=4)
    np.testing.assert_array_equal(r["rho"], rho_a)
    np.testing.assert_array_equal(r["supp"], supp_a)
    np.testing.assert_array_equal(r["err"], err_a)
    assert r["best"] == int(np.argmin(err_a))
    assert r["status"] == 0 and r["t_arrival"] <= r["t_admit"] <= r["t_finish"]
    assert st["bytes_in_use"] == 0 and st["completed"] == 1


@pytest.mark.parametrize("n", (256, 384))
def test_server_uses_the_context_variant(ctx, B, n):
    # a server created while the alternative plan is selected runs it: its
    # shot equals the population run on that plan bit for bit (and, since the
    # plans differ only in column-tile width, the default plan's densities)
    c = Case(n, 3, seed=n + 61)
    s = plain(B, ctx, G=2)
    base = alone_population(ctx, B, c, s)
    ctx.set_variant(n, 1)
    try:
        rho_a, supp_a, err_a = alone_population(ctx, B, c, s)
        (r,), _ = serve(ctx, B, [c], s, P=3)
    finally:
        ctx.set_variant(n, 0)
    np.testing.assert_array_equal(r["rho"], rho_a)
    np.testing.assert_array_equal(r["supp"], supp_a)
    np.testing.assert_array_equal(r["err"], err_a)
    np.testing.assert_array_equal(rho_a, base[0])
    np.testing.assert_allclose(err_a, base[2], rtol=1e-14, atol=0)


def test_alone_equals_mix(ctx, B):
    specs = [(64, 51), (96, 52), (64, 53), (128, 54), (32, 55), (96, 56)]
    cases = [Case(n, 4, seed=sd) for n, sd in specs]
    seeds = [1000 + sd for _, sd in specs]
    s = plain(B, ctx, G=4)
    alone = [serve(ctx, B, [c], s, P=4, seeds=[sd])[0][0] for c, sd in zip(cases, seeds)]
    # engine thread, shots arriving while others run
    mix, st = serve(ctx, B, cases, s, P=4, seeds=seeds, manual=False, stagger=0.002)
    assert st["completed"] == len(cases)
    for a, m in zip(alone, mix):
        np.testing.assert_array_equal(m["rho"], a["rho"])
        np.testing.assert_array_equal(m["supp"], a["supp"])
        np.testing.assert_array_equal(m["err"], a["err"])
    # the device random-phase start agrees with a population created the same way
    rho_p, supp_p, err_p = alone_population(ctx, B, cases[1], s, seed=seeds[1])
    np.testing.assert_array_equal(alone[1]["rho"], rho_p)
    np.testing.assert_array_equal(alone[1]["err"], err_p)


def test_best_member_record(ctx, B):
    cases = [Case(64, 4, seed=61), Case(32, 4, seed=62)]
    s = plain(B, ctx)
    full, _ = serve(ctx, B, cases, s, P=4, seeds=[7, 8])
    best, _ = serve(ctx, B, cases, s, P=4, seeds=[7, 8], all_members=False)
    for f, b in zip(full, best):
        assert b["members"] == 1 and b["best"] == f["best"] == int(np.argmin(f["err"]))
        np.testing.assert_array_equal(b["rho"][0], f["rho"][f["best"]])
        np.testing.assert_array_equal(b["supp"][0], f["supp"][f["best"]])
        np.testing.assert_array_equal(b["err"], f["err"])


def test_chunks_split_across_shots(ctx, B):
    # 512^2 members: 64 fit one iteration chunk, so the third shot of 24 members is split
    cases = [Case(512, 24, seed=70 + i) for i in range(3)]
    s = B.sched_ops([B.op(B.OP_RAAR, count=3, beta=0.9, chi=0.5), B.op(B.OP_ER, count=2, chi=0.5),
                     B.op(B.OP_GET_ERROR)], ctx)
    served, _ = serve(ctx, B, cases, s, P=24, seeds=[1, 2, 3])
    for c, sd, r in zip(cases, [1, 2, 3], served):
        rho_a, supp_a, err_a = alone_population(ctx, B, c, s, seed=sd)
        np.testing.assert_array_equal(r["rho"], rho_a)
        np.testing.assert_array_equal(r["err"], err_a)


def test_served_er_run_matches_oracle(ctx, B):
    n, P, seed = 96, 3, 2024
    c = Case(n, P, seed=81)
    s = B.sched_ops([B.op(B.OP_ER, count=20, chi=0.5), B.op(B.OP_GET_ERROR)], ctx)
    (r,), _ = serve(ctx, B, [c], s, P=P, seeds=[seed])
    x0 = mpr.random_phase_start(c.M, c.known, P, seed)
    for p in range(P):
        x = mpr.sequence(x0[p], c.S[0], c.M, c.known, 0.5, "HIO", 0.9, 0, 20)
        assert rel(r["rho"][p], x) <= 1e-3
        e = mpr.get_error(x, c.S[0], c.M, c.known)
        assert abs(r["err"][p] - e) <= 1e-3 * e


def test_server_rejects(ctx, B):
    s = plain(B, ctx)
    with pytest.raises(B.SprError):
        B.Server(ctx, s, P=4, hbm_budget=1 << 20, max_shots=2)  # budget below the work buffers
    # the server reserves two work buffers of 3/8 of the context's cache budget
    # each: with 2 x 96 MiB of them, a 200 MiB budget leaves too little for
    # the 4 members of a 1024^2 shot (their densities alone take 32 MiB)
    ctx.set_cache_budget(256 << 20)
    sv = B.Server(ctx, s, P=4, hbm_budget=(200 << 20), max_shots=2, manual=True)
    big = Case(1024, 1, seed=1)
    with pytest.raises(B.SprError) as e:
        sv.submit(big.amp32, big.mask8, big.supp8[0], seed=1)  # 4 members of 1024^2 do not fit
    assert e.value.code == B.E_ADMISSION
    sv.close()


def test_read_member(ctx, B):
    c = Case(64, 4, seed=91)
    sh, pop = c.population(ctx)
    pop.run(B.sched_ops([B.op(B.OP_ER, count=3, chi=0.5), B.op(B.OP_SHRINKWRAP, sigma=1.0, tau=0.1)], ctx))
    rho, supp, err = pop.read()
    for p in range(4):
        r1, s1 = pop.read_member(p)
        np.testing.assert_array_equal(r1, rho[p])
        np.testing.assert_array_equal(s1, supp[p])
    with pytest.raises(B.SprError):
        pop.read_member(4)
    np.testing.assert_array_equal(pop.errors(), err)
    pop.close()
    sh.close()
