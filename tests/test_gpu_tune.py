"""Kernel variants and the run-time tuner: every compiled variant meets the
single-operator bar against the oracle, and the tuner's choice is kept on
the context and used by shots created afterwards."""

import numpy as np
import pytest

from oracle import mpr

from gpu_cases import Case, rel

pytestmark = pytest.mark.gpu

VARIANT_SIZES = (128, 256, 384, 512, 768, 1024)


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


@pytest.mark.parametrize("n", VARIANT_SIZES)
def test_variant_one_parity(ctx, B, n):
    import torch
    assert B.load().spr_size_variants(n) == 2
    ctx.set_variant(n, 1)
    try:
        rng = np.random.default_rng(n)
        x = (rng.standard_normal((2, n, n)) + 1j * rng.standard_normal((2, n, n))).astype(np.complex64)
        xi = torch.from_numpy(x).cuda()
        xo = torch.empty_like(xi)
        ctx.fft2(xi, xo)
        got = xo.cpu().numpy()
        for b in range(2):
            assert rel(got[b], mpr.fft2(x[b].astype(np.complex128))) <= 1e-5
        c = Case(n, 2, seed=n + 9)
        sh, pop = c.population(ctx)
        pop.run(B.sched_ops([B.op(B.OP_RAAR, count=1, beta=0.9, chi=0.5), B.op(B.OP_GET_ERROR)], ctx))
        rho, _, err = pop.read()
        for p in range(2):
            ref = mpr.raar(c.rho[p], c.S[p], c.M, c.known, 0.5, 0.9)
            assert rel(rho[p], ref) <= 1e-5
            e = mpr.get_error(ref, c.S[p], c.M, c.known)
            assert abs(err[p] - e) <= 1e-5 * e
        pop.close()
        sh.close()
    finally:
        ctx.set_variant(n, 0)


def test_autotune_keeps_its_choice(ctx, B):
    r = ctx.autotune(256, 64)
    assert r["n"] == 256 and r["variant"] in (0, 1) and 1 <= r["chunk_members"] <= 64
    assert len(r["candidates"]) >= 2
    best = max(c["member_iterations_per_s"] for c in r["candidates"])
    assert r["member_iterations_per_s"] == best > 0
    assert ctx.tuning(256) == (r["variant"], r["chunk_members"])
    ctx.set_variant(256, 0)


def test_autotune_times_the_resident_variant(ctx, B):
    # at 128^2 variant 1 is the resident Sequence: the tuner times it beside
    # the launch pairs (a candidate whose barrier wait ran out would report 0)
    r = ctx.autotune(128, 8)
    rates = {c["variant"]: c["member_iterations_per_s"] for c in r["candidates"]}
    assert set(rates) == {0, 1} and min(rates.values()) > 0
    print(f"autotune 128^2, 8 members: {rates}")
    ctx.set_variant(128, 0)


def test_batch_rejects_mixed_variants(ctx, B):
    a, b = Case(256, 2, seed=1), Case(256, 2, seed=2)
    ctx.set_variant(256, 0)
    sa, pa = a.population(ctx)
    ctx.set_variant(256, 1)
    sb, pb = b.population(ctx)
    ctx.set_variant(256, 0)
    s = B.sched_ops([B.op(B.OP_ER, count=1)], ctx)
    with pytest.raises(B.SprError):
        ctx.run_batch([pa, pb], [s, s])
    for x in (pa, pb, sa, sb):
        x.close()
