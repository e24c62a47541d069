"""Per-iteration Fourier-error traces (SPR_ITER_TRACE) against the oracle."""

import numpy as np
import pytest

from oracle import mpr

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


@pytest.mark.parametrize("n,alg,n_ia,n_er", [(64, "RAAR", 3, 5), (96, "HIO", 2, 4), (128, "RAAR", 0, 6)])
def test_trace_matches_oracle(ctx, B, n, alg, n_ia, n_er):
    P = 3
    c = Case(n, P, seed=n + 11)
    sh, pop = c.population(ctx)
    kind = B.OP_RAAR if alg == "RAAR" else B.OP_HIO
    ops = []
    if n_ia:
        ops.append(B.op(kind, count=n_ia, beta=0.9, chi=0.5, which=B.ITER_TRACE))
    ops.append(B.op(B.OP_ER, count=n_er, chi=0.5, which=B.ITER_TRACE))
    pop.run(B.sched_ops(ops, ctx))
    tr = pop.trace()
    assert tr.shape == (n_ia + n_er, P)
    for p in range(P):
        _, ref = mpr.sequence_trace(c.rho[p], c.S[p], c.M, c.known, 0.5, alg, 0.9, n_ia, n_er)
        np.testing.assert_allclose(tr[:, p], ref, rtol=1e-4, atol=1e-6)  # errors are relative to |M|: FP32 floor ~1e-7
    pop.close()
    sh.close()


@pytest.mark.parametrize("n", (256, 384, 512, 768, 1024))
@pytest.mark.parametrize("variant", (0, 1))
def test_trace_every_plan(ctx, B, n, variant):
    # the tracing column pass of both plans of each tuned size (its per-tile
    # FP64 partials follow the tile width, its workgroup size C*T up to 1024)
    P = 2
    c = Case(n, P, seed=n + 3 * variant + 17)
    ctx.set_variant(n, variant)
    try:
        sh, pop = c.population(ctx)
        pop.run(B.sched_ops([B.op(B.OP_RAAR, count=2, beta=0.9, chi=0.5, which=B.ITER_TRACE),
                             B.op(B.OP_ER, count=2, chi=0.5, which=B.ITER_TRACE)], ctx))
        tr = pop.trace()
        pop.close()
        sh.close()
    finally:
        ctx.set_variant(n, 0)
    assert tr.shape == (4, P)
    for p in range(P):
        _, ref = mpr.sequence_trace(c.rho[p], c.S[p], c.M, c.known, 0.5, "RAAR", 0.9, 2, 2)
        np.testing.assert_allclose(tr[:, p], ref, rtol=1e-4, atol=1e-6)


def test_trace_scope_chunks_and_untraced_ops(ctx, B):
    # children only: parents' columns stay NaN; member chunks smaller than the
    # scope; an untraced op in between adds no row
    n, P = 64, 4
    c = Case(n, P, seed=5)
    sh, pop = c.population(ctx, memetic=True, seed=1)
    pop.write(rho=c.rho32, supp=c.supp8, children=True)
    ctx.set_cache_budget(2 * 2 * n * n * 8)  # two members per launch
    try:
        ops = [B.op(B.OP_ER, count=2, chi=0.5, scope=B.SCOPE_CHILDREN, which=B.ITER_TRACE),
               B.op(B.OP_ER, count=1, chi=0.5, scope=B.SCOPE_CHILDREN),
               B.op(B.OP_ER, count=1, chi=0.5, scope=B.SCOPE_CHILDREN, which=B.ITER_TRACE)]
        pop.run(B.sched_ops(ops, ctx))
    finally:
        ctx.set_cache_budget(256 << 20)
    tr = pop.trace()
    assert tr.shape == (3, 2 * P)
    assert np.isnan(tr[:, :P]).all()
    for p in range(P):
        _, ref = mpr.sequence_trace(c.rho[p], c.S[p], c.M, c.known, 0.5, "RAAR", 0.9, 0, 4)
        np.testing.assert_allclose(tr[:, P + p], [ref[0], ref[1], ref[3]], rtol=1e-4, atol=1e-6)
    # a run without traced ops leaves the last trace in place
    pop.run(B.sched_ops([B.op(B.OP_GET_ERROR, scope=B.SCOPE_CHILDREN)], ctx))
    assert pop.trace().shape == (3, 2 * P)
    pop.close()
    sh.close()


def test_trace_rejected_outside_single_populations(ctx, B):
    c = Case(64, 2, seed=2)
    sh, pop = c.population(ctx)
    s = B.sched_ops([B.op(B.OP_ER, count=2, chi=0.5, which=B.ITER_TRACE)], ctx)
    with pytest.raises(B.SprError):
        ctx.run_batch([pop], [s])
    with pytest.raises(B.SprError):
        B.sched_ops([B.op(B.OP_ER, count=2, chi=0.5, which=2)], ctx)
    pop.close()
    sh.close()
