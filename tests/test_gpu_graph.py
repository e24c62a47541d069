"""Captured schedules: every replay of a graph gives the same result, bit for
bit, as running the schedule eagerly on a twin population, with eager work
and synchronisations between the replays."""

import numpy as np
import pytest

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


def _eager_noise(ctx, n=64):
    """Unrelated eager work on the context stream between replays."""
    import torch
    x = torch.randn(2, n, n, dtype=torch.complex64, device="cuda")
    y = torch.empty_like(x)
    ctx.fft2(x, y)
    torch.cuda.synchronize()


def _same(pa, pb, children=False):
    a, b = pa.read(children), pb.read(children)
    for u, v in zip(a, b):
        np.testing.assert_array_equal(u, v)


@pytest.mark.parametrize("n,variant", [(32, 0), (128, 0), (128, 1), (384, 1), (512, 0)])
def test_population_graph_replays_match_eager(ctx, B, n, variant):
    # (384, 1): a graph recorded on a size's alternative plan, taken from the
    # context when the populations are created; (128, 1): eager runs use the
    # resident Sequence, the captured graph the launch pairs it falls back to
    ctx.set_variant(n, variant)
    try:
        _graph_replays(ctx, B, n)
    finally:
        ctx.set_variant(n, 0)


def _graph_replays(ctx, B, n):
    c = Case(n, 4, seed=n + 1)
    s = B.sched_ops([B.op(B.OP_RAAR, count=3, beta=0.9, chi=0.5), B.op(B.OP_SHRINKWRAP, sigma=1.5, tau=0.1),
                     B.op(B.OP_ER, count=2, chi=0.5),
                     B.op(B.OP_SUPPORT_AREA, sigma=1.0, which=B.AREA_ABS, alpha=0.05 * n * n),
                     B.op(B.OP_GET_ERROR)], ctx)
    sa, pa = c.population(ctx)
    sb, pb = c.population(ctx)
    g = pa.graph(s)
    for _ in range(4):
        g.launch()
        pb.run(s)
        _same(pa, pb)
        _eager_noise(ctx)
    g.close()
    for x in (pa, pb, sa, sb):
        x.close()


def test_memetic_generation_graph_matches_eager(ctx, B):
    c = Case(64, 6, seed=7)
    s = B.sched_mpr(ctx, alg=B.ALG_RAAR, G=3, R=2, j=3, j_er=2, j_end=0, j_eval=2, t_min=4, t_max=8,
                    gen_first=1, gen_count=1, init_error=1, beta=0.9, chi=0.5, sigma=2.0, sigma_end=0.5,
                    tau=0.1, tau_end=0.0667, c_p=0.6, c_w=0.4)
    sa, pa = c.population(ctx, memetic=True, seed=11)
    sb, pb = c.population(ctx, memetic=True, seed=11)
    g = pa.graph(s)
    for _ in range(3):
        g.launch()
        pb.run(s)
        _same(pa, pb)
        _same(pa, pb, children=True)
        assert [tuple(r.a for r in pa.xover())] == [tuple(r.a for r in pb.xover())]
        _eager_noise(ctx)
    g.close()
    for x in (pa, pb, sa, sb):
        x.close()


def test_batch_graph_matches_eager_batch(ctx, B):
    cases = [Case(64, 3, seed=21), Case(32, 4, seed=22), Case(64, 2, seed=23)]
    s = B.sched_ops([B.op(B.OP_HIO, count=4, beta=0.9, chi=0.5), B.op(B.OP_SHRINKWRAP, sigma=1.0, tau=0.1),
                     B.op(B.OP_ER, count=2, chi=0.5), B.op(B.OP_GET_ERROR)], ctx)
    A = [c.population(ctx) for c in cases]
    Bp = [c.population(ctx) for c in cases]
    g = ctx.graph_batch([p for _, p in A], [s] * len(A))
    for _ in range(3):
        g.launch()
        ctx.run_batch([p for _, p in Bp], [s] * len(Bp))
        for (_, pa), (_, pb) in zip(A, Bp):
            _same(pa, pb)
        _eager_noise(ctx)
    g.close()
    for sh, p in A + Bp:
        p.close()
        sh.close()


def test_population_with_graph_cannot_be_destroyed(ctx, B):
    c = Case(32, 2, seed=3)
    sh, pop = c.population(ctx)
    g = pop.graph(B.sched_ops([B.op(B.OP_ER, count=1)], ctx))
    assert ctx.lib.spr_pop_destroy(pop.h) == B.E_BUSY
    g.close()
    pop.close()
    sh.close()
