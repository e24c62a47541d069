"""Population average (aligned to the best member) and the average-modulus
crossover term against the oracle.  Members are translated, twinned and
phase-shifted copies of one object plus small noise, so that every alignment
is unambiguous and the comparison is element by element."""

import numpy as np
import pytest

from oracle import mpr
from paper_2409_07413_amd import synth

from gpu_cases import rel

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


def copies(n, P, seed):
    """A noiseless shot of a compact object and P transformed noisy copies."""
    kw = dict(count=8, radius=(0.02 * n, 0.06 * n), spread=0.05 * n, extent=0.3 * n)
    sh = synth.shot(n, "spheres", seed, 1e8, beamstop=max(2, n // 16), gap=2, noiseless=True, **kw)
    x = sh["obj"] * sh["scale"]
    S = mpr.smooth(x, 1.0) > 0.02 * x.max()
    rng = np.random.default_rng(seed)
    xs, Ss = [], []
    for p in range(P):
        twin = bool(p % 3 == 2)
        y = np.conj(np.roll(x[::-1, ::-1], 1, axis=(0, 1))) if twin else x.astype(complex)
        sy = np.roll(S[::-1, ::-1], 1, axis=(0, 1)) if twin else S
        d = tuple(int(v) for v in rng.integers(-n // 8, n // 8, size=2))
        ph = rng.uniform(-np.pi, np.pi)
        noise = 0.02 * x.max() * (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)))
        xs.append((np.exp(1j * ph) * np.roll(y, d, axis=(0, 1)) + noise).astype(np.complex64))
        Ss.append(np.roll(sy, d, axis=(0, 1)))
    amp = sh["amp"].astype(np.float32)
    mask = sh["mask"].astype(np.uint8)
    return amp, mask, np.stack(xs), np.stack(Ss)


AVG_CASES = [(64, 5, 0), (128, 6, 0), (256, 4, 0), (384, 4, 0), (512, 4, 0), (768, 4, 0), (1024, 4, 0),
             (256, 4, 1), (384, 4, 1), (512, 4, 1), (768, 4, 1), (1024, 4, 1)]


@pytest.mark.parametrize("n,P,variant", AVG_CASES)
def test_average_matches_oracle(ctx, B, n, P, variant):
    # every size on both plans of the tuned sizes: Reshift to the best member
    # (correlations, argmax, alignment), the average spectra and support
    amp, mask, xs, Ss = copies(n, P, seed=n + 7 * variant)
    M = mpr.to_fft_order(amp.astype(np.float64))
    known = mpr.to_fft_order(mask.astype(bool))
    if variant:
        ctx.set_variant(n, variant)
    try:
        sh = ctx.shot(amp, mask)
        pop = sh.population(xs, Ss.astype(np.uint8))
        pop.run(B.sched_ops([B.op(B.OP_GET_ERROR), B.op(B.OP_AVERAGE, scope=B.SCOPE_PARENTS)], ctx))
        rho, supp, e_avg = pop.average()
        err = pop.errors()
    finally:
        if variant:
            ctx.set_variant(n, 0)
    x64 = [x.astype(np.complex128) for x in xs]
    E = [mpr.get_error(x, S, M, known) for x, S in zip(x64, Ss)]
    assert int(np.argmin(err)) == int(np.argmin(E))
    ref = mpr.average(x64, list(Ss), E, known)
    assert rel(rho, ref["rho"]) <= 1e-5
    np.testing.assert_array_equal(supp, ref["S"])
    e_ref = mpr.get_error(ref["rho"], ref["S"], M, known)
    assert abs(e_avg - e_ref) <= 1e-5 * e_ref
    pop.close()
    sh.close()


def test_crossover_with_average_modulus_matches_oracle(ctx, B):
    n, P, seed = 64, 6, 41
    amp, mask, xs, Ss = copies(n, P, seed=7)
    M = mpr.to_fft_order(amp.astype(np.float64))
    known = mpr.to_fft_order(mask.astype(bool))
    sh = ctx.shot(amp, mask)
    pop = sh.population(xs, Ss.astype(np.uint8), memetic=True, seed=seed)
    ops = [B.op(B.OP_GET_ERROR, scope=B.SCOPE_PARENTS), B.op(B.OP_AVERAGE, scope=B.SCOPE_PARENTS),
           B.op(B.OP_CROSSOVER, gen=1, c_p=0.6, c_w=0.4, c_a=0.5, t_min=4, t_max=8)]
    pop.run(B.sched_ops(ops, ctx))
    kids, ksupp, _ = pop.read(children=True)
    x64 = [x.astype(np.complex128) for x in xs]
    E = [mpr.get_error(x, S, M, known) for x, S in zip(x64, Ss)]
    avg = mpr.average(x64, list(Ss), E, known)
    kx, kS, _ = mpr.crossover(x64, list(Ss), known, 1, seed, 0.6, 0.4, 4, 8, c_a=0.5, avg=avg)
    for p in range(P):
        assert rel(kids[p], kx[p]) <= 1e-5
        np.testing.assert_array_equal(ksupp[p], kS[p])
    pop.close()
    sh.close()


def test_crossover_with_ca_needs_an_average(ctx, B):
    amp, mask, xs, Ss = copies(32, 4, seed=3)
    sh = ctx.shot(amp, mask)
    pop = sh.population(xs, Ss.astype(np.uint8), memetic=True, seed=1)
    with pytest.raises(B.SprError):
        pop.run(B.sched_ops([B.op(B.OP_CROSSOVER, gen=1, c_p=0.6, c_w=0.4, c_a=0.5, t_min=4, t_max=4)], ctx))
    with pytest.raises(B.SprError):
        pop.average()
    pop.close()
    sh.close()
