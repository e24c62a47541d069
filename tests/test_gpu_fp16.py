"""FP16 storage of the measured modulus: the device path against the oracle
given the same stored values (the FP32 single-operator bar), and against the
oracle with the exact modulus (bounded by the FP16 rounding of M)."""

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


@pytest.mark.parametrize("n", [32, 128, 384, 512, 1024])
def test_fp16_single_iteration_and_error(ctx, B, n):
    c = Case(n, 3, seed=n + 5, photons=1e8)
    Mq, s = mpr.fp16_modulus(c.M, c.known)
    sh = ctx.shot(c.amp32, c.mask8, fp16=True)
    pop = sh.population(c.rho32, c.supp8)
    pop.run(B.sched_ops([B.op(B.OP_RAAR, count=1, beta=0.9, chi=0.5), B.op(B.OP_GET_ERROR)], ctx))
    rho, _, err = pop.read()
    for p in range(c.P):
        ref_q = mpr.raar(c.rho[p], c.S[p], Mq, c.known, 0.5, 0.9)
        ref = mpr.raar(c.rho[p], c.S[p], c.M, c.known, 0.5, 0.9)
        assert rel(rho[p], ref_q) <= 1e-5
        assert rel(rho[p], ref) <= 1e-3  # FP16 rounding of M: at most 2^-11 relative per pixel
        e_q = mpr.get_error(ref_q, c.S[p], Mq, c.known)
        assert abs(err[p] - e_q) <= 1e-5 * e_q
    pop.close()
    sh.close()


def test_fp16_random_start_and_served_equal_population(ctx, B):
    n, P = 96, 3
    c = Case(n, P, seed=17)
    Mq, _ = mpr.fp16_modulus(c.M, c.known)
    sh = ctx.shot(c.amp32, c.mask8, fp16=True)
    pop = sh.population(None, c.supp8[0], seed=321, P=P)
    rho0, _, _ = pop.read()
    ref = mpr.random_phase_start(Mq, c.known, P, 321)
    for p in range(P):
        assert rel(rho0[p], ref[p]) <= 1e-5
    s = B.sched_plain(ctx, alg=B.ALG_HIO, G=2, j=5, j_er=3, j_end=0, beta=0.9, chi=0.5, sigma=2.0,
                      sigma_end=1.0, tau=0.1, tau_end=0.1)
    pop.run(s)
    rho_a, supp_a, err_a = pop.read()
    pop.close()
    sh.close()
    sv = B.Server(ctx, s, P=P, hbm_budget=1 << 30, max_shots=2, manual=True, all_members=True)
    t = sv.submit(c.amp32, c.mask8, c.supp8[0], seed=321, fp16=True)
    assert sv.drain(60.0)
    r = sv.poll(t)
    sv.close()
    np.testing.assert_array_equal(r["rho"], rho_a)
    np.testing.assert_array_equal(r["supp"], supp_a)
    np.testing.assert_array_equal(r["err"], err_a)
