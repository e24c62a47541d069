"""Device-side random-phase start against the oracle (single operator: the
counter-driven phases and one unitary inverse 2D DFT)."""

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


@pytest.mark.parametrize("n,P,seed", [(12, 3, 5), (64, 4, 2**33 + 7), (96, 2, 11), (256, 3, 123456789), (1024, 2, 77)])
def test_random_phase_start_matches_oracle(ctx, n, P, seed):
    c = Case(n, 1, seed=n)
    sh = c.shot(ctx)
    pop = sh.population(None, c.supp8[0], seed=seed, P=P)
    rho, supp, err = pop.read()
    ref = mpr.random_phase_start(c.M, c.known, P, seed)
    for p in range(P):
        assert rel(rho[p], ref[p]) <= 1e-5, (n, p)
    np.testing.assert_array_equal(supp, np.broadcast_to(c.S[0], supp.shape))
    pop.close()
    sh.close()
