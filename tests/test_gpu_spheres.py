"""Device sphere start (the paper's Initialize) against the oracle's."""

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


@pytest.mark.parametrize("n,P,sigma,n_init,phase,gamma,fp16", [
    (64, 3, 24.0, 5, (0.0, 0.0), 1.0, False),
    (128, 4, 50.0, 3, (-0.5, 0.5), 0.7, False),
    (96, 2, 40.0, 8, (0.0, 0.0), 1.5, True),
])
def test_sphere_start_matches_oracle(ctx, n, P, sigma, n_init, phase, gamma, fp16):
    c = Case(n, P, seed=n + 3, gap=4)
    sh = ctx.shot(c.amp32, c.mask8, fp16=fp16)
    pop = sh.population(c.rho32, c.supp8, seed=1234 + n, memetic=True)
    pop.init_spheres(sigma, n_init=n_init, phase=phase, gamma=gamma)
    rho, supp, _ = pop.read()
    M = mpr.fp16_modulus(c.M, c.known)[0] if fp16 else c.M
    ref = mpr.sphere_start(M, c.known, P, 1234 + n, sigma, n_init=n_init, phase=phase, gamma=gamma)
    for p in range(P):
        assert rel(rho[p], ref[p]) <= 1e-5
    y, x = np.mgrid[0:n, 0:n] - n / 2.0
    square = (np.abs(y) <= sigma / 2) & (np.abs(x) <= sigma / 2)
    for p in range(P):
        np.testing.assert_array_equal(supp[p], square)
    pop.close()
    sh.close()
