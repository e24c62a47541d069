"""The method at work: on a noiseless, fully measured 128 x 128 shot, MPR with
the paper's default operators (RAAR beta 0.9 and ER, shrink-wrap, crossover
C_p 0.6 / C_w 0.4, selection) recovers the object up to the trivial
ambiguities of phase retrieval (translation, twin, global phase).  This is a
functional check of the whole pipeline, not parity: phase retrieval from
random starts can stagnate, so the bounds leave a margin of about two over
the values this fixed-seed run reaches (fitness 0.012, aligned distance 0.12)."""

import numpy as np
import pytest

from oracle import mpr

pytestmark = pytest.mark.gpu


def test_mpr_recovers_a_noiseless_object():
    from paper_2409_07413_amd import binding as B
    from paper_2409_07413_amd import synth
    n, P, G, seed = 128, 8, 10, 7
    sh = synth.shot(n, "ellipses", seed, 1e6, beamstop=0, noiseless=True, count=4, semi=(2.0, 0.09 * n),
                    disk_diameter=0.3 * n)
    obj = (sh["obj"] * sh["scale"]).astype(np.complex128)
    ctx = B.Context(0)
    try:
        shot = ctx.shot(sh["amp"].astype(np.float32), sh["mask"].astype(np.uint8))
        pop = shot.population(None, synth.centred_square(n, int(0.45 * n)).astype(np.uint8), memetic=True,
                              seed=seed + 100, P=P)
        s = ctx.sched_mpr(alg=B.ALG_RAAR, G=G, R=3, j=16, j_er=4, j_end=0, j_eval=20, t_min=4, t_max=n // 8,
                          gen_first=1, gen_count=G, init_error=1, beta=0.9, chi=0.5, sigma=2.0, sigma_end=0.5,
                          tau=0.10, tau_end=0.10 * 2 / 3, c_p=0.6, c_w=0.4)
        pop.run(s)
        rho, supp, err = pop.read()
        pop.close()
        s.close()
        shot.close()
    finally:
        ctx.close()
    b = int(np.argmin(err))
    # align the best member to the object (shift, twin, global phase) with the
    # oracle's Reshift on the full Fourier domain
    X, _, _ = mpr.reshift(mpr.fft2(rho[b].astype(np.complex128)), supp[b].astype(bool), mpr.fft2(obj),
                          np.ones((n, n), bool))
    dist = np.linalg.norm(mpr.ifft2(X) - obj) / np.linalg.norm(obj)
    print(f"best fitness {err[b]:.4f}, aligned distance to the object {dist:.4f}")
    assert err[b] < 0.05
    assert dist < 0.3
