"""CPU checks of the step-chained parity helper (tests/chained.py): its HIO
step is the oracle's HIO wherever the band rule takes no decision, a device
output with a flipped decision outside the band is caught, and the step
list and cut schedules follow the op list."""

import numpy as np

from oracle import mpr
from paper_2409_07413_amd import synth

import chained


def _case(n=32, seed=3):
    sh = synth.shot(n, "ellipses", seed, 1e6, beamstop=4, count=3, semi=(2.0, 5.0), disk_diameter=14.0)
    M = mpr.to_fft_order(sh["amp"])
    known = mpr.to_fft_order(sh["mask"])
    x = synth.random_phase_starts(sh["amp"], sh["mask"], 1, seed + 1)[0]
    S = synth.centred_square(n, 16).astype(bool)
    return x, S, M, known


def test_banded_hio_is_the_oracle_step():
    x, S, M, known = _case()
    for chi in (0.5, 0.3, 1.0):
        ref = mpr.hio(x, S, M, known, chi, 0.9)
        out, nb, hard = chained.hio_step_banded(x, ref, S, M, known, chi, 0.9)
        assert hard == 0
        np.testing.assert_array_equal(out, ref)
        if chi == 1.0:
            assert nb == 0


def test_banded_hio_catches_a_flipped_decision():
    x, S, M, known = _case()
    chi, beta = 0.5, 0.9
    ref = mpr.hio(x, S, M, known, chi, beta)
    y = mpr.proj_modulus(x, M, known)
    margin = chained.feasibility_margin(y, chi)
    # a pixel inside S whose decision is far from the band, flipped
    cand = np.argwhere(S & (np.abs(margin) > 1e-2 * np.abs(y).max()) &
                       (np.abs(x - (1 + beta) * y) > 1e-3 * np.abs(y).max()))
    i, j = cand[0]
    bad = ref.copy()
    bad[i, j] = y[i, j] if ref[i, j] != y[i, j] else x[i, j] - beta * y[i, j]
    _, _, hard = chained.hio_step_banded(x, bad, S, M, known, chi, beta)
    assert hard == 1
    # a pixel inside the band takes the device's decision and is counted
    k = np.unravel_index(np.argmin(np.where(S, np.abs(margin), np.inf)), margin.shape)
    wide = np.abs(margin[k]) / np.abs(y).max() * 1.01
    flipped = ref.copy()
    flipped[k] = y[k] if ref[k] != y[k] else x[k] - beta * y[k]
    out, nb, hard = chained.hio_step_banded(x, flipped, S, M, known, chi, beta, band=wide)
    assert hard == 0 and nb >= 1
    np.testing.assert_array_equal(out[k], flipped[k])


def test_steps_and_cuts_follow_the_op_list():
    from paper_2409_07413_amd import binding as B
    ops = [B.op(B.OP_RAAR, count=3, beta=0.9), B.op(B.OP_SHRINKWRAP, sigma=2.0, tau=0.1),
           B.op(B.OP_ER, count=2), B.op(B.OP_GET_ERROR)]
    assert chained.steps(ops) == [(0, 1), (0, 2), (0, 3), (1, None), (2, 1), (2, 2), (3, None)]
    sub = chained.cut(B, ops, 2, 1)
    assert [(o.kind, o.count) for o in sub] == [(B.OP_RAAR, 3), (B.OP_SHRINKWRAP, 0), (B.OP_ER, 1)]
    assert sub[0].beta == 0.9 and sub[1].sigma == 2.0
    assert chained.cut(B, ops, -1, None) == []
