"""Pins of the per-iteration Fourier-error trace of the oracle."""

import numpy as np

from oracle import mpr
from paper_2409_07413_amd import synth


def _shot(n=16, seed=3):
    rng = np.random.default_rng(seed)
    obj = np.zeros((n, n))
    obj[3:9, 4:10] = rng.uniform(0.5, 1.5, size=(6, 6))
    M = np.abs(mpr.fft2(obj))
    known = np.ones((n, n), bool)
    known[0, :2] = False
    known[-1, -1] = False
    S = np.zeros((n, n), bool)
    S[2:11, 3:12] = True
    return obj, M, known, S


def test_fourier_error_is_the_fitness_with_a_full_support():
    obj, M, known, S = _shot()
    x = np.random.default_rng(1).standard_normal(M.shape) + 1j * np.random.default_rng(2).standard_normal(M.shape)
    assert abs(mpr.fourier_error(x, M, known) - mpr.get_error(x, np.ones_like(S), M, known)) < 1e-14


def test_fourier_error_closed_forms():
    obj, M, known, S = _shot()
    assert mpr.fourier_error(np.zeros_like(M, dtype=complex), M, known) == 1.0  # |0 - M| / |M|
    assert mpr.fourier_error(obj, M, known) < 1e-13                         # the object itself
    x0 = synth.random_phase_starts(np.fft.fftshift(M), np.fft.fftshift(known), 1, 9)[0]  # modulus exact on Xi
    assert mpr.fourier_error(x0, M, known) < 1e-13
    assert abs(mpr.fourier_error(1.7 * obj, M, known) - 0.7) < 1e-12       # |c - 1| for F[x] = c M e^{i phi}


def test_trace_follows_the_sequence_and_er_does_not_increase():
    obj, M, known, S = _shot()
    x0 = synth.random_phase_starts(np.fft.fftshift(M), np.fft.fftshift(known), 1, 4)[0]
    x, errs = mpr.sequence_trace(x0, S, M, known, 0.5, "RAAR", 0.9, 3, 12)
    np.testing.assert_allclose(x, mpr.sequence(x0, S, M, known, 0.5, "RAAR", 0.9, 3, 12), rtol=0, atol=1e-13)
    assert len(errs) == 15
    assert errs[0] == mpr.fourier_error(x0, M, known)
    x3 = mpr.sequence(x0, S, M, known, 0.5, "RAAR", 0.9, 3, 0)
    assert errs[3] == mpr.fourier_error(mpr.proj_constraint(x3, S, 0.5), M, known)
    # alternating projections: the distance of P_C x to the modulus set never grows
    er = errs[3:]
    assert all(b <= a + 1e-12 for a, b in zip(er, er[1:]))
