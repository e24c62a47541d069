"""Pins of the oracle's vectorised Philox and of the random-phase start."""

import numpy as np

from oracle import mpr, philox


def test_vectorised_philox_matches_scalar_rounds():
    rng = np.random.default_rng(5)
    c = rng.integers(0, 2**32, size=(4, 64), dtype=np.uint64)
    key = (0x9A3F17C2, 0x01234567)
    out = philox.philox4x32_10_array(c[0], c[1], c[2], c[3], key)
    for i in range(64):
        ref = philox.philox4x32_10(tuple(int(v) for v in c[:, i]), key)
        assert [int(o[i]) for o in out] == ref


def test_vectorised_philox_known_answers():
    # the same Random123 known-answer vectors that pin the scalar rounds
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.txt")
    rows = [l.split() for l in open(path) if l.strip() and not l.startswith("#")]
    for r in rows:
        v = [int(x, 16) for x in r]
        ctr, key, exp = v[0:4], v[4:6], v[6:10]
        out = philox.philox4x32_10_array(*[np.array([x], dtype=np.uint64) for x in ctr], key)
        assert [int(o[0]) for o in out] == exp


def test_draws_array_follows_the_draw_convention():
    d = philox.draws_array(2**40 + 17, philox.PURPOSE_INIT, 0, 5, 23)
    assert [int(x) for x in d] == [philox.draw(2**40 + 17, philox.PURPOSE_INIT, 0, 5, i) for i in range(23)]


def _shot(n, seed=3):
    rng = np.random.default_rng(seed)
    M = np.abs(rng.standard_normal((n, n))) + 0.1
    known = np.ones((n, n), bool)
    known[:3, :3] = False
    known[-2:, :] = False
    return M, known


def test_random_phase_start_has_measured_modulus():
    M, known = _shot(24)
    x0 = mpr.random_phase_start(M, known, 3, seed=11)
    for p in range(3):
        X = mpr.fft2(x0[p])
        assert np.allclose(np.abs(X)[known], M[known], rtol=1e-12, atol=1e-12)
        assert np.abs(X[~known]).max() < 1e-12
        # a point of the modulus set is left unchanged by P_M
        assert np.allclose(mpr.proj_modulus(x0[p], M, known), x0[p], atol=1e-12)


def test_random_phase_start_phases_uniform_and_member_distinct():
    n = 64
    M = np.ones((n, n))
    known = np.ones((n, n), bool)
    x0 = mpr.random_phase_start(M, known, 2, seed=7)
    ph = np.angle(mpr.fft2(x0[0])).ravel() % (2 * np.pi)
    hist, _ = np.histogram(ph, bins=16, range=(0, 2 * np.pi))
    exp = ph.size / 16
    chi2 = float(((hist - exp) ** 2 / exp).sum())
    assert chi2 < 37.7  # 99.9% quantile of chi^2 with 15 degrees of freedom
    assert not np.allclose(x0[0], x0[1])
    again = mpr.random_phase_start(M, known, 2, seed=7)
    np.testing.assert_array_equal(again, x0)
    other = mpr.random_phase_start(M, known, 1, seed=8)
    assert not np.allclose(other[0], x0[0])


def test_random_phase_start_angle_matches_the_generator():
    # at one known pixel the phase is the generator's draw mapped to [0, 2 pi)
    M, known = _shot(16)
    x0 = mpr.random_phase_start(M, known, 2, seed=99)
    X = mpr.fft2(x0[1])
    k = 5 * 16 + 9
    u = philox.draw(99, philox.PURPOSE_INIT, 0, 1, k)
    phi = 2 * np.pi * (u + 0.5) / 2**32
    assert abs(np.exp(1j * np.angle(X.ravel()[k])) - np.exp(1j * phi)) < 1e-12


def test_fp16_modulus_scale_and_rounding_bound():
    rng = np.random.default_rng(9)
    M = rng.uniform(0.0, 3.0e5, size=(32, 32))
    known = rng.random((32, 32)) > 0.1
    Mq, s = mpr.fp16_modulus(M, known)
    assert np.log2(s) == int(np.log2(s))           # a power of two
    top = M[known].max() / s
    assert 2.0 ** 13 <= top <= 2.0 ** 14            # largest value in the top binade
    k = known & (M / s >= 2.0 ** -14)               # normal FP16 range
    assert np.all(np.abs(Mq[k] - M[k]) <= 2.0 ** -11 * M[k])   # half-ulp bound of 11-bit significands
    assert np.array_equal(Mq[~known], M[~known])


def test_fp16_modulus_exact_values_unchanged():
    # integers below 2^11 times a power of two are FP16 numbers
    M = np.arange(64, dtype=np.float64).reshape(8, 8) * 16.0
    M[0, 0] = 2.0 ** 14 * 16.0 / 2.0        # largest value 2^17 -> s = 2^3
    known = np.ones((8, 8), bool)
    Mq, s = mpr.fp16_modulus(M, known)
    assert s == 8.0
    np.testing.assert_array_equal(Mq, M)


def test_fp16_modulus_rounds_ties_to_even():
    # with s = 1: 2049 lies halfway between 2048 and 2050 -> 2048 (even significand)
    M = np.array([[2.0 ** 14, 2049.0], [2051.0, 1.0]])
    Mq, s = mpr.fp16_modulus(M, np.ones((2, 2), bool))
    assert s == 1.0
    assert Mq[0, 1] == 2048.0 and Mq[1, 0] == 2052.0 and Mq[1, 1] == 1.0


def test_sphere_start_single_centred_sphere_closed_form():
    n = 32
    M = np.abs(np.random.default_rng(1).standard_normal((n, n))) + 0.5
    known = np.ones((n, n), bool)
    known[:2, :2] = False
    # one sphere whose diameter equals the square: centred, radius 6
    x0 = mpr.sphere_start(M, known, 1, seed=3, sigma_init=12, n_init=1, diam=(1.0, 1.0))[0]
    y, x = np.mgrid[0:n, 0:n] - n / 2.0
    prof = 2 * np.sqrt(np.clip(36.0 - y ** 2 - x ** 2, 0, None))
    c = x0.real.max() / prof.max()
    np.testing.assert_allclose(x0, c * prof, atol=1e-12 * prof.max() * c)
    # Eq. norm: the known part of the Fourier power equals the known intensities
    assert abs(np.sum(np.abs(mpr.fft2(x0))[known] ** 2) - np.sum(M[known] ** 2)) < 1e-9 * np.sum(M[known] ** 2)


def test_sphere_start_square_phase_gamma():
    n = 48
    M = np.ones((n, n))
    known = np.ones((n, n), bool)
    xs = mpr.sphere_start(M, known, 3, seed=9, sigma_init=20, phase=(0.7, 0.7))
    y, x = np.mgrid[0:n, 0:n] - n / 2.0
    inside = (np.abs(y) <= 10) & (np.abs(x) <= 10)
    for x0 in xs:
        assert np.all(x0[~inside] == 0)                          # inside the sigma_init square
        nz = np.abs(x0) > 0
        np.testing.assert_allclose(np.angle(x0[nz]), 0.7)          # constant phase
    g1 = mpr.sphere_start(M, known, 1, seed=9, sigma_init=20, gamma=1.0)[0]
    g5 = mpr.sphere_start(M, known, 1, seed=9, sigma_init=20, gamma=0.5)[0]
    nz = np.abs(g1) > 0
    ratio = np.abs(g5[nz]) / np.sqrt(np.abs(g1[nz]))               # |rho|^0.5 up to one scale
    np.testing.assert_allclose(ratio, ratio[0], rtol=1e-10)
    assert not np.allclose(xs[0], xs[1])                           # members differ


def test_sphere_start_draw_mapping():
    n = 64
    M = np.ones((n, n))
    known = np.ones((n, n), bool)
    # one sphere of random diameter in [0.2, 0.9] x 30: its support width follows draw 0
    x0 = mpr.sphere_start(M, known, 1, seed=2024, sigma_init=30, n_init=1)[0]
    from oracle import philox
    u0 = philox.draw(2024, philox.PURPOSE_SPHERES, 0, 0, 0) / 2 ** 32
    D = (0.2 + 0.7 * u0) * 30
    rows = np.nonzero(np.abs(x0).sum(axis=1))[0]
    assert abs((rows[-1] - rows[0] + 1) - D) <= 2.0
