"""Pins of the upper-bound modulus projector (appendix on missing intensities,
Eq. avgint, Eq. stdint, Eq. upperbound, Eq. pm_bounds)."""

import numpy as np

from oracle import mpr


def test_radial_bins_values():
    b = mpr.radial_bins(8)
    assert b[0, 0] == 0 and b[0, 3] == 3 and b[3, 4] == 5 and b[4, 4] == 6
    assert b[0, 7] == 1 and b[7, 7] == 1  # signed frequency -1
    np.testing.assert_array_equal(b, b.T)


def _ring(N, q):
    return mpr.radial_bins(N) == q


def test_bound_of_a_constant_ring_is_its_amplitude():
    N = 16
    M = np.full((N, N), 3.0)
    known = np.ones((N, N), bool)
    ring = _ring(N, 5)
    idx = np.argwhere(ring)
    known[tuple(idx[0])] = False  # one unknown pixel out of many
    U = mpr.upper_bounds(M, known, eta=1.5)
    assert U[tuple(idx[0])] == 3.0  # sigma = 0: the bound is sqrt(mu) = M
    assert np.isnan(U[known]).all()


def test_bound_closed_form_two_values():
    # ring with known intensities {1, 4} in equal numbers: mu = 2.5, sigma = 1.5
    N = 32
    ring = _ring(N, 9)
    pix = np.argwhere(ring)
    M = np.zeros((N, N))
    known = np.ones((N, N), bool)
    for k, (i, j) in enumerate(pix):
        M[i, j] = 1.0 if k % 2 == 0 else 2.0
    # one unknown pair keeps the ring balanced
    known[tuple(pix[0])] = False
    known[tuple(pix[1])] = False
    U = mpr.upper_bounds(M, known, eta=1.5)
    assert abs(U[tuple(pix[0])] - np.sqrt(2.5 + 1.5 * 1.5)) < 1e-12


def test_bound_needs_eighty_percent_known():
    N = 32
    ring = _ring(N, 10)
    pix = np.argwhere(ring)
    M = np.ones((N, N))
    kmax = int(np.floor(0.2 * len(pix)))  # most unknown pixels a bounded ring may have
    for k, has in ((kmax, True), (kmax + 1, False)):
        known = np.ones((N, N), bool)
        for i, j in pix[:k]:
            known[i, j] = False
        U = mpr.upper_bounds(M, known)
        assert bool(np.isfinite(U[tuple(pix[0])])) == has


def test_saturated_pixels_get_no_bound():
    # constant ring (bound = M): the unknown pixels that are saturated get no
    # bound, the other unknown pixels keep theirs; no mask means no saturation
    N = 32
    pix = np.argwhere(_ring(N, 10))
    M = np.full((N, N), 2.0)
    known = np.ones((N, N), bool)
    for i, j in pix[:4]:
        known[i, j] = False
    sat = np.zeros((N, N), bool)
    sat[tuple(pix[0])] = True  # 1 of the ring's pixels: below 5 %
    assert len(pix) > 20
    U = mpr.upper_bounds(M, known, saturated=sat)
    assert np.isnan(U[tuple(pix[0])])
    for i, j in pix[1:4]:
        assert U[i, j] == 2.0
    np.testing.assert_array_equal(mpr.upper_bounds(M, known, saturated=np.zeros((N, N), bool)),
                                  mpr.upper_bounds(M, known))


def test_ring_more_than_five_percent_saturated_gets_no_bound():
    N = 32
    pix = np.argwhere(_ring(N, 10))
    M = np.ones((N, N))
    smax = int(np.floor(0.05 * len(pix)))  # most saturated pixels a bounded ring may have
    assert smax >= 1
    for k, has in ((smax, True), (smax + 1, False)):
        known = np.ones((N, N), bool)
        sat = np.zeros((N, N), bool)
        for i, j in pix[:k]:
            known[i, j] = False
            sat[i, j] = True
        free = tuple(pix[k])  # an unknown pixel that is not saturated
        known[free] = False
        U = mpr.upper_bounds(M, known, saturated=sat)
        assert bool(np.isfinite(U[free])) == has
        # the threshold follows max_saturated
        U0 = mpr.upper_bounds(M, known, saturated=sat, max_saturated=0.0)
        assert np.isnan(U0[free])
    # other rings are untouched by the saturated pixels of ring 10
    other = tuple(np.argwhere(_ring(N, 6))[0])
    known = np.ones((N, N), bool)
    known[other] = False
    sat = np.zeros((N, N), bool)
    for i, j in pix[:smax + 1]:
        known[i, j] = False
        sat[i, j] = True
    assert mpr.upper_bounds(M, known, saturated=sat)[other] == 1.0


def test_saturated_pixel_must_be_unknown():
    N = 16
    known = np.ones((N, N), bool)
    sat = np.zeros((N, N), bool)
    sat[3, 4] = True
    try:
        mpr.upper_bounds(np.ones((N, N)), known, saturated=sat)
    except ValueError:
        return
    raise AssertionError("a known saturated pixel was accepted")


def test_bounded_projector_properties():
    rng = np.random.default_rng(3)
    N = 24
    X = rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N))
    M = np.abs(rng.standard_normal((N, N)))
    known = rng.random((N, N)) > 0.3
    bound = np.where(known, np.nan, np.where(rng.random((N, N)) > 0.5, 0.8, np.nan))
    Y = mpr.modulus_fourier_bounded(X, M, known, bound)
    # known pixels: as Eq. pm_full
    np.testing.assert_allclose(Y[known], mpr.modulus_fourier(X, M, known)[known])
    b = np.isfinite(bound)
    assert np.all(np.abs(Y[b]) <= 0.8 + 1e-12)
    inside = b & (np.abs(X) <= 0.8)
    np.testing.assert_array_equal(Y[inside], X[inside])
    free = ~known & ~b
    np.testing.assert_array_equal(Y[free], X[free])
    # idempotent
    np.testing.assert_allclose(mpr.modulus_fourier_bounded(Y, M, known, bound), Y, atol=1e-12)
    # nearest point of the disc |z| <= b, by brute force on a polar grid
    z = X[b & (np.abs(X) > 0.8)][:5]
    r = np.linspace(0, 0.8, 161)
    th = np.linspace(-np.pi, np.pi, 2049)
    grid = (r[:, None] * np.exp(1j * th[None, :])).ravel()
    for zz, yy in zip(z, Y[b & (np.abs(X) > 0.8)][:5]):
        d = np.abs(grid - zz).min()
        assert abs(abs(zz - yy) - d) < 2e-3
    # no bounds: the plain projector
    none = np.full((N, N), np.nan)
    np.testing.assert_array_equal(mpr.modulus_fourier_bounded(X, M, known, none), mpr.modulus_fourier(X, M, known))


def test_true_object_is_a_fixed_point_with_bounds():
    # noiseless pattern with a gap: the true object satisfies every bound that
    # its own unknown amplitudes satisfy, so it stays a fixed point
    rng = np.random.default_rng(8)
    N = 32
    x = np.zeros((N, N))
    x[12:20, 10:22] = rng.random((8, 12))
    S = x > 0
    X = mpr.fft2(x)
    M = np.abs(X)
    known = np.ones((N, N), bool)
    known[:, 14:18] = False
    U = mpr.upper_bounds(M, known, eta=50.0)
    ok = ~np.isfinite(U) | (M <= U)
    U = np.where(ok, U, np.nan)
    for f in (lambda z: mpr.er(z, S, M, known, 0.5, bound=U),
              lambda z: mpr.hio(z, S, M, known, 0.5, 0.9, bound=U),
              lambda z: mpr.raar(z, S, M, known, 0.5, 0.9, bound=U)):
        np.testing.assert_allclose(f(x.astype(complex)), x, atol=1e-12)
