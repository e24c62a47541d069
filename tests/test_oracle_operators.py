"""Pins of the oracle's operators against brute force, closed forms and invariants.

Nothing here re-types an oracle formula: each check uses a definition written
differently (explicit sums, geometry, algebraic identities of the method).
"""

import numpy as np
import pytest

from oracle import mpr
from paper_2409_07413_amd import synth


def brute_dft2(x, sign=-1):
    """Unitary 2D DFT as explicit sums over exp(sign 2 pi i (km + ln)/N)."""
    n = x.shape[0]
    out = np.zeros((n, n), dtype=np.complex128)
    for k in range(n):
        for l in range(n):
            acc = 0j
            for m in range(n):
                for q in range(n):
                    acc += x[m, q] * np.exp(sign * 2j * np.pi * (k * m + l * q) / n)
            out[k, l] = acc / n
    return out


def dft_matrix(n, sign=-1):
    k = np.arange(n)
    return np.exp(sign * 2j * np.pi * np.outer(k, k) / n) / np.sqrt(n)


@pytest.mark.parametrize("n", [8])
def test_fft_matches_explicit_sums(n):
    x = synth.random_complex((n, n), 11)
    np.testing.assert_allclose(mpr.fft2(x), brute_dft2(x, -1), atol=1e-12)
    np.testing.assert_allclose(mpr.ifft2(x), brute_dft2(x, +1), atol=1e-12)


@pytest.mark.parametrize("n", [12, 16, 24, 32])
def test_fft_matches_dft_matrix(n):
    x = synth.random_complex((n, n), n)
    W = dft_matrix(n, -1)
    np.testing.assert_allclose(mpr.fft2(x), W @ x @ W.T, atol=1e-11)
    Wi = dft_matrix(n, +1)
    np.testing.assert_allclose(mpr.ifft2(x), Wi @ x @ Wi.T, atol=1e-11)


@pytest.mark.parametrize("n", [8, 24, 64])
def test_parseval_and_inverse(n):
    x = synth.random_complex((n, n), 3 * n)
    X = mpr.fft2(x)
    assert abs(np.sum(np.abs(x) ** 2) - np.sum(np.abs(X) ** 2)) < 1e-9 * np.sum(np.abs(x) ** 2)
    np.testing.assert_allclose(mpr.ifft2(X), x, atol=1e-12)


def test_fft_delta_and_shift():
    n = 16
    x = np.zeros((n, n), complex)
    x[0, 0] = 1.0
    np.testing.assert_allclose(mpr.fft2(x), np.full((n, n), 1.0 / n), atol=1e-14)
    # a unit impulse at (a, b) has spectrum exp(-2 pi i (k a + l b)/N)/N
    x[:] = 0
    x[3, 5] = 1.0
    k = np.arange(n)
    ref = np.exp(-2j * np.pi * (k[:, None] * 3 + k[None, :] * 5) / n) / n
    np.testing.assert_allclose(mpr.fft2(x), ref, atol=1e-14)


def _pattern(n=32, seed=5, gap=2, bs=4):
    obj = synth.ellipses(n, seed, count=3, semi=(2.0, 5.0), disk_diameter=14.0)
    amp, scale = synth.diffraction(obj, 1e6, seed=seed, noiseless=True)
    mask = synth.beamstop_gap_mask(n, bs, gap)
    M = mpr.to_fft_order(amp)
    known = mpr.to_fft_order(mask)
    return obj * scale, M, known


def test_modulus_projector_properties():
    _, M, known = _pattern()
    n = M.shape[0]
    x = synth.random_complex((n, n), 17)
    y = mpr.proj_modulus(x, M, known)
    Y = mpr.fft2(y)
    X = mpr.fft2(x)
    # measured pixels carry exactly the measured modulus, others are untouched
    np.testing.assert_allclose(np.abs(Y[known]), M[known], rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(Y[~known], X[~known], atol=1e-12)
    # phases are kept where |X| > 0
    ph = np.angle(Y[known] * np.conj(X[known]))
    assert np.max(np.abs(ph)) < 1e-9
    # projector: applying twice changes nothing
    np.testing.assert_allclose(mpr.proj_modulus(y, M, known), y, atol=1e-12)
    # nearest point: the distance moved equals the modulus residual on known pixels
    dist = np.linalg.norm(x - y)
    res = np.sqrt(np.sum((np.abs(X[known]) - M[known]) ** 2))
    assert abs(dist - res) < 1e-10 * res


def test_modulus_projector_is_nearest_point_per_pixel():
    # brute force: among points of modulus M on a fine phase grid none is closer
    rng = np.random.default_rng(2)
    for _ in range(50):
        X = complex(*rng.standard_normal(2))
        Mv = abs(rng.standard_normal())
        got = mpr.modulus_fourier(np.array([X]), np.array([Mv]), np.array([True]))[0]
        ph = np.linspace(0, 2 * np.pi, 20001)
        best = np.min(np.abs(Mv * np.exp(1j * ph) - X))
        assert abs(got - X) <= best + 1e-6
    # zero spectrum value -> the measured modulus with phase 0
    got = mpr.modulus_fourier(np.array([0j]), np.array([2.5]), np.array([True]))[0]
    assert got == 2.5 + 0j


@pytest.mark.parametrize("chi", [0.1, 0.25, 0.5, 0.7, 0.9])
def test_phase_projection_nearest_point(chi):
    rng = np.random.default_rng(int(chi * 100))
    z = rng.standard_normal(400) + 1j * rng.standard_normal(400)
    p = mpr.proj_phase(z, chi)
    # allowed set sampled on a polar grid: rays at angles in [-chi pi, chi pi]
    ang = np.linspace(-chi * np.pi, chi * np.pi, 721)
    rad = np.linspace(0, 4, 801)
    pts = (rad[:, None] * np.exp(1j * ang[None, :])).ravel()
    for zi, pi in zip(z, p):
        # result lies in the set
        assert abs(np.angle(pi)) <= chi * np.pi + 1e-12 or abs(pi) < 1e-15
        best = np.min(np.abs(pts - zi))
        assert abs(pi - zi) <= best + 1e-9
    # idempotent
    np.testing.assert_allclose(mpr.proj_phase(p, chi), p, atol=1e-14)


def test_phase_projection_special_cases():
    z = np.array([1 + 1j, -1 + 2j, -3 - 1j, 2 - 5j])
    np.testing.assert_array_equal(mpr.proj_phase(z, 1.0), z)
    np.testing.assert_array_equal(mpr.proj_phase(z, 0.0), z)
    np.testing.assert_array_equal(mpr.proj_phase(z, 0.5), np.array([1 + 1j, 2j, -1j, 2 - 5j]))


def test_support_projector_idempotent():
    n = 16
    x = synth.random_complex((n, n), 4)
    S = synth.centred_square(n, 6)
    for chi in (1.0, 0.5, 0.3):
        y = mpr.proj_constraint(x, S, chi)
        assert np.all(y[~S] == 0)
        np.testing.assert_allclose(mpr.proj_constraint(y, S, chi), y, atol=1e-15)
    np.testing.assert_array_equal(mpr.proj_constraint(x, S, 1.0), np.where(S, x, 0))


def test_true_object_is_fixed_point_with_zero_error():
    rho, M, known = _pattern()
    n = M.shape[0]
    S = np.abs(rho) > 0
    x = rho.astype(complex)
    assert mpr.get_error(x, S, M, known) < 1e-12
    for chi in (1.0, 0.5):
        np.testing.assert_allclose(mpr.er(x, S, M, known, chi), x, atol=1e-10)
        np.testing.assert_allclose(mpr.hio(x, S, M, known, chi, 0.9), x, atol=1e-10)
        np.testing.assert_allclose(mpr.raar(x, S, M, known, chi, 0.9), x, atol=1e-10)
    # a larger support keeps the fixed point
    S2 = synth.centred_square(n, 20) | S
    np.testing.assert_allclose(mpr.er(x, S2, M, known, 0.5), x, atol=1e-10)


def test_er_monotone():
    rho, M, known = _pattern(seed=9)
    n = M.shape[0]
    S = synth.centred_square(n, 18)
    x = synth.random_phase_starts(np.fft.fftshift(M), np.fft.fftshift(known), 1, 3)[0]

    def dist_to_modulus(z):
        Z = np.fft.fft2(z, norm="ortho")
        return np.sqrt(np.sum((np.abs(Z[known]) - M[known]) ** 2))

    for chi in (1.0, 0.5):
        xk = x.copy()
        prev = np.inf
        prevE = np.inf
        for _ in range(30):
            xk = mpr.er(xk, S, M, known, chi)
            d = dist_to_modulus(mpr.proj_constraint(xk, S, chi))
            assert d <= prev * (1 + 1e-12) + 1e-12
            prev = d
            if chi == 1.0:   # then P_C = P_S and Eq. error_calc is the same distance
                E = mpr.get_error(xk, S, M, known)
                assert E <= prevE * (1 + 1e-12) + 1e-12
                prevE = E


def test_raar_equals_hio_at_beta_one_without_phase_constraint():
    rho, M, known = _pattern(seed=4)
    n = M.shape[0]
    S = synth.centred_square(n, 14)
    x = synth.random_complex((n, n), 8)
    np.testing.assert_allclose(mpr.raar(x, S, M, known, 1.0, 1.0),
                               mpr.hio(x, S, M, known, 1.0, 1.0), atol=1e-12)
    # and they differ for beta < 1 (the terms are not dropped)
    assert np.max(np.abs(mpr.raar(x, S, M, known, 1.0, 0.9) - mpr.hio(x, S, M, known, 1.0, 0.9))) > 1e-3


def test_hio_outside_support_is_x_minus_beta_y():
    rho, M, known = _pattern(seed=6)
    n = M.shape[0]
    S = synth.centred_square(n, 10)
    x = synth.random_complex((n, n), 1)
    y = mpr.proj_modulus(x, M, known)
    out = mpr.hio(x, S, M, known, 0.5, 0.7)
    np.testing.assert_allclose(out[~S], (x - 0.7 * y)[~S], atol=1e-13)
    inside = S & (y.real >= 0)
    np.testing.assert_allclose(out[inside], y[inside], atol=1e-13)
    neg = S & (y.real < 0)
    np.testing.assert_allclose(out[neg], (x - 0.7 * y)[neg], atol=1e-13)


def brute_error(x, S, M, known):
    n = x.shape[0]
    X = brute_dft2(np.where(S, x, 0), -1)
    num = den = 0.0
    for i in range(n):
        for j in range(n):
            if known[i, j]:
                num += (abs(X[i, j]) - M[i, j]) ** 2
                den += M[i, j] ** 2
    return np.sqrt(num / den)


def test_error_bruteforce_8():
    n = 8
    x = synth.random_complex((n, n), 21)
    S = synth.centred_square(n, 4)
    M = np.abs(synth.random_complex((n, n), 22))
    known = synth.beamstop_gap_mask(n, 2, 0)
    assert abs(mpr.get_error(x, S, M, known) - brute_error(x, S, M, known)) < 1e-12


def test_error_invariances():
    rho, M, known = _pattern(seed=12)
    n = M.shape[0]
    x = synth.random_complex((n, n), 5)
    S = synth.centred_square(n, 12)
    e0 = mpr.get_error(x, S, M, known)
    # joint translation
    xs, Ss = np.roll(x, (3, -5), axis=(0, 1)), np.roll(S, (3, -5), axis=(0, 1))
    assert abs(mpr.get_error(xs, Ss, M, known) - e0) < 1e-12
    # global phase
    assert abs(mpr.get_error(np.exp(0.7j) * x, S, M, known) - e0) < 1e-12
    # twin: conj(x(-r)), support S(-r)
    xt = np.conj(np.roll(x[::-1, ::-1], 1, axis=(0, 1)))
    St = np.roll(S[::-1, ::-1], 1, axis=(0, 1))
    assert abs(mpr.get_error(xt, St, M, known) - e0) < 1e-12
    # a support change does change the error (support multiplies, term not dropped)
    assert abs(mpr.get_error(x, synth.centred_square(n, 8), M, known) - e0) > 1e-3


def brute_conv2(a, w):
    """Direct periodic 2D convolution with the outer-product kernel w w^T."""
    n = a.shape[0]
    r = (len(w) - 1) // 2
    out = np.zeros_like(a)
    for i in range(n):
        for j in range(n):
            acc = 0.0
            for p in range(-r, r + 1):
                for q in range(-r, r + 1):
                    acc += w[p + r] * w[q + r] * a[(i + p) % n, (j + q) % n]
            out[i, j] = acc
    return out


def test_smoothing_matches_direct_convolution():
    n = 24
    a = np.abs(synth.random_complex((n, n), 31))
    for sigma in (0.8, 2.0):
        w = np.exp(-np.arange(-int(np.ceil(4 * sigma)), int(np.ceil(4 * sigma)) + 1) ** 2
                   / (2 * sigma ** 2))
        w /= w.sum()
        np.testing.assert_allclose(mpr.smooth(a, sigma), brute_conv2(a, w), rtol=1e-12)
    np.testing.assert_array_equal(mpr.smooth(a, 0.0), a)
    assert len(mpr.gauss_taps(2.0)) == 17


def test_update_support_threshold():
    n = 32
    x = synth.random_complex((n, n), 41) * synth.centred_square(n, 10)
    S0 = np.zeros((n, n), bool)
    # sigma = 0 and a tiny tau keep exactly the non-zero pixels
    np.testing.assert_array_equal(mpr.update_support(x, S0, 0.0, 1e-12), np.abs(x) > 0)
    # tau = 0.5 without smoothing: strict comparison against half the maximum
    a = np.abs(x)
    np.testing.assert_array_equal(mpr.update_support(x, S0, 0.0, 0.5), a > 0.5 * a.max())
    # zero density leaves the support unchanged
    S1 = synth.centred_square(n, 4)
    np.testing.assert_array_equal(mpr.update_support(np.zeros((n, n), complex), S1, 2.0, 0.1), S1)


def test_support_area_count_rounds_half_up_and_clamps():
    # round(alpha) with halves rounded up, at least one pixel, at most N^2
    assert mpr.area_count(2.5, 100) == 3
    assert mpr.area_count(2.499, 100) == 2
    assert mpr.area_count(3.0, 100) == 3
    assert mpr.area_count(0.4, 100) == 1
    assert mpr.area_count(-7.0, 100) == 1
    assert mpr.area_count(99.5, 100) == 100
    assert mpr.area_count(1e9, 100) == 100


def test_update_support_size_exact_topk_with_index_ties():
    n = 16
    rng = np.random.default_rng(0)
    # heavy ties: few distinct values
    x = rng.integers(0, 5, size=(n, n)).astype(complex)
    for alpha in (1.0, 17.4, 17.5, 100.0, 255.6, 1000.0):
        S = mpr.update_support_size(x, 0.0, alpha)
        k = min(max(int(np.floor(alpha + 0.5)), 1), n * n)
        assert S.sum() == k
        # brute force: sort (value desc, index asc)
        flat = np.abs(x).ravel()
        pairs = sorted(range(n * n), key=lambda i: (-flat[i], i))
        ref = np.zeros(n * n, bool)
        ref[pairs[:k]] = True
        np.testing.assert_array_equal(S.ravel(), ref)
    # nesting S(k) subset of S(k+1)
    y = synth.random_complex((n, n), 3)
    prev = mpr.update_support_size(y, 1.0, 10)
    for k in range(11, 40):
        cur = mpr.update_support_size(y, 1.0, k)
        assert np.all(cur[prev])
        prev = cur


def test_schedule_endpoints():
    for G in (1, 2, 10, 100):
        j1, e1, s1, t1 = mpr.schedule_at(1, G, 40, 40, 0, 2.0, 0.5, 0.1, 0.1 * 2 / 3)
        assert (j1, e1, s1, t1) == (40, 40, 2.0, 0.1)
        jG, eG, sG, tG = mpr.schedule_at(G, G, 40, 40, 0, 2.0, 0.5, 0.1, 0.1 * 2 / 3)
        if G > 1:
            assert jG == 0 and eG == 80 and abs(sG - 0.5) < 1e-15 and abs(tG - 0.1 * 2 / 3) < 1e-15
        for g in range(1, G + 1):
            jg, eg, _, _ = mpr.schedule_at(g, G, 40, 40, 0, 2.0, 0.5, 0.1, 0.1)
            assert jg + eg == 80 and 0 <= jg <= 40
    # config-1 style decay 16 -> 0 in 10 blocks
    js = [mpr.schedule_at(g, 10, 16, 4, 0, 2, 1, 0.1, 0.1)[0] for g in range(1, 11)]
    assert js == [int(np.floor(16 * (1 - b / 9) + 0.5)) for b in range(10)]


def test_generation_stats_bruteforce():
    n = 8
    Ss = [np.zeros((n, n), bool) for _ in range(4)]
    Ss[0][0, :3] = True
    Ss[1][1, :5] = True
    Ss[2][0, :2] = True
    Ss[3][7, 7] = True
    E = [0.3, 0.2, 0.2, 0.5]      # tie between 1 and 2 -> lowest index 1
    st = mpr.generation_stats(E, Ss, 3, 10)
    assert st["best"] == 1 and st["alpha_best"] == 5
    assert st["alpha_all"] == 3 + 5 + 1      # union: row0 cols0-2, row1 cols0-4, (7,7)
    assert abs(st["alpha_eval"] - (0.3 * 5 + 0.7 * 9)) < 1e-12
    assert mpr.generation_stats(E, Ss, 10, 10)["alpha_eval"] == 5
    assert abs(st["oversampling"] - 64 / 5) < 1e-12
