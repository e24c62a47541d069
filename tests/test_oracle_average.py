"""Pins of the population average (Eq. avgrec with aligned members) and of the
average-modulus crossover term (Eq. avgint1, Eq. avgint2, Eq. crossavg)."""

import numpy as np

from oracle import mpr


def _object(N, seed):
    rng = np.random.default_rng(seed)
    x = np.zeros((N, N), complex)
    x[5:13, 6:15] = rng.random((8, 9)) + 0.2
    return x


def test_average_of_shifted_twinned_phased_copies_is_the_object():
    N = 24
    x = _object(N, 1)
    S = np.abs(x) > 0
    known = np.ones((N, N), bool)
    copies, supps = [], []
    for (dr, dc), twin, ph in (((0, 0), False, 0.0), ((3, -2), False, 0.7), ((5, 4), True, -1.1),
                               ((-4, 7), True, 2.0)):
        y = np.conj(np.roll(x[::-1, ::-1], 1, axis=(0, 1))) if twin else x
        sy = np.roll(S[::-1, ::-1], 1, axis=(0, 1)) if twin else S
        copies.append(np.exp(1j * ph) * np.roll(y, (dr, dc), axis=(0, 1)))
        supps.append(np.roll(sy, (dr, dc), axis=(0, 1)))
    E = [0.1, 0.2, 0.3, 0.4]  # the unshifted copy is the reference
    avg = mpr.average(copies, supps, E, known)
    np.testing.assert_allclose(avg["rho"], x, atol=1e-12)
    np.testing.assert_array_equal(avg["S"], S)
    np.testing.assert_allclose(avg["Mdot"], avg["Mddot"], atol=1e-12)  # equal phases: equality


def test_average_of_one_member_is_the_member():
    N = 16
    x = _object(N, 2)[:N, :N]
    S = np.abs(x) > 0
    known = np.ones((N, N), bool)
    known[:2, :2] = False
    avg = mpr.average([x], [S], [0.5], known)
    np.testing.assert_allclose(avg["rho"], x, atol=1e-12)
    np.testing.assert_array_equal(avg["S"], S)


def test_average_moduli_ordering():
    rng = np.random.default_rng(4)
    N = 16
    xs = [rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N)) for _ in range(5)]
    Ss = [np.ones((N, N), bool)] * 5
    avg = mpr.average(xs, Ss, [0.3, 0.1, 0.5, 0.2, 0.4], np.ones((N, N), bool))
    assert avg["best"] == 1
    assert np.all(avg["Mdot"] <= avg["Mddot"] + 1e-12)  # triangle inequality (appendix on unconstrained modes)


def test_crossavg_limits():
    rng = np.random.default_rng(6)
    N = 8
    Xa = rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N))
    Mdot, Mddot = np.abs(rng.standard_normal((N, N))), np.abs(rng.standard_normal((N, N))) + 1
    np.testing.assert_allclose(mpr.mix_average_modulus(Xa, Mdot, Mddot, 0.0), Xa, rtol=1e-14)
    one = mpr.mix_average_modulus(Xa, Mdot, Mddot, 1.0)
    np.testing.assert_allclose(np.abs(one), 0.5 * (Mdot + Mddot))
    np.testing.assert_allclose(np.angle(one), np.angle(Xa))
    half = mpr.mix_average_modulus(Xa, Mdot, Mddot, 0.5)
    np.testing.assert_allclose(np.abs(half), 0.25 * (Mdot + Mddot) + 0.5 * np.abs(Xa))
    z = mpr.mix_average_modulus(np.zeros((N, N), complex), Mdot, Mddot, 0.4)
    np.testing.assert_allclose(z, 0.2 * (Mdot + Mddot))


def test_crossover_with_ca_zero_is_the_plain_crossover_and_ca_one_sets_the_modulus():
    rng = np.random.default_rng(11)
    N, P = 16, 5
    xs = [rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N)) for _ in range(P)]
    Ss = [rng.random((N, N)) > 0.3 for _ in range(P)]
    known = np.ones((N, N), bool)
    avg = mpr.average(xs, Ss, list(range(P)), known)
    a = mpr.crossover(xs, Ss, known, 2, 7, 0.6, 0.4, 4, 4)
    b = mpr.crossover(xs, Ss, known, 2, 7, 0.6, 0.4, 4, 4, c_a=0.0, avg=avg)
    for u, v in zip(a[0], b[0]):
        np.testing.assert_array_equal(u, v)
    # C_p = 1 (whole map), C_w = 0, C_a = 1: every child spectrum has the average modulus
    c = mpr.crossover(xs, Ss, known, 2, 7, 1.0, 0.0, 4, 4, c_a=1.0, avg=avg)
    for x in c[0]:
        np.testing.assert_allclose(np.abs(mpr.fft2(x)), 0.5 * (avg["Mdot"] + avg["Mddot"]), atol=1e-10)


def test_complexity_closed_forms():
    x = np.zeros((4, 4), complex)
    x[1, 1], x[2, 2] = 3.0, 1.0
    assert mpr.complexity(x) == 0.0                       # constant phase
    x[2, 2] = 1j * 3.0
    assert abs(mpr.complexity(x) - (1 - np.sqrt(18) / 6)) < 1e-15
    x[2, 2] = -3.0
    assert mpr.complexity(x) == 1.0                       # opposite phases cancel
    assert mpr.complexity(np.exp(0.4j) * np.abs(x)) < 1e-15  # global phase does not count


def test_monitor_statistics_by_hand():
    xs = [np.full((2, 2), 1.0 + 0j), np.full((2, 2), 3.0 + 0j), np.array([[1, -1], [1j, -1j]], complex)]
    m = mpr.monitors(xs, [0.3, 0.1, 0.2])
    assert m["err_best"] == 0.1 and m["err_median"] == 0.2 and m["err_worst"] == 0.3
    assert abs(m["err_mean"] - 0.2) < 1e-15
    sums = np.array([4.0, 12.0, 0.0])
    assert abs(m["sum_mean"] - sums.mean()) < 1e-12
    assert abs(m["sum_rel_std"] - sums.std() / sums.mean()) < 1e-12
    assert abs(m["gamma_mean"] - (0 + 0 + 1) / 3) < 1e-15
    m4 = mpr.monitors(xs + [xs[0]], [0.4, 0.1, 0.2, 0.3])
    assert m4["err_median"] == 0.2                          # lower of the two middle values
