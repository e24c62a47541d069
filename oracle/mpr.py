"""FP64 oracle of Memetic Phase Retrieval: operators, memetic steps, drivers.

Test infrastructure only: a plain, slow reference for the HIP library.  Only
``tests/``, ``__graft_entry__.smoke()`` and ``bench.py``'s ``cpu_baseline`` leg
may import it.  Everything is NumPy complex128/float64; NumPy's FFT serves as
the library primitive for the discrete Fourier transform.

Conventions (shared with the GPU path by specification, not by code):

* Arrays are N x N.  Fourier-domain arrays (M, the mask, spectra) are in FFT
  order (zero frequency at [0, 0]); ``to_fft_order`` converts a detector-style
  centred image.  Real-space arrays use natural indices (origin at [0, 0]).
* ``known`` is the boolean mask Xi (True = measured) of the appendix on missing
  intensities.
* Supports are boolean N x N arrays.

Readings of passages that are silent or ambiguous are stated at each function;
the same list is kept in the design notes.
"""

import numpy as np

from . import philox

# ----------------------------------------------------------------------------
# Fourier transform (appendix "phase problem as an optimisation problem",
# Eq. pm; initialisation appendix, Parseval and Eq. norm)
# ----------------------------------------------------------------------------


def fft2(x):
    """Unitary forward 2D DFT, X[k,l] = N^-1 sum x[m,n] exp(-2 pi i (km+ln)/N).

    The paper fixes neither sign nor normalisation; it uses Parseval without
    factors (initialisation appendix), which reads as the unitary transform.
    """
    return np.fft.fft2(np.asarray(x, dtype=np.complex128), norm="ortho")


def ifft2(X):
    """Unitary inverse 2D DFT (exp(+2 pi i ...), factor 1/N)."""
    return np.fft.ifft2(np.asarray(X, dtype=np.complex128), norm="ortho")


def to_fft_order(img):
    """Centred detector layout (DC at [N/2, N/2]) -> FFT order (DC at [0, 0])."""
    return np.fft.ifftshift(np.asarray(img))


def sphere_start(M, known, P, seed, sigma_init, n_init=5, diam=(0.2, 0.9), phase=(0.0, 0.0), gamma=1.0):
    """The paper's Initialize (initialisation appendix): every member fills a
    centred sigma_init-wide square with n_init projected spheres (optical depth
    2 sqrt(R^2 - r^2)) of diameters in [diam[0], diam[1]] * sigma_init, each
    with a global phase in [phase[0], phase[1]]; the modulus of the sum is
    raised to gamma (phase kept) and the density is scaled by sqrt(nu), nu the
    ratio of Eq. norm (known intensities over the known part of |F[rho]|^2).

    Readings: sphere centres are uniform over the positions that keep the
    sphere inside the square (the centre of the square when it is narrower
    than the sphere), measured from the array centre (n/2, n/2); the random
    numbers are the shared generator's draws 4k..4k+3 of (seed, purpose 5,
    generation 0, member) for sphere k, mapped to [0, 1) as u / 2^32.
    """
    M = np.asarray(M, dtype=np.float64)
    n = M.shape[0]
    y, x = np.mgrid[0:n, 0:n].astype(np.float64)
    y -= n / 2.0
    x -= n / 2.0
    half = sigma_init / 2.0
    den = float(np.sum(M[known] ** 2))
    out = np.empty((P, n, n), dtype=np.complex128)
    for p in range(P):
        u = philox.draws_array(seed, philox.PURPOSE_SPHERES, 0, p, 4 * n_init).astype(np.float64) / 4294967296.0
        rho = np.zeros((n, n), dtype=np.complex128)
        for k in range(n_init):
            D = (diam[0] + (diam[1] - diam[0]) * u[4 * k]) * sigma_init
            R = D / 2.0
            cy = cx = 0.0
            if half > R:
                cy = -half + R + 2.0 * (half - R) * u[4 * k + 1]
                cx = -half + R + 2.0 * (half - R) * u[4 * k + 2]
            ph = phase[0] + (phase[1] - phase[0]) * u[4 * k + 3]
            r2 = (y - cy) ** 2 + (x - cx) ** 2
            rho = rho + 2.0 * np.sqrt(np.clip(R * R - r2, 0.0, None)) * np.exp(1j * ph)
        A = np.abs(rho)
        unit = np.where(A > 0, rho / np.where(A > 0, A, 1.0), 0.0)
        rho = A ** gamma * unit
        power = float(np.sum(np.abs(fft2(rho))[known] ** 2))
        out[p] = rho * np.sqrt(den / power) if power > 0 else rho
    return out


def fp16_modulus(M, known):
    """The measured modulus as the FP16 storage represents it.

    The paper fixes no storage precision.  The reading taken: the values kept
    are M / s rounded to the nearest FP16 number (ties to even), with s the
    power of two that puts the largest measured M / s in [2^13, 2^14]; the
    arithmetic then uses s * fp16(M / s) everywhere the modulus enters, the
    normaliser sum Xi M^2 of Eq. error_calc included.  Unknown pixels are
    irrelevant.  Returns (M_stored, s) in float64.
    """
    M = np.asarray(M, dtype=np.float64)
    mx = float(M[known].max()) if np.any(known) else 0.0
    s = 2.0 ** (int(np.ceil(np.log2(mx))) - 14) if mx > 0 else 1.0
    q = M.copy()
    q[known] = (M[known] / s).astype(np.float16).astype(np.float64) * s
    return q, s


def random_phase_start(M, known, P, seed):
    """Random-phase starting densities rho0_p = F^-1[Xi * M * exp(i phi_p)].

    This start is not the paper's Initialize (projected spheres, initialisation
    appendix); it is the classic random-phase start of the iterative methods
    the paper builds on.  The phases come from the shared counter generator so
    that both implementations produce the same start: at FFT-order pixel k
    (row-major) of member p, u = Philox draw k of (seed, INIT, generation 0,
    member p) and phi = 2 pi (u + 1/2) / 2^32.  Unknown pixels get 0.
    """
    M = np.asarray(M, dtype=np.float64)
    n = M.shape[0]
    out = np.empty((P, n, n), dtype=np.complex128)
    two_pi = 2.0 * np.pi
    for p in range(P):
        u = philox.draws_array(seed, philox.PURPOSE_INIT, 0, p, n * n).astype(np.float64)
        phi = (two_pi * (u + 0.5) / 4294967296.0).reshape(n, n)
        out[p] = ifft2(np.where(known, M, 0.0) * np.exp(1j * phi))
    return out


# ----------------------------------------------------------------------------
# Projectors
# ----------------------------------------------------------------------------


def modulus_fourier(X, M, known):
    """Masked modulus replacement in the Fourier domain (Eq. pm_full).

    Where known: M * X / |X|; where |X| = 0 every phase is equally near, and
    the reading taken is phase 0, i.e. the value M.  Elsewhere X is kept.
    """
    X = np.asarray(X, dtype=np.complex128)
    out = X.copy()
    absX = np.abs(X)
    nz = known & (absX > 0)
    out[nz] = M[nz] * (X[nz] / absX[nz])
    z = known & (absX == 0)
    out[z] = M[z]
    return out


def radial_bins(N):
    """Ring index of every FFT-order pixel: the distance of its signed
    frequency (u, v) from the zero frequency, rounded half up to an integer."""
    f = np.fft.fftfreq(N) * N
    q = np.sqrt(f[:, None] ** 2 + f[None, :] ** 2)
    return np.floor(q + 0.5).astype(np.int64)


def upper_bounds(M, known, eta=1.5, max_unknown=0.2, saturated=None, max_saturated=0.05):
    """Amplitude upper bounds for unknown pixels (appendix on missing
    intensities, Eq. avgint, Eq. stdint, Eq. upperbound).

    Per ring q (integer distance from the centre): mu = mean of I = M^2 over
    the ring's known pixels, sigma = sqrt(mean(I^2) - mu^2) over the same,
    U(q) = mu + eta * sigma.  A ring gets a bound only when its unknown pixels
    are at most `max_unknown` of the ring (and it has a known pixel).
    Readings: Eq. pm_bounds compares |rho~| with U, an amplitude with an
    intensity; the amplitude bound taken is sqrt(U).
    Saturation rules of the same appendix, with `saturated` (FFT order, a
    subset of the unknown pixels, since saturated pixels carry no valid
    measurement): a saturated pixel gets no bound, and a ring with more than
    `max_saturated` (the paper's 5 %) of its pixels saturated gets none.
    Saturated pixels count as unknown in the `max_unknown` rule.
    Returns the bound per pixel (NaN where there is none; known pixels get
    NaN too).
    """
    M = np.asarray(M, dtype=np.float64)
    N = M.shape[0]
    sat = np.zeros((N, N), bool) if saturated is None else np.asarray(saturated, dtype=bool)
    if np.any(sat & known):
        raise ValueError("a saturated pixel must be unknown")
    bins = radial_bins(N)
    out = np.full((N, N), np.nan)
    for q in np.unique(bins):
        ring = bins == q
        kn = ring & known
        unk = ring & ~known
        if not kn.any() or unk.sum() > max_unknown * ring.sum():
            continue
        if (ring & sat).sum() > max_saturated * ring.sum():
            continue
        I = M[kn] ** 2
        mu = I.mean()
        var = max((I ** 2).mean() - mu ** 2, 0.0)
        out[unk & ~sat] = np.sqrt(mu + eta * np.sqrt(var))
    return out


def modulus_fourier_bounded(X, M, known, bound):
    """Eq. pm_bounds: measured pixels as in Eq. pm_full; an unknown pixel with
    a bound b and |X| > b is brought to modulus b with its phase; every other
    pixel is kept.  This is the nearest point of the set {|z| <= b}."""
    out = modulus_fourier(X, M, known)
    A = np.abs(X)
    clamp = ~known & np.isfinite(bound) & (A > np.where(np.isfinite(bound), bound, np.inf))
    out = np.where(clamp, X * (np.where(clamp, bound, 0.0) / np.where(clamp, A, 1.0)), out)
    return out


def proj_modulus_bounded(x, M, known, bound):
    """P_M with upper bounds on the unknown pixels, in real space."""
    return ifft2(modulus_fourier_bounded(fft2(x), M, known, bound))


def proj_modulus(x, M, known):
    """P_M of Eq. pm with the mask of Eq. pm_full: F^-1[modulus_fourier(F[x])]."""
    return ifft2(modulus_fourier(fft2(x), M, known))


def phase_off(chi):
    """True when chi leaves the phase unconstrained.

    The real-space constraints appendix limits arg(rho) to [-chi pi, chi pi]
    with chi in (0, 1]; the complex-density section asks for chi = 0 when
    positivity must not be enforced.  Reading: chi >= 1 and chi <= 0 both mean
    "no phase constraint".
    """
    return chi >= 1.0 or chi <= 0.0


def proj_phase(z, chi):
    """Nearest-point projection onto {z : |arg z| <= chi*pi} (real-space
    constraints appendix).  chi = 0.5 (positivity) is (max(Re z, 0), Im z)."""
    z = np.asarray(z, dtype=np.complex128)
    if phase_off(chi):
        return z.copy()
    if chi == 0.5:
        return np.maximum(z.real, 0.0) + 1j * z.imag
    theta = chi * np.pi
    c, s = np.cos(theta), np.sin(theta)
    re, im = z.real, z.imag
    aim = np.abs(im)
    inside = aim * c <= re * s
    sgn = np.where(im < 0, -1.0, 1.0)
    p = np.maximum(re * c + aim * s, 0.0)   # component along the nearer edge ray
    edge = p * c + 1j * sgn * p * s
    return np.where(inside, z, edge)


def proj_constraint(x, S, chi):
    """P_C = support projector (Eq. ps) combined with the phase constraint."""
    return np.where(S, proj_phase(x, chi), 0.0)


# ----------------------------------------------------------------------------
# Iterative algorithms (phase-problem section; appendix on ER)
# ----------------------------------------------------------------------------


def _pm(x, M, known, bound):
    return proj_modulus(x, M, known) if bound is None else proj_modulus_bounded(x, M, known, bound)


def er(x, S, M, known, chi, bound=None):
    """Error Reduction, x' = P_M P_C x (optimisation-problem appendix).
    With `bound`, P_M is the upper-bounded projector of Eq. pm_bounds."""
    return _pm(proj_constraint(x, S, chi), M, known, bound)


def hio(x, S, M, known, chi, beta, bound=None):
    """Hybrid Input-Output (cited, not written out, in the paper).

    Fienup's rule with y = P_M x: x' = y where y satisfies the real-space
    constraints (inside S and P_C y = y), otherwise x - beta*y.
    """
    y = _pm(x, M, known, bound)
    feasible = S & (proj_phase(y, chi) == y)
    return np.where(feasible, y, x - beta * y)


def raar(x, S, M, known, chi, beta, bound=None):
    """Relaxed Averaged Alternating Reflections (cited, not written out).

    Luke's form beta/2 (R_C R_M + I) x + (1 - beta) P_M x with R = 2P - I,
    i.e. x' = beta*P_C(2y - x) + beta*x + (1 - 2 beta)*y, y = P_M x.
    """
    y = _pm(x, M, known, bound)
    return beta * proj_constraint(2.0 * y - x, S, chi) + beta * x + (1.0 - 2.0 * beta) * y


def sequence(x, S, M, known, chi, alg, beta, n_ia, n_er):
    """Eq. sequence: n_ia iterations of the IA (HIO or RAAR), then n_er of ER."""
    step = {"HIO": hio, "RAAR": raar}[alg]
    for _ in range(n_ia):
        x = step(x, S, M, known, chi, beta)
    for _ in range(n_er):
        x = er(x, S, M, known, chi)
    return x


def fourier_error(x, M, known):
    """The measure of Eq. error_calc applied to an iterate without its support:
    sqrt(sum Xi (|F[x]| - M)^2 / sum Xi M^2), the distance of F[x] from the
    measured moduli relative to their norm (the per-iteration trace)."""
    den = float(np.sum(M[known] ** 2))
    A = np.abs(fft2(x))
    return float(np.sqrt(np.sum((A[known] - M[known]) ** 2) / den))


def sequence_trace(x, S, M, known, chi, alg, beta, n_ia, n_er):
    """Eq. sequence, recording before every iteration the Fourier error of the
    density whose spectrum that iteration projects: x for the HIO/RAAR steps,
    P_C x for the ER steps.  Returns (final x, list of errors)."""
    step = {"HIO": hio, "RAAR": raar}[alg]
    errs = []
    for _ in range(n_ia):
        errs.append(fourier_error(x, M, known))
        x = step(x, S, M, known, chi, beta)
    for _ in range(n_er):
        errs.append(fourier_error(proj_constraint(x, S, chi), M, known))
        x = er(x, S, M, known, chi)
    return x, errs


def schedule_at(g, G, j, j_er, j_end, sigma, sigma_end, tau, tau_end):
    """Linear parameter changes over generations (appendix "changing values").

    Interpolation and rounding are not given; reading: t = (g-1)/(G-1) (t = 0
    when G = 1), j(g) = floor(j + t (j_end - j) + 1/2), the ER count keeps the
    sequence length constant (j + j_ER), sigma and tau interpolate linearly.
    """
    t = 0.0 if G <= 1 else (g - 1) / (G - 1)
    jg = int(np.floor(j + t * (j_end - j) + 0.5))
    jer = j + j_er - jg
    return jg, jer, sigma + t * (sigma_end - sigma), tau + t * (tau_end - tau)


# ----------------------------------------------------------------------------
# Fitness (Eq. error_calc)
# ----------------------------------------------------------------------------


def get_error(x, S, M, known):
    """E = sqrt( sum Xi (|F[S x]| - M)^2 / sum Xi M^2 ), Eq. error_calc.

    The support alone multiplies x (no phase constraint), as the equation is
    written.  A pattern with sum Xi M^2 = 0 is invalid input.
    """
    den = float(np.sum(M[known] ** 2))
    if not den > 0:
        raise ValueError("sum of known M^2 must be positive")
    A = np.abs(fft2(np.where(S, x, 0.0)))
    num = float(np.sum((A[known] - M[known]) ** 2))
    return float(np.sqrt(num / den))


# ----------------------------------------------------------------------------
# Shrink-wrap (Eq. shrinkwrap) and the modified shrink-wrap (UpdateSupportSize)
# ----------------------------------------------------------------------------


def gauss_taps(sigma):
    """1D Gaussian taps w_k ~ exp(-k^2 / 2 sigma^2), |k| <= ceil(4 sigma), sum 1.

    The kernel support and normalisation are not given; reading: radius
    ceil(4 sigma), unit sum, periodic boundary.  sigma = 0 means no smoothing.
    """
    if sigma <= 0:
        return np.array([1.0])
    r = int(np.ceil(4.0 * sigma))
    k = np.arange(-r, r + 1, dtype=np.float64)
    w = np.exp(-(k * k) / (2.0 * sigma * sigma))
    return w / w.sum()


def smooth(a, sigma):
    """Circular separable Gaussian smoothing of a real image (rows, then columns)."""
    w = gauss_taps(sigma)
    r = (len(w) - 1) // 2
    a = np.asarray(a, dtype=np.float64)
    rows = np.zeros_like(a)
    for i, k in enumerate(range(-r, r + 1)):
        rows += w[i] * np.roll(a, -k, axis=1)      # out[., j] += w_k a[., j+k]
    out = np.zeros_like(a)
    for i, k in enumerate(range(-r, r + 1)):
        out += w[i] * np.roll(rows, -k, axis=0)
    return out


def update_support(x, S, sigma, tau):
    """Shrink-wrap UpdateSupport: S' = {a_sigma > tau * max a_sigma}, a = |x|.

    Reading: the modulus |x| is smoothed (complex smoothing is not implied by
    the text).  If max a_sigma = 0 the support is left unchanged.
    """
    a = smooth(np.abs(x), sigma)
    m = a.max()
    if not m > 0:
        return S.copy()
    return a > tau * m


def area_count(alpha, n_pix):
    """Support size used by UpdateSupportSize: round half up, clamped to [1, N^2]."""
    return int(min(max(np.floor(alpha + 0.5), 1), n_pix))


def update_support_size(x, sigma, alpha):
    """Modified shrink-wrap: the round(alpha) largest smoothed values form S'.

    Ties at the threshold go to the lower linear index.
    """
    a = smooth(np.abs(x), sigma).ravel()
    k = area_count(alpha, a.size)
    order = np.lexsort((np.arange(a.size), -a))   # descending value, then index
    S = np.zeros(a.size, dtype=bool)
    S[order[:k]] = True
    return S.reshape(x.shape)


# ----------------------------------------------------------------------------
# Population statistics (self-improvement appendix; oversampling Eq.)
# ----------------------------------------------------------------------------


def generation_stats(E_par, S_par, g, G):
    """alpha_best, alpha_all, alpha_eval of Alg. improve from the parents.

    best = lowest error, ties to the lowest index; alpha_all = area of the union
    of the parents' supports; alpha_eval = (g/G) alpha_best + (1 - g/G) alpha_all.
    """
    b = int(np.argmin(np.asarray(E_par, dtype=np.float64)))
    a_best = int(np.count_nonzero(S_par[b]))
    union = np.zeros_like(S_par[0], dtype=bool)
    for S in S_par:
        union |= S
    a_all = int(np.count_nonzero(union))
    a_eval = (g / G) * a_best + (1.0 - g / G) * a_all
    n2 = S_par[0].size
    return {"best": b, "alpha_best": a_best, "alpha_all": a_all,
            "alpha_eval": a_eval, "oversampling": n2 / max(a_best, 1)}


# ----------------------------------------------------------------------------
# Crossover appendix: RandomChoice, Reshift, CrossoverMap, mixing
# ----------------------------------------------------------------------------


def random_choice(p, P, seed, g):
    """Three distinct parents, all different from p (RandomChoice).

    The method is not given; reading: uniform draws over the remaining indices
    by skip-mapping (draw in [0, P-1-n) and step past the excluded indices in
    ascending order), which needs no rejection loop.
    """
    chosen = []
    excluded = [p]
    for i in range(3):
        r = philox.uniform_int(philox.draw(seed, philox.PURPOSE_CHOICE, g, p, i),
                               P - 1 - i)
        for e in sorted(excluded):
            if r >= e:
                r += 1
        chosen.append(r)
        excluded.append(r)
    return tuple(chosen)


def reshift(Xq, Sq, Xref, known):
    """Align parent q to the reference (Reshift; Eq. crosscorr).

    Cross-correlations through the masked convolution theorem:
    C1 = F^-1[Xi conj(Xq) Xref] (parent as is) and C2 = F^-1[Xi Xq Xref]
    (the twin rho*(-x), whose transform is conj(Xq)).  d = argmax |C| (ties to
    the lowest FFT-order index), the twin is kept iff its peak is strictly
    higher, phi = arg C(d).  Result: X' = e^{i phi} e^{-2 pi i k.d/N} (Xq or
    conj Xq), S'(y) = S(y - d) or S(d - y).
    """
    N = Xq.shape[0]
    C1 = ifft2(known * np.conj(Xq) * Xref)
    C2 = ifft2(known * Xq * Xref)
    m1, m2 = np.abs(C1).ravel(), np.abs(C2).ravel()
    d1, d2 = int(np.argmax(m1)), int(np.argmax(m2))
    twin = bool(m2[d2] > m1[d1])
    d = d2 if twin else d1
    val = (C2 if twin else C1).ravel()[d]
    phase = np.exp(1j * np.angle(val)) if abs(val) > 0 else 1.0 + 0j
    dr, dc = divmod(d, N)
    k = np.arange(N)
    ramp_idx = (k[:, None] * dr + k[None, :] * dc) % N
    ramp = np.exp(-2j * np.pi * ramp_idx / N)
    Xb = np.conj(Xq) if twin else Xq
    Xout = phase * ramp * Xb
    if twin:
        St = np.roll(Sq[::-1, ::-1], 1, axis=(0, 1))   # S(-y)
        Sout = np.roll(St, (dr, dc), axis=(0, 1))       # S(d - y)
    else:
        Sout = np.roll(Sq, (dr, dc), axis=(0, 1))       # S(y - d)
    info = {"shift": (dr, dc), "twin": twin, "phase": complex(phase),
            "peak1": float(m1[d1]), "peak2": float(m2[d2]),
            "second1": float(np.partition(m1, -2)[-2]) if m1.size > 1 else 0.0,
            "second2": float(np.partition(m2, -2)[-2]) if m2.size > 1 else 0.0}
    return Xout, Sout, info


# Integer rotations (a, b, h) with a^2 + b^2 = h^2: cos = a/h, sin = b/h.
# Angles 0, 16.3, 22.6, 28.1, 36.9, 53.1, 61.9, 67.4, 73.7 degrees; rotating a
# rectangular tiling by 90 degrees only swaps the tile sides, so [0, 90) covers
# the distinct grids.
ROTATIONS = ((1, 0, 1), (24, 7, 25), (12, 5, 13), (15, 8, 17), (4, 3, 5),
             (3, 4, 5), (8, 15, 17), (5, 12, 13), (7, 24, 25))


def map_params(N, seed, g, p, t_min, t_max):
    """Tile sides, grid shift and rotation of one crossover map.

    Reading: one (t_x, t_y) per map drawn uniformly from [t_min, t_max], a
    shift uniform in [0, t) per axis, and a rotation from ROTATIONS.
    """
    d = [philox.draw(seed, philox.PURPOSE_MAPPARAM, g, p, i) for i in range(5)]
    span = t_max - t_min + 1
    tx = t_min + philox.uniform_int(d[0], span)
    ty = t_min + philox.uniform_int(d[1], span)
    sx = philox.uniform_int(d[2], tx)
    sy = philox.uniform_int(d[3], ty)
    rot = philox.uniform_int(d[4], len(ROTATIONS))
    return tx, ty, sx, sy, rot


def tile_key(qx, qy):
    return ((qx & 0xFFFF) << 16) | (qy & 0xFFFF)


def crossover_map(N, seed, g, p, c_p, t_min, t_max):
    """Binary crossover map of the Fourier domain (CrossoverMap, Fig. crossmap).

    The domain (signed frequencies u for rows, v for columns) is tiled by
    t_x x t_y rectangles, rotated by an integer Pythagorean rotation and
    shifted; each tile is elected with probability C_p.
    """
    return crossover_map_with(N, map_params(N, seed, g, p, t_min, t_max), seed, g, p, c_p)


def crossover_map_with(N, params, seed, g, p, c_p):
    """Crossover map for given (t_x, t_y, s_x, s_y, rotation index)."""
    tx, ty, sx, sy, rot = params
    a, b, h = ROTATIONS[rot]
    thr = philox.bernoulli_threshold(c_p)
    cache = {}
    out = np.zeros((N, N), dtype=bool)
    for i in range(N):
        u = i if i < N // 2 else i - N
        for j in range(N):
            v = j if j < N // 2 else j - N
            ur = a * u + b * v
            vr = -b * u + a * v
            qx = (ur + h * sx) // (h * tx)
            qy = (vr + h * sy) // (h * ty)
            key = tile_key(qx, qy)
            if key not in cache:
                w = philox.philox4x32_10((key, p, g, philox.PURPOSE_TILE),
                                         philox.seed_key(seed))[0]
                cache[key] = w < thr
            out[i, j] = cache[key]
    return out


def default_t_max(N, t_min=4):
    """Example value t_max = N/8 of the crossover appendix, kept >= t_min."""
    return max(t_min, N // 8)


def average(xs, Ss, E, known):
    """The population average (Alg. mpr's final Average, Eq. avgrec), with the
    members aligned first.

    The densities of a population are defined up to translation, twin and a
    global phase; the paper resolves these before any operation on several
    densities (appendix on aligning the reconstructions).  Reading: every
    member is aligned by Reshift to the member with the lowest error (ties to
    the lower index), then rho_avg = mean of the aligned densities and S_avg
    = union of the aligned supports (Eq. avgrec read as the union over
    p = 1..P).  Also returns the two average moduli of the appendix on
    unconstrained modes: Mdot = |F[rho_avg]| (Eq. avgint1) and Mddot = mean of
    |F[rho_p]| (Eq. avgint2), and the alignment records.
    """
    b = int(np.argmin(E))
    Xs = [fft2(x) for x in xs]
    al = [reshift(X, S, Xs[b], known) for X, S in zip(Xs, Ss)]
    Xavg = sum(a[0] for a in al) / len(xs)
    S_avg = np.zeros_like(Ss[0], dtype=bool)
    for a in al:
        S_avg = S_avg | a[1]
    Mddot = sum(np.abs(X) for X in Xs) / len(xs)
    return {"rho": ifft2(Xavg), "S": S_avg, "Mdot": np.abs(Xavg), "Mddot": Mddot, "best": b,
            "align": [a[2] for a in al]}


def complexity(x):
    """Eq. complexity: Gamma = 1 - |sum rho| / sum |rho| (0 for a constant phase)."""
    x = np.asarray(x, dtype=np.complex128)
    a = float(np.sum(np.abs(x)))
    return 1.0 - abs(complex(np.sum(x))) / a if a > 0 else 0.0


def monitors(xs, E, avg=None, avg_err=None):
    """Per-generation indicators of the monitoring section and the appendix on
    unconstrained modes: best, lower-median, worst and mean error; mean
    complexity Gamma over the members; mean density sum |sum rho| and its
    standard deviation relative to the mean (population standard deviation);
    for the average reconstruction, its Gamma and error.  Readings: the median
    of an even count is the lower of the two middle values (an actual member's
    error)."""
    E = np.asarray(E, dtype=np.float64)
    sums = np.array([abs(complex(np.sum(np.asarray(x, dtype=np.complex128)))) for x in xs])
    Es = np.sort(E)
    out = {"err_best": float(Es[0]), "err_median": float(Es[(len(Es) - 1) // 2]), "err_worst": float(Es[-1]),
           "err_mean": float(E.mean()), "gamma_mean": float(np.mean([complexity(x) for x in xs])),
           "sum_mean": float(sums.mean()),
           "sum_rel_std": float(sums.std() / sums.mean()) if sums.mean() > 0 else 0.0}
    if avg is not None:
        out["gamma_avg"] = complexity(avg)
        out["err_avg"] = float(avg_err) if avg_err is not None else float("nan")
    return out


def mix_average_modulus(Xa, Mdot, Mddot, c_a):
    """Eq. crossavg: the parent a keeps its Fourier phases and takes the modulus
    C_a (Mdot + Mddot)/2 + (1 - C_a)|Xa| (phase 0 where Xa = 0)."""
    A = np.abs(Xa)
    unit = np.where(A > 0, Xa / np.where(A > 0, A, 1.0), 1.0)
    return (c_a * 0.5 * (Mdot + Mddot) + (1.0 - c_a) * A) * unit


def crossover(xs, Ss, known, g, seed, c_p, c_w, t_min, t_max, c_a=0.0, avg=None):
    """Alg. crossover: one child per parent p from three aligned parents.

    Non-map Fourier pixels keep the child's own parent p ("Copy"); map pixels
    take X_a + C_w (X_b - X_c); the support is S_a OR (S_b AND S_c AND S_p);
    the child density is the inverse transform of the mixed spectrum.  With
    C_a > 0 the aligned parent a first takes the modulus of Eq. crossavg from
    the population average `avg` (see `average`).
    """
    P = len(xs)
    N = xs[0].shape[0]
    Xs = [fft2(x) for x in xs]
    kids_x, kids_S, infos = [], [], []
    for p in range(P):
        abc = random_choice(p, P, seed, g)
        aligned = [reshift(Xs[q], Ss[q], Xs[p], known) for q in abc]
        cmap = crossover_map(N, seed, g, p, c_p, t_min, t_max)
        (Xa, Sa, ia), (Xb, Sb, ib), (Xc, Sc, ic) = aligned
        if c_a > 0.0:
            Xa = mix_average_modulus(Xa, avg["Mdot"], avg["Mddot"], c_a)
        Xn = np.where(cmap, Xa + c_w * (Xb - Xc), Xs[p])
        Sn = Sa | (Sb & Sc & Ss[p])
        kids_x.append(ifft2(Xn))
        kids_S.append(Sn)
        infos.append({"abc": abc, "align": (ia, ib, ic), "map": cmap})
    return kids_x, kids_S, infos


def select(E_old, E_new):
    """Alg. select: child p replaces parent p iff E_new < E_old (strict)."""
    return [bool(en < eo) for eo, en in zip(E_old, E_new)]


# ----------------------------------------------------------------------------
# Drivers: Alg. randomsearch + normalimprove (plain) and Alg. mpr + improve
# ----------------------------------------------------------------------------


def _bcast_supports(S0, P):
    S0 = np.asarray(S0, dtype=bool)
    if S0.ndim == 2:
        return [S0.copy() for _ in range(P)]
    return [s.copy() for s in S0]


def run_plain(M, known, x0, S0, prm):
    """Plain multi-start reconstruction (Alg. randomsearch with normalimprove).

    ``prm`` keys: alg, beta, chi, G, j, j_er, j_end, sigma, sigma_end, tau,
    tau_end.  Each generation runs Sequence then UpdateSupport on every member;
    the error of every member is evaluated at the end and Best is the lowest
    (ties to the lowest index).
    """
    xs = [np.asarray(x, dtype=np.complex128).copy() for x in x0]
    Ss = _bcast_supports(S0, len(xs))
    for g in range(1, prm["G"] + 1):
        jg, jer, sg, tg = schedule_at(g, prm["G"], prm["j"], prm["j_er"], prm.get("j_end", 0),
                                      prm["sigma"], prm["sigma_end"], prm["tau"], prm["tau_end"])
        for m in range(len(xs)):
            xs[m] = sequence(xs[m], Ss[m], M, known, prm["chi"], prm["alg"], prm["beta"], jg, jer)
            Ss[m] = update_support(xs[m], Ss[m], sg, tg)
    E = [get_error(x, S, M, known) for x, S in zip(xs, Ss)]
    return {"x": xs, "S": Ss, "E": E, "best": int(np.argmin(E))}


def improve_member(x, S, M, known, prm, g, stats):
    """Alg. improve for one reconstruction (both populations run this)."""
    jg, jer, sg, tg = schedule_at(g, prm["G"], prm["j"], prm["j_er"], prm.get("j_end", 0),
                                  prm["sigma"], prm["sigma_end"], prm["tau"], prm["tau_end"])
    chi, alg, beta = prm["chi"], prm["alg"], prm["beta"]
    for _ in range(prm["R"] - 2):
        x = sequence(x, S, M, known, chi, alg, beta, jg, jer)
        S = update_support(x, S, sg, tg)
    x = sequence(x, S, M, known, chi, alg, beta, jg, jer)
    S = update_support_size(x, sg, stats["alpha_best"])
    x = sequence(x, S, M, known, chi, alg, beta, jg, jer)
    S = update_support_size(x, sg, stats["alpha_eval"])
    x = sequence(x, S, M, known, chi, alg, beta, 0, prm["j_eval"])
    E = get_error(x, S, M, known)
    S = update_support(x, S, sg, tg)
    return x, S, E


def run_mpr(M, known, x0, S0, prm, seed, gen_offset=0, generations=None):
    """Alg. mpr: crossover, improve both, select; the final Average is
    returned under "average".

    ``prm`` adds R, j_eval, c_p, c_w, t_min, t_max (and optionally c_a, the
    weight of Eq. crossavg) to the plain keys.  The
    errors of the initial population are evaluated first (GetError), since the
    first generation's statistics need them.  Generations gen_offset+1 ..
    gen_offset+generations are run (all G by default).
    """
    xs = [np.asarray(x, dtype=np.complex128).copy() for x in x0]
    P = len(xs)
    Ss = _bcast_supports(S0, P)
    E = [get_error(x, S, M, known) for x, S in zip(xs, Ss)]
    G = prm["G"]
    n_gen = G - gen_offset if generations is None else generations
    history = []
    for g in range(gen_offset + 1, gen_offset + n_gen + 1):
        c_a = prm.get("c_a", 0.0)
        avg = average(xs, Ss, E, known) if c_a > 0.0 else None
        kx, kS, infos = crossover(xs, Ss, known, g, seed, prm["c_p"], prm["c_w"],
                                  prm["t_min"], prm["t_max"], c_a=c_a, avg=avg)
        stats = generation_stats(E, Ss, g, G)
        new_par = [improve_member(xs[p], Ss[p], M, known, prm, g, stats) for p in range(P)]
        new_kid = [improve_member(kx[p], kS[p], M, known, prm, g, stats) for p in range(P)]
        repl = select([e for _, _, e in new_par], [e for _, _, e in new_kid])
        xs, Ss, E = [], [], []
        for p in range(P):
            src = new_kid[p] if repl[p] else new_par[p]
            xs.append(src[0]); Ss.append(src[1]); E.append(src[2])
        history.append({"g": g, "stats": stats, "replaced": repl, "crossover": infos,
                        "E_par": [e for _, _, e in new_par], "E_kid": [e for _, _, e in new_kid]})
    return {"x": xs, "S": Ss, "E": E, "history": history, "average": average(xs, Ss, E, known)}
