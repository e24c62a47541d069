"""Seeded synthetic inputs shaped like single-shot XFEL diffraction data.

The paper's experimental datasets are not available, so seeded synthetic
patterns stand in for them: compact objects (uniform ellipses, clustered
projected spheres), far-field amplitudes with Poisson photon noise, a central
beamstop and a horizontal detector gap, and initial populations.  This module
holds input generation only (NumPy PCG64 generators with explicit seeds); it
contains none of the reconstruction arithmetic and is used alike by the test
oracle, the tests and the benchmark.

Layouts: amplitude and mask images are returned in the *centred* detector
layout (zero frequency at [N/2, N/2]); densities and supports in real space
with the object around the array centre.
"""

import numpy as np


def _rng(seed):
    return np.random.Generator(np.random.PCG64(int(seed)))


def _grid(n):
    y, x = np.mgrid[0:n, 0:n].astype(np.float64)
    return y - n / 2.0, x - n / 2.0


def ellipses(n, seed, count=5, semi=(4.0, 15.0), disk_diameter=40.0):
    """Union of `count` uniform-density (value 1) ellipses inside a centred disk."""
    rng = _rng(seed)
    yy, xx = _grid(n)
    obj = np.zeros((n, n))
    rad = disk_diameter / 2.0
    for _ in range(count):
        a, b = rng.uniform(semi[0], semi[1], size=2)
        ang = rng.uniform(0.0, np.pi)
        reach = max(a, b)
        if reach > rad:
            raise ValueError(f"an ellipse with semi-axis {reach:.2f} does not fit a disk of radius {rad:.2f}")
        while True:
            c = rng.uniform(-rad, rad, size=2)
            if np.hypot(c[0], c[1]) + reach <= rad:
                break
        ca, sa = np.cos(ang), np.sin(ang)
        dy, dx = yy - c[0], xx - c[1]
        u = ca * dx + sa * dy
        v = -sa * dx + ca * dy
        obj[(u / a) ** 2 + (v / b) ** 2 <= 1.0] = 1.0
    return obj


def projected_sphere(n, cy, cx, radius):
    """Optical depth 2 sqrt(R^2 - r^2) of a sphere centred at (cy, cx) from the array centre."""
    yy, xx = _grid(n)
    r2 = (yy - cy) ** 2 + (xx - cx) ** 2
    return 2.0 * np.sqrt(np.clip(radius * radius - r2, 0.0, None))


def clustered_spheres(n, seed, count=12, radius=(6.0, 24.0), spread=30.0, extent=150.0):
    """Sum of projected spheres with Gaussian-clustered centres inside a disk of
    diameter `extent`."""
    rng = _rng(seed)
    obj = np.zeros((n, n))
    lim = extent / 2.0
    for _ in range(count):
        R = rng.uniform(radius[0], radius[1])
        while True:
            c = rng.normal(0.0, spread, size=2)
            if np.hypot(c[0], c[1]) + R <= lim:
                break
        obj += projected_sphere(n, c[0], c[1], R)
    return obj


def beamstop_gap_mask(n, beamstop=8, gap=0):
    """Centred mask (True = measured): b x b central beamstop and a horizontal gap.

    Beamstop rows/columns n/2-b/2 .. n/2+b/2-1; gap rows n/2-gap/2 .. n/2+gap/2-1
    across the full width.
    """
    m = np.ones((n, n), dtype=bool)
    if beamstop > 0:
        lo = n // 2 - beamstop // 2
        m[lo:lo + beamstop, lo:lo + beamstop] = False
    if gap > 0:
        lo = n // 2 - gap // 2
        m[lo:lo + gap, :] = False
    return m


def diffraction(obj, photons, seed=None, noiseless=False):
    """Centred amplitudes M = sqrt(I) of a real object.

    Expected counts lambda = photons |Y|^2 / sum |Y|^2 with Y the unitary DFT of
    the object; I ~ Poisson(lambda) unless noiseless (then M = sqrt(lambda)).
    Returns (amp_centred float64, scale) where scale * obj is the density whose
    unitary transform has modulus sqrt(lambda).
    """
    Y = np.fft.fft2(obj, norm="ortho")
    p = np.abs(Y) ** 2
    tot = p.sum()
    lam = photons * p / tot
    if noiseless:
        I = lam
    else:
        I = _rng(seed).poisson(lam).astype(np.float64)
    amp = np.sqrt(I)
    return np.fft.fftshift(amp), float(np.sqrt(photons / tot))


def centred_square(n, side):
    """Boolean square support of the given side, centred in the array."""
    s = np.zeros((n, n), dtype=bool)
    lo = n // 2 - side // 2
    s[lo:lo + side, lo:lo + side] = True
    return s


def random_phase_starts(amp_centred, mask_centred, P, seed):
    """rho0 = F^-1[Xi * M * exp(i phi)], phi ~ U[0, 2 pi): a common random start."""
    rng = _rng(seed)
    amp = np.fft.ifftshift(amp_centred)
    known = np.fft.ifftshift(mask_centred)
    n = amp.shape[0]
    out = np.empty((P, n, n), dtype=np.complex128)
    for p in range(P):
        phi = rng.uniform(0.0, 2.0 * np.pi, size=(n, n))
        out[p] = np.fft.ifft2(np.where(known, amp, 0.0) * np.exp(1j * phi), norm="ortho")
    return out


def sphere_starts(amp_centred, mask_centred, P, seed, sigma_init, n_init=5,
                  diam=(0.2, 0.9), gamma=1.0):
    """Initial densities filled with projected spheres inside a centred
    sigma_init-wide square (initialisation appendix), gamma applied to the
    modulus, phase 0, scaled so that the partial Fourier norm over the known
    pixels matches the data (Eq. norm gives the squared-norm ratio nu, so the
    density is multiplied by sqrt(nu))."""
    rng = _rng(seed)
    amp = np.fft.ifftshift(amp_centred)
    known = np.fft.ifftshift(mask_centred)
    n = amp.shape[0]
    out = np.empty((P, n, n), dtype=np.complex128)
    half = sigma_init / 2.0
    for p in range(P):
        rho = np.zeros((n, n))
        for _ in range(n_init):
            D = rng.uniform(diam[0] * sigma_init, diam[1] * sigma_init)
            R = D / 2.0
            c = rng.uniform(-half + R, half - R, size=2) if half > R else np.zeros(2)
            rho += projected_sphere(n, c[0], c[1], R)
        rho = np.abs(rho) ** gamma
        Y = np.fft.fft2(rho, norm="ortho")
        nu = np.sum(amp[known] ** 2) / max(np.sum(np.abs(Y[known]) ** 2), 1e-300)
        out[p] = rho * np.sqrt(nu)
    return out


def shot(n, kind, seed, photons, beamstop, gap=0, noiseless=False, **kw):
    """One synthetic shot: dict with obj, amp (centred), mask (centred), scale."""
    if kind == "ellipses":
        obj = ellipses(n, seed, **kw)
    elif kind == "spheres":
        obj = clustered_spheres(n, seed, **kw)
    else:
        raise ValueError(kind)
    amp, scale = diffraction(obj, photons, seed=seed + 7919, noiseless=noiseless)
    mask = beamstop_gap_mask(n, beamstop, gap)
    return {"obj": obj, "amp": amp, "mask": mask, "scale": scale, "n": n}


def random_complex(shape, seed, scale=1.0):
    """Seeded complex Gaussian array (generic operator-test input)."""
    rng = _rng(seed)
    return scale * (rng.standard_normal(shape) + 1j * rng.standard_normal(shape))
