"""Seeded cases shared by the GPU parity tests: the same FP32 inputs go to the
HIP library (through the C ABI) and, promoted to FP64, to the oracle."""

import numpy as np

from oracle import mpr
from paper_2409_07413_amd import synth


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(np.asarray(b)), 1e-300))


class Case:
    """One shot plus a population, as float32 library inputs and FP64 oracle inputs."""

    def __init__(self, n, P, seed=1, photons=1e6, gap=None, kind="ellipses", side=None, per_member_supp=False):
        if kind == "ellipses":
            semi = (max(1.0, 0.03 * n), max(1.5, 0.11 * n))
            kw = dict(count=5, semi=semi, disk_diameter=max(0.32 * n, 2.0 * semi[1] + 0.5))
        else:
            kw = dict(count=12, radius=(0.012 * n, 0.047 * n), spread=0.06 * n, extent=0.3 * n)
        bs = max(2, n // 16)
        gp = (4 if n >= 64 else 2) if gap is None else gap
        sh = synth.shot(n, kind, seed, photons, beamstop=bs, gap=gp, **kw)
        self.n, self.P = n, P
        self.amp32 = sh["amp"].astype(np.float32)
        self.mask8 = sh["mask"].astype(np.uint8)
        self.M = mpr.to_fft_order(self.amp32.astype(np.float64))
        self.known = mpr.to_fft_order(sh["mask"])
        self.obj = sh["obj"] * sh["scale"]
        rho = synth.random_phase_starts(self.amp32.astype(np.float64), sh["mask"], P, seed + 100)
        self.rho32 = rho.astype(np.complex64)
        self.rho = self.rho32.astype(np.complex128)
        side = side or n // 2
        if per_member_supp:
            S = np.stack([np.roll(synth.centred_square(n, side), (p, -p), axis=(0, 1)) for p in range(P)])
        else:
            S = np.stack([synth.centred_square(n, side)] * P)
        self.S = S
        self.supp8 = S.astype(np.uint8)

    def shot(self, ctx):
        return ctx.shot(self.amp32, self.mask8)

    def population(self, ctx, memetic=False, seed=0):
        sh = self.shot(ctx)
        pop = sh.population(self.rho32, self.supp8, memetic=memetic, seed=seed)
        return sh, pop


def perturbed(x, rng, eps=1e-7):
    """x plus complex Gaussian noise of size eps * max|x| (FP32 rounding scale)."""
    return x + eps * np.abs(x).max() * (rng.standard_normal(x.shape) + 1j * rng.standard_normal(x.shape))


def self_sensitivity(fn, x, seed=0, eps=1e-7):
    """Relative change of the FP64 oracle map fn under an FP32-rounding-size
    perturbation of its input: how far any FP32 evaluation can legitimately be
    from the FP64 trajectory."""
    rng = np.random.default_rng(seed)
    return rel(fn(perturbed(x, rng, eps)), fn(x))


class NearSolutionCase(Case):
    """Noiseless clustered-sphere pattern, support from the smoothed object and
    a start 5% away from the true density: the regime in which the projection
    iterations are well conditioned."""

    def __init__(self, n, P, seed=1):
        kw = dict(count=12, radius=(0.012 * n, 0.047 * n), spread=0.06 * n, extent=0.3 * n)
        sh = synth.shot(n, "spheres", seed, 1e8, beamstop=max(2, n // 21), gap=4, noiseless=True, **kw)
        self.n, self.P = n, P
        self.amp32 = sh["amp"].astype(np.float32)
        self.mask8 = sh["mask"].astype(np.uint8)
        self.M = mpr.to_fft_order(self.amp32.astype(np.float64))
        self.known = mpr.to_fft_order(sh["mask"])
        xt = sh["obj"] * sh["scale"]
        self.obj = xt
        S = mpr.smooth(xt, 2.0) > 0.01 * xt.max()
        rng = np.random.default_rng(seed + 1)
        xs = [xt + 0.05 * xt.max() * rng.standard_normal(xt.shape) * S for _ in range(P)]
        self.rho32 = np.stack(xs).astype(np.complex64)
        self.rho = self.rho32.astype(np.complex128)
        self.S = np.stack([S] * P)
        self.supp8 = self.S.astype(np.uint8)
