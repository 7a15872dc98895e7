"""Seeded synthetic inputs for ptychographic reconstruction.

This module only builds the *ingredients* of a ptychography experiment: a
complex test object, a (multi-mode) probe, scan positions, and Poisson count
draws for a given expected intensity.  It contains none of the reconstruction
arithmetic (no exit waves, no projection, no object or probe update): the
forward model that turns object, probe and positions into expected
intensities is implemented separately by each consumer.

Seeding: every random stream is ``numpy.random.default_rng([cfg, ..., stream])``
with the stream numbers

    0 object amplitude, 1 object phase, 2 probe phase plate, 3 position jitter,
    4 Poisson draw, 5 dataset parameters (batched configuration),
    6 network training objects, 7 network weight init.

The five workloads (probe size N, modes K, positions J, object H x W, photons
per pattern) are described in :data:`CONFIGS`.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Sequence

import numpy as np

__all__ = [
    "stream",
    "smooth_noise",
    "make_object",
    "probe_modes_orthonormal",
    "make_probe",
    "raster_positions",
    "spiral_positions",
    "spiral_object_side",
    "poisson_counts",
    "Workload",
    "CONFIGS",
    "workload",
    "POWER_WEIGHTS",
    "sim_object",
    "sim_probe",
]

# Relative power of the incoherent probe modes, K = 1..4.
POWER_WEIGHTS = {
    1: (1.0,),
    2: (0.85, 0.15),
    3: (0.80, 0.15, 0.05),
    4: (0.70, 0.15, 0.10, 0.05),
}


def stream(cfg: int, s: int, *extra: int) -> np.random.Generator:
    """The generator for configuration ``cfg``, stream ``s`` (extra keys go in between)."""
    return np.random.default_rng([int(cfg), *[int(e) for e in extra], int(s)])


def smooth_noise(rng: np.random.Generator, shape: Sequence[int], sigma: float) -> np.ndarray:
    """White N(0,1) noise filtered by a periodic Gaussian of width ``sigma`` pixels.

    The filter is applied in the Fourier domain with the transfer function
    exp(-2 pi^2 sigma^2 (fy^2 + fx^2)), fy and fx in cycles per pixel.
    """
    h, w = int(shape[0]), int(shape[1])
    white = rng.standard_normal((h, w))
    fy = np.fft.fftfreq(h)[:, None]
    fx = np.fft.fftfreq(w)[None, :]
    kern = np.exp(-2.0 * math.pi**2 * sigma**2 * (fy**2 + fx**2))
    return np.real(np.fft.ifft2(np.fft.fft2(white) * kern))


def _minmax(x: np.ndarray, lo: float, hi: float) -> np.ndarray:
    x0, x1 = float(x.min()), float(x.max())
    if x1 == x0:
        return np.full_like(x, 0.5 * (lo + hi))
    return lo + (hi - lo) * (x - x0) / (x1 - x0)


def make_object(cfg: int, h: int, w: int, sigma_o: float, *extra: int,
                amp=(0.8, 1.0), phase=(-0.5, 0.5)) -> np.ndarray:
    """Complex128 test object: smooth amplitude in ``amp`` and smooth phase in ``phase``."""
    a = _minmax(smooth_noise(stream(cfg, 0, *extra), (h, w), sigma_o), *amp)
    p = _minmax(smooth_noise(stream(cfg, 1, *extra), (h, w), sigma_o), *phase)
    return a * np.exp(1j * p)


def probe_modes_orthonormal(cfg: int, n: int, k: int, d: float, sigma_e: float,
                            sigma_p: float, n_fresnel: float, *extra: int) -> np.ndarray:
    """K orthonormal probe modes (each of unit L2 norm, mutually orthogonal).

    Mode 0: a circular aperture of diameter ``d`` centred at (n/2, n/2) with a
    Gaussian edge of width ``sigma_e`` outside the radius, times a smooth phase
    plate within +-0.3 rad, propagated by the paraxial (Fresnel) transfer
    function exp(-i pi zeta (p^2 + q^2) / n^2) with zeta = (d/2)^2 / n_fresnel and
    p, q the signed frequency indices.  Further modes are mode 0 times the first
    moments x - <x>, y - <y> and their product (moments under |mode 0|^2),
    orthonormalised by Gram-Schmidt in float64.
    """
    if not 1 <= k <= 4:
        raise ValueError("1 <= K <= 4")
    yy, xx = np.meshgrid(np.arange(n) - n / 2.0, np.arange(n) - n / 2.0, indexing="ij")
    rho = np.hypot(yy, xx)
    r0 = d / 2.0
    amp = np.where(rho <= r0, 1.0, np.exp(-((rho - r0) ** 2) / (2.0 * sigma_e**2)))
    plate = _minmax(smooth_noise(stream(cfg, 2, *extra), (n, n), sigma_p), -0.3, 0.3)
    p0 = amp * np.exp(1j * plate)
    zeta = r0**2 / n_fresnel
    f = np.fft.fftfreq(n) * n
    tf = np.exp(-1j * math.pi * zeta * (f[:, None] ** 2 + f[None, :] ** 2) / float(n * n))
    p0 = np.fft.ifft2(np.fft.fft2(p0) * tf)

    wgt = np.abs(p0) ** 2
    wsum = wgt.sum()
    my = (yy * wgt).sum() / wsum
    mx = (xx * wgt).sum() / wsum
    sy = math.sqrt(((yy - my) ** 2 * wgt).sum() / wsum)
    sx = math.sqrt(((xx - mx) ** 2 * wgt).sum() / wsum)
    cands = [p0, p0 * (xx - mx) / sx, p0 * (yy - my) / sy, p0 * (xx - mx) * (yy - my) / (sx * sy)]
    basis: list[np.ndarray] = []
    for c in cands[:k]:
        v = c.astype(np.complex128).copy()
        for b in basis:
            v = v - np.vdot(b, v) * b
        v = v / math.sqrt(np.vdot(v, v).real)
        basis.append(v)
    return np.stack(basis)


def make_probe(cfg: int, n: int, k: int, d: float, sigma_e: float, sigma_p: float,
               n_fresnel: float, *extra: int) -> np.ndarray:
    """Power-weighted probe modes: ||P_k||^2 = POWER_WEIGHTS[K][k] (total power 1)."""
    e = probe_modes_orthonormal(cfg, n, k, d, sigma_e, sigma_p, n_fresnel, *extra)
    w = np.sqrt(np.asarray(POWER_WEIGHTS[k], dtype=np.float64))
    return e * w[:, None, None]


def raster_positions(rows: int, cols: int, step: float, offset: float) -> np.ndarray:
    """Top-left corners (y, x) of a row-major raster: (offset + step*r, offset + step*c)."""
    r, c = np.meshgrid(np.arange(rows), np.arange(cols), indexing="ij")
    return np.stack([offset + step * r.ravel(), offset + step * c.ravel()], axis=1).astype(np.float64)


def spiral_positions(j: int, c: float, centre: float, n: int,
                     jitter_rng: np.random.Generator | None = None, jitter: float = 0.5) -> np.ndarray:
    """Fermat-spiral scan: r_m = c sqrt(m), theta_m = m pi (3 - sqrt 5), m = 0..J-1.

    Returns top-left corners (y, x) = centre - n/2 + (r sin theta, r cos theta),
    plus a uniform [-jitter, jitter] offset per axis when a generator is given.
    """
    m = np.arange(j, dtype=np.float64)
    r = c * np.sqrt(m)
    th = m * math.pi * (3.0 - math.sqrt(5.0))
    pos = np.stack([centre - n / 2.0 + r * np.sin(th), centre - n / 2.0 + r * np.cos(th)], axis=1)
    if jitter_rng is not None:
        pos = pos + jitter_rng.uniform(-jitter, jitter, size=pos.shape)
    return pos


def spiral_object_side(j: int, c: float, n: int, margin: float) -> int:
    """Side of a square object that holds a J-point spiral of pitch c with N windows."""
    return int(math.ceil(2.0 * c * math.sqrt(max(j - 1, 0)) + n + 2 + 2 * margin))


def poisson_counts(expected: np.ndarray, rng: np.random.Generator) -> np.ndarray:
    """One Poisson draw per pixel of ``expected`` (photon counts), as float32."""
    lam = np.clip(np.asarray(expected, dtype=np.float64), 0.0, None)
    return rng.poisson(lam).astype(np.float32)


@dataclasses.dataclass(frozen=True)
class Workload:
    """Shapes and generator settings of one synthetic workload."""

    cfg: int
    n: int            # probe window N (square)
    k: int            # probe modes K
    j: int            # scan positions J
    h: int            # object height
    w: int            # object width
    d: float          # aperture diameter (px)
    sigma_e: float    # aperture edge width (px)
    sigma_p: float    # phase-plate smoothing (px)
    n_fresnel: float  # Fresnel number of the propagation
    sigma_o: float    # object smoothing (px)
    photons: float    # mean photons per pattern
    iters: int        # iterations of the reconstruction
    probe_start: int  # first iteration with probe updates
    scan: str         # "raster" or "spiral"
    step: float = 0.0       # raster step (px)
    offset: float = 0.0     # raster offset (px)
    rows: int = 0
    cols: int = 0
    pitch: float = 0.0      # spiral c (px)
    centre: float = 0.0     # spiral centre (px)
    jitter: bool = False

    def obj(self) -> np.ndarray:
        return make_object(self.cfg, self.h, self.w, self.sigma_o)

    def probe(self) -> np.ndarray:
        """Probe modes with total power 1 (scale to the photon budget with the forward model)."""
        return make_probe(self.cfg, self.n, self.k, self.d, self.sigma_e, self.sigma_p, self.n_fresnel)

    def positions(self) -> np.ndarray:
        if self.scan == "raster":
            return raster_positions(self.rows, self.cols, self.step, self.offset)
        rng = stream(self.cfg, 3) if self.jitter else None
        return spiral_positions(self.j, self.pitch, self.centre, self.n, rng)

    def noise_rng(self) -> np.random.Generator:
        return stream(self.cfg, 4)


CONFIGS = {
    # tiny: 64^2 window, 1 mode, 10x10 raster with 8 px step, 160^2 object
    1: Workload(cfg=1, n=64, k=1, j=100, h=160, w=160, d=26.0, sigma_e=1.5, sigma_p=4.0,
                n_fresnel=5.0, sigma_o=2.0, photons=1e6, iters=50, probe_start=10,
                scan="raster", step=8.0, offset=12.0, rows=10, cols=10),
    # production: 256^2 window, 3 modes, 2,500-point Fermat spiral, 1700^2 object
    2: Workload(cfg=2, n=256, k=3, j=2500, h=1700, w=1700, d=84.0, sigma_e=3.0, sigma_p=12.0,
                n_fresnel=5.0, sigma_o=4.0, photons=1e8, iters=100, probe_start=10,
                scan="spiral", pitch=14.0, centre=850.0, jitter=True),
    # adjoint: 128^2 window, 4 modes, 1,000-point spiral, 600^2 object
    3: Workload(cfg=3, n=128, k=4, j=1000, h=600, w=600, d=42.0, sigma_e=2.0, sigma_p=6.0,
                n_fresnel=5.0, sigma_o=3.0, photons=1e6, iters=1, probe_start=0,
                scan="spiral", pitch=7.0, centre=300.0, jitter=True),
    # learned initialiser evaluation: 128^2 window, 1 mode, 4,096-point spiral, 1200^2 object
    4: Workload(cfg=4, n=128, k=1, j=4096, h=1200, w=1200, d=48.0, sigma_e=2.0, sigma_p=6.0,
                n_fresnel=5.0, sigma_o=3.0, photons=1e8, iters=200, probe_start=1 << 30,
                scan="spiral", pitch=8.0, centre=600.0, jitter=True),
}


def workload(cfg: int) -> Workload:
    return CONFIGS[cfg]


def scaled(wl: Workload, **changes) -> Workload:
    """A copy of ``wl`` with fields replaced (used for reduced test shapes)."""
    return dataclasses.replace(wl, **changes)


def sim_object(shape, seed: int = 0, corr: float = 4.0) -> np.ndarray:
    """A seeded phase-and-amplitude test object standing in for the paper's
    simulation image (the command front end's simulation mode):
    Gaussian-correlated noise (correlation length ``corr`` pixels), amplitude
    in [0.8, 1], phase in [-0.5, 0.5] rad."""
    rng = np.random.default_rng([2202, 3144, seed])
    ky = np.fft.fftfreq(shape[0])[:, None]
    kx = np.fft.fftfreq(shape[1])[None, :]
    g = np.exp(-2.0 * (math.pi * corr) ** 2 * (ky * ky + kx * kx))

    def field():
        f = np.real(np.fft.ifft2(np.fft.fft2(rng.standard_normal(shape)) * g))
        return (f - f.min()) / (f.max() - f.min())
    return ((0.8 + 0.2 * field()) * np.exp(1j * (field() - 0.5))).astype(np.complex64)


def sim_probe(n: int, modes: int, beam_px: float) -> np.ndarray:
    """The known probe of the simulation: a disk of the beam diameter with a
    defocus-like quadratic phase (0.8 rad at the rim), later modes weaker
    copies times x, y ramps, total power 1 (the forward model rescales it)."""
    c = (n - 1) / 2.0
    u, v = np.meshgrid(np.arange(n) - c, np.arange(n) - c, indexing="ij")
    rr = (u * u + v * v) / (beam_px / 2.0) ** 2
    disk = (rr <= 1.0) * np.exp(1j * 0.8 * rr)
    shapes = [disk, disk * v / (beam_px / 2), disk * u / (beam_px / 2), disk * u * v / (beam_px / 2) ** 2]
    p = np.stack([shapes[k] * (0.5 ** k) for k in range(modes)])
    return (p / math.sqrt(float(np.sum(np.abs(p) ** 2)))).astype(np.complex64)
