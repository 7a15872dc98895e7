"""Seeded synthetic cases shared by the parity tests.

Ingredients come from ``ptysynth``; the counts come from the oracle's forward
model plus a Poisson draw, so no test input is produced by the HIP path.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

import oracle
import ptysynth


@dataclasses.dataclass
class Case:
    n: int
    k: int
    obj_true: np.ndarray
    probe: np.ndarray
    pos: np.ndarray
    counts: np.ndarray     # float32, centred
    amp: np.ndarray        # float64 natural-order moduli of the float32 counts

    @property
    def j(self):
        return len(self.pos)

    @property
    def shape(self):
        return self.obj_true.shape


def spiral_case(n: int, k: int, j: int, cfg: int = 90, photons: float = 1e6, jitter: bool = True,
                noise: bool = True, margin: float = 3.0) -> Case:
    """Fermat-spiral case with the configuration-2 proportions scaled to N."""
    c = 14.0 * n / 256.0
    side = ptysynth.spiral_object_side(j, c, n, margin)
    obj = ptysynth.make_object(cfg, side, side, max(2.0, 4.0 * n / 256.0))
    probe = ptysynth.make_probe(cfg, n, k, 84.0 * n / 256.0, max(1.0, 3.0 * n / 256), max(2.0, 12.0 * n / 256),
                                5.0)
    pos = ptysynth.spiral_positions(j, c, side / 2.0, n, ptysynth.stream(cfg, 3) if jitter else None)
    return _finish(n, k, obj, probe, pos, photons, cfg, noise)


def raster_case(n: int, k: int, rows: int, cols: int, step: float, offset: float, side: int,
                cfg: int = 91, photons: float = 1e6, noise: bool = True) -> Case:
    obj = ptysynth.make_object(cfg, side, side, 2.0)
    probe = ptysynth.make_probe(cfg, n, k, 26.0 * n / 64.0, 1.5, 4.0, 5.0)
    pos = ptysynth.raster_positions(rows, cols, step, offset)
    return _finish(n, k, obj, probe, pos, photons, cfg, noise)


def workload_case(cfg: int, noise: bool = True) -> Case:
    wl = ptysynth.workload(cfg)
    return _finish(wl.n, wl.k, wl.obj(), wl.probe(), wl.positions(), wl.photons, cfg, noise)


def _finish(n, k, obj, probe, pos, photons, cfg, noise):
    expected, probe = oracle.simulate(obj, probe, pos, photons)
    counts = ptysynth.poisson_counts(expected, ptysynth.stream(cfg, 4)) if noise else expected.astype(np.float32)
    return Case(n, k, obj, probe, pos, counts, oracle.amplitude(counts.astype(np.float64)))


def c64(x):
    return np.asarray(x, dtype=np.complex64)


def rel(x, y) -> float:
    """Phase-aligned relative L2 error (global phase removed)."""
    return oracle.phase_aligned_rel(np.asarray(x, np.complex128), np.asarray(y, np.complex128))


def start_state(case: Case, perturb: float = 0.0, seed: int = 5):
    """Initial object (flat, optionally perturbed) and probe (the truth in float32)."""
    rng = np.random.default_rng(seed)
    o0 = np.ones(case.shape, np.complex128)
    if perturb:
        o0 = o0 + perturb * (rng.standard_normal(case.shape) + 1j * rng.standard_normal(case.shape))
    # both sides start from the same float32-representable values
    return c64(o0).astype(np.complex128), c64(case.probe).astype(np.complex128)
