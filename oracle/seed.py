"""FP64 reference of the learned seed's data path (test infrastructure).

Network input and training targets, and the stitching of predicted
64 x 64 patches into an object seed:

* placement: the central 64 x 64 of window j, at the window's nearest
  integer position (floor(p + 1/2)) plus (32, 32);
* phase offsets: a sequential chain over the patches in position order on
  the coarse grid of object pixels whose coordinates are multiples of 16:
  z_j = sum over patch j's coarse samples of S conj(c_j), e_j = z_j / |z_j|
  (1 if z_j = 0), then S += c_j e_j on those samples;
* the seed: the mean of c_j e_j over the patches covering a pixel, 1 where no
  patch covers it.

c_j = a_j exp(i phi_j) from the predicted amplitude a_j and phase phi_j.
"""
from __future__ import annotations

import numpy as np

PATCH = 64
GRID = 16


def network_input(counts, photons):
    """log1p(max(d, 0)) / log1p(photons) of centred counts."""
    return np.log1p(np.maximum(np.asarray(counts, np.float64), 0.0)) / np.log1p(photons)


def targets(obj, pos, n=128):
    """Amplitude and phase relative to the mean phasor of the central n/2 x n/2
    patch of each window at integer positions pos (J, 2): (J, n/2, n/2, 2)."""
    m, q = n // 2, n // 4
    out = np.empty((len(pos), m, m, 2))
    for j, (y, x) in enumerate(np.asarray(pos)):
        y, x = int(y), int(x)
        o = np.asarray(obj, np.complex128)[y + q:y + q + m, x + q:x + q + m]
        s = o.sum()
        ph = s / abs(s) if abs(s) > 0 else 1.0
        out[j, ..., 0] = np.abs(o)
        out[j, ..., 1] = np.angle(o * np.conj(ph))
    return out


def placements(pos, n=128):
    """Top-left object pixel of each patch: nearest integer position + n/4."""
    return np.floor(np.asarray(pos, np.float64) + 0.5).astype(np.int64) + n // 4


def stitch(patches, pos, h, w, n=128):
    """Object seed (h, w) from patches (J, 64, 64, 2) of amplitude and phase."""
    p = np.asarray(patches, np.float64)
    c = p[..., 0] * np.exp(1j * p[..., 1])
    t = placements(pos, n)
    S = np.zeros(((h + GRID - 1) // GRID, (w + GRID - 1) // GRID), np.complex128)
    e = np.ones(len(t), np.complex128)
    for j, (ty, tx) in enumerate(t):
        gy, gx = -(-ty // GRID) * GRID, -(-tx // GRID) * GRID   # first grid points inside
        samples = c[j, gy - ty::GRID, gx - tx::GRID]               # 4 x 4
        win = S[gy // GRID:gy // GRID + samples.shape[0], gx // GRID:gx // GRID + samples.shape[1]]
        z = np.sum(win * np.conj(samples))
        e[j] = z / abs(z) if abs(z) > 0 else 1.0
        win += samples * e[j]
    acc = np.zeros((h, w), np.complex128)
    cnt = np.zeros((h, w))
    for j, (ty, tx) in enumerate(t):
        acc[ty:ty + PATCH, tx:tx + PATCH] += c[j] * e[j]
        cnt[ty:ty + PATCH, tx:tx + PATCH] += 1
    out = np.ones((h, w), np.complex128)
    cov = cnt > 0
    out[cov] = acc[cov] / cnt[cov]
    return out, e
