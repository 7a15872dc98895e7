"""FP64 reference of the learned seed's data path (test infrastructure).

Network input (a real-space estimate of the patch from the pattern and the
known probe) and training targets, and the stitching of predicted 64 x 64
patches into an object seed:

* placement: the central 64 x 64 of window j, at the window's nearest
  integer position (floor(p + 1/2)) plus (32, 32);
* phase offsets (for patches of unknown relative phase): a sequential chain
  over the patches in position order on the coarse grid of object pixels
  whose coordinates are multiples of 8:
  z_j = sum over patch j's coarse samples of S conj(c_j), e_j = z_j / |z_j|
  (1 if z_j = 0), then S += c_j e_j on those samples;
* the stitched object: the mean of c_j e_j over the patches covering a pixel,
  1 where no patch covers it;
* the learned seed: the same mean of the predicted c_j without phase factors
  (the network's input fixes each patch's phase relative to the known probe).

c_j = a_j exp(i phi_j) from the predicted amplitude a_j and phase phi_j.
"""
from __future__ import annotations

import numpy as np

PATCH = 64
GRID = 8


EST_EPS = 0.01   # regulariser of the probe division, relative to max |P|^2


def probe_planes(probe):
    """For a single-mode probe P (N x N, or 1 x N x N): the phase of its far
    field, u = F(P) / |F(P)| (1 where F(P) = 0), and the regularised inverse
    of the probe, g = conj(P) / (|P|^2 + EST_EPS max |P|^2)."""
    p = np.asarray(probe, np.complex128).reshape(np.shape(probe)[-2:])
    n = p.shape[-1]
    fp = np.fft.fft2(p) / n
    a = np.abs(fp)
    u = np.where(a > 0, fp / np.where(a > 0, a, 1.0), 1.0)
    p2 = np.abs(p) ** 2
    return u, np.conj(p) / (p2 + EST_EPS * p2.max())


def network_input(counts, probe):
    """Real-space estimate of each window's object patch from its centred
    counts (..., N, N): the measured moduli in natural order, A = sqrt(max(d,
    0)), given the known probe's far-field phase, taken back to the sample
    plane by the unitary inverse transform and multiplied by g,
        est = g * F^-1(A u)  (= O for a flat, noise-free O times a real
        constant, up to the regulariser);
    its central (N/2) x (N/2) is upsampled 2x (nearest) to N x N, so that the
    network's (N/2) x (N/2) output grid lies on the target patch's pixels.
    Returns (..., N, N, 2): channels Re, Im."""
    d = np.asarray(counts, np.float64)
    n = d.shape[-1]
    u, g = probe_planes(probe)
    a = np.sqrt(np.maximum(np.fft.ifftshift(d, axes=(-2, -1)), 0.0))
    x = np.fft.ifft2(a * u, axes=(-2, -1)) * n
    est = (g * x)[..., n // 4:3 * n // 4, n // 4:3 * n // 4]
    est = np.repeat(np.repeat(est, 2, axis=-2), 2, axis=-1)
    return np.stack([est.real, est.imag], axis=-1)


def targets(obj, pos, n=128):
    """Amplitude and phase of the central n/2 x n/2 patch of each window at
    integer positions pos (J, 2): (J, n/2, n/2, 2)."""
    m, q = n // 2, n // 4
    out = np.empty((len(pos), m, m, 2))
    for j, (y, x) in enumerate(np.asarray(pos)):
        y, x = int(y), int(x)
        o = np.asarray(obj, np.complex128)[y + q:y + q + m, x + q:x + q + m]
        out[j, ..., 0] = np.abs(o)
        out[j, ..., 1] = np.angle(o)
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


def average(patches, pos, h, w, n=128):
    """Learned seed (h, w): the mean of the patches (J, 64, 64, 2) of amplitude
    and phase over the windows covering each pixel, placed as in stitch, with
    no phase factors; 1 where no patch covers a pixel."""
    p = np.asarray(patches, np.float64)
    c = p[..., 0] * np.exp(1j * p[..., 1])
    acc = np.zeros((h, w), np.complex128)
    cnt = np.zeros((h, w))
    for j, (ty, tx) in enumerate(placements(pos, n)):
        acc[ty:ty + PATCH, tx:tx + PATCH] += c[j]
        cnt[ty:ty + PATCH, tx:tx + PATCH] += 1
    out = np.ones((h, w), np.complex128)
    cov = cnt > 0
    out[cov] = acc[cov] / cnt[cov]
    return out
