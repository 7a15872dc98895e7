"""Pins of the FP64 reference of the learned seed's data path: stitching
recovers an object exactly from consistent patches with arbitrary per-patch
phase offsets, the chain's special cases, targets and inputs in closed form."""
import numpy as np

import ptysynth
from oracle import seed


def _object(h, w, s=5):
    rng = np.random.default_rng(s)
    amp = 0.8 + 0.2 * rng.uniform(size=(h, w))
    ph = rng.uniform(-2.5, 2.5, size=(h, w))
    return amp * np.exp(1j * ph)


def _cut(obj, pos, rng):
    """Patches of the object at the oracle's placements, each with a random phase offset."""
    t = seed.placements(pos)
    out = np.empty((len(t), 64, 64, 2))
    for j, (ty, tx) in enumerate(t):
        o = obj[ty:ty + 64, tx:tx + 64] * np.exp(1j * rng.uniform(-np.pi, np.pi))
        out[j, ..., 0] = np.abs(o)
        out[j, ..., 1] = np.angle(o)
    return out, t


def test_stitch_recovers_consistent_patches_up_to_global_phase():
    h, w = 300, 280
    obj = _object(h, w)
    pos = ptysynth.spiral_positions(60, 6.0, 140.0, 128)
    pos += np.random.default_rng(1).uniform(0.0, 1.0, pos.shape)   # fractional parts round both ways
    rng = np.random.default_rng(2)
    patches, t = _cut(obj, pos, rng)
    out, e = seed.stitch(patches, pos, h, w)
    cov = np.zeros((h, w), bool)
    for ty, tx in t:
        cov[ty:ty + 64, tx:tx + 64] = True
    g = out[cov] / obj[cov]
    assert np.allclose(np.abs(g), 1.0, atol=1e-12)
    assert np.allclose(g, g[0], atol=1e-10)          # one global phase everywhere
    assert np.all(out[~cov] == 1.0)
    assert abs(e[0] - 1.0) == 0.0                     # the first patch has nothing to align to


def test_stitch_single_patch_and_disjoint_patches():
    h, w = 256, 256
    rng = np.random.default_rng(3)
    p = np.stack([rng.uniform(0.5, 1.0, (2, 64, 64)), rng.uniform(-3, 3, (2, 64, 64))], axis=-1)
    pos = np.array([[0.2, 0.4], [120.0, 110.6]])     # placements (32, 32) and (152, 143): disjoint
    out, e = seed.stitch(p, pos, h, w)
    np.testing.assert_allclose(out[32:96, 32:96], p[0, ..., 0] * np.exp(1j * p[0, ..., 1]), atol=1e-13)
    np.testing.assert_allclose(out[152:216, 143:207], p[1, ..., 0] * np.exp(1j * p[1, ..., 1]), atol=1e-13)
    assert np.all(e == 1.0)
    assert np.all(out[:32] == 1.0)


def test_placement_rounding():
    t = seed.placements(np.array([[10.49, 10.5], [0.0, 7.999]]))
    assert t.tolist() == [[42, 43], [32, 40]]


def test_targets_closed_form():
    rng = np.random.default_rng(4)
    obj = _object(200, 220, 6)
    pos = rng.integers(0, 70, size=(5, 2))
    tg = seed.targets(obj, pos)
    for j, (y, x) in enumerate(pos):
        o = obj[y + 32:y + 96, x + 32:x + 96]
        v = tg[j, ..., 0] * np.exp(1j * tg[j, ..., 1])
        # amplitude and phase of the patch itself: they recombine to it
        np.testing.assert_allclose(v, o, atol=1e-12)
        assert np.all(tg[j, ..., 0] >= 0) and np.all(np.abs(tg[j, ..., 1]) <= np.pi)


def test_average_of_patches():
    """Patches cut from an object (consistent phases) average back to it on
    every covered pixel, exactly; a pixel covered by two patches gets their
    mean; uncovered pixels are 1."""
    rng = np.random.default_rng(7)
    obj = _object(300, 280, 8)
    pos = rng.uniform(0, 150, size=(30, 2))
    t = seed.placements(pos)
    p = np.empty((len(pos), 64, 64, 2))
    for j, (ty, tx) in enumerate(t):
        o = obj[ty:ty + 64, tx:tx + 64]
        p[j, ..., 0], p[j, ..., 1] = np.abs(o), np.angle(o)
    out = seed.average(p, pos, 300, 280)
    cov = np.zeros((300, 280), bool)
    for ty, tx in t:
        cov[ty:ty + 64, tx:tx + 64] = True
    np.testing.assert_allclose(out[cov], obj[cov], atol=1e-12)
    assert np.all(out[~cov] == 1.0)
    # two overlapping patches of different values: their mean where they overlap
    q = np.zeros((2, 64, 64, 2))
    q[0, ..., 0], q[1, ..., 0], q[1, ..., 1] = 1.0, 2.0, np.pi / 2
    two = seed.average(q, np.array([[0.0, 0.0], [0.0, 32.0]]), 128, 160)
    assert two[40, 40] == 1.0 and abs(two[40, 70] - (1 + 2j) / 2) < 1e-12 and abs(two[40, 100] - 2j) < 1e-12


def _probe(n, rng):
    y, x = np.mgrid[:n, :n] - n / 2
    amp = np.exp(-(x ** 2 + y ** 2) / (2 * (n / 6) ** 2))
    return amp * np.exp(1j * (0.3 * rng.standard_normal((n, n)) + 0.02 * (x ** 2 + y ** 2)))


def _input_brute_force(d, p):
    """The network input written out for a tiny window: DFT sums, index
    arithmetic for the centring, the crop and the 2x repetition."""
    n = p.shape[0]
    # far-field phase of the probe by the DFT definition (unitary)
    fp = np.zeros((n, n), complex)
    for a in range(n):
        for b in range(n):
            fp[a, b] = sum(p[u, v] * np.exp(-2j * np.pi * (a * u + b * v) / n)
                           for u in range(n) for v in range(n)) / n
    uphase = fp / np.abs(fp)
    p2 = np.abs(p) ** 2
    g = np.conj(p) / (p2 + 0.01 * p2.max())
    # natural-order moduli: natural frequency a sits at centred index (a + n/2) mod n
    amp = np.array([[np.sqrt(max(d[(a + n // 2) % n, (b + n // 2) % n], 0.0)) for b in range(n)]
                    for a in range(n)])
    out = np.zeros((n, n, 2))
    for y in range(n):
        for xx in range(n):
            r, c = n // 4 + y // 2, n // 4 + xx // 2
            v = sum(amp[a, b] * uphase[a, b] * np.exp(2j * np.pi * (a * r + b * c) / n)
                    for a in range(n) for b in range(n)) / n
            v *= g[r, c]
            out[y, xx] = v.real, v.imag
    return out


def test_network_input_brute_force():
    """Against the definition on an 8 x 8 window (any slip in the centring,
    the transform direction or scale, the crop or the repetition changes it)."""
    rng = np.random.default_rng(12)
    p = _probe(8, rng)
    d = rng.uniform(0.0, 40.0, (8, 8))
    d[0, 3] = -2.0   # negative counts read as 0
    np.testing.assert_allclose(seed.network_input(d, p), _input_brute_force(d, p), atol=1e-12)
    # two planted mistakes the check catches: the forward transform, and the
    # centred pattern used without moving zero frequency to the corner
    wrong_dir = np.fft.fft2(np.sqrt(np.maximum(np.fft.ifftshift(d), 0)) * seed.probe_planes(p)[0]) / 8
    assert not np.allclose((seed.probe_planes(p)[1] * wrong_dir)[2:6, 2:6].real,
                           _input_brute_force(d, p)[::2, ::2, 0], atol=1e-3)
    shifted = seed.network_input(np.fft.ifftshift(d), p)
    assert not np.allclose(shifted, _input_brute_force(d, p), atol=1e-3)


def test_network_input_of_a_flat_object():
    """O = c (constant, complex) and noise-free counts: the estimate is
    |c| |P|^2 / (|P|^2 + 0.01 max |P|^2), real, on the window's centre (the
    pattern fixes O only up to a global phase)."""
    rng = np.random.default_rng(13)
    n = 32
    p = _probe(n, rng)
    c = 0.9 * np.exp(0.7j)
    d = np.fft.fftshift(np.abs(np.fft.fft2(c * p) / n) ** 2)
    x = seed.network_input(d, p)
    p2 = np.abs(p) ** 2
    want = abs(c) * p2 / (p2 + 0.01 * p2.max())
    want = np.repeat(np.repeat(want[n // 4:3 * n // 4, n // 4:3 * n // 4], 2, axis=0), 2, axis=1)
    np.testing.assert_allclose(x[..., 0], want, atol=1e-12)
    np.testing.assert_allclose(x[..., 1], 0.0, atol=1e-12)
    # batched counts give the same per pattern
    xb = seed.network_input(np.stack([d, 4 * d]), p)
    np.testing.assert_allclose(xb[1], 2 * x, atol=1e-12)
