"""Pins of the oracle's blind probe start: power by Parseval (every mode
photons / K, and the forward model of a flat object gives patterns whose
mean total is the photon count), support on the disk, orthogonal modes, the
constant first mode in closed form, and the count estimate."""
import math

import numpy as np
import pytest

import oracle


@pytest.mark.parametrize("k", [1, 2, 3, 4])
def test_guess_power_support_and_orthogonality(k):
    n, dia, photons = 32, 13.0, 2.5e6
    p = oracle.probe_guess(n, k, dia, photons)
    pw = np.sum(np.abs(p) ** 2, axis=(1, 2))
    assert np.max(np.abs(pw - photons / k)) <= 1e-9 * photons
    c = (n - 1) / 2
    u, v = np.meshgrid(np.arange(n) - c, np.arange(n) - c, indexing="ij")
    outside = u * u + v * v > (dia / 2) ** 2
    assert np.max(np.abs(p[:, outside])) == 0.0
    g = np.einsum("kxy,lxy->kl", p.conj(), p)
    assert np.max(np.abs(g - np.diag(np.diag(g)))) <= 1e-9 * photons
    # the first mode is the constant disk
    npix = int(np.count_nonzero(~outside))
    inside = p[0, ~outside]
    assert np.max(np.abs(inside - math.sqrt(photons / k / npix))) <= 1e-9 * abs(inside[0])
    # a flat object: mean pattern total = photons (unitary transform)
    pos = np.array([[0.0, 0.0], [1.5, 2.25]])
    cnt, _ = oracle.simulate(np.ones((40, 40), complex), p, pos)
    assert np.max(np.abs(np.sum(cnt, axis=(1, 2)) - photons)) <= 1e-8 * photons


def test_disk_pixel_count_for_an_odd_window():
    # pixel centres on integers around the centre of a 5 x 5 window: the
    # diameter-2 disk holds the centre and its 4 neighbours
    p = oracle.probe_guess(5, 1, 2.0, 5.0)
    assert np.count_nonzero(p) == 5 and np.allclose(np.abs(p[0, 2, 2]) ** 2, 1.0)


def test_photons_from_counts():
    d = np.zeros((3, 4, 4))
    d[0, 1, 1] = 6.0
    d[1] = 1.0
    d[2, 0, 0] = -5.0          # negative counts count as 0
    assert oracle.photons_from_counts(d) == (6.0 + 16.0 + 0.0) / 3
