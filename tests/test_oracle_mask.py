"""Pins of the oracle's detector mask (pixels without a measurement, Sec. 2.2's
saturated-pixel and noise-threshold preprocessing): no measurement means the
projection keeps the model there and the pixel adds nothing to the error or
the likelihood.  Checked against brute-force pixel loops, the projection's
own properties on the measured set, independence of the result from the
unmeasured counts, and finite differences of the masked likelihood."""
import numpy as np
import pytest

import oracle
import ptysynth


def _rng(seed):
    return np.random.default_rng([23, seed])


def _crandn(rng, *shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def _beamstop_mask(n, dead_col=None):
    """Centred mask: a 3 x 3 beam stop on the zero frequency and one dead column."""
    m = np.ones((n, n), np.uint8)
    c = n // 2
    m[c - 1:c + 2, c - 1:c + 2] = 0
    m[:, n // 4 if dead_col is None else dead_col] = 0
    return m


def test_mask_layout_follows_the_counts():
    n = 8
    d = np.arange(2 * n * n, dtype=float).reshape(2, n, n)
    m = np.ones((n, n), np.uint8)
    m[n // 2, n // 2] = 0           # the zero frequency, centred
    m[1, 6] = 0
    a = oracle.amplitude(d, m)
    assert np.isnan(a[:, 0, 0]).all()                                  # centre -> origin
    assert np.isnan(a[:, (1 + n // 2) % n, (6 + n // 2) % n]).all()
    assert np.count_nonzero(np.isnan(a)) == 4
    ok = ~np.isnan(a)
    assert np.array_equal(a[ok], oracle.amplitude(d)[ok])


def test_masked_projection_keeps_model_and_projects_the_rest():
    rng = _rng(1)
    psi = _crandn(rng, 3, 16, 16)
    a = rng.uniform(0.1, 4.0, (16, 16))
    a[2:5, 7] = np.nan
    a[11, 3] = np.nan
    d, _, _ = oracle.project_delta(psi, a)
    p1 = psi + d
    un = np.isnan(a)
    assert np.array_equal(p1[:, un], psi[:, un])                        # untouched, bit for bit
    mod = np.sqrt(np.sum(np.abs(p1) ** 2, axis=0))
    assert np.max(np.abs(mod[~un] - a[~un])) <= 1e-12                   # measured: modulus = A
    d2, _, _ = oracle.project_delta(p1, a)
    assert np.max(np.abs(d2)) <= 1e-12                                  # idempotent


def test_masked_error_sums_equal_pixel_loops():
    rng = _rng(2)
    n, k = 8, 2
    psi = _crandn(rng, k, n, n)
    a = rng.uniform(0.0, 3.0, (n, n))
    a[[0, 3, 3, 7], [0, 1, 2, 5]] = np.nan
    _, e1, e2 = oracle.project_delta(psi, a)
    s1 = s2 = 0.0
    for u in range(n):
        for v in range(n):
            if a[u, v] != a[u, v]:          # NaN: no measurement
                continue
            i = sum(abs(complex(psi[m, u, v])) ** 2 for m in range(k))
            s1 += (i ** 0.5 - a[u, v]) ** 2
            s2 += a[u, v] ** 2
    assert abs(e1 - s1) <= 1e-12 * s1 and abs(e2 - s2) <= 1e-12 * s2


def _tiny(k=2, n=32):
    wl = ptysynth.scaled(ptysynth.workload(1), cfg=41, n=n, k=k, h=80, w=80, d=13.0,
                         rows=5, cols=5, step=8.0, offset=6.0, j=25, photons=1e6)
    o = wl.obj()
    pos = wl.positions()
    cnt, p = oracle.simulate(o, wl.probe(), pos, wl.photons)
    cnt = ptysynth.poisson_counts(cnt, wl.noise_rng()).astype(np.float64)
    return o, p, pos, cnt


def _one_iteration(algo, o0, p0, a, pos):
    if algo == "epie":
        o, p, e = oracle.epie(o0, p0, a, pos, 1, start=0)
    elif algo == "dm":
        o, p, _, e = oracle.dm(o0, p0, oracle.dm_init(o0, p0, pos), a, pos, 1, start=0)
    else:
        o, p, e = oracle.lsqml(o0, p0, a, pos, 1, start=0, batch=10)
    return o, p, np.asarray(e)


@pytest.mark.parametrize("algo", ["epie", "dm", "lsqml"])
def test_reconstruction_ignores_unmeasured_counts(algo):
    o, p, pos, cnt = _tiny()
    n = p.shape[-1]
    m = _beamstop_mask(n)
    o0 = np.ones_like(o)
    garbage = cnt.copy()
    garbage[:, m == 0] = _rng(3).uniform(0, 1e7, (len(pos), int(np.count_nonzero(m == 0))))
    r1 = _one_iteration(algo, o0, p, oracle.amplitude(cnt, m), pos)
    r2 = _one_iteration(algo, o0, p, oracle.amplitude(garbage, m), pos)
    for x, y in zip(r1, r2):
        assert np.array_equal(x, y)
    # and the mask does change the iteration (the beam stop holds most counts;
    # DM's first object update precedes its first projection, so compare all)
    r0 = _one_iteration(algo, o0, p, oracle.amplitude(cnt), pos)
    assert any(not np.array_equal(x, y) for x, y in zip(r0, r1))


def test_masked_truth_stays_a_fixed_point():
    o, p, pos, _ = _tiny()
    cnt, _ = oracle.simulate(o, p, pos)             # noise-free, probe already scaled
    a = oracle.amplitude(cnt, _beamstop_mask(p.shape[-1]))
    o1, p1, e = oracle.epie(o, p, a, pos, 1, start=0)
    assert np.max(np.abs(o1 - o)) <= 1e-9 and np.max(np.abs(p1 - p)) <= 1e-9
    assert e[0] <= 1e-20


def test_masked_nll_loss_and_gradient():
    wl = ptysynth.scaled(ptysynth.workload(3), cfg=31, n=32, k=2, h=48, w=48, d=11.0,
                         sigma_e=1.0, sigma_p=3.0, photons=1e4)
    rng = _rng(4)
    pos = ptysynth.raster_positions(3, 3, 5.0, 1.0) + rng.uniform(0.1, 0.9, (9, 2))
    o = wl.obj()
    cnt, p = oracle.simulate(o, wl.probe(), pos, wl.photons)
    cnt = ptysynth.poisson_counts(cnt, wl.noise_rng()).astype(np.float64)
    o = o * (1 + 0.05 * _crandn(rng, *o.shape))
    m = _beamstop_mask(32, dead_col=3)
    loss, g_o, g_p, g_r = oracle.nll_grad(o, p, pos, cnt, mask=m)
    # the loss is the plain per-pixel sum over measured pixels
    valid = np.fft.ifftshift(m != 0)
    dn = np.fft.ifftshift(cnt, axes=(-2, -1))
    ref = 0.0
    for j, r in enumerate(pos):
        inten = oracle.forward_intensity(o, p, r)
        ref += float(np.sum((inten - dn[j] * np.log(inten + oracle.EPS_L))[valid]))
    assert abs(loss - ref) <= 1e-12 * abs(ref)
    assert abs(loss - oracle.nll(o, p, pos, cnt, mask=m)) <= 1e-12 * abs(loss)
    # changing unmeasured counts changes nothing
    g2 = cnt.copy()
    g2[:, m == 0] += 1e3
    l2, go2, gp2, gr2 = oracle.nll_grad(o, p, pos, g2, mask=m)
    assert l2 == loss and np.array_equal(go2, g_o) and np.array_equal(gp2, g_p) and np.array_equal(gr2, g_r)
    # central differences of the masked loss
    h = 1e-5
    d_o = _crandn(rng, *o.shape) * np.sqrt(np.mean(np.abs(o) ** 2))
    fd = (oracle.nll(o + h * d_o, p, pos, cnt, mask=m) - oracle.nll(o - h * d_o, p, pos, cnt, mask=m)) / (2 * h)
    an = float(np.real(np.vdot(g_o, d_o)))
    assert abs(fd - an) <= 1e-6 * abs(an)
    e = np.zeros_like(pos)
    e[4, 1] = 1e-4
    fd = (oracle.nll(o, p, pos + e, cnt, mask=m) - oracle.nll(o, p, pos - e, cnt, mask=m)) / 2e-4
    assert abs(fd - g_r[4, 1]) <= 1e-6 * abs(g_r[4, 1])
