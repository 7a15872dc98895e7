"""Pins of the oracle's Poisson exit-wave update (LSQML with the Poisson
likelihood, Odstrcil et al. 2018 as cited for LSQML in Sec. 2.3):

* its step is the minimiser along the ray of the likelihood evaluated from
  its definition (a direct sum over modes), found by a brute-force 1-D
  minimisation (a dense grid, then scipy's bounded scalar minimiser);
* with a uniform measured/model ratio c the step has the closed form
  1 / (1 + sqrt(c)) and moves every intensity onto the data;
* its direction is the likelihood gradient that ``nll_grad`` gives (itself
  pinned by finite differences);
* unmeasured pixels take no part in it;
* on consistent data the update vanishes, and LSQML with it lowers the
  Poisson likelihood of a perturbed start."""
import numpy as np
import pytest

import oracle
import ptysynth


def _crandn(rng, *shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def _field(k=3, n=16, seed=0):
    rng = np.random.default_rng([77, seed])
    psi = _crandn(rng, k, n, n) * 4.0
    inten = np.sum(np.abs(psi) ** 2, axis=0)
    d = rng.poisson(inten).astype(np.float64)
    return psi, inten, d


def _likelihood_on_ray(psi, d, g, alpha):
    """L(alpha) of the far field Psi (1 - alpha g), summed from the modes
    (eps = 0, log(d!) dropped)."""
    moved = psi * (1.0 - alpha * g)[None]
    inten = np.sum(np.abs(moved) ** 2, axis=0)
    with np.errstate(divide="ignore"):
        logs = np.where(d > 0, d * np.log(np.where(d > 0, inten, 1.0)), 0.0)   # 0 log 0 = 0
    return float(np.sum(inten - logs))


def _brute_minimiser(psi, d, g):
    """argmin over [0, 1] of the likelihood on the ray: the best of 20,001 grid
    points, then scipy's bounded minimiser around it."""
    from scipy.optimize import minimize_scalar
    grid = np.linspace(0.0, 1.0, 20001)
    vals = [_likelihood_on_ray(psi, d, g, a) for a in grid]
    k = int(np.argmin(vals))
    lo, hi = grid[max(k - 1, 0)], grid[min(k + 1, len(grid) - 1)]
    r = minimize_scalar(lambda a: _likelihood_on_ray(psi, d, g, a), bounds=(lo, hi), method="bounded",
                        options={"xatol": 1e-12})
    return float(r.x)


@pytest.mark.parametrize("seed,dose", [(0, 4.0), (3, 0.3), (4, 30.0)])
def test_step_minimises_the_likelihood_on_the_ray(seed, dose):
    rng = np.random.default_rng([78, seed])
    psi = _crandn(rng, 3, 16, 16) * dose
    inten = np.sum(np.abs(psi) ** 2, axis=0)
    d = rng.poisson(inten).astype(np.float64)
    d[0, :3] = 5.0 * inten[0, :3] + 3.0           # a few pixels far above the model
    g = 1.0 - d / inten
    want = _brute_minimiser(psi, d, g)
    got = oracle.poisson_step(inten, d, eps=0.0)
    assert 0.0 < got <= 1.0
    assert abs(got - want) <= 1e-6 * want, (got, want)
    # no point of the ray has a lower likelihood
    l_got = _likelihood_on_ray(psi, d, g, got)
    for a in np.linspace(0.0, 1.0, 101):
        assert l_got <= _likelihood_on_ray(psi, d, g, a) + 1e-9 * abs(l_got)
    # a planted mistake the pin catches: one Newton step from 0 instead
    num = float(np.sum(inten * g * g))
    den = float(np.sum((inten + d) * g * g))
    assert abs(num / den - want) > 1e-3 * want


@pytest.mark.parametrize("c", [0.25, 0.9, 1.0, 1.7, 4.0])
def test_uniform_ratio_closed_form(c):
    psi, inten, _ = _field(seed=1)
    d = c * inten
    a = oracle.poisson_step(inten, d, eps=0.0)
    if c == 1.0:
        assert a == 0.0                      # nothing to correct
        return
    assert abs(a - 1.0 / (1.0 + np.sqrt(c))) <= 1e-12
    delta, alpha, _, _ = oracle.poisson_delta(psi, np.sqrt(d), eps=0.0)
    # every mode scaled by s = 1 - alpha (1 - c) = sqrt(c): the moved intensity is the data
    assert np.max(np.abs(psi + delta - np.sqrt(c) * psi)) <= 1e-12 * np.max(np.abs(psi))


def test_direction_is_the_likelihood_gradient():
    # one position over a flat object: nll_grad's probe gradient is 2 g_psi,
    # g_psi = F^-1[(1 - d / (I + eps)) Psi], and the update is -alpha_R g_psi
    rng = np.random.default_rng(5)
    n, k = 16, 2
    probe = _crandn(rng, k, n, n) * 0.5
    obj = np.ones((n, n), complex)
    pos = np.zeros((1, 2))
    inten = oracle.forward_intensity(obj, probe, pos[0])
    d = rng.poisson(inten).astype(np.float64)
    centred = np.fft.fftshift(d)
    _, _, g_p, _ = oracle.nll_grad(obj, probe, pos, centred[None])
    delta, _, _, _ = oracle.poisson_delta(oracle.fft2u(probe * obj[None]), oracle.amplitude(centred))
    chi = oracle.ifft2u(delta)
    alpha = oracle.poisson_step(inten, d)
    assert alpha > 0
    assert np.max(np.abs(chi + alpha * g_p / 2)) <= 1e-12 * np.max(np.abs(chi))


def test_unmeasured_pixels_take_no_part():
    psi, inten, d = _field(seed=2)
    mask = np.ones(d.shape, bool)
    mask[3:7, 5:9] = False
    a = np.where(mask, np.sqrt(d), np.nan)
    delta, alpha, e1, e2 = oracle.poisson_delta(psi, a)
    assert np.all(delta[:, ~mask] == 0)
    # the same step as from the measured pixels alone
    assert alpha == pytest.approx(oracle.poisson_step(inten[mask], d[mask]), rel=1e-14)
    # changing the data under the mask changes nothing
    d2 = d.copy()
    d2[~mask] *= 7.0
    delta2, alpha2, _, _ = oracle.poisson_delta(psi, np.where(mask, np.sqrt(d2), np.nan))
    assert alpha2 == alpha and np.array_equal(delta2, delta)


def _tiny(noise):
    wl = ptysynth.scaled(ptysynth.workload(1), cfg=44, n=32, k=2, h=80, w=80, d=13.0,
                         rows=5, cols=5, step=8.0, offset=6.0, j=25, photons=1e6)
    o = wl.obj()
    pos = wl.positions()
    cnt, p = oracle.simulate(o, wl.probe(), pos, wl.photons)
    if noise:
        cnt = ptysynth.poisson_counts(cnt, wl.noise_rng()).astype(np.float64)
    return o, p, pos, cnt


def test_consistent_data_leave_the_state():
    o, p, pos, cnt = _tiny(noise=False)
    a = oracle.amplitude(cnt)
    o1, p1, err = oracle.lsqml(o, p, a, pos, 1, start=0, batch=10, likelihood="poisson")
    assert np.max(np.abs(o1 - o)) <= 1e-6 * np.max(np.abs(o))
    assert np.max(np.abs(p1 - p)) <= 1e-6 * np.max(np.abs(p))
    assert err[0] <= 1e-12                    # rounding only


def test_poisson_lsqml_lowers_the_likelihood():
    o, p, pos, cnt = _tiny(noise=True)
    a = oracle.amplitude(cnt)
    rng = np.random.default_rng(6)
    o0 = o * (1 + 0.1 * _crandn(rng, *o.shape))
    p0 = p * (1 + 0.05 * _crandn(rng, *p.shape))
    l_prev = oracle.nll(o0, p0, pos, cnt)
    o1, p1 = o0, p0
    for _ in range(3):
        o1, p1, _ = oracle.lsqml(o1, p1, a, pos, 1, start=0, batch=10, likelihood="poisson")
        l_now = oracle.nll(o1, p1, pos, cnt)
        assert l_now < l_prev
        l_prev = l_now


def test_unknown_likelihood_is_rejected():
    o, p, pos, cnt = _tiny(noise=False)
    with pytest.raises(ValueError):
        oracle.lsqml(o, p, oracle.amplitude(cnt), pos, 1, likelihood="gauss")
