"""Pins of the FP64 oracle against what mathematics and the cited methods fix.

None of these re-derives the oracle from its own formulas: each compares it to
a brute-force definition, a closed form, an invariant, a special case that
reduces to a textbook routine, or a library solver.
"""
import math

import numpy as np
import pytest

import oracle
import ptysynth


def _rng(seed):
    return np.random.default_rng(seed)


def _crandn(rng, *shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


# ---------------------------------------------------------------------------
# F: unitary 2-D DFT, natural order
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("n", [2, 3, 4, 8, 16])
def test_fft_equals_bruteforce_dft(n):
    rng = _rng(n)
    x = _crandn(rng, n, n)
    idx = np.arange(n)
    w = np.exp(-2j * math.pi * np.outer(idx, idx) / n)  # 1-D DFT matrix
    ref = (w @ x @ w.T) / n                              # N^-1 sum over both axes
    assert np.max(np.abs(oracle.fft2u(x) - ref)) <= 1e-12
    assert np.max(np.abs(oracle.ifft2u(ref) - x)) <= 1e-12


def test_fft_parseval_inverse_and_dc():
    rng = _rng(1)
    x = _crandn(rng, 3, 32, 32)
    y = oracle.fft2u(x)
    assert abs(np.sum(np.abs(x) ** 2) - np.sum(np.abs(y) ** 2)) <= 1e-10 * np.sum(np.abs(x) ** 2)
    assert np.max(np.abs(oracle.ifft2u(y) - x)) <= 1e-14 * 1e2
    c = np.full((16, 16), 2.5 - 1.0j)
    yc = oracle.fft2u(c)
    assert abs(yc[0, 0] - 16 * (2.5 - 1.0j)) <= 1e-12
    yc[0, 0] = 0
    assert np.max(np.abs(yc)) <= 1e-12


# ---------------------------------------------------------------------------
# Gather S_j and its adjoint
# ---------------------------------------------------------------------------
def test_gather_scatter_adjoint():
    rng = _rng(2)
    h, w, n = 40, 37, 16
    for _ in range(10):
        r = rng.uniform(0, [h - n - 1, w - n - 1])
        x = _crandn(rng, h, w)
        y = _crandn(rng, n, n)
        lhs = np.vdot(oracle.gather(x, r, n), y)
        acc = np.zeros((h, w), complex)
        oracle.scatter_add(acc, y, r)
        rhs = np.vdot(x, acc)
        assert abs(lhs - rhs) <= 1e-13 * max(1.0, abs(lhs)) * 10


def test_gather_integer_is_slice_and_constants_preserved():
    rng = _rng(3)
    o = _crandn(rng, 30, 30)
    np.testing.assert_array_equal(oracle.gather(o, (5.0, 7.0), 8), o[5:13, 7:15])
    # the last valid integer position reads the last rows without touching row H
    np.testing.assert_array_equal(oracle.gather(o, (22.0, 22.0), 8), o[22:30, 22:30])
    c = np.full((30, 30), 0.3 + 0.2j)
    p = oracle.gather(c, (4.37, 9.91), 8)
    assert np.max(np.abs(p - (0.3 + 0.2j))) <= 1e-15


def test_gather_reproduces_linear_ramps():
    # bilinear interpolation is exact on affine functions: O = a + b y + c x
    h = w = 32
    yy, xx = np.meshgrid(np.arange(h), np.arange(w), indexing="ij")
    a, b, c = 0.7 - 0.1j, 0.03 + 0.02j, -0.05 + 0.04j
    o = a + b * yy + c * xx
    for r in [(3.25, 4.75), (10.9, 0.1), (0.5, 12.0)]:
        u, v = np.meshgrid(np.arange(8), np.arange(8), indexing="ij")
        ref = a + b * (r[0] + u) + c * (r[1] + v)
        assert np.max(np.abs(oracle.gather(o, r, 8) - ref)) <= 1e-13


def test_gather_grad_matches_finite_difference():
    rng = _rng(4)
    o = _crandn(rng, 24, 24)
    r = np.array([5.3, 7.6])
    dy, dx = oracle.gather_grad(o, r, 8)
    h = 1e-6
    fy = (oracle.gather(o, r + [h, 0], 8) - oracle.gather(o, r - [h, 0], 8)) / (2 * h)
    fx = (oracle.gather(o, r + [0, h], 8) - oracle.gather(o, r - [0, h], 8)) / (2 * h)
    assert np.max(np.abs(dy - fy)) <= 1e-8
    assert np.max(np.abs(dx - fx)) <= 1e-8


# ---------------------------------------------------------------------------
# Modulus projection
# ---------------------------------------------------------------------------
def _proj(psi_f, a):
    d, _, _ = oracle.project_delta(psi_f, a)
    return psi_f + d


def test_projection_modulus_idempotence_and_shared_ratio():
    rng = _rng(5)
    psi = _crandn(rng, 3, 16, 16)
    a = rng.uniform(0.1, 4.0, (16, 16))
    p1 = _proj(psi, a)
    # the mode-summed modulus equals the measurement exactly
    assert np.max(np.abs(np.sqrt(np.sum(np.abs(p1) ** 2, axis=0)) - a)) <= 1e-12
    # idempotent
    assert np.max(np.abs(_proj(p1, a) - p1)) <= 1e-12
    # every mode is scaled by the same real non-negative ratio
    ratio = p1 / psi
    assert np.max(np.abs(ratio.imag)) <= 1e-12
    assert np.max(np.abs(ratio - ratio[0:1])) <= 1e-12
    assert np.all(ratio.real >= 0)


def test_projection_is_nearest_point():
    rng = _rng(6)
    psi = _crandn(rng, 2, 12, 12)
    a = rng.uniform(0.1, 3.0, (12, 12))
    p = _proj(psi, a)
    best = np.linalg.norm(p - psi)
    for _ in range(50):
        x = _crandn(rng, 2, 12, 12)
        x = x * (a / np.sqrt(np.sum(np.abs(x) ** 2, axis=0)))[None]   # same moduli
        assert np.linalg.norm(x - psi) >= best - 1e-12


def test_projection_zero_data_and_zero_field():
    rng = _rng(7)
    psi = _crandn(rng, 2, 8, 8)
    assert np.max(np.abs(_proj(psi, np.zeros((8, 8))))) == 0.0
    z = np.zeros((2, 8, 8), complex)
    assert np.max(np.abs(_proj(z, np.ones((8, 8))))) == 0.0


def test_amplitude_moves_centre_to_origin():
    d = np.zeros((8, 8))
    d[4, 4] = 9.0
    a = oracle.amplitude(d)
    assert a[0, 0] == 3.0 and np.count_nonzero(a) == 1


# ---------------------------------------------------------------------------
# Synthetic inputs and the error metric
# ---------------------------------------------------------------------------
def _tiny(k=1, n=32, noise=False, seed_cfg=11):
    wl = ptysynth.scaled(ptysynth.workload(1), cfg=seed_cfg, n=n, k=k, h=80, w=80, d=13.0,
                         rows=5, cols=5, step=8.0, offset=6.0, j=25, photons=1e6)
    o = wl.obj()
    p0 = wl.probe()
    pos = wl.positions()
    cnt, p = oracle.simulate(o, p0, pos, wl.photons)
    if noise:
        cnt = ptysynth.poisson_counts(cnt, wl.noise_rng()).astype(np.float64)
    return wl, o, p, pos, cnt


def test_generator_photons_modes_and_coverage():
    wl, o, p, pos, cnt = _tiny(k=3)
    assert abs(np.mean(np.sum(cnt, axis=(1, 2))) - wl.photons) <= 1e-9 * wl.photons
    e = ptysynth.probe_modes_orthonormal(wl.cfg, wl.n, 3, wl.d, wl.sigma_e, wl.sigma_p, wl.n_fresnel)
    gram = np.einsum("kij,lij->kl", e.conj(), e)
    assert np.max(np.abs(gram - np.eye(3))) <= 1e-12
    for cfg in (1, 2, 3, 4):
        w = ptysynth.workload(cfg)
        q = w.positions()
        assert q.shape == (w.j, 2)
        assert q.min() >= 0 and np.all(np.floor(q) + w.n + 1 <= [w.h, w.w])
    amp = np.abs(o)
    assert amp.min() >= 0.8 - 1e-12 and amp.max() <= 1.0 + 1e-12


def test_error_zero_at_truth_and_invariances():
    wl, o, p, pos, cnt = _tiny(k=3)
    a = oracle.amplitude(cnt)
    assert oracle.model_error(o, p, a, pos) <= 1e-24
    rng = _rng(8)
    o2 = o * np.exp(1j * 0.1) * 1.1
    p2 = p * (1.0 + 0.05 * _crandn(rng, *p.shape))
    e_ref = oracle.model_error(o2, p2, a, pos)
    c = 0.7 * np.exp(0.3j)
    assert abs(oracle.model_error(o2 * c, p2 / c, a, pos) - e_ref) <= 1e-10 * e_ref
    q, _ = np.linalg.qr(_crandn(rng, 3, 3))   # unitary mode mixing
    p3 = np.einsum("kl,lij->kij", q, p2)
    assert abs(oracle.model_error(o2, p3, a, pos) - e_ref) <= 1e-10 * e_ref


# ---------------------------------------------------------------------------
# ePIE
# ---------------------------------------------------------------------------
def _er_step(o, a):
    """Error reduction with a pure Fourier-modulus constraint (Fienup 1982), via numpy.fft."""
    f = np.fft.fft2(o)
    return np.fft.ifft2(a * f / np.abs(f)) if a.ndim == 2 else None


def test_epie_fixed_point_at_truth():
    wl, o, p, pos, cnt = _tiny(k=2)
    a = oracle.amplitude(cnt)
    o1, p1, err = oracle.epie(o, p, a, pos, 1, start=0)
    assert np.max(np.abs(o1 - o)) <= 1e-12 and np.max(np.abs(p1 - p)) <= 1e-12
    assert err[0] <= 1e-24


def test_epie_single_flat_position_is_error_reduction():
    rng = _rng(9)
    n = 16
    o = _crandn(rng, n, n)
    a = rng.uniform(0.5, 2.0, (n, n)) * n   # moduli of the unitary far field
    p = np.ones((1, n, n), complex)
    o1, p1, _ = oracle.epie(o, p, a[None], np.array([[0.0, 0.0]]), 1, start=1)
    # numpy.fft uses the unnormalised forward transform: the measured moduli scale by N
    ref = _er_step(o, a * n)
    assert np.max(np.abs(o1 - ref)) <= 1e-12
    np.testing.assert_array_equal(p1, p)


def test_epie_order_is_seeded_permutation():
    assert list(oracle.epie_order(7, 0, 3)) == list(range(7))
    s = oracle.epie_order(50, 12345, 2)
    assert sorted(s) == list(range(50)) and list(s) != list(range(50))
    assert list(s) == list(oracle.epie_order(50, 12345, 2))
    assert list(s) != list(oracle.epie_order(50, 12345, 3))


def test_splitmix64_published_outputs():
    # first two outputs of SplitMix64 from state 0 (Steele, Lea & Flood 2014, as
    # in the public-domain reference splitmix64.c)
    g = oracle.splitmix64_stream(0)
    assert next(g) == 0xE220A8397B1DCDAF
    assert next(g) == 0x6E789E6AA1B965F4


# ---------------------------------------------------------------------------
# DM
# ---------------------------------------------------------------------------
def test_dm_fixed_point_at_truth():
    wl, o, p, pos, cnt = _tiny(k=2)
    a = oracle.amplitude(cnt)
    psi = oracle.dm_init(o, p, pos)
    o1, p1, psi1, err = oracle.dm(o, p, psi, a, pos, 1, start=0)
    assert np.max(np.abs(o1 - o)) <= 1e-12
    assert np.max(np.abs(p1 - p)) <= 1e-12
    assert np.max(np.abs(psi1 - psi)) <= 1e-12
    assert err[0] <= 1e-24


def test_dm_single_flat_position_is_error_reduction():
    rng = _rng(10)
    n = 16
    o = _crandn(rng, n, n)
    a = rng.uniform(0.5, 2.0, (n, n)) * n
    p = np.ones((1, n, n), complex)
    pos = np.array([[0.0, 0.0]])
    psi = oracle.dm_init(o, p, pos)
    o1, _, psi1, _ = oracle.dm(o, p, psi, a[None], pos, 1, start=5)
    assert np.max(np.abs(o1 - o)) <= 1e-12
    assert np.max(np.abs(psi1[0, 0] - _er_step(o, a * n))) <= 1e-12


def test_dm_overlap_steps_solve_normal_equations():
    rng = _rng(11)
    n, h = 16, 48
    pos = ptysynth.raster_positions(4, 4, 8.0, 4.0)
    o = _crandn(rng, h, h)
    p = _crandn(rng, 2, n, n)
    psi = _crandn(rng, len(pos), 2, n, n)
    a = np.ones((len(pos), n, n))
    # object step only (probe update later than this iteration)
    o1, _, _, _ = oracle.dm(o, p, psi, a, pos, 1, start=5, gamma_obj=1e-14)
    res = np.zeros((h, h), complex)
    cov = np.zeros((h, h))
    for j, r in enumerate(pos):
        oj = o1[int(r[0]):int(r[0]) + n, int(r[1]):int(r[1]) + n]
        res[int(r[0]):int(r[0]) + n, int(r[1]):int(r[1]) + n] += np.sum(np.conj(p) * (p * oj - psi[j]), axis=0)
        cov[int(r[0]):int(r[0]) + n, int(r[1]):int(r[1]) + n] += 1
    scale = np.max(np.abs(np.sum(np.conj(p) * psi[0], axis=0)))
    assert np.max(np.abs(res[cov > 0])) <= 1e-10 * scale
    # probe step with the new object
    _, p1, _, _ = oracle.dm(o, p, psi, a, pos, 1, start=0, gamma_obj=1e-14, gamma_probe=1e-14)
    resp = np.zeros_like(p)
    for j, r in enumerate(pos):
        oj = o1[int(r[0]):int(r[0]) + n, int(r[1]):int(r[1]) + n]
        resp += np.conj(oj)[None] * (p1 * oj[None] - psi[j])
    assert np.max(np.abs(resp)) <= 1e-10 * np.max(np.abs(np.conj(o1[:n, :n])[None] * psi[0]))


# ---------------------------------------------------------------------------
# LSQML
# ---------------------------------------------------------------------------
def test_lsqml_step_equals_regularised_lstsq():
    rng = _rng(12)
    for probe_on in (True, False):
        for _ in range(20):
            av = _crandn(rng, 2, 8, 8)
            bv = _crandn(rng, 2, 8, 8) if probe_on else np.zeros((2, 8, 8), complex)
            chi = _crandn(rng, 2, 8, 8)
            m00 = float(np.sum(np.abs(av) ** 2))
            m11 = float(np.sum(np.abs(bv) ** 2))
            m01 = float(np.real(np.vdot(av, bv)))
            v0 = float(np.real(np.vdot(av, chi)))
            v1 = float(np.real(np.vdot(bv, chi)))
            got = oracle.lsqml_solve2(m00, m11, m01, v0, v1, probe_on)
            eta = 1e-6 * max(m00, m11)
            cols = [np.concatenate([av.real.ravel(), av.imag.ravel()])]
            if probe_on:
                cols.append(np.concatenate([bv.real.ravel(), bv.imag.ravel()]))
            mat = np.stack(cols, axis=1)
            rhs = np.concatenate([chi.real.ravel(), chi.imag.ravel()])
            # Tikhonov-regularised least squares, written as an augmented system
            aug = np.vstack([mat, math.sqrt(eta) * np.eye(mat.shape[1])])
            sol = np.linalg.lstsq(aug, np.concatenate([rhs, np.zeros(mat.shape[1])]), rcond=None)[0]
            if not probe_on:
                sol = np.array([sol[0], 0.0])
            assert np.max(np.abs(np.asarray(got) - sol)) <= 1e-10 * max(1.0, np.max(np.abs(sol)))
    assert oracle.lsqml_solve2(0.0, 0.0, 0.0, 1.0, 1.0) == (0.0, 0.0)


def test_lsqml_single_flat_position_is_error_reduction():
    rng = _rng(13)
    n = 16
    o = _crandn(rng, n, n)
    a = rng.uniform(0.5, 2.0, (n, n)) * n
    p = np.ones((1, n, n), complex)
    o1, _, _ = oracle.lsqml(o, p, a[None], np.array([[0.0, 0.0]]), 1, start=5)
    # den_O = 1, so the direction is chi / (1 + 1e-3); the optimal step length is
    # (1 + 1e-3) / (1 + 1e-6) (eta = 1e-6 |a|^2), hence O1 = O + chi / (1 + 1e-6)
    er = _er_step(o, a * n)
    ref = o + (er - o) / (1.0 + 1e-6)
    assert np.max(np.abs(o1 - ref)) <= 1e-12 * np.max(np.abs(er))


def test_lsqml_fixed_point_at_truth():
    wl, o, p, pos, cnt = _tiny(k=2)
    a = oracle.amplitude(cnt)
    o1, p1, err = oracle.lsqml(o, p, a, pos, 1, start=0)
    assert np.max(np.abs(o1 - o)) <= 1e-12 and np.max(np.abs(p1 - p)) <= 1e-12
    assert err[0] <= 1e-24


# ---------------------------------------------------------------------------
# Convergence on noise-free data with the true probe, and NRMSE
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("algo", ["epie", "dm", "lsqml"])
def test_noise_free_convergence(algo):
    wl, o_true, p, pos, cnt = _tiny(k=1)
    a = oracle.amplitude(cnt)
    o0 = np.ones_like(o_true)
    mask = oracle.roi_mask(p, pos, wl.h, wl.w)
    start = 10
    if algo == "epie":
        o1, _, err = oracle.epie(o0, p, a, pos, 50, start=start)
    elif algo == "dm":
        o1, _, _, err = oracle.dm(o0, p, oracle.dm_init(o0, p, pos), a, pos, 50, start=start)
    else:
        o1, _, err = oracle.lsqml(o0, p, a, pos, 50, start=start)
    assert err[-1] <= 0.1 * err[0]
    assert oracle.nrmse(o1, o_true, mask) < 0.5 * oracle.nrmse(o0, o_true, mask)


def test_nrmse_invariance_and_closed_form():
    rng = _rng(14)
    t = _crandn(rng, 20, 20)
    mask = np.ones((20, 20), bool)
    mask[:3] = False
    for c in (1.0, -2.0, 0.3 + 4j, 1e-3j):
        assert oracle.nrmse(c * t, t, mask) <= 1e-14
    o = t + 0.1 * _crandn(rng, 20, 20)
    # closed form: the optimum over c of ||cO - T|| is sqrt(1 - |<O,T>|^2 / (|O|^2 |T|^2))
    om, tm = o[mask], t[mask]
    ref = math.sqrt(1 - abs(np.vdot(om, tm)) ** 2 / (np.vdot(om, om).real * np.vdot(tm, tm).real))
    assert abs(oracle.nrmse(o, t, mask) - ref) <= 1e-12


# ---------------------------------------------------------------------------
# Poisson NLL adjoint
# ---------------------------------------------------------------------------
def _fd_case():
    wl = ptysynth.scaled(ptysynth.workload(3), cfg=31, n=32, k=4, h=48, w=48, d=11.0,
                         sigma_e=1.0, sigma_p=3.0, photons=1e4)
    rng = _rng(15)
    pos = ptysynth.raster_positions(4, 4, 4.0, 1.0) + rng.uniform(0.1, 0.9, (16, 2))
    o = wl.obj()
    p = wl.probe()
    cnt, p = oracle.simulate(o, p, pos, wl.photons)
    cnt = ptysynth.poisson_counts(cnt, wl.noise_rng()).astype(np.float64)
    # evaluate the gradient away from the truth
    o = o * (1 + 0.05 * _crandn(rng, *o.shape))
    p = p * (1 + 0.05 * _crandn(rng, *p.shape))
    return o, p, pos, cnt, rng


def test_nll_gradient_finite_differences():
    o, p, pos, cnt, rng = _fd_case()
    loss, g_o, g_p, g_r = oracle.nll_grad(o, p, pos, cnt)
    assert abs(loss - oracle.nll(o, p, pos, cnt)) <= 1e-12 * abs(loss)
    # |L| ~ 7e5, so each step trades float64 cancellation against truncation
    h = 1e-5
    for _ in range(3):
        # random complex directions scaled to the variable: dL = Re<g, dO> in the (Re, Im) convention
        d_o = _crandn(rng, *o.shape) * np.sqrt(np.mean(np.abs(o) ** 2))
        fd = (oracle.nll(o + h * d_o, p, pos, cnt) - oracle.nll(o - h * d_o, p, pos, cnt)) / (2 * h)
        an = float(np.real(np.vdot(g_o, d_o)))
        assert abs(fd - an) <= 1e-6 * abs(an)
        d_p = _crandn(rng, *p.shape) * np.sqrt(np.mean(np.abs(p) ** 2))
        fd = (oracle.nll(o, p + h * d_p, pos, cnt) - oracle.nll(o, p - h * d_p, pos, cnt)) / (2 * h)
        an = float(np.real(np.vdot(g_p, d_p)))
        assert abs(fd - an) <= 1e-6 * abs(an)
    h = 1e-4
    for j in (0, 5, 15):
        for ax in (0, 1):
            e = np.zeros_like(pos)
            e[j, ax] = h
            fd = (oracle.nll(o, p, pos + e, cnt) - oracle.nll(o, p, pos - e, cnt)) / (2 * h)
            assert abs(fd - g_r[j, ax]) <= 1e-6 * abs(g_r[j, ax])


def test_nll_gradient_vanishes_at_truth():
    wl, o, p, pos, cnt = _tiny(k=2)
    _, g_o, g_p, g_r = oracle.nll_grad(o, p, pos, cnt, eps=1e-14)
    _, g_o2, _, _ = oracle.nll_grad(o * 1.01, p, pos, cnt, eps=1e-14)
    assert np.max(np.abs(g_o)) <= 1e-8 * np.max(np.abs(g_o2))
    assert np.max(np.abs(g_r)) <= 1e-6


def test_nll_gradient_swap_symmetry():
    # one position at an integer corner with N = object size: the model is
    # symmetric in (O, P), so g_P(O, P) equals g_O with the roles exchanged
    rng = _rng(16)
    n = 16
    x = _crandn(rng, n, n)
    y = _crandn(rng, n, n)
    d = np.fft.fftshift(rng.poisson(20.0, (1, n, n)).astype(float), axes=(-2, -1))
    pos = np.zeros((1, 2))
    _, g_o, g_p, _ = oracle.nll_grad(x, y[None], pos, d)
    _, g_o2, g_p2, _ = oracle.nll_grad(y, x[None], pos, d)
    assert np.max(np.abs(g_p[0] - g_o2)) <= 1e-12 * np.max(np.abs(g_o2))
    assert np.max(np.abs(g_o - g_p2[0])) <= 1e-12 * np.max(np.abs(g_o))
