"""Pins of the oracle's LSQML position refinement (least-squares shift of each
position from its exit-wave update, Odstrcil et al. 2018): the shift is the
vertex of the residual's quadratic in the shift, zero at the truth, recovers
known position errors when iterated with the true object and probe, and
inside LSQML lowers the position error while keeping every patch in the
object."""
import numpy as np
import pytest

import oracle
import ptysynth
from oracle import ptycho


def _case(seed=51, jitter=0.3):
    wl = ptysynth.scaled(ptysynth.workload(1), cfg=seed, n=32, k=2, h=80, w=80, d=13.0,
                         rows=5, cols=5, step=8.0, offset=6.0, j=25, photons=1e6)
    o = wl.obj()
    pos_true = wl.positions()
    cnt, p = oracle.simulate(o, wl.probe(), pos_true, wl.photons)
    rng = np.random.default_rng([31, seed])
    nominal = pos_true + rng.uniform(-jitter, jitter, pos_true.shape)
    return o, p, pos_true, nominal, oracle.amplitude(cnt)


def _chi(o, p, r, a):
    chi, _, _ = ptycho._exit_diff(p, oracle.gather(o, r, p.shape[-1]), a)
    return chi


def test_shift_is_the_vertex_of_the_residual_quadratic():
    rng = np.random.default_rng(5)
    o = rng.standard_normal((40, 40)) + 1j * rng.standard_normal((40, 40))
    p = rng.standard_normal((2, 16, 16)) + 1j * rng.standard_normal((2, 16, 16))
    chi = rng.standard_normal((2, 16, 16)) + 1j * rng.standard_normal((2, 16, 16))
    r = (7.3, 11.6)
    s = oracle.position_shift(o, p, chi, r, max_shift=1e9)
    dy, dx = oracle.gather_grad(o, r, 16)
    for ax, d in enumerate((dy, dx)):
        dpsi = p * d[None]
        f = [float(np.sum(np.abs(chi - t * dpsi) ** 2)) for t in (-1.0, 0.0, 1.0)]
        vertex = 0.5 * (f[0] - f[2]) / (f[0] - 2 * f[1] + f[2])
        assert abs(s[ax] - vertex) <= 1e-10 * max(1.0, abs(vertex))
    # the clip
    big = oracle.position_shift(o, p, 1e6 * chi, r, max_shift=0.25)
    assert np.all(np.abs(big) <= 0.25) and np.any(np.abs(big) == 0.25)


def test_shift_is_zero_at_the_truth():
    o, p, pos_true, _, a = _case()
    for j in (0, 7, 24):
        s = oracle.position_shift(o, p, _chi(o, p, pos_true[j], a[j]), pos_true[j], 0.5)
        assert np.max(np.abs(s)) <= 1e-9


def test_iterated_shifts_recover_known_position_errors():
    o, p, pos_true, pos, a = _case()
    err0 = np.sqrt(np.mean((pos - pos_true) ** 2))
    prev = err0
    for _ in range(8):
        pos = pos + np.array([oracle.position_shift(o, p, _chi(o, p, r, a[j]), r, 0.5)
                              for j, r in enumerate(pos)])
        err = np.sqrt(np.mean((pos - pos_true) ** 2))
        assert err < prev
        prev = err
    assert prev <= 0.2 * err0


def test_lsqml_refinement_recovers_positions_on_a_spiral_scan():
    # noise-free spiral scan (a regular raster has near-null directions of its
    # own, so a spiral is the fair test), solver given positions off by up to
    # 0.4 px; the refined positions approach the true ones up to the global
    # shift that object and positions can share
    from _cases import spiral_case
    case = spiral_case(32, 1, 60, cfg=61, noise=False)
    rng = np.random.default_rng(9)
    lim = np.array(case.shape, dtype=float) - 32
    nominal = np.clip(case.pos + rng.uniform(-0.4, 0.4, case.pos.shape), 0.0, lim)
    nominal[0] = (0.0, lim[1])                      # one at the object's edge
    o0 = np.ones(case.shape, complex)
    kw = dict(start=1 << 30, batch=20)
    o_ref, _, e_ref, pos_ref = oracle.lsqml(o0, case.probe, case.amp, nominal, 20, pos_start=5, max_shift=0.5,
                                            return_positions=True, **kw)
    o_plain, _, e_plain = oracle.lsqml(o0, case.probe, case.amp, nominal, 20, **kw)
    assert np.all(pos_ref >= 0.0) and np.all(pos_ref <= lim)

    def err(pp):
        d = (pp - case.pos)[1:]
        return float(np.sqrt(np.mean((d - d.mean(0)) ** 2)))
    assert err(pos_ref) <= 0.25 * err(nominal)
    roi = oracle.roi_mask(case.probe, case.pos, *case.shape)
    assert oracle.nrmse(o_ref, case.obj_true, roi) < 0.5 * oracle.nrmse(o_plain, case.obj_true, roi)
    assert e_ref[-1] < 0.1 * e_plain[-1]
    # before pos_start the two runs are the same iterations
    assert e_ref[:5] == e_plain[:5]
