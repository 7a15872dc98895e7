"""Pins of the oracle's ePIE and LSQML probe updates, with probe updates on.

The error-reduction and fixed-point pins elsewhere run with the probe fixed or
with a zero exit-wave update, so they hold for any probe rule.  The pins here
fix the probe rules themselves:

* swap symmetry: one position at the origin of an object as large as the
  window makes the exit wave P O symmetric in (O, P), so the probe update must
  be the object update with the two exchanged (ePIE, Maiden & Rodenburg 2009;
  LSQML, Odstrcil et al. 2018), and the object update is pinned to Fienup's
  error reduction elsewhere;
* ePIE as a proximal least-squares step: each update is the minimiser of
  sum_k |P_k o' - psi_k|^2 + (max sum_k |P_k|^2 - sum_k |P_k|^2) |o' - o|^2
  (and likewise for each probe mode with the pre-update patch), solved here
  pixel by pixel with numpy.linalg.lstsq;
* LSQML on a phase-only object with a flat probe, where the 2 x 2 step system
  is singular and the regularised solve has a closed form around Fienup's
  error-reduction step.

Each pin is then shown to fail on a copy of the oracle with a planted mistake
(the post-update patch in ePIE's probe step; LSQML's probe update computed
from the updated object; a dropped conjugate).
"""
import inspect
import math

import numpy as np
import pytest

import oracle
import oracle.ptycho as optycho


def _rng(seed):
    return np.random.default_rng(seed)


def _crandn(rng, *shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def _target(probe, patch, a):
    """Projected exit waves F^-1 Pi(F(P patch)) by numpy.fft (unitary), all modes."""
    f = np.fft.fft2(probe * patch[None], norm="ortho")
    mod = np.sqrt(np.sum(np.abs(f) ** 2, axis=0))
    return np.fft.ifft2(f * (a / mod)[None], norm="ortho")


def _er_step(o, a):
    """Fienup's error reduction with a pure modulus constraint (numpy.fft, unitary)."""
    f = np.fft.fft2(o, norm="ortho")
    return np.fft.ifft2(a * f / np.abs(f), norm="ortho")


def _prox(coef, target, old):
    """Pixel-wise minimiser of sum_k |coef_k x - target_k|^2 + (m - sum_k |coef_k|^2) |x - old|^2,
    m = max over pixels of sum_k |coef_k|^2, each pixel solved by numpy.linalg.lstsq."""
    k = coef.shape[0]
    w = np.sum(np.abs(coef) ** 2, axis=0)
    m = float(w.max())
    out = np.empty(old.shape, complex)
    for idx in np.ndindex(old.shape):
        r = math.sqrt(max(m - w[idx], 0.0))
        mat = np.array([coef[(kk,) + idx] for kk in range(k)] + [r], complex)[:, None]
        rhs = np.array([target[(kk,) + idx] for kk in range(k)] + [r * old[idx]], complex)
        out[idx] = np.linalg.lstsq(mat, rhs, rcond=None)[0][0]
    return out


def _moduli(rng, n):
    return rng.uniform(0.5, 2.0, (n, n))


# ---------------------------------------------------------------------------
# ePIE
# ---------------------------------------------------------------------------
def _check_epie_swap(epie):
    rng = _rng(31)
    n = 16
    x, y = _crandn(rng, n, n), _crandn(rng, n, n)
    a = _moduli(rng, n)[None] * math.sqrt(np.sum(np.abs(x * y) ** 2)) / n
    pos = np.zeros((1, 2))
    o1, p1, _ = epie(x, y[None], a, pos, 1, start=0)
    o2, p2, _ = epie(y, x[None], a, pos, 1, start=0)
    scale = max(np.max(np.abs(o1)), np.max(np.abs(p1)))
    return max(np.max(np.abs(p1[0] - o2)), np.max(np.abs(o1 - p2[0]))) / scale


def _check_epie_prox(epie):
    # one integer position inside a larger object, two modes, probe update on
    rng = _rng(32)
    n, h = 8, 13
    o = _crandn(rng, h, h)
    p = _crandn(rng, 2, n, n)
    r = np.array([[3.0, 2.0]])
    patch = o[3:3 + n, 2:2 + n].copy()
    a = _moduli(rng, n) * math.sqrt(np.sum(np.abs(p * patch[None]) ** 2)) / n
    o1, p1, _ = epie(o, p, a[None], r, 1, start=0)
    tgt = _target(p, patch, a)
    ref_o = o.copy()
    ref_o[3:3 + n, 2:2 + n] = _prox(p, tgt, patch)
    ref_p = np.stack([_prox(patch[None], tgt[k][None], p[k]) for k in range(2)])
    scale = max(np.max(np.abs(ref_o)), np.max(np.abs(ref_p)))
    return max(np.max(np.abs(o1 - ref_o)), np.max(np.abs(p1 - ref_p))) / scale


def _check_epie_sequence(epie):
    # two overlapping integer positions: the second sees the first one's object and probe
    rng = _rng(33)
    n, h = 8, 12
    o = _crandn(rng, h, h)
    p = _crandn(rng, 1, n, n)
    pos = np.array([[0.0, 0.0], [3.0, 4.0]])
    a = np.stack([_moduli(rng, n) for _ in pos]) * math.sqrt(np.sum(np.abs(p) ** 2) * 2) / n
    o1, p1, _ = epie(o, p, a, pos, 1, start=0)
    ro, rp = o.copy(), p.copy()
    for j, (yy, xx) in enumerate(pos.astype(int)):
        patch = ro[yy:yy + n, xx:xx + n].copy()
        tgt = _target(rp, patch, a[j])
        ro[yy:yy + n, xx:xx + n] = _prox(rp, tgt, patch)
        rp = _prox(patch[None], tgt, rp[0])[None]
    scale = max(np.max(np.abs(ro)), np.max(np.abs(rp)))
    return max(np.max(np.abs(o1 - ro)), np.max(np.abs(p1 - rp))) / scale


def test_epie_probe_update_is_object_update_swapped():
    assert _check_epie_swap(oracle.epie) <= 1e-12


def test_epie_updates_are_proximal_least_squares():
    assert _check_epie_prox(oracle.epie) <= 1e-12


def test_epie_positions_are_sequential_proximal_steps():
    assert _check_epie_sequence(oracle.epie) <= 1e-12


# ---------------------------------------------------------------------------
# LSQML
# ---------------------------------------------------------------------------
def _check_lsqml_swap(lsqml):
    rng = _rng(34)
    n = 16
    x, y = _crandn(rng, n, n), _crandn(rng, n, n)
    a = _moduli(rng, n)[None] * math.sqrt(np.sum(np.abs(x * y) ** 2)) / n
    pos = np.zeros((1, 2))
    o1, p1, _ = lsqml(x, y[None], a, pos, 1, start=0)
    o2, p2, _ = lsqml(y, x[None], a, pos, 1, start=0)
    scale = max(np.max(np.abs(o1)), np.max(np.abs(p1)))
    return max(np.max(np.abs(p1[0] - o2)), np.max(np.abs(o1 - p2[0]))) / scale


def _check_lsqml_phase_object(lsqml):
    # flat probe, phase-only object |O| = c: the object and probe directions give
    # the same exit-wave change chi / (1 + gamma), so M is singular with equal
    # entries m; (M + eta I) alpha = v gives alpha_O = alpha_P = (1 + gamma) / (2 + 1e-6)
    # and, with chi = ER(O) - O from Fienup's error reduction,
    #   O' = O + chi / (2 + 1e-6),   P' = 1 + conj(O) chi / (c^2 (2 + 1e-6)).
    rng = _rng(35)
    n, c = 16, 1.3
    o = c * np.exp(1j * rng.uniform(-math.pi, math.pi, (n, n)))
    a = _moduli(rng, n) * c
    p = np.ones((1, n, n), complex)
    o1, p1, _ = lsqml(o, p, a[None], np.zeros((1, 2)), 1, start=0)
    chi = _er_step(o, a) - o
    ref_o = o + chi / (2.0 + 1e-6)
    ref_p = 1.0 + np.conj(o) * chi / (c * c * (2.0 + 1e-6))
    return max(np.max(np.abs(o1 - ref_o)) / c, np.max(np.abs(p1[0] - ref_p)))


def test_lsqml_probe_update_is_object_update_swapped():
    assert _check_lsqml_swap(oracle.lsqml) <= 1e-12


def test_lsqml_phase_object_closed_form():
    # (M + eta I) has condition number (2 m + eta) / eta = 2e6 here, which
    # amplifies the ~1e-16 rounding of M's entries into the step lengths
    assert _check_lsqml_phase_object(oracle.lsqml) <= 1e-8


# ---------------------------------------------------------------------------
# Planted mistakes: each must fail at least one of the pins above
# ---------------------------------------------------------------------------
def _mutant(fn, old, new, extra=None):
    """A copy of oracle function ``fn`` with the source fragment ``old`` replaced by ``new``."""
    src = inspect.getsource(fn)
    assert src.count(old) == 1, old
    ns = dict(vars(optycho))
    if extra:
        ns.update(extra)
    exec(compile(src.replace(old, new), f"<mutant {fn.__name__}>", "exec"), ns)
    return ns[fn.__name__]


def _post_patch(obj, probe, chi, r, n, alpha, pmax):
    """The patch after this position's object update (the planted mistake's input)."""
    o = np.array(obj)
    optycho.scatter_add(o, alpha * np.sum(np.conj(probe) * chi, axis=0) / pmax, r)
    return optycho.gather(o, r, n)


EPIE_MUTANTS = {
    "post-update patch in the probe step": (
        "new_probe = probe + beta * np.conj(oj)[None] * chi / omax",
        "new_probe = probe + beta * np.conj(_post_patch(obj, probe, chi, pos[j], n, alpha, pmax))[None]"
        " * chi / omax"),
    "mean instead of max in the probe normaliser": (
        "omax = float(np.max(np.abs(oj) ** 2))",
        "omax = float(np.mean(np.abs(oj) ** 2))"),
    "updated probe in the object step": (
        "scatter_add(obj, alpha * np.sum(np.conj(probe) * chi, axis=0) / pmax, pos[j])",
        "scatter_add(obj, alpha * np.sum(np.conj(new_probe) * chi, axis=0) / pmax, pos[j])"),
}

LSQML_MUTANTS = {
    "probe update from the updated object": (
        "                probe = probe + beta_probe * upd_p / (den_p + d_p)",
        "                upd_p = sum(alpha[j, 1] * np.conj(gather(obj, pos[j], n))[None] * chis[j] for j in idx)\n"
        "                probe = probe + beta_probe * upd_p / (den_p + d_p)"),
    "conjugate dropped in the probe direction": (
        "num_p += np.conj(oj)[None] * chi",
        "num_p += oj[None] * chi"),
    "probe denominator from the probe": (
        "den_p += np.abs(oj) ** 2",
        "den_p += pint"),
}


@pytest.mark.parametrize("name", sorted(EPIE_MUTANTS))
def test_epie_pins_catch_planted_mistake(name):
    old, new = EPIE_MUTANTS[name]
    bad = _mutant(optycho.epie, old, new, {"_post_patch": _post_patch})
    errs = [_check_epie_swap(bad), _check_epie_prox(bad), _check_epie_sequence(bad)]
    assert max(errs) > 1e-6, (name, errs)


@pytest.mark.parametrize("name", sorted(LSQML_MUTANTS))
def test_lsqml_pins_catch_planted_mistake(name):
    old, new = LSQML_MUTANTS[name]
    bad = _mutant(optycho.lsqml, old, new)
    errs = [_check_lsqml_swap(bad), _check_lsqml_phase_object(bad)]
    assert max(errs) > 1e-6, (name, errs)
