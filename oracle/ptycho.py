"""FP64 reference implementation of multi-mode ptychographic reconstruction.

Test infrastructure: imported only by the tests, the smoke check and the
benchmark's CPU-baseline leg.  Nothing in the product library calls it.

Notation (used by every function):

* N probe window (square), K probe modes, J scan positions, object H x W.
* O: (H, W) complex object.  P: (K, N, N) complex probe modes.
* R_j = (y_j, x_j): top-left corner of patch j in object pixels, 0-based,
  real-valued; i_j = floor(R_j), f_j = R_j - i_j.
* Gather S_j (bilinear, exact slicing when f_j = 0):
  (S_j O)[u, v] = sum_{a,b in {0,1}} w_a(f^y) w_b(f^x) O[i^y+u+a, i^x+v+b],
  w_0(f) = 1 - f, w_1(f) = f.  S_j^T is its exact adjoint (a scatter with the
  same real weights).
* F: unitary 2-D DFT in natural order, (F x)[p,q] = N^-1 sum x[u,v] e^{-2 pi i (pu+qv)/N};
  F^-1 = F^H.
* Data d_j: photon counts with the zero frequency at (N/2, N/2) (detector
  convention); the measured moduli are A_j = sqrt(ifftshift(d_j)).
* Modulus projection of a multi-mode far field Psi (mixed states, Thibault &
  Menzel 2013): I = sum_k |Psi_k|^2, Pi(Psi)_k = Psi_k A / max(sqrt(I), eps_M),
  eps_M = 1e-6; the difference Delta = Pi(Psi) - Psi = (ratio - 1) Psi.
* Amplitude error of one iteration:
  E = sum_j sum_q (sqrt(I_jq) - A_jq)^2 / sum_j sum_q A_jq^2,
  on the far field that enters the projection in that iteration.
* Regularisers: delta = gamma * max(den) for a denominator plane ``den``.

The update rules are those of the methods the paper names in Sec. 2.3 (ePIE:
Maiden & Rodenburg 2009; DM: Thibault et al. 2008/2009; LSQML: Odstrcil,
Menzel & Guizar-Sicairos 2018), written from those papers.
"""
from __future__ import annotations

import math
import os
from typing import Iterable

import numpy as np
import scipy.fft as sfft

__all__ = [
    "EPS_M",
    "EPS_L",
    "fft2u",
    "ifft2u",
    "split_position",
    "gather",
    "gather_all",
    "gather_grad",
    "scatter_add",
    "amplitude",
    "project_delta",
    "poisson_step",
    "POISSON_NEWTON_STEPS",
    "poisson_delta",
    "forward_intensity",
    "simulate",
    "model_error",
    "photons_from_counts",
    "probe_guess",
    "mode_basis",
    "orthogonalise_modes",
    "splitmix64_stream",
    "epie_order",
    "epie",
    "dm_init",
    "dm",
    "lsqml_solve2",
    "position_shift",
    "lsqml",
    "illumination",
    "roi_mask",
    "nrmse",
    "phase_aligned_rel",
    "nll",
    "nll_grad",
]

EPS_M = 1e-6   # floor of the model modulus in the projection (sqrt(counts))
EPS_L = 1e-6   # offset inside the log of the Poisson likelihood
WORKERS = os.cpu_count() or 1


# ---------------------------------------------------------------------------
# Transform, gather, scatter
# ---------------------------------------------------------------------------
def fft2u(x: np.ndarray) -> np.ndarray:
    """Unitary forward 2-D DFT over the last two axes, natural order."""
    return sfft.fft2(np.asarray(x, dtype=np.complex128), norm="ortho", workers=WORKERS)


def ifft2u(x: np.ndarray) -> np.ndarray:
    """Unitary inverse 2-D DFT over the last two axes (the adjoint of fft2u)."""
    return sfft.ifft2(np.asarray(x, dtype=np.complex128), norm="ortho", workers=WORKERS)


def split_position(r: float) -> tuple[int, float]:
    """Integer floor and fractional part of one coordinate of R_j."""
    i = math.floor(r)
    return int(i), float(r - i)


def _taps(r: Iterable[float]):
    (iy, fy), (ix, fx) = (split_position(v) for v in r)
    return iy, ix, ((0, 0, (1 - fy) * (1 - fx)), (0, 1, (1 - fy) * fx),
                    (1, 0, fy * (1 - fx)), (1, 1, fy * fx))


def gather(obj: np.ndarray, r, n: int) -> np.ndarray:
    """(S_j O): the N x N bilinear patch of ``obj`` at top-left ``r`` = (y, x).

    Taps with zero weight are skipped, so an integer position reads exactly the
    slice obj[y:y+N, x:x+N].
    """
    iy, ix, taps = _taps(r)
    out = np.zeros((n, n), dtype=np.result_type(obj.dtype, np.float64))
    for a, b, w in taps:
        if w != 0.0:
            out += w * obj[iy + a: iy + a + n, ix + b: ix + b + n]
    return out


def gather_all(obj: np.ndarray, pos: np.ndarray, n: int) -> np.ndarray:
    return np.stack([gather(obj, r, n) for r in pos])


def gather_grad(obj: np.ndarray, r, n: int) -> tuple[np.ndarray, np.ndarray]:
    """Derivatives of the bilinear patch with respect to y_j and x_j.

    Uses dw_0/df = -1 and dw_1/df = +1 at fixed floor (the right derivative at
    integer positions).  Pixels beyond the object's last row or column count as
    zero (only an integer position on the far edge reaches them).
    """
    (iy, fy), (ix, fx) = (split_position(v) for v in r)
    obj = np.pad(obj, ((0, 1), (0, 1)))

    def sl(a, b):
        return obj[iy + a: iy + a + n, ix + b: ix + b + n]

    dy = (1 - fx) * (sl(1, 0) - sl(0, 0)) + fx * (sl(1, 1) - sl(0, 1))
    dx = (1 - fy) * (sl(0, 1) - sl(0, 0)) + fy * (sl(1, 1) - sl(1, 0))
    return dy, dx


def scatter_add(acc: np.ndarray, y: np.ndarray, r) -> None:
    """acc += S_j^T y, the exact adjoint of :func:`gather` (in place)."""
    n = y.shape[-1]
    iy, ix, taps = _taps(r)
    for a, b, w in taps:
        if w != 0.0:
            acc[iy + a: iy + a + n, ix + b: ix + b + n] += w * y


# ---------------------------------------------------------------------------
# Data, projection, forward model
# ---------------------------------------------------------------------------
def amplitude(d: np.ndarray, mask: np.ndarray | None = None) -> np.ndarray:
    """Measured moduli in natural order: A = sqrt(ifftshift(d)) (Sec. 3.2 normalisation).

    ``mask``: optional detector mask in the same centred layout as one pattern,
    nonzero where the pixel measured something (saturated or dead pixels and
    a beam stop are the excluded ones, Sec. 2.2's preprocessing parameters).
    Unmeasured pixels get NaN: no measurement.
    """
    d = np.asarray(d, dtype=np.float64)
    a = np.sqrt(np.fft.ifftshift(d, axes=(-2, -1)))
    if mask is not None:
        valid = np.fft.ifftshift(np.asarray(mask) != 0)
        a = np.where(valid, a, np.nan)
    return a


def project_delta(psi_f: np.ndarray, a: np.ndarray):
    """Difference Delta = Pi(Psi) - Psi of the multi-mode modulus projection.

    ``psi_f``: (K, N, N) far field; ``a``: (N, N) measured moduli, NaN where
    nothing was measured: there the projection keeps the model (Delta = 0)
    and the pixel adds nothing to either error sum.
    Returns (Delta, sum (sqrt(I) - A)^2, sum A^2) over the measured pixels.
    """
    inten = np.sum(np.abs(psi_f) ** 2, axis=0)
    mod = np.sqrt(inten)
    valid = np.isfinite(a)
    am = np.where(valid, a, 0.0)
    ratio = np.where(valid, am / np.maximum(mod, EPS_M), 1.0)
    delta = (ratio - 1.0)[None] * psi_f
    return delta, float(np.sum(np.where(valid, (mod - am) ** 2, 0.0))), float(np.sum(am * am))


POISSON_NEWTON_STEPS = 12
POISSON_STEP_TOL = 1e-7


def poisson_step(inten: np.ndarray, d: np.ndarray, eps: float = EPS_L) -> float:
    """Step length alpha_R of the Poisson exit-wave update of one pattern.

    ``inten``: (N, N) model intensity I; ``d``: (N, N) measured counts, NaN
    where nothing was measured (those pixels add nothing).  Along the negative
    gradient of the Poisson likelihood in the detector plane the far field
    becomes Psi (1 - alpha g), g = 1 - d / (I + eps), so every intensity
    becomes I s^2 with s = 1 - alpha g.  alpha_R minimises the pattern's
    likelihood along that ray,

        L(alpha) = sum [I s^2 - d log(I s^2 + eps)],
        L'(alpha) = -2 sum I g s (1 - r),
        L''(alpha) = 2 sum I g^2 (1 - r + 2 r I s^2 / (I s^2 + eps)),
        r = d / (I s^2 + eps),

    on [0, 1]: L'(0) = -2 sum I g^2 < 0 unless the pattern is already met,
    and every pixel's own minimiser 1 / (1 + sqrt(d / I)) (eps -> 0) lies in
    (0, 1].  It is found by POISSON_NEWTON_STEPS Newton steps from 1/2 inside
    the bracket [lo, hi] that the sign of L' keeps (a step that would leave
    the closed bracket, or a non-positive L'', bisects it instead), stopping
    early once a Newton step moves alpha by at most POISSON_STEP_TOL; 0 when
    sum I g^2 = 0.  For a uniform ratio d = c I (eps = 0) it is
    1 / (1 + sqrt(c)), where the moved intensity equals d.
    """
    valid = np.isfinite(d)
    dm = np.where(valid, d, 0.0)
    g = np.where(valid, 1.0 - dm / (inten + eps), 0.0)
    if float(np.sum(inten * g * g)) <= 0.0:
        return 0.0
    lo, hi, a = 0.0, 1.0, 0.5
    for _ in range(POISSON_NEWTON_STEPS):
        s = 1.0 - a * g
        u = inten * s * s
        t = u + eps
        r = dm / t
        d1 = float(np.sum(np.where(valid, -2.0 * inten * g * s * (1.0 - r), 0.0)))
        d2 = float(np.sum(np.where(valid, 2.0 * inten * g * g * (1.0 - r + 2.0 * r * u / t), 0.0)))
        if d1 < 0.0:
            lo = a
        else:
            hi = a
        nxt = a - d1 / d2 if d2 > 0.0 else -1.0
        if not (lo <= nxt <= hi):
            nxt = 0.5 * (lo + hi)
        elif abs(nxt - a) <= POISSON_STEP_TOL:
            return nxt                      # converged
        a = nxt
    return a


def poisson_delta(psi_f: np.ndarray, a: np.ndarray, eps: float = EPS_L):
    """Difference Delta = -alpha_R g Psi of the Poisson exit-wave update.

    ``psi_f``: (K, N, N) far field; ``a``: (N, N) measured moduli (d = a^2),
    NaN where nothing was measured (g = 0 there).  alpha_R from
    :func:`poisson_step`.  Returns (Delta, alpha_R, and the amplitude-error
    partials of :func:`project_delta`: sum (sqrt(I) - A)^2, sum A^2).
    """
    inten = np.sum(np.abs(psi_f) ** 2, axis=0)
    valid = np.isfinite(a)
    am = np.where(valid, a, 0.0)
    d = np.where(valid, am * am, np.nan)
    alpha = poisson_step(inten, d, eps)
    g = np.where(valid, 1.0 - am * am / (inten + eps), 0.0)
    delta = (-alpha * g)[None] * psi_f
    mod = np.sqrt(inten)
    return delta, alpha, float(np.sum(np.where(valid, (mod - am) ** 2, 0.0))), float(np.sum(am * am))


def forward_intensity(obj: np.ndarray, probe: np.ndarray, r) -> np.ndarray:
    """I_j = sum_k |F(P_k S_j O)|^2 in natural order (mixed-state forward model)."""
    n = probe.shape[-1]
    return np.sum(np.abs(fft2u(probe * gather(obj, r, n)[None])) ** 2, axis=0)


def simulate(obj: np.ndarray, probe: np.ndarray, pos: np.ndarray, photons: float | None = None):
    """Expected counts of every pattern, centred (zero frequency at (N/2, N/2)).

    With ``photons`` given, the probe is rescaled so that the mean over
    patterns of the total expected counts equals ``photons``; the function then
    returns (counts, scaled probe).  Without it, (counts, probe).
    """
    inten = np.stack([forward_intensity(obj, probe, r) for r in pos])
    if photons is not None:
        s = photons / float(np.mean(np.sum(inten, axis=(1, 2))))
        inten = inten * s
        probe = probe * math.sqrt(s)
    return np.fft.fftshift(inten, axes=(-2, -1)), probe


def model_error(obj: np.ndarray, probe: np.ndarray, a: np.ndarray, pos: np.ndarray) -> float:
    """E evaluated on the far fields of the current object and probe."""
    n = probe.shape[-1]
    num = den = 0.0
    for j, r in enumerate(pos):
        _, e1, e2 = project_delta(fft2u(probe * gather(obj, r, n)[None]), a[j])
        num += e1
        den += e2
    return num / den


def _exit_diff(probe: np.ndarray, oj: np.ndarray, a: np.ndarray, z: np.ndarray | None = None,
               likelihood: str = "amplitude"):
    """chi = F^-1 Delta(F z) with z = P (S_j O) unless given; plus the error
    partials.  Delta: the modulus projection's (``likelihood="amplitude"``) or
    the Poisson update's (``"poisson"``, :func:`poisson_delta`)."""
    if z is None:
        z = probe * oj[None]
    if likelihood == "poisson":
        delta, _, e1, e2 = poisson_delta(fft2u(z), a)
    elif likelihood == "amplitude":
        delta, e1, e2 = project_delta(fft2u(z), a)
    else:
        raise ValueError(f"unknown likelihood {likelihood!r}")
    return ifft2u(delta), e1, e2


# ---------------------------------------------------------------------------
# Blind probe start
# ---------------------------------------------------------------------------
def photons_from_counts(d) -> float:
    """Mean over patterns of the total counts, negative counts taken as 0."""
    d = np.maximum(np.asarray(d, dtype=np.float64), 0.0)
    return float(np.mean(np.sum(d, axis=(-2, -1))))


def probe_guess(n: int, k: int, diameter: float, photons: float) -> np.ndarray:
    """Starting probe when none is known (Sec. 2.2: the guess of the probe size
    and the number of modes): an unaberrated aperture, a uniform real disk of
    the given diameter (pixels) centred on the window (pixel centres at
    distance <= diameter / 2 from ((n-1)/2, (n-1)/2)), and for k > 1 the disk
    times x, y and x*y (centred pixel coordinates) made orthogonal to the
    lower modes by Gram-Schmidt in that order; every mode has power
    photons / k, so that with the unitary transform the mean pattern total
    of a flat object equals ``photons`` (Sec. 3.2's normalisation)."""
    c = (n - 1) / 2.0
    u, v = np.meshgrid(np.arange(n) - c, np.arange(n) - c, indexing="ij")
    disk = (u * u + v * v <= (diameter / 2.0) ** 2).astype(np.float64)
    shapes = [disk, disk * v, disk * u, disk * u * v]
    modes = []
    for f in shapes[:k]:
        g = f.astype(np.complex128)
        for m in modes:
            g = g - np.vdot(m, g) / np.vdot(m, m) * m
        modes.append(g)
    out = np.stack(modes)
    for i in range(k):
        out[i] *= math.sqrt(photons / k / float(np.sum(np.abs(out[i]) ** 2)))
    return out


# ---------------------------------------------------------------------------
# Probe-mode orthogonalisation (mixed states, Thibault & Menzel 2013)
# ---------------------------------------------------------------------------
def mode_basis(probe) -> np.ndarray:
    """Unitary K x K matrix V of the eigenvectors of the modes' Gram matrix
    G_kl = sum_r P_k(r) conj(P_l(r)), columns in order of decreasing
    eigenvalue, each column's phase set so that its largest-magnitude entry
    (the first of equal ones) is real and positive."""
    p = np.asarray(probe, dtype=np.complex128).reshape(len(probe), -1)
    g = p @ p.conj().T
    lam, v = np.linalg.eigh(g)
    order = np.argsort(-lam, kind="stable")
    v = v[:, order]
    for k in range(v.shape[1]):
        i = int(np.argmax(np.abs(v[:, k])))
        v[:, k] *= np.conj(v[i, k]) / abs(v[i, k])
    return v


def orthogonalise_modes(probe, psi=None):
    """P'_k = sum_l conj(V_lk) P_l with V = mode_basis(P): orthogonal modes in
    order of decreasing power, the same incoherent sum sum_k |P_k|^2 and the
    same mutual coherence.  DM exit waves, if given (J, K, N, N), are mixed
    with the same matrix so that they stay paired with their modes.  Returns
    (P', psi') (psi' None without psi)."""
    v = mode_basis(probe)
    m = v.conj().T
    p2 = np.einsum("kl,l...->k...", m, np.asarray(probe, dtype=np.complex128))
    psi2 = None if psi is None else np.einsum("kl,jl...->jk...", m, np.asarray(psi, dtype=np.complex128))
    return p2, psi2


# ---------------------------------------------------------------------------
# ePIE (Maiden & Rodenburg 2009): sequential over positions
# ---------------------------------------------------------------------------
_M64 = (1 << 64) - 1


def splitmix64_stream(state: int):
    """SplitMix64 (Steele, Lea & Flood 2014): yields successive 64-bit outputs."""
    s = state & _M64
    while True:
        s = (s + 0x9E3779B97F4A7C15) & _M64
        z = s
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _M64
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _M64
        yield z ^ (z >> 31)


def epie_order(j: int, seed: int, t: int) -> np.ndarray:
    """Visiting order of iteration t: identity if seed == 0, else a Fisher-Yates
    shuffle of the identity driven by SplitMix64 with state seed + t."""
    order = list(range(j))
    if seed == 0:
        return np.asarray(order)
    gen = splitmix64_stream(seed + t)
    for i in range(j - 1, 0, -1):
        k = next(gen) % (i + 1)
        order[i], order[k] = order[k], order[i]
    return np.asarray(order)


def epie(obj, probe, a, pos, n_iter, t0=0, alpha=1.0, beta=1.0, start=0, order_seed=0, ortho=False):
    """``n_iter`` ePIE iterations; returns (object, probe, [E per iteration]).

    For each position j in the iteration's order, with chi = F^-1 Delta(F(P S_j O))
    and the pre-update patch O_j0 = S_j O:

        O   += alpha S_j^T (sum_k conj(P_k) chi_k) / max_r sum_k |P_k|^2
        P_k += beta conj(O_j0) chi_k / max_r |O_j0|^2       (iteration t >= start)

    both right-hand sides evaluated with the values before this position's
    update.  A zero maximum skips that update.  E accumulates over positions as
    they are visited.  ``a``: (J, N, N) moduli in natural order.  ``ortho``:
    after every iteration that updated the probe, :func:`orthogonalise_modes`.
    """
    obj = np.array(obj, dtype=np.complex128)
    probe = np.array(probe, dtype=np.complex128)
    n = probe.shape[-1]
    errs = []
    for t in range(t0, t0 + n_iter):
        num = den = 0.0
        for j in epie_order(len(pos), order_seed, t):
            oj = gather(obj, pos[j], n)
            chi, e1, e2 = _exit_diff(probe, oj, a[j])
            num += e1
            den += e2
            pmax = float(np.max(np.sum(np.abs(probe) ** 2, axis=0)))
            omax = float(np.max(np.abs(oj) ** 2))
            new_probe = probe
            if t >= start and omax > 0.0:
                new_probe = probe + beta * np.conj(oj)[None] * chi / omax
            if pmax > 0.0:
                scatter_add(obj, alpha * np.sum(np.conj(probe) * chi, axis=0) / pmax, pos[j])
            probe = new_probe
        errs.append(num / den)
        if ortho and t >= start:
            probe, _ = orthogonalise_modes(probe)
    return obj, probe, errs


# ---------------------------------------------------------------------------
# Difference map (Thibault et al. 2008, 2009), beta_DM = 1, Gauss-Seidel overlap
# ---------------------------------------------------------------------------
def dm_init(obj, probe, pos) -> np.ndarray:
    """Initial exit waves psi_jk = P_k S_j O, shape (J, K, N, N)."""
    n = probe.shape[-1]
    return np.stack([probe * gather(obj, r, n)[None] for r in pos]).astype(np.complex128)


def dm(obj, probe, psi, a, pos, n_iter, t0=0, start=0, gamma_obj=1e-6, gamma_probe=1e-6, ortho=False):
    """``n_iter`` DM iterations from exit-wave state ``psi``.

    Returns (object, probe, psi, [E per iteration]).  Each iteration:

    1. overlap projection for the object:
       O = (sum_j S_j^T sum_k conj(P_k) psi_jk + dO O) / (sum_j S_j^T sum_k |P_k|^2 + dO)
    2. if t >= start, the probe with the new object:
       P_k = (sum_j conj(S_j O) psi_jk + dP P_k) / (sum_j |S_j O|^2 + dP)
    3. phi = P S_j O;  Z = F(2 phi - psi);  psi <- phi + F^-1 Delta(Z)
       (= psi + F^-1 Pi(Z) - phi); E is measured on Z.

    dO = gamma_obj max(den_O), dP = gamma_probe max(den_P).  ``ortho``: after
    every iteration that updated the probe, :func:`orthogonalise_modes` of the
    probe with the exit waves.
    """
    obj = np.array(obj, dtype=np.complex128)
    probe = np.array(probe, dtype=np.complex128)
    psi = np.array(psi, dtype=np.complex128)
    n = probe.shape[-1]
    errs = []
    for t in range(t0, t0 + n_iter):
        num_o = np.zeros_like(obj)
        den_o = np.zeros(obj.shape)
        pint = np.sum(np.abs(probe) ** 2, axis=0)
        for j, r in enumerate(pos):
            scatter_add(num_o, np.sum(np.conj(probe) * psi[j], axis=0), r)
            scatter_add(den_o, pint, r)
        d_o = gamma_obj * float(den_o.max())
        obj = (num_o + d_o * obj) / (den_o + d_o)

        if t >= start:
            num_p = np.zeros_like(probe)
            den_p = np.zeros(probe.shape[1:])
            for j, r in enumerate(pos):
                oj = gather(obj, r, n)
                num_p += np.conj(oj)[None] * psi[j]
                den_p += np.abs(oj) ** 2
            d_p = gamma_probe * float(den_p.max())
            probe = (num_p + d_p * probe) / (den_p + d_p)

        e_num = e_den = 0.0
        for j, r in enumerate(pos):
            phi = probe * gather(obj, r, n)[None]
            chi, e1, e2 = _exit_diff(probe, None, a[j], z=2.0 * phi - psi[j])
            psi[j] = phi + chi
            e_num += e1
            e_den += e2
        errs.append(e_num / e_den)
        if ortho and t >= start:
            probe, psi = orthogonalise_modes(probe, psi)
    return obj, probe, psi, errs


# ---------------------------------------------------------------------------
# LSQML (Odstrcil, Menzel & Guizar-Sicairos 2018), amplitude likelihood
# ---------------------------------------------------------------------------
def lsqml_solve2(m00, m11, m01, v0, v1, probe_on=True):
    """Per-position step lengths (alpha_O, alpha_P) from the 2x2 normal equations.

    (M + eta I) alpha = v with M = [[m00, m01], [m01, m11]], eta = 1e-6 max(m00, m11);
    alpha = 0 when max(m00, m11) = 0; without probe update alpha_P = 0 and
    alpha_O = v0 / (m00 + eta).
    """
    m = max(m00, m11)
    if m <= 0.0:
        return 0.0, 0.0
    eta = 1e-6 * m
    if not probe_on:
        return v0 / (m00 + eta), 0.0
    a00, a11 = m00 + eta, m11 + eta
    det = a00 * a11 - m01 * m01
    return (a11 * v0 - m01 * v1) / det, (a00 * v1 - m01 * v0) / det


def position_shift(obj, probe, chi, r, max_shift):
    """Least-squares shift of one position from its exit-wave update (LSQML's
    position correction, Odstrcil et al. 2018): with d_y psi_k = P_k d_y(S_j O)
    (and likewise x), the shift along each axis that best explains chi,
    sum Re(conj(d psi) chi) / sum |d psi|^2 (0 where the denominator is 0),
    clipped to [-max_shift, max_shift]."""
    n = probe.shape[-1]
    dy, dx = gather_grad(obj, r, n)
    out = np.zeros(2)
    for ax, d in enumerate((dy, dx)):
        dpsi = probe * d[None]
        den = float(np.sum(np.abs(dpsi) ** 2))
        if den > 0.0:
            out[ax] = float(np.real(np.vdot(dpsi, chi))) / den
    return np.clip(out, -max_shift, max_shift)


def lsqml(obj, probe, a, pos, n_iter, t0=0, start=0, batch=512, gamma_obj=1e-3,
          gamma_probe=1e-3, beta_obj=1.0, beta_probe=1.0, return_alpha=False,
          pos_start=-1, max_shift=0.5, return_positions=False, ortho=False, likelihood="amplitude"):
    """``n_iter`` LSQML iterations; returns (object, probe, [E], alpha of last iteration).

    Positions are split into G = ceil(J / batch) interleaved groups
    {j : j mod G = g}, processed in order g = 0..G-1.  For each group, all
    quantities use the object and probe at the start of the group:

    * pass A: chi_j = F^-1 Delta(F(P S_j O)); directions
      dO = sum S_j^T sum_k conj(P_k) chi_jk / (den_O + delta_O),
      dP_k = sum conj(S_j O) chi_jk / (den_P + delta_P), with
      den_O = sum S_j^T sum_k |P_k|^2, den_P = sum |S_j O|^2 over the group;
    * pass B: a_jk = P_k S_j dO, b_jk = dP_k S_j O and the step lengths of
      :func:`lsqml_solve2` from sums over pixels and modes of |a|^2, |b|^2,
      Re conj(a) b, Re conj(a) chi, Re conj(b) chi;
    * update: O += beta_O sum S_j^T(alpha_O,j sum_k conj(P_k) chi_jk) / (den_O + delta_O),
      P_k += beta_P sum alpha_P,j conj(S_j O) chi_jk / (den_P + delta_P)  (t >= start);
    * position refinement (t >= pos_start >= 0): after the group's update each
      of its positions moves by :func:`position_shift` of its pass-A chi
      (object and probe at the start of the group), kept inside the object
      (0 <= R <= size - N).  ``return_positions`` adds the refined positions
      to the returned tuple;
    * ``ortho``: after every iteration that updated the probe,
      :func:`orthogonalise_modes`;
    * ``likelihood="poisson"``: chi_j = F^-1 of :func:`poisson_delta` (the
      Poisson exit-wave update) in place of the modulus projection's; every
      other step is the same least-squares solver (E stays the amplitude
      error).
    """
    obj = np.array(obj, dtype=np.complex128)
    probe = np.array(probe, dtype=np.complex128)
    pos = np.array(pos, dtype=np.float64)
    lim = np.array([obj.shape[0] - probe.shape[-1], obj.shape[1] - probe.shape[-1]], dtype=np.float64)
    n = probe.shape[-1]
    jn = len(pos)
    g_count = max(1, -(-jn // batch))
    errs = []
    alpha = np.zeros((jn, 2))
    for t in range(t0, t0 + n_iter):
        probe_on = t >= start
        refine = 0 <= pos_start <= t
        e_num = e_den = 0.0
        for g in range(g_count):
            idx = range(g, jn, g_count)
            pint = np.sum(np.abs(probe) ** 2, axis=0)
            num_o = np.zeros_like(obj)
            den_o = np.zeros(obj.shape)
            num_p = np.zeros_like(probe)
            den_p = np.zeros(probe.shape[1:])
            chis, ojs = {}, {}
            for j in idx:
                oj = gather(obj, pos[j], n)
                chi, e1, e2 = _exit_diff(probe, oj, a[j], likelihood=likelihood)
                e_num += e1
                e_den += e2
                chis[j], ojs[j] = chi, oj
                scatter_add(num_o, np.sum(np.conj(probe) * chi, axis=0), pos[j])
                scatter_add(den_o, pint, pos[j])
                num_p += np.conj(oj)[None] * chi
                den_p += np.abs(oj) ** 2
            d_o = gamma_obj * float(den_o.max())
            dir_o = num_o / (den_o + d_o)
            d_p = gamma_probe * float(den_p.max())
            dir_p = num_p / (den_p + d_p) if probe_on else np.zeros_like(probe)

            shifts = {j: position_shift(obj, probe, chis[j], pos[j], max_shift) for j in idx} if refine else {}
            for j in idx:
                av = probe * gather(dir_o, pos[j], n)[None]
                bv = dir_p * ojs[j][None]
                chi = chis[j]
                m00 = float(np.sum(np.abs(av) ** 2))
                m11 = float(np.sum(np.abs(bv) ** 2))
                m01 = float(np.real(np.vdot(av, bv)))
                v0 = float(np.real(np.vdot(av, chi)))
                v1 = float(np.real(np.vdot(bv, chi)))
                alpha[j] = lsqml_solve2(m00, m11, m01, v0, v1, probe_on)

            upd_o = np.zeros_like(obj)
            upd_p = np.zeros_like(probe)
            for j in idx:
                scatter_add(upd_o, alpha[j, 0] * np.sum(np.conj(probe) * chis[j], axis=0), pos[j])
                upd_p += alpha[j, 1] * np.conj(ojs[j])[None] * chis[j]
            obj = obj + beta_obj * upd_o / (den_o + d_o)
            if probe_on:
                probe = probe + beta_probe * upd_p / (den_p + d_p)
            for j, sh in shifts.items():
                pos[j] = np.clip(pos[j] + sh, 0.0, lim)
        errs.append(e_num / e_den)
        if ortho and probe_on:
            probe, _ = orthogonalise_modes(probe)
    out = (obj, probe, errs) + ((alpha,) if return_alpha else ()) + ((pos,) if return_positions else ())
    return out


# ---------------------------------------------------------------------------
# Metrics
# ---------------------------------------------------------------------------
def illumination(probe, pos, h, w) -> np.ndarray:
    """Ill = sum_j S_j^T sum_k |P_k|^2 on the object grid."""
    ill = np.zeros((h, w))
    pint = np.sum(np.abs(probe) ** 2, axis=0)
    for r in pos:
        scatter_add(ill, pint, r)
    return ill


def roi_mask(probe_true, pos, h, w, frac=0.3) -> np.ndarray:
    ill = illumination(probe_true, pos, h, w)
    return ill >= frac * ill.max()


def nrmse(obj, obj_true, mask) -> float:
    """Invariant NRMSE (Fienup 1997): min over complex c of ||c O - O_true|| / ||O_true|| on the ROI.

    The optimal c = <O, O_true> / <O, O> with <a, b> = sum conj(a) b.
    """
    o = np.asarray(obj)[mask]
    t = np.asarray(obj_true)[mask]
    oo = np.vdot(o, o).real
    c = np.vdot(o, t) / oo if oo > 0 else 0.0
    return float(np.linalg.norm(c * o - t) / np.linalg.norm(t))


def phase_aligned_rel(x, y) -> float:
    """min over theta of ||e^{i theta} X - Y|| / ||Y||, theta = arg <X, Y>."""
    x = np.asarray(x, dtype=np.complex128).ravel()
    y = np.asarray(y, dtype=np.complex128).ravel()
    ip = np.vdot(x, y)
    ph = ip / abs(ip) if abs(ip) > 0 else 1.0
    ny = np.linalg.norm(y)
    return float(np.linalg.norm(ph * x - y) / (ny if ny > 0 else 1.0))


# ---------------------------------------------------------------------------
# Poisson negative log-likelihood and its gradients
# ---------------------------------------------------------------------------
def _measured(mask, n):
    """Natural-order boolean plane of measured pixels (all of them without a mask)."""
    if mask is None:
        return np.ones((n, n), dtype=bool)
    return np.fft.ifftshift(np.asarray(mask) != 0)


def nll(obj, probe, pos, d, eps=EPS_L, mask=None) -> float:
    """L = sum_j sum_q [I_jq - d_jq log(I_jq + eps)] over the measured pixels,
    d given centred (log(d!) dropped); ``mask`` as in ``amplitude``."""
    n = probe.shape[-1]
    dn = np.fft.ifftshift(np.asarray(d, dtype=np.float64), axes=(-2, -1))
    valid = _measured(mask, n)
    total = 0.0
    for j, r in enumerate(pos):
        inten = np.sum(np.abs(fft2u(probe * gather(obj, r, n)[None])) ** 2, axis=0)
        total += float(np.sum(np.where(valid, inten - dn[j] * np.log(inten + eps), 0.0)))
    return total


def nll_grad(obj, probe, pos, d, eps=EPS_L, mask=None):
    """(L, g_O, g_P, g_R) in PyTorch's convention for complex leaves.

    For a real loss of complex z the gradient is dL/dRe z + i dL/dIm z.  With
    g_psi = F^-1[(1 - d/(I + eps)) Psi] (the derivative with respect to conj(psi)):
    g_O = 2 sum_j S_j^T sum_k conj(P_k) g_psi,jk;  g_P,k = 2 sum_j conj(S_j O) g_psi,jk;
    dL/dy_j = 2 Re sum_k sum_r conj(g_psi,jk) P_k d_y(S_j O), likewise for x.
    Unmeasured pixels (``mask`` as in ``amplitude``) add nothing to L, so their
    factor (1 - d/(I + eps)) is 0.
    """
    obj = np.asarray(obj, dtype=np.complex128)
    probe = np.asarray(probe, dtype=np.complex128)
    n = probe.shape[-1]
    dn = np.fft.ifftshift(np.asarray(d, dtype=np.float64), axes=(-2, -1))
    valid = _measured(mask, n)
    g_o = np.zeros_like(obj)
    g_p = np.zeros_like(probe)
    g_r = np.zeros((len(pos), 2))
    total = 0.0
    for j, r in enumerate(pos):
        oj = gather(obj, r, n)
        psi_f = fft2u(probe * oj[None])
        inten = np.sum(np.abs(psi_f) ** 2, axis=0)
        total += float(np.sum(np.where(valid, inten - dn[j] * np.log(inten + eps), 0.0)))
        g_psi = ifft2u(np.where(valid, 1.0 - dn[j] / (inten + eps), 0.0)[None] * psi_f)
        scatter_add(g_o, 2.0 * np.sum(np.conj(probe) * g_psi, axis=0), r)
        g_p += 2.0 * np.conj(oj)[None] * g_psi
        dy, dx = gather_grad(obj, r, n)
        g_r[j, 0] = 2.0 * float(np.real(np.sum(np.conj(g_psi) * probe * dy[None])))
        g_r[j, 1] = 2.0 * float(np.real(np.sum(np.conj(g_psi) * probe * dx[None])))
    return total, g_o, g_p, g_r
