"""Pins of the oracle's probe-mode orthogonalisation (mixed states, Thibault &
Menzel 2013): the new modes are orthogonal, ordered by power, carry the same
incoherent sum and mutual coherence, their powers are the Gram matrix's
eigenvalues (closed form for two modes), the basis follows its phase
convention and is the identity on already-orthogonal modes, and — because
every update rule here is equivariant under a unitary mixing of the modes —
a reconstruction with orthogonalisation follows the same object trajectory."""
import numpy as np
import pytest

import oracle
import ptysynth


def _crandn(rng, *shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def _modes(k=3, n=12, seed=1):
    rng = np.random.default_rng([41, seed])
    p = _crandn(rng, k, n, n)
    p[1] += 0.6 * p[0]               # far from orthogonal
    return p


def test_orthogonal_sorted_same_density_and_coherence():
    p = _modes()
    q, _ = oracle.orthogonalise_modes(p)
    g = np.einsum("kxy,lxy->kl", q, q.conj())
    off = g - np.diag(np.diag(g))
    assert np.max(np.abs(off)) <= 1e-12 * np.max(np.abs(g))
    pw = np.real(np.diag(g))
    assert np.all(np.diff(pw) < 0)
    assert np.max(np.abs(np.sum(np.abs(q) ** 2, 0) - np.sum(np.abs(p) ** 2, 0))) <= 1e-12 * np.max(np.abs(p)) ** 2
    rng = np.random.default_rng(2)
    for _ in range(10):
        r1, r2 = rng.integers(0, 12, 2), rng.integers(0, 12, 2)
        c_p = np.sum(p[:, r1[0], r1[1]] * np.conj(p[:, r2[0], r2[1]]))
        c_q = np.sum(q[:, r1[0], r1[1]] * np.conj(q[:, r2[0], r2[1]]))
        assert abs(c_p - c_q) <= 1e-12 * max(1.0, abs(c_p))


def test_two_mode_powers_match_closed_form_eigenvalues():
    p = _modes(k=2)
    a = float(np.sum(np.abs(p[0]) ** 2))
    d = float(np.sum(np.abs(p[1]) ** 2))
    b = complex(np.sum(p[0] * np.conj(p[1])))
    mid, rad = 0.5 * (a + d), np.sqrt((0.5 * (a - d)) ** 2 + abs(b) ** 2)
    q, _ = oracle.orthogonalise_modes(p)
    pw = np.sum(np.abs(q) ** 2, axis=(1, 2))
    assert abs(pw[0] - (mid + rad)) <= 1e-12 * (mid + rad)
    assert abs(pw[1] - (mid - rad)) <= 1e-10 * (mid + rad)


def test_basis_convention_and_identity_on_orthogonal_modes():
    p = _modes(k=4, seed=3)
    v = oracle.mode_basis(p)
    assert np.max(np.abs(v.conj().T @ v - np.eye(4))) <= 1e-12
    for k in range(4):
        i = int(np.argmax(np.abs(v[:, k])))
        assert abs(v[i, k].imag) <= 1e-15 and v[i, k].real > 0
    q, _ = oracle.orthogonalise_modes(p)
    assert np.max(np.abs(oracle.mode_basis(q) - np.eye(4))) <= 1e-12
    q2, _ = oracle.orthogonalise_modes(q)
    assert np.max(np.abs(q2 - q)) <= 1e-12 * np.max(np.abs(q))


def _tiny():
    wl = ptysynth.scaled(ptysynth.workload(1), cfg=43, n=32, k=2, h=80, w=80, d=13.0,
                         rows=5, cols=5, step=8.0, offset=6.0, j=25, photons=1e6)
    o = wl.obj()
    pos = wl.positions()
    cnt, p = oracle.simulate(o, wl.probe(), pos, wl.photons)
    cnt = ptysynth.poisson_counts(cnt, wl.noise_rng()).astype(np.float64)
    rng = np.random.default_rng(4)
    p0 = p.copy()
    p0[1] += 0.5 * p0[0]             # a non-orthogonal start
    p0 = p0 * (1 + 0.05 * _crandn(rng, *p0.shape))
    return np.ones_like(o), p0, pos, oracle.amplitude(cnt)


@pytest.mark.parametrize("algo", ["epie", "dm", "lsqml"])
def test_reconstruction_with_orthogonalisation_follows_the_same_object(algo):
    o0, p0, pos, a = _tiny()
    runs = []
    for ortho in (False, True):
        if algo == "epie":
            o, p, e = oracle.epie(o0, p0, a, pos, 3, start=0, ortho=ortho)
        elif algo == "dm":
            o, p, _, e = oracle.dm(o0, p0, oracle.dm_init(o0, p0, pos), a, pos, 3, start=0, ortho=ortho)
        else:
            o, p, e = oracle.lsqml(o0, p0, a, pos, 3, start=0, batch=10, ortho=ortho)
        runs.append((o, p, np.asarray(e)))
    (o1, p1, e1), (o2, p2, e2) = runs
    assert np.max(np.abs(o2 - o1)) <= 1e-9 * np.max(np.abs(o1))
    assert np.max(np.abs(e2 - e1)) <= 1e-9 * np.max(e1)
    assert np.max(np.abs(np.sum(np.abs(p2) ** 2, 0) - np.sum(np.abs(p1) ** 2, 0))) <= 1e-9 * np.max(np.abs(p1)) ** 2
    # and the modes themselves did change: orthogonal now
    g = np.einsum("kxy,lxy->kl", p2, p2.conj())
    assert abs(g[0, 1]) <= 1e-9 * abs(g[0, 0])
    g1 = np.einsum("kxy,lxy->kl", p1, p1.conj())
    assert abs(g1[0, 1]) > 1e-3 * abs(g1[0, 0])
