"""LSQML with the Poisson exit-wave update on the GPU vs the FP64 oracle
(whose update is pinned in test_oracle_poisson.py): object, probe and errors
after iterations at the parity tolerance, with and without a detector mask,
over the chunked column pass and its mode split; graph replays equal eager
iterations bit for bit; the likelihood falls; ePIE and DM refuse the flag."""
import numpy as np
import pytest

import oracle
from _cases import c64, rel, spiral_case, start_state

pytestmark = pytest.mark.gpu

TOL = 1e-4


def _plan(case, o0, p0, mask=None):
    from paper_2202_03144_amd import Plan
    pl = Plan(case.n, case.k, case.j, case.shape)
    pl.load_patterns(case.counts)
    if mask is not None:
        pl.set_mask(mask)
    pl.load_positions(case.pos)
    pl.set_object(c64(o0))
    pl.set_probe(c64(p0))
    return pl


def _mask(n):
    m = np.ones((n, n), np.uint8)
    c = n // 2
    m[c - 2:c + 3, c - 2:c + 3] = 0      # beam stop over the zero frequency
    m[:, n // 3] = 0                     # dead column
    return m


# (N, K, J, chunk, lsqml batch, probe update start, masked): a ragged last
# chunk, the 4-mode split of the column pass, the production window, 512^2
@pytest.mark.parametrize("n,k,j,chunk,batch,start,masked", [
    (64, 2, 40, 7, 12, 1, False),
    (64, 1, 20, 5, 20, 0, True),
    (128, 4, 12, 5, 6, 0, False),
    (128, 4, 9, 4, 9, 0, True),
    (256, 3, 10, 4, 6, 1, False),
    (512, 2, 4, 3, 4, 0, False),
])
def test_poisson_lsqml_matches_oracle(n, k, j, chunk, batch, start, masked):
    case = spiral_case(n, k, j, cfg=64)
    o0, p0 = start_state(case, perturb=0.05)
    m = _mask(n) if masked else None
    a = oracle.amplitude(case.counts.astype(np.float64), m)
    pl = _plan(case, o0, p0, m)
    iters = 2 if n <= 256 else 1
    pl.iterate("lsqml", iters, likelihood="poisson", probe_update_start=start, chunk=chunk, lsqml_batch=batch)
    o1, p1, err = oracle.lsqml(o0, p0, a, case.pos, iters, start=start, batch=batch, likelihood="poisson")
    assert rel(pl.object(), o1) <= TOL
    assert rel(pl.probe(), p1) <= TOL
    e = pl.errors()
    assert np.all(np.abs(e - np.asarray(err)) <= TOL * np.asarray(err))
    pl.close()


def test_graph_replay_is_exact_and_the_likelihood_falls():
    import torch
    case = spiral_case(64, 2, 40, cfg=64)
    o0, p0 = start_state(case, perturb=0.05)
    a, b = _plan(case, o0, p0), _plan(case, o0, p0)
    params = dict(likelihood="poisson", probe_update_start=0, lsqml_batch=12)
    nll = [oracle.nll(o0, p0, case.pos, case.counts.astype(np.float64))]
    for _ in range(3):
        a.iterate("lsqml", 1, **params)
        b.iterate("lsqml", 1, graph=True, **params)
        torch.cuda.synchronize()
        assert np.array_equal(a.object(), b.object())
        assert np.array_equal(a.probe(), b.probe())
        nll.append(oracle.nll(a.object().astype(np.complex128), a.probe().astype(np.complex128), case.pos,
                              case.counts.astype(np.float64)))
    assert np.array_equal(a.errors(), b.errors())
    assert all(y < x for x, y in zip(nll, nll[1:]))
    a.close()
    b.close()


def test_poisson_differs_from_amplitude_and_is_refused_outside_lsqml():
    from paper_2202_03144_amd import PtyError
    case = spiral_case(64, 1, 20, cfg=64)
    o0, p0 = start_state(case, perturb=0.05)
    a, b = _plan(case, o0, p0), _plan(case, o0, p0)
    for algo in ("epie", "dm"):
        with pytest.raises(PtyError, match="UNSUPPORTED"):
            a.iterate(algo, 1, likelihood="poisson")
    with pytest.raises(ValueError):
        a.iterate("lsqml", 1, likelihood="gaussian")
    assert len(a.errors()) == 0
    a.iterate("lsqml", 1, likelihood="poisson", probe_update_start=0)
    b.iterate("lsqml", 1, probe_update_start=0)
    assert not np.array_equal(a.object(), b.object())
    assert np.allclose(a.errors(), b.errors(), rtol=1e-6, atol=0)   # the same far field enters
    a.close()
    b.close()
