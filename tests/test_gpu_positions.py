"""LSQML position refinement on the GPU vs the FP64 oracle (whose shift rule
is pinned in test_oracle_positions.py): object, probe, errors and refined
positions after iterations that refine from the second one on, at the parity
tolerance; refined positions within 1e-4 px.  Plus the refusals (ePIE, DM,
graph replay, a non-positive clip) and the positions round trip."""
import numpy as np
import pytest

import oracle
from _cases import c64, rel, spiral_case, start_state

pytestmark = pytest.mark.gpu

TOL = 1e-4


def _nominal(case, seed=9, err=0.4):
    rng = np.random.default_rng(seed)
    lim = np.array(case.shape, dtype=float) - case.n
    return np.clip(case.pos + rng.uniform(-err, err, case.pos.shape), 0.0, lim)


def _plan(case, pos, o0, p0):
    from paper_2202_03144_amd import Plan
    pl = Plan(case.n, case.k, case.j, case.shape)
    pl.load_patterns(case.counts)
    pl.load_positions(pos)
    pl.set_object(c64(o0))
    pl.set_probe(c64(p0))
    return pl


# (N, K, J, chunk, lsqml batch, probe update start)
@pytest.mark.parametrize("n,k,j,chunk,batch,start", [(64, 2, 40, 7, 12, 1), (128, 1, 20, 6, 8, 0),
                                                     (256, 3, 10, 4, 6, 1)])
def test_refined_lsqml_matches_oracle(n, k, j, chunk, batch, start):
    case = spiral_case(n, k, j, cfg=62)
    pos0 = _nominal(case)
    o0, p0 = start_state(case, perturb=0.05)
    pl = _plan(case, pos0, o0, p0)
    params = dict(probe_update_start=start, chunk=chunk, lsqml_batch=batch, position_start=1,
                  position_max_shift=0.5)
    pl.iterate("lsqml", 3, **params)
    o1, p1, err, pos1 = oracle.lsqml(o0, p0, case.amp, pos0, 3, start=start, batch=batch, pos_start=1,
                                     max_shift=0.5, return_positions=True)
    got = pl.positions()
    assert np.max(np.abs(got - pos1)) <= 1e-4
    assert np.max(np.abs(got - pos0)) > 1e-2          # they did move
    assert rel(pl.object(), o1) <= TOL
    assert rel(pl.probe(), p1) <= TOL
    e = pl.errors()
    assert np.all(np.abs(e - np.asarray(err)) <= TOL * np.asarray(err))
    # a later iteration without refinement keeps the refined positions
    pl.iterate("lsqml", 1, probe_update_start=start, chunk=chunk, lsqml_batch=batch)
    assert np.array_equal(pl.positions(), got)
    pl.close()


def test_refinement_refusals_and_positions_round_trip():
    from paper_2202_03144_amd import PtyError
    case = spiral_case(64, 1, 20, cfg=62)
    pos0 = _nominal(case)
    o0, p0 = start_state(case)
    pl = _plan(case, pos0, o0, p0)
    assert np.max(np.abs(pl.positions() - pos0)) <= 1e-6
    for algo in ("epie", "dm"):
        with pytest.raises(PtyError, match="UNSUPPORTED"):
            pl.iterate(algo, 1, position_start=0)
    with pytest.raises(PtyError, match="UNSUPPORTED"):
        pl.iterate("lsqml", 1, graph=True, position_start=0)
    with pytest.raises(PtyError, match="INVALID"):
        pl.iterate("lsqml", 1, position_start=0, position_max_shift=0.0)
    assert len(pl.errors()) == 0
    assert np.max(np.abs(pl.positions() - pos0)) <= 1e-6
    pl.close()


def test_resume_with_refined_positions_is_exact():
    from paper_2202_03144_amd import Plan
    case = spiral_case(64, 2, 40, cfg=62)
    pos0 = _nominal(case)
    o0, p0 = start_state(case, perturb=0.05)
    params = dict(probe_update_start=0, lsqml_batch=12, position_start=1)
    ref = _plan(case, pos0, o0, p0)
    ref.iterate("lsqml", 4, **params)
    want = (ref.object(), ref.probe(), ref.errors(), ref.positions())
    ref.close()
    first = _plan(case, pos0, o0, p0)
    first.iterate("lsqml", 2, **params)
    blob, obj, probe, pos = first.state(), first.object(), first.probe(), first.positions()
    first.close()
    resumed = Plan(case.n, case.k, case.j, case.shape)
    resumed.load_patterns(case.counts)
    resumed.load_positions(pos)
    resumed.set_object(obj)
    resumed.set_probe(probe)
    resumed.set_state(blob)
    resumed.iterate("lsqml", 2, **params)
    got = (resumed.object(), resumed.probe(), resumed.errors(), resumed.positions())
    resumed.close()
    for name, a, b in zip(("object", "probe", "E", "positions"), got, want):
        assert np.array_equal(a, b), name
