"""Checkpoint / resume and the failure statuses that need a device.

* n iterations, checkpoint (object, probe, state), a new plan restored from
  it, n more iterations: bit-identical to 2n uninterrupted iterations
  (object, probe, error and NRMSE histories), for each algorithm, with the
  probe update switching on after the checkpoint;
* a checkpoint of the wrong shape, a truncated or foreign buffer is refused
  with the context unchanged;
* NaN in the probe gives PTY_E_NUMERIC from the error history; restoring the
  checkpoint taken before it continues the clean run exactly;
* a device-memory cap (PTY_MEM_LIMIT) gives PTY_E_NOMEM from the iteration
  that would exceed it, without exceeding the cap, and leaves the context
  usable."""
import os

import numpy as np
import pytest

from _cases import c64, spiral_case

pytestmark = pytest.mark.gpu


def _plan(case, truth=True):
    from paper_2202_03144_amd import Plan
    pl = Plan(case.n, case.k, case.j, case.shape)
    pl.load_patterns(case.counts)
    pl.load_positions(case.pos)
    pl.set_object(c64(np.ones(case.shape)))
    pl.set_probe(c64(case.probe))
    if truth:
        pl.set_truth(c64(case.obj_true), 0.3)
    return pl


def _snapshot(pl):
    return pl.object(), pl.probe(), pl.errors(), pl.nrmse_history()


@pytest.mark.parametrize("algo,params", [
    ("dm", dict(probe_update_start=3)),
    ("lsqml", dict(probe_update_start=3, lsqml_batch=9)),
    ("epie", dict(probe_update_start=3, order_seed=11)),
])
def test_resume_from_checkpoint_matches_uninterrupted_run(algo, params):
    case = spiral_case(64, 2, 30, cfg=97)
    ref = _plan(case)
    ref.iterate(algo, 5, **params)
    want = _snapshot(ref)
    ref.close()

    first = _plan(case)
    first.iterate(algo, 2, **params)
    blob, obj, probe = first.state(), first.object(), first.probe()
    first.close()

    resumed = _plan(case)
    resumed.set_object(obj)
    resumed.set_probe(probe)
    resumed.set_state(blob)
    assert len(resumed.errors()) == 2
    resumed.iterate(algo, 3, **params)
    got = _snapshot(resumed)
    resumed.close()
    for name, a, b in zip(("object", "probe", "E", "NRMSE"), got, want):
        assert np.array_equal(a, b), name


def test_dm_checkpoint_carries_exit_waves():
    case = spiral_case(64, 1, 20, cfg=98)
    pl = _plan(case, truth=False)
    pl.iterate("dm", 2, probe_update_start=0)
    blob = pl.state()
    psi = pl.exit_waves()
    other = _plan(case, truth=False)
    other.set_object(pl.object())
    other.set_probe(pl.probe())
    other.set_state(blob)
    assert np.array_equal(other.exit_waves(), psi)
    # without exit waves in the state, DM restarts them from object and probe
    pl.set_object(pl.object())                      # discards the exit waves
    assert len(pl.state()) < len(blob)
    pl.close()
    other.close()


def test_bad_checkpoints_are_refused_and_leave_the_context():
    from paper_2202_03144_amd import PtyError
    case = spiral_case(64, 1, 20, cfg=98)
    pl = _plan(case, truth=False)
    pl.iterate("lsqml", 2, lsqml_batch=10)
    blob = pl.state()
    other_shape = spiral_case(64, 2, 20, cfg=98)
    with _plan(other_shape, truth=False) as wrong:
        with pytest.raises(PtyError, match="INVALID.*shape"):
            wrong.set_state(blob)
        assert len(wrong.errors()) == 0
    target = _plan(case, truth=False)
    target.iterate("lsqml", 1, lsqml_batch=10)
    before = target.errors()
    with pytest.raises(PtyError, match="INVALID.*size"):
        target.set_state(blob[:-8])
    with pytest.raises(PtyError, match="INVALID.*not a state"):
        target.set_state(b"X" + blob[1:])
    with pytest.raises(PtyError, match="INVALID.*header"):
        target.set_state(blob[:20])
    assert np.array_equal(target.errors(), before)
    pl.close()
    target.close()


def test_nan_probe_reports_numeric_and_checkpoint_recovers():
    from paper_2202_03144_amd import PtyError
    case = spiral_case(64, 1, 20, cfg=98)
    ref = _plan(case, truth=False)
    ref.iterate("dm", 3, probe_update_start=0)
    want = _snapshot(ref)[:3]
    ref.close()

    pl = _plan(case, truth=False)
    pl.iterate("dm", 2, probe_update_start=0)
    blob, obj, probe = pl.state(), pl.object(), pl.probe()
    bad = probe.copy()
    bad[0, 32, 32] = np.nan
    pl.set_probe(bad)
    pl.iterate("dm", 1, probe_update_start=0)
    with pytest.raises(PtyError, match="NUMERIC"):
        pl.errors()
    # the state is kept, NaN and all (the object update skips pixels whose
    # denominator is not positive, so the NaN shows in the probe)
    assert np.isnan(pl.probe()).any()
    pl.set_object(obj)
    pl.set_probe(probe)
    pl.set_state(blob)
    pl.iterate("dm", 1, probe_update_start=0)
    got = (pl.object(), pl.probe(), pl.errors())
    pl.close()
    for name, a, b in zip(("object", "probe", "E"), got, want):
        assert np.array_equal(a, b), name


def test_memory_cap_reports_nomem_and_keeps_the_context():
    from paper_2202_03144_amd import Plan, PtyError
    case = spiral_case(64, 2, 30, cfg=97)
    probe_plan = _plan(case, truth=False)
    loaded = probe_plan.mem_bytes()
    probe_plan.close()
    # room for the host upload's temporary copy of the counts and a few small
    # buffers, not for the iteration's work buffers
    cap = loaded + case.j * case.n * case.n * 4 + (64 << 10)
    os.environ["PTY_MEM_LIMIT"] = str(cap)
    try:
        pl = Plan(case.n, case.k, case.j, case.shape)
    finally:
        del os.environ["PTY_MEM_LIMIT"]
    pl.load_patterns(case.counts)
    pl.load_positions(case.pos)
    o0 = c64(np.ones(case.shape))
    pl.set_object(o0)
    pl.set_probe(c64(case.probe))
    with pytest.raises(PtyError, match="NOMEM"):
        pl.iterate("dm", 1)
    assert pl.mem_bytes() <= cap
    assert np.array_equal(pl.object(), o0)
    assert len(pl.errors()) == 0
    pl.close()
