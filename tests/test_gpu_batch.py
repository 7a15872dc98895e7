"""Graph-replayed iterations, batches of uneven datasets and the autotuner
against eager single-dataset iterations, and the batched, graph-replayed path
against the FP64 oracle.

Graphs and batches only change how the same kernels are launched (captured
once and replayed; several contexts on their own streams), never what they
compute, so their results must be bit-identical to eager iterations of each
dataset alone; the autotuner's probe-sum slicing reorders sums (rounding)."""
import json

import numpy as np
import pytest

import oracle
from _cases import c64, raster_case, rel, spiral_case

pytestmark = pytest.mark.gpu


def _plan(case, stream=None, truth=False):
    import torch
    from paper_2202_03144_amd import Plan
    pl = Plan(case.n, case.k, case.j, case.shape, stream=stream)
    pl.load_patterns(case.counts)
    pl.load_positions(case.pos)
    pl.set_object(c64(np.ones(case.shape)))
    pl.set_probe(c64(case.probe))
    if truth:
        pl.set_truth(c64(case.obj_true), 0.3)
    return pl


def _state(pl):
    return pl.object(), pl.probe(), pl.errors()


def _same(a, b):
    return all(np.array_equal(x, y) for x, y in zip(a, b))


@pytest.mark.parametrize("algo,params", [
    ("dm", dict(probe_update_start=2)),
    ("lsqml", dict(probe_update_start=1, lsqml_batch=12)),
])
def test_graph_replays_match_eager(algo, params):
    import torch
    case = spiral_case(64, 2, 30, cfg=97)
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    eager = _plan(case, s1, truth=True)
    graph = _plan(case, s2, truth=True)
    for it in range(5):
        eager.iterate(algo, 1, **params)
        graph.iterate(algo, 1, graph=True, **params)
        # eager work and synchronisation between the replays
        a, b = _state(eager), _state(graph)
        assert _same(a, b), f"iteration {it}"
        assert np.array_equal(eager.nrmse_history(), graph.nrmse_history())
    # several replays in one call
    eager.iterate(algo, 3, **params)
    graph.iterate(algo, 3, graph=True, **params)
    assert _same(_state(eager), _state(graph))
    # switching back to eager iterations continues the same trajectory
    eager.iterate(algo, 1, **params)
    graph.iterate(algo, 1, **params)
    assert _same(_state(eager), _state(graph))
    eager.close()
    graph.close()


def _uneven_cases():
    return [spiral_case(64, 1, 20, cfg=98), spiral_case(128, 1, 12, cfg=99),
            raster_case(64, 2, 5, 6, 7.0, 4.0, 110, cfg=100), spiral_case(32, 3, 40, cfg=101)]


@pytest.mark.parametrize("graph", [False, True])
def test_batch_matches_individual(graph):
    import torch
    from paper_2202_03144_amd import Batch
    cases = _uneven_cases()
    params = dict(probe_update_start=1, lsqml_batch=8)
    singles = [_plan(c) for c in cases]
    for pl in singles:
        pl.iterate("lsqml", 3, **params)
    batched = [_plan(c, torch.cuda.Stream()) for c in cases]
    with Batch(batched) as b:
        b.iterate("lsqml", 3, graph=graph, **params)
        b.sync()
    for i, (x, y) in enumerate(zip(singles, batched)):
        assert _same(_state(x), _state(y)), f"dataset {i}"
    for pl in singles + batched:
        pl.close()


def test_batch_reports_failing_context():
    from paper_2202_03144_amd import Batch, Plan, PtyError
    case = spiral_case(64, 1, 20, cfg=98)
    good = _plan(case)
    empty = Plan(64, 1, 20, case.shape)      # nothing loaded
    with Batch([good, empty]) as b:
        with pytest.raises(PtyError, match="STATE.*context 1"):
            b.iterate("dm", 1)
    good.close()
    empty.close()


def test_autotune_keeps_results_and_caches(tmp_path):
    case = spiral_case(64, 2, 30, cfg=97)
    params = dict(probe_update_start=0, lsqml_batch=15)
    ref = _plan(case)
    ref.iterate("lsqml", 2, chunk=7, **params)
    tuned = _plan(case)
    cache = str(tmp_path / "tune.json")
    ch = tuned.autotune("lsqml", cache, **params)
    assert ch in (8, 16, 24, 32, 48, 64, 96, 128, 192, 256)
    ch2, sl = tuned.tuning()
    assert ch2 == ch and sl in (8, 16, 32)
    tuned.iterate("lsqml", 2, **params)         # uses the tuned chunk and probe-sum slices
    # the chunk changes only how the passes are launched; the slice size the
    # order of the probe sums, so the results agree to rounding
    a, b = _state(ref), _state(tuned)
    for x, y in zip(a, b):
        assert np.linalg.norm(x - y) <= 1e-5 * np.linalg.norm(y)
    data = json.load(open(cache))
    key = [k for k in data if not k.endswith(" slice")]
    assert len(key) == 1 and "n=64 k=2 j=30 lsqml b=15" in key[0]
    assert data[key[0]] == ch and data[key[0] + " slice"] == sl
    # a second plan of the same shape reads the cache
    again = _plan(case)
    assert again.autotune("lsqml", cache, **params) == ch and again.tuning() == (ch, sl)
    for pl in (ref, tuned, again):
        pl.close()


def test_error_paths_of_the_newer_entry_points():
    """State and shape errors are reported as statuses, before any device work."""
    import torch
    from paper_2202_03144_amd import Plan, PtyError
    from paper_2202_03144_amd.cnn import Net
    case = spiral_case(64, 1, 20, cfg=98)
    with Plan(64, 1, 20, case.shape) as pl:
        with pytest.raises(PtyError, match="STATE"):
            pl.set_truth(c64(case.obj_true))          # no positions yet
        with pytest.raises(PtyError, match="STATE"):
            pl.nrmse()                                # no truth
        with pytest.raises(PtyError, match="STATE"):
            pl.model_error()                          # nothing loaded
        pl.load_patterns(case.counts)
        pl.load_positions(case.pos)
        pl.set_object(c64(np.ones(case.shape)))
        pl.set_probe(c64(case.probe))
        with pytest.raises(PtyError, match="UNSUPPORTED"):
            pl.autotune("epie")
        with pytest.raises(PtyError, match="UNSUPPORTED"):
            pl.stitch(torch.zeros((20, 64, 64, 2), dtype=torch.float32, device="cuda"))
        with Net(4, seed=0) as net:
            with pytest.raises(PtyError, match="UNSUPPORTED"):
                pl.seed_object(net, batch=4)     # the network takes 128 x 128 windows
        with pytest.raises(PtyError, match="INVALID"):
            pl.set_truth(c64(case.obj_true), 1.5)     # roi_frac outside [0, 1]
        with pytest.raises(PtyError, match="INVALID"):
            pl.training_targets(torch.zeros((20, 32, 32, 2), dtype=torch.float32, device="cuda"))
        # state survives the failed calls
        pl.iterate("dm", 1)
        assert np.isfinite(pl.errors()).all()


def test_batched_graph_iteration_matches_oracle_per_size_class():
    """One dataset of each window size of the batched workload (64, 128, 256;
    1-3 modes; LSQML in several groups, probe updates on), iterated together
    through pty_batch_iterate with graph replay: each against one FP64 oracle
    LSQML iteration from the same state (phase-aligned relative L2 <= 1e-4)."""
    import torch
    from paper_2202_03144_amd import Batch
    cases = [spiral_case(64, 2, 40, cfg=102), spiral_case(128, 1, 30, cfg=103), spiral_case(256, 3, 20, cfg=104)]
    batch = 12
    plans = [_plan(c, torch.cuda.Stream()) for c in cases]
    with Batch(plans) as b:
        b.iterate("lsqml", 1, graph=True, probe_update_start=0, lsqml_batch=batch)
        b.sync()
    for c, pl in zip(cases, plans):
        o0 = np.ones(c.shape, np.complex128)
        p0 = c64(c.probe).astype(np.complex128)
        ro, rp, re = oracle.lsqml(o0, p0, c.amp, c.pos, 1, start=0, batch=batch)
        eo, ep = rel(pl.object(), ro), rel(pl.probe(), rp)
        ee = abs(pl.errors()[0] - re[0]) / re[0]
        print(f"[batch-oracle] N={c.n} K={c.k} J={c.j}: object {eo:.2e} probe {ep:.2e} E {ee:.2e}", flush=True)
        assert eo <= 1e-4 and ep <= 1e-4 and ee <= 1e-4, (c.n, eo, ep, ee)
        pl.close()
