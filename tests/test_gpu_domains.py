"""Strip decomposition (pty_domains_*) against one context: the strips, run
one after another on one GPU with their halo and probe messages exchanged,
give the single-context DM and LSQML iteration from an identical state up to
the order of the sums (relative L2 <= 1e-6 for object, probe and error; one
strip is bit-identical).  A second iteration continues from the two
slightly different states, and DM's reflection amplifies their rounding
differences (the noisy 64^2 workload moves ~25x per DM iteration), so the
second is held to 1e-4.  Cases: a 64^2 two-mode spiral split into 1, 3 and 4
strips, and the production shape (256^2, 3 modes, 2,500 positions, 1700^2
object) split into 8 strips, one GPU's share each."""
import numpy as np
import pytest

import ptysynth
from _cases import c64, spiral_case

pytestmark = pytest.mark.gpu

TOL = 1e-6
TOL_NEXT = 1e-4


def _rel(x, y):
    x = np.asarray(x, np.complex128).ravel()
    y = np.asarray(y, np.complex128).ravel()
    return float(np.linalg.norm(x - y) / np.linalg.norm(y))


def _pair(n, k, pos, shape, counts, o0, p0, strips):
    from paper_2202_03144_amd import Plan
    from paper_2202_03144_amd.plan import Domains
    pl = Plan(n, k, len(pos), shape)
    pl.load_patterns(counts)
    pl.load_positions(pos)
    pl.set_object(o0)
    pl.set_probe(p0)
    dd = Domains(n, k, pos, shape, strips)
    dd.load_patterns(counts)
    dd.set_object(o0)
    dd.set_probe(p0)
    return pl, dd


def _check_strips(dd, pos, n, h):
    """owned rows partition the object; every strip holds its patches' rows"""
    info = [dd.strip(s) for s in range(dd.strips)]
    assert info[0]["own_lo"] == 0 and info[-1]["own_hi"] == h
    for a, b in zip(info, info[1:]):
        assert a["own_hi"] == b["own_lo"]
    for s in info:
        assert s["lo"] <= s["own_lo"] <= s["own_hi"] <= s["hi"]
    assert sum(s["positions"] for s in info) == len(pos)


def _compare(pl, dd, label, tol=TOL):
    eo = _rel(dd.object(), pl.object())
    ep = _rel(dd.probe(), pl.probe())
    ee = _rel(dd.errors(), pl.errors())
    print(f"[domains] {label}: object {eo:.2e} probe {ep:.2e} error {ee:.2e}", flush=True)
    assert eo <= tol and ep <= tol and ee <= tol, (label, eo, ep, ee)
    return eo


def _reset_to(pl, dd):
    """both to the single context's object and probe (DM restarts its exit waves)"""
    o, p = pl.object(), pl.probe()
    pl.set_object(o)
    pl.set_probe(p)
    dd.set_object(o)
    dd.set_probe(p)


@pytest.mark.parametrize("strips", [1, 3, 4])
@pytest.mark.parametrize("algo", ["dm", "lsqml"])
def test_strips_equal_one_context_small(algo, strips):
    case = spiral_case(64, 2, 300, cfg=97)
    o0 = np.ones(case.obj_true.shape, np.complex64)
    p0 = c64(case.probe)
    print(f"\n[domains] 64^2 x 2, 300 positions, {strips} strips, {algo}", flush=True)
    pl, dd = _pair(64, 2, case.pos, case.obj_true.shape, case.counts, o0, p0, strips)
    with pl, dd:
        _check_strips(dd, case.pos, 64, case.obj_true.shape[0])
        params = dict(probe_update_start=0)
        if algo == "lsqml":
            params["lsqml_batch"] = 100
        pl.iterate(algo, 1, **params)
        dd.iterate(algo, 1, **params)
        _compare(pl, dd, f"{algo} {strips} strips, iteration 1")
        pl.iterate(algo, 1, **params)
        dd.iterate(algo, 1, **params)
        _compare(pl, dd, f"{algo} {strips} strips, iteration 2 (continued)", TOL_NEXT)
        _reset_to(pl, dd)
        pl.iterate(algo, 1, **params)
        dd.iterate(algo, 1, **params)
        _compare(pl, dd, f"{algo} {strips} strips, iteration 3 from the same state")
        halo, probe = dd.traffic()
        if strips == 1:
            assert halo == 0
        else:
            assert halo > 0 and probe > 0


def test_strips_equal_one_context_production_shape():
    import torch
    from paper_2202_03144_amd import Plan
    wl = ptysynth.workload(2)
    obj = wl.obj().astype(np.complex64)
    pos = wl.positions()
    expected = torch.empty((wl.j, wl.n, wl.n), dtype=torch.float32, device="cuda")
    with Plan(wl.n, wl.k, wl.j, (wl.h, wl.w)) as sim:
        sim.load_positions(pos)
        sim.set_object(obj)
        sim.set_probe(wl.probe().astype(np.complex64))
        sim.simulate(wl.photons, out=expected)
        probe = sim.probe()
    counts = expected.cpu().numpy()
    o0 = np.ones((wl.h, wl.w), np.complex64)
    print("\n[domains] 256^2 x 3, 2500 positions, 8 strips", flush=True)
    pl, dd = _pair(wl.n, wl.k, pos, (wl.h, wl.w), counts, o0, probe, 8)
    with pl, dd:
        _check_strips(dd, pos, wl.n, wl.h)
        shares = [dd.strip(s)["positions"] for s in range(8)]
        assert max(shares) - min(shares) <= 1
        pl.iterate("dm", 1, probe_update_start=0)
        dd.iterate("dm", 1, probe_update_start=0)
        _compare(pl, dd, "production DM, 8 strips")
        _reset_to(pl, dd)
        pl.iterate("lsqml", 1, probe_update_start=0, lsqml_batch=500)
        dd.iterate("lsqml", 1, probe_update_start=0, lsqml_batch=500)
        _compare(pl, dd, "production LSQML, 8 strips")


def test_strips_reject_what_is_not_decomposed():
    from paper_2202_03144_amd import PtyError
    from paper_2202_03144_amd import _lib as L
    case = spiral_case(64, 1, 40, cfg=98)
    o0 = np.ones(case.obj_true.shape, np.complex64)
    pl, dd = _pair(64, 1, case.pos, case.obj_true.shape, case.counts, o0, c64(case.probe), 2)
    with pl, dd:
        for algo, params in (("epie", {}), ("dm", {"flags": L.ITER_GRAPH}), ("lsqml", {"position_start": 0})):
            with pytest.raises(PtyError) as e:
                dd.iterate(algo, 1, **params)
            assert e.value.status == L.E_UNSUPPORTED
