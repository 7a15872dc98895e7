"""The allocation-free Poisson likelihood (pty_nll_forward_noalloc), called
through the C ABI, against the allocating pty_nll_forward: two calls in a row
on one context, the second over fewer positions, each compared with
pty_nll_forward on a context that holds exactly those positions.  Both entry
points sum the same per-block partials in the same order, so the losses agree
to rounding (relative 1e-12 here; the float32 kernels' own error against the
FP64 oracle is covered by the adjoint tests)."""
import ctypes as C

import numpy as np
import pytest

from _cases import c64, spiral_case

pytestmark = pytest.mark.gpu


def _plan(case, count):
    from paper_2202_03144_amd import Plan
    pl = Plan(case.n, case.k, count, case.obj_true.shape)
    pl.load_patterns(np.ascontiguousarray(case.counts[:count]))
    pl.load_positions(np.ascontiguousarray(case.pos[:count]))
    return pl


def _noalloc(pl, ot, pt, pos, count):
    import torch
    from paper_2202_03144_amd import _lib as L
    lib = L.lib()
    out = torch.full((1,), float("nan"), dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    st = lib.pty_nll_forward_noalloc(pl._live(), C.c_void_p(ot.data_ptr()), C.c_void_p(pt.data_ptr()),
                                     None if pos is None else C.c_void_p(pos.data_ptr()), count,
                                     C.c_void_p(out.data_ptr()))
    assert st == L.OK, lib.pty_last_error(pl._live())
    pl.sync()
    return float(out.cpu()[0])


def _rel(a, b):
    return abs(a - b) / abs(b)


@pytest.mark.parametrize("n,k,j,small", [(256, 3, 100, 37), (64, 2, 60, 9)])
def test_noalloc_forward_matches_allocating_forward(n, k, j, small):
    import torch
    from paper_2202_03144_amd import _lib as L
    case = spiral_case(n, k, j, cfg=96)
    rng = np.random.default_rng(7)
    o = c64(case.obj_true * (1 + 0.05 * rng.standard_normal(case.obj_true.shape)))
    p = c64(case.probe * (1 + 0.05 * rng.standard_normal(case.probe.shape)))
    ot = torch.from_numpy(o).cuda()
    pt = torch.from_numpy(p).cuda()
    pos = torch.from_numpy(case.pos.astype(np.float32)).cuda()
    print(f"\n[noalloc] n={n} k={k} j={j} small={small}", flush=True)
    with _plan(case, j) as full, _plan(case, small) as part:
        ref_full = full.nll_forward(ot, pt, pos)
        ref_part = part.nll_forward(ot, pt, pos[:small].contiguous())
        ref_part_loaded = part.nll_forward(ot, pt)   # float64 positions of pty_load_positions
        # first call: every position, device positions (several transform chunks at 256^2)
        l1 = _noalloc(full, ot, pt, pos, j)
        assert _rel(l1, ref_full) <= 1e-12, (l1, ref_full)
        # second call, smaller: the first `small` positions as loaded
        l2 = _noalloc(full, ot, pt, None, small)
        assert _rel(l2, ref_part_loaded) <= 1e-12, (l2, ref_part_loaded)
        # and once more from device positions, after the smaller call
        l3 = _noalloc(full, ot, pt, pos[:small].contiguous(), small)
        assert _rel(l3, ref_part) <= 1e-12, (l3, ref_part)
        # out-of-range counts are rejected before any device work
        lib = L.lib()
        out = torch.zeros(1, dtype=torch.float64, device="cuda")
        for bad in (0, j + 1):
            st = lib.pty_nll_forward_noalloc(full._live(), C.c_void_p(ot.data_ptr()), C.c_void_p(pt.data_ptr()),
                                             None, bad, C.c_void_p(out.data_ptr()))
            assert st == L.E_INVALID
            assert b"count" in lib.pty_last_error(full._live())
