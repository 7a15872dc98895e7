"""Detector mask on the GPU vs the FP64 oracle (whose masked projection,
error and likelihood are pinned in test_oracle_mask.py): one iteration of
each algorithm and the Poisson-NLL gradients with a beam stop and a dead
column masked, at the parity tolerance (phase-aligned relative L2 1e-4);
mask before or after the patterns, and clearing it, give bit-identical
results to the corresponding unmasked or masked plan."""
import numpy as np
import pytest

import oracle
import ptysynth
from _cases import c64, rel, spiral_case, start_state

pytestmark = pytest.mark.gpu

TOL = 1e-4

# (N, K, J, chunk, lsqml batch): the fused ePIE path (64^2), the per-position
# launches with the mode split of the column pass (128^2, 4 modes), the
# production window (256^2, 3 modes) and the wavefront-per-line ePIE
# launches (512^2)
SHAPES = [(64, 2, 20, 7, 6), (128, 4, 9, 4, 4), (256, 3, 8, 3, 4), (512, 1, 4, 2, 2)]


def _mask(n):
    m = np.ones((n, n), np.uint8)
    c = n // 2
    m[c - 2:c + 3, c - 2:c + 3] = 0      # beam stop over the zero frequency
    m[:, n // 3] = 0                     # dead column
    m[5, 7] = 0                          # one hot pixel
    return m


def _plan(case, o0, p0, mask, mask_first=False):
    from paper_2202_03144_amd import Plan
    pl = Plan(case.n, case.k, case.j, case.shape)
    if mask_first:
        pl.set_mask(mask)
    pl.load_patterns(case.counts)
    if not mask_first:
        pl.set_mask(mask)
    pl.load_positions(case.pos)
    pl.set_object(c64(o0))
    pl.set_probe(c64(p0))
    return pl


@pytest.mark.parametrize("algo", ["epie", "dm", "lsqml"])
@pytest.mark.parametrize("n,k,j,chunk,batch", SHAPES)
def test_masked_iteration_matches_oracle(algo, n, k, j, chunk, batch):
    case = spiral_case(n, k, j, cfg=88)
    m = _mask(n)
    a = oracle.amplitude(case.counts.astype(np.float64), m)
    o0, p0 = start_state(case, perturb=0.05)
    pl = _plan(case, o0, p0, m)
    if algo == "epie":
        pl.iterate("epie", 1, probe_update_start=0, order_seed=3)
        o1, p1, err = oracle.epie(o0, p0, a, case.pos, 1, start=0, order_seed=3)
    elif algo == "dm":
        pl.iterate("dm", 2, probe_update_start=0, chunk=chunk)
        o1, p1, _, err = oracle.dm(o0, p0, oracle.dm_init(o0, p0, case.pos), a, case.pos, 2, start=0)
    else:
        pl.iterate("lsqml", 1, probe_update_start=0, chunk=chunk, lsqml_batch=batch)
        o1, p1, err = oracle.lsqml(o0, p0, a, case.pos, 1, start=0, batch=batch)
    assert rel(pl.object(), o1) <= TOL
    assert rel(pl.probe(), p1) <= TOL
    e = pl.errors()
    assert np.all(np.abs(e - np.asarray(err)) <= TOL * np.asarray(err))
    # the evaluation pass uses the same masked projection
    assert abs(pl.model_error() - oracle.model_error(pl.object().astype(np.complex128),
                                                     pl.probe().astype(np.complex128), a, case.pos)) \
        <= 1e-4 * pl.model_error()
    pl.close()


def test_mask_order_and_clearing_are_exact():
    case = spiral_case(64, 2, 20, cfg=88)
    m = _mask(64)
    o0, p0 = start_state(case, perturb=0.05)
    runs = []
    for first in (False, True):
        pl = _plan(case, o0, p0, m, mask_first=first)
        pl.iterate("lsqml", 2, probe_update_start=0, lsqml_batch=6)
        runs.append((pl.object(), pl.probe(), pl.errors()))
        pl.close()
    assert all(np.array_equal(x, y) for x, y in zip(*runs))
    # masked, then cleared: identical to a plan that never had a mask
    from paper_2202_03144_amd import Plan
    cleared = _plan(case, o0, p0, m)
    cleared.set_mask(None)
    plain = Plan(case.n, case.k, case.j, case.shape)
    plain.load_patterns(case.counts)
    plain.load_positions(case.pos)
    plain.set_object(c64(o0))
    plain.set_probe(c64(p0))
    for pl in (cleared, plain):
        pl.iterate("dm", 2, probe_update_start=0)
    assert np.array_equal(cleared.object(), plain.object())
    assert np.array_equal(cleared.errors(), plain.errors())
    cleared.close()
    plain.close()


def test_masked_nll_gradients_match_oracle():
    import torch
    from paper_2202_03144_amd import Plan
    wl = ptysynth.scaled(ptysynth.workload(3), cfg=31, n=32, k=4, h=48, w=48, d=11.0,
                         sigma_e=1.0, sigma_p=3.0, photons=1e4)
    rng = np.random.default_rng(17)
    pos = ptysynth.raster_positions(4, 4, 4.0, 1.0) + rng.uniform(0.1, 0.9, (16, 2))
    o = wl.obj()
    cnt, p = oracle.simulate(o, wl.probe(), pos, wl.photons)
    cnt = ptysynth.poisson_counts(cnt, wl.noise_rng())
    o = c64(o * (1 + 0.05 * (rng.standard_normal(o.shape) + 1j * rng.standard_normal(o.shape))))
    p = c64(p)
    m = _mask(32)
    pl = Plan(32, 4, len(pos), o.shape)
    pl.load_patterns(cnt)
    pl.load_positions(pos)
    pl.set_mask(m)
    ot, pt = torch.from_numpy(o).cuda(), torch.from_numpy(p).cuda()
    go, gp = torch.empty_like(ot), torch.empty_like(pt)
    gr = torch.empty((len(pos), 2), dtype=torch.float32, device="cuda")
    loss = pl.nll_backward(ot, pt, 1.0, go, gp, gr)
    lf = pl.nll_forward(ot, pt)
    pl.close()
    ref_l, ref_go, ref_gp, ref_gr = oracle.nll_grad(o.astype(np.complex128), p.astype(np.complex128), pos,
                                                    cnt.astype(np.float64), mask=m)
    assert abs(loss - ref_l) <= 1e-5 * abs(ref_l) and abs(lf - ref_l) <= 1e-5 * abs(ref_l)
    for got, ref in ((go.cpu().numpy(), ref_go), (gp.cpu().numpy(), ref_gp)):
        assert np.linalg.norm(got - ref) <= TOL * np.linalg.norm(ref)
    g = gr.cpu().numpy()
    assert np.linalg.norm(g - ref_gr) <= TOL * np.linalg.norm(ref_gr)
