"""HIP path vs the FP64 oracle, element by element, through the C ABI.

Tolerance: relative L2 error <= 1e-4 after global-phase alignment for object,
probe, DM exit waves and LSQML step lengths after one iteration from an
identical state; relative 1e-4 on the iteration error; final NRMSE within 2%
of the oracle's on the full 64^2 / 100-position workload.
"""
import numpy as np
import pytest

import oracle
from _cases import c64, raster_case, rel, spiral_case, start_state, workload_case

pytestmark = pytest.mark.gpu

TOL = 1e-4

# (N, K, J, chunk, lsqml batch): ragged chunk tails and group sizes
SHAPES = [
    (32, 2, 13, 5, 5),
    (64, 1, 24, 7, 10),
    (128, 4, 9, 4, 4),
    (256, 3, 10, 3, 4),
    (256, 4, 6, 4, 4),     # modes split over two lane groups in the column pass
    (512, 2, 5, 3, 3),     # 512-wide windows: two column blocks per row band
]


def _plan(case, o0, p0):
    from paper_2202_03144_amd import Plan
    pl = Plan(case.n, case.k, case.j, case.shape)
    pl.load_patterns(case.counts)
    pl.load_positions(case.pos)
    pl.set_object(c64(o0))
    pl.set_probe(c64(p0))
    return pl


_CACHE = {}


def _case(n, k, j):
    key = (n, k, j)
    if key not in _CACHE:
        _CACHE[key] = spiral_case(n, k, j)
    return _CACHE[key]


@pytest.mark.parametrize("n,k,j,chunk,batch", SHAPES)
def test_simulate_matches_forward_model(n, k, j, chunk, batch):
    case = _case(n, k, j)
    pl = _plan(case, case.obj_true, case.probe)
    got = pl.simulate(0.0)
    ref, _ = oracle.simulate(c64(case.obj_true), c64(case.probe), case.pos)
    assert np.linalg.norm(got - ref) / np.linalg.norm(ref) <= 1e-5
    pl.close()


@pytest.mark.parametrize("start", [0, 1])
@pytest.mark.parametrize("n,k,j,chunk,batch", SHAPES)
def test_dm_one_iteration(n, k, j, chunk, batch, start):
    case = _case(n, k, j)
    o0, p0 = start_state(case, perturb=0.05)
    pl = _plan(case, o0, p0)
    pl.iterate("dm", 1, probe_update_start=start, chunk=chunk)
    psi0 = oracle.dm_init(o0, p0, case.pos)
    o1, p1, psi1, err = oracle.dm(o0, p0, psi0, case.amp, case.pos, 1, start=start)
    assert rel(pl.object(), o1) <= TOL
    assert rel(pl.probe(), p1) <= TOL
    assert rel(pl.exit_waves(), psi1) <= TOL
    e = pl.errors()
    assert len(e) == 1 and abs(e[0] - err[0]) <= TOL * err[0]
    # a second call continues from the stored exit waves
    pl.iterate("dm", 1, probe_update_start=start, chunk=chunk)
    o2, p2, psi2, err2 = oracle.dm(o1, p1, psi1, case.amp, case.pos, 1, t0=1, start=start)
    assert rel(pl.object(), o2) <= TOL
    assert rel(pl.probe(), p2) <= TOL
    assert abs(pl.errors()[1] - err2[0]) <= TOL * err2[0]
    pl.close()


@pytest.mark.parametrize("start", [0, 5])
@pytest.mark.parametrize("n,k,j,chunk,batch", SHAPES)
def test_lsqml_one_iteration(n, k, j, chunk, batch, start):
    case = _case(n, k, j)
    o0, p0 = start_state(case, perturb=0.05)
    pl = _plan(case, o0, p0)
    pl.iterate("lsqml", 1, probe_update_start=start, chunk=chunk, lsqml_batch=batch)
    o1, p1, err, alpha = oracle.lsqml(o0, p0, case.amp, case.pos, 1, start=start, batch=batch,
                                      return_alpha=True)
    assert rel(pl.object(), o1) <= TOL
    assert rel(pl.probe(), p1) <= TOL
    a = pl.lsqml_steps().astype(np.float64)
    assert np.linalg.norm(a - alpha) <= TOL * np.linalg.norm(alpha)
    assert abs(pl.errors()[0] - err[0]) <= TOL * err[0]
    pl.close()


@pytest.mark.parametrize("seed", [0, 77])
@pytest.mark.parametrize("n,k,j,chunk,batch", SHAPES)
def test_epie_one_iteration(n, k, j, chunk, batch, seed):
    case = _case(n, k, j)
    o0, p0 = start_state(case, perturb=0.05)
    pl = _plan(case, o0, p0)
    pl.iterate("epie", 1, probe_update_start=0, order_seed=seed)
    o1, p1, err = oracle.epie(o0, p0, case.amp, case.pos, 1, start=0, order_seed=seed)
    assert rel(pl.object(), o1) <= TOL
    assert rel(pl.probe(), p1) <= TOL
    assert abs(pl.errors()[0] - err[0]) <= TOL * err[0]
    pl.close()


# ePIE windows of each kernel family: the one-workgroup kernels (32^2 and
# 64^2 up to four modes), the per-position launches (128^2) and the
# wavefront-per-line launches (512^2, one and two modes); odd and even
# position counts (the probe's final buffer)
EPIE_WINDOWS = [(32, 4, 13), (64, 2, 12), (64, 3, 9), (64, 4, 7), (128, 1, 9), (128, 1, 8),
                (512, 1, 5), (512, 2, 4)]


@pytest.mark.parametrize("n,k,j", EPIE_WINDOWS)
def test_epie_window_two_iterations(n, k, j):
    case = _case(n, k, j)
    o0, p0 = start_state(case, perturb=0.05)
    pl = _plan(case, o0, p0)
    pl.iterate("epie", 2, probe_update_start=0, order_seed=5)
    o1, p1, err = oracle.epie(o0, p0, case.amp, case.pos, 2, start=0, order_seed=5)
    assert rel(pl.object(), o1) <= TOL
    assert rel(pl.probe(), p1) <= TOL
    assert np.allclose(pl.errors()[:2], err[:2], rtol=TOL, atol=0)
    pl.close()


def _oracle_run(algo, case, o0, p0, n_iter, start):
    if algo == "epie":
        o, _, err = oracle.epie(o0, p0, case.amp, case.pos, n_iter, start=start)
    elif algo == "dm":
        o, _, _, err = oracle.dm(o0, p0, oracle.dm_init(o0, p0, case.pos), case.amp, case.pos, n_iter, start=start)
    else:
        o, _, err = oracle.lsqml(o0, p0, case.amp, case.pos, n_iter, start=start)
    return o, err


@pytest.mark.parametrize("noise", [False, True])
@pytest.mark.parametrize("algo", ["epie", "dm", "lsqml"])
def test_raster64_final_nrmse_within_2pct(algo, noise):
    """The full 64^2, 1-mode, 10x10 raster workload: 50 iterations, probe updates from 10.

    DM on Poisson data does not converge on this workload: its final NRMSE moves
    by ~2.5% when the FP64 oracle's probe is perturbed by 1e-7 (relative), so
    there the GPU result is checked against the oracle's own spread under such
    perturbations, widened by 2%.
    """
    case = workload_case(1, noise=noise)
    o0 = np.ones(case.shape, np.complex128)
    p0 = c64(case.probe).astype(np.complex128)
    mask = oracle.roi_mask(case.probe, case.pos, *case.shape)
    pl = _plan(case, o0, p0)
    pl.iterate(algo, 50, probe_update_start=10)
    n_gpu = oracle.nrmse(pl.object().astype(np.complex128), case.obj_true, mask)
    e = pl.errors()
    pl.close()
    assert len(e) == 50 and np.all(np.isfinite(e))
    o_ref, err = _oracle_run(algo, case, o0, p0, 50, 10)
    n_ref = oracle.nrmse(o_ref, case.obj_true, mask)
    if noise and algo == "dm":
        spread = [n_ref]
        rng = np.random.default_rng(1)
        for _ in range(3):
            pp = p0 * (1 + 1e-7 * rng.standard_normal(p0.shape))
            spread.append(oracle.nrmse(_oracle_run(algo, case, o0, pp, 50, 10)[0], case.obj_true, mask))
        assert 0.98 * min(spread) <= n_gpu <= 1.02 * max(spread), (n_gpu, spread)
        return
    assert abs(n_gpu - n_ref) <= 0.02 * n_ref, (n_gpu, n_ref)
    assert abs(e[-1] - err[-1]) <= 0.02 * err[-1], (e[-1], err[-1])


def test_integer_positions_and_edge_patch():
    """Integer positions (exact slices), including a patch on the object's far edge."""
    case = raster_case(32, 1, 4, 4, 10.0, 0.0, 62)
    assert case.pos.max() + 32 == 62
    o0, p0 = start_state(case, perturb=0.05)
    for algo in ("dm", "lsqml", "epie"):
        pl = _plan(case, o0, p0)
        pl.iterate(algo, 1, probe_update_start=0, lsqml_batch=7)
        if algo == "dm":
            o1, p1, _, _ = oracle.dm(o0, p0, oracle.dm_init(o0, p0, case.pos), case.amp, case.pos, 1, start=0)
        elif algo == "lsqml":
            o1, p1, _ = oracle.lsqml(o0, p0, case.amp, case.pos, 1, start=0, batch=7)
        else:
            o1, p1, _ = oracle.epie(o0, p0, case.amp, case.pos, 1, start=0)
        assert rel(pl.object(), o1) <= TOL, algo
        assert rel(pl.probe(), p1) <= TOL, algo
        pl.close()


def test_single_position():
    case = spiral_case(64, 2, 1)
    o0, p0 = start_state(case, perturb=0.05)
    for algo in ("dm", "lsqml", "epie"):
        pl = _plan(case, o0, p0)
        pl.iterate(algo, 2, probe_update_start=1)
        if algo == "dm":
            o1, p1, _, _ = oracle.dm(o0, p0, oracle.dm_init(o0, p0, case.pos), case.amp, case.pos, 2, start=1)
        elif algo == "lsqml":
            o1, p1, _ = oracle.lsqml(o0, p0, case.amp, case.pos, 2, start=1)
        else:
            o1, p1, _ = oracle.epie(o0, p0, case.amp, case.pos, 2, start=1)
        assert rel(pl.object(), o1) <= TOL, algo
        assert rel(pl.probe(), p1) <= TOL, algo
        pl.close()


def test_algorithm_switch_reinitialises_dm():
    case = spiral_case(64, 1, 16)
    o0, p0 = start_state(case, perturb=0.05)
    pl = _plan(case, o0, p0)
    pl.iterate("lsqml", 1, probe_update_start=0)
    pl.iterate("dm", 1, probe_update_start=0)
    o1, p1, _ = oracle.lsqml(o0, p0, case.amp, case.pos, 1, start=0)
    o2, p2, _, _ = oracle.dm(o1, p1, oracle.dm_init(o1, p1, case.pos), case.amp, case.pos, 1, t0=1, start=0)
    assert rel(pl.object(), o2) <= TOL
    assert rel(pl.probe(), p2) <= TOL
    assert len(pl.errors()) == 2
    pl.close()
