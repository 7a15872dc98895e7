"""Learned initialiser on the GPU vs the FP64 references (oracle.unet,
oracle.seed, oracle.ptycho), which are pinned on the CPU.

The network computes with bf16 weights and activations and float32
accumulation; the reference is evaluated in FP64 with the same bf16-rounded
weights, so the tolerance covers only the rounding of activations and
gradients to bf16 (8 significant bits): relative L2 error 1e-2 for outputs
and 3e-2 per layer for gradients."""
import numpy as np
import pytest

import oracle
import ptysynth
from oracle import seed as oseed
from oracle import unet
from _cases import c64

pytestmark = pytest.mark.gpu

TOL_Y = 1e-2
TOL_G = 3e-2


def _bf16(a):
    """float32 -> nearest bf16 (ties to even), returned as float32."""
    a = np.ascontiguousarray(a, np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32)


def _as_kernel_sees(flat32):
    """FP64 parameters as the kernels use them: bf16 weights, float32 biases."""
    ps = unet.unflatten(flat32.astype(np.float64))
    for i in range(0, len(ps), 2):
        ps[i] = _bf16(ps[i].astype(np.float32)).astype(np.float64)
    return unet.flatten(ps)


def _rel(a, b):
    a = np.asarray(a, np.float64).ravel()
    b = np.asarray(b, np.float64).ravel()
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _params(seed=11):
    flat = unet.init_params(seed).astype(np.float32)
    # non-zero biases so that they are exercised
    rng = np.random.default_rng(seed)
    ps = unet.unflatten(flat.astype(np.float64))
    for i in range(1, len(ps), 2):
        ps[i] = 0.05 * rng.standard_normal(ps[i].shape)
    return unet.flatten(ps).astype(np.float32)


def _inputs(b, seed=12):
    """Network inputs of simulated patterns (config-4 proportions) at integer positions."""
    wl = ptysynth.workload(4)
    obj = ptysynth.make_object(40 + seed, 128 + 16 * b, 144, wl.sigma_o)
    probe = wl.probe()
    pos = np.array([[16.0 * i, 8.0] for i in range(b)])
    cnt, pr = oracle.simulate(obj, probe, pos, wl.photons)
    return oseed.network_input(cnt, pr), obj, pos


def _net(b, flat):
    from paper_2202_03144_amd.cnn import Net
    net = Net(b, seed=0)
    net.set_params(flat)
    return net


def test_forward_matches_oracle():
    import torch
    b = 3
    flat = _params()
    x, _, _ = _inputs(b)
    net = _net(b, flat)
    xt = torch.from_numpy(x.astype(np.float32)).cuda()
    y = torch.empty((b, 64, 64, 2), dtype=torch.float32, device="cuda")
    net.forward(xt, y)
    ref, _ = unet.forward(_as_kernel_sees(flat), x.astype(np.float32).astype(np.float64))
    err = _rel(y.cpu().numpy(), ref)
    print("forward rel err", err)
    assert err <= TOL_Y
    # params round trip exactly (float32 masters)
    assert np.array_equal(net.params(), flat)
    net.close()


def test_gradient_matches_oracle():
    import torch
    b = 2
    flat = _params(13)
    x, _, _ = _inputs(b, 14)
    rng = np.random.default_rng(15)
    t = (0.3 * rng.standard_normal((b, 64, 64, 2))).astype(np.float32)
    net = _net(b, flat)
    loss, g = net.grad(torch.from_numpy(x.astype(np.float32)).cuda(), torch.from_numpy(t).cuda())
    rl, rg = unet.loss_and_grad(_as_kernel_sees(flat), x.astype(np.float32).astype(np.float64),
                                t.astype(np.float64))
    print("loss", loss, rl)
    assert abs(loss - rl) <= TOL_Y * rl
    off = 0
    for li, (cin, cout, _, _) in enumerate(unet.LAYERS):
        nw = 9 * cin * cout
        for name, sl in (("w", slice(off, off + nw)), ("b", slice(off + nw, off + nw + cout))):
            e = _rel(g[sl], rg[sl])
            print(f"layer {li} {name} rel err {e:.3e}")
            assert e <= TOL_G, (li, name, e)
        off += nw + cout
    assert np.array_equal(net.params(), flat)   # grad leaves the parameters alone
    net.close()


def test_train_steps_reduce_loss():
    import torch
    b = 8
    x, obj, pos = _inputs(b, 16)
    from paper_2202_03144_amd import Plan
    with Plan(128, 1, b, obj.shape) as pl:
        pl.load_positions(pos)
        pl.set_object(c64(obj))
        tg = torch.empty((b, 64, 64, 2), dtype=torch.float32, device="cuda")
        pl.training_targets(tg)
    np.testing.assert_allclose(tg.cpu().numpy(), oseed.targets(obj.astype(np.complex64).astype(np.complex128), pos),
                               rtol=0, atol=2e-5)
    from paper_2202_03144_amd.cnn import Net
    net = Net(b, seed=3)
    xt = torch.from_numpy(x.astype(np.float32)).cuda()
    losses = [net.train_step(xt, tg, 1e-3) for _ in range(30)]
    print("losses", losses[0], losses[-1])
    assert losses[-1] < 0.5 * losses[0]
    net.close()


def test_bad_arguments():
    import torch
    from paper_2202_03144_amd import PtyError
    from paper_2202_03144_amd.cnn import Net
    net = Net(2, seed=0)
    x = torch.zeros((3, 128, 128, 2), dtype=torch.float32, device="cuda")
    y = torch.zeros((3, 64, 64, 2), dtype=torch.float32, device="cuda")
    with pytest.raises(PtyError, match="INVALID"):
        net.forward(x, y)            # batch above max_batch
    with pytest.raises(PtyError, match="INVALID"):
        net.train_step(x[:2], y[:2], -1.0)
    with pytest.raises(ValueError):
        net.set_params(np.zeros(5, np.float32))
    net.close()


def test_poisson_statistics():
    """Device Poisson sampler (inversion below 10, Hormann's PTRS above): mean,
    variance, reproducibility, and a chi-square test of the histogram against
    the exact pmf (scipy.stats.poisson) at every rate, including the ones the
    rejection method covers."""
    import torch
    from scipy import stats
    from paper_2202_03144_amd import Plan
    lam_values = [0.3, 4.0, 9.9, 10.0, 40.0, 200.0, 5e4]
    n = 400_000
    lam = torch.tensor(np.repeat(lam_values, n).astype(np.float32), device="cuda")
    out = torch.empty_like(lam)
    with Plan(32, 1, 1, (33, 33)) as pl:
        pl.poisson(lam, out, seed=99)
        a = out.cpu().numpy().reshape(len(lam_values), n)
        out2 = torch.empty_like(lam)
        pl.poisson(lam, out2, seed=99)
        assert torch.equal(out, out2)              # counter-based: same seed, same draws
    assert np.all(a == np.round(a)) and np.all(a >= 0)
    for i, l in enumerate(lam_values):
        m, v = a[i].mean(), a[i].var()
        se = np.sqrt(l / n)
        assert abs(m - l) <= 5 * se + 0.5 / n, (l, m)
        assert abs(v / l - 1) <= 0.03, (l, v)
        # chi-square against the exact pmf over bins of expected count >= 50
        lo, hi = int(stats.poisson.ppf(1e-6, l)), int(stats.poisson.ppf(1 - 1e-6, l))
        edges = np.arange(lo, hi + 2)
        p = stats.poisson.pmf(edges[:-1], l)
        obs = np.histogram(a[i], bins=edges)[0].astype(np.float64)
        groups, cur_p, cur_o = [], 0.0, 0.0
        for pk, ok in zip(p, obs):
            cur_p, cur_o = cur_p + pk, cur_o + ok
            if cur_p * n >= 50:
                groups.append((cur_p, cur_o))
                cur_p, cur_o = 0.0, 0.0
        if cur_p > 0:
            groups[-1] = (groups[-1][0] + cur_p, groups[-1][1] + cur_o)
        gp = np.array([g[0] for g in groups])
        go = np.array([g[1] for g in groups])
        gp = gp / gp.sum()
        chi2 = float(((go - n * gp) ** 2 / (n * gp)).sum())
        pval = float(stats.chi2.sf(chi2, len(groups) - 1))
        print(f"[poisson] lambda {l}: chi2 {chi2:.1f} on {len(groups) - 1} dof, p {pval:.3g}", flush=True)
        assert pval > 1e-4, (l, chi2, len(groups), pval)


def _spiral_patches(j=60, h=300, w=280):
    obj = ptysynth.make_object(77, h, w, 3.0)
    pos = ptysynth.spiral_positions(j, 6.0, 140.0, 128, ptysynth.stream(77, 3))
    rng = np.random.default_rng(8)
    t = oseed.placements(pos)
    p = np.empty((j, 64, 64, 2), np.float32)
    for i, (ty, tx) in enumerate(t):
        o = obj[ty:ty + 64, tx:tx + 64] * np.exp(1j * rng.uniform(-np.pi, np.pi))
        o = o * (1 + 0.05 * rng.standard_normal(o.shape))        # inconsistent patches
        p[i, ..., 0] = np.abs(o)
        p[i, ..., 1] = np.angle(o)
    return p, pos, obj


def test_stitch_matches_oracle():
    import torch
    from paper_2202_03144_amd import Plan
    p, pos, obj = _spiral_patches()
    h, w = obj.shape
    with Plan(128, 1, len(pos), (h, w)) as pl:
        pl.load_positions(pos)
        out = torch.empty((h, w), dtype=torch.complex64, device="cuda")
        pl.stitch(torch.from_numpy(p).cuda(), out)
        got = out.cpu().numpy()
    ref, _ = oseed.stitch(p.astype(np.float64), pos, h, w)
    err = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
    print("stitch rel err", err)
    assert err <= 1e-5
    # uncovered pixels are exactly 1
    assert np.all(got[ref == 1.0] == 1.0)


def _seed_case(j=10):
    wl = ptysynth.workload(4)
    h = w = 300
    obj = ptysynth.make_object(81, h, w, wl.sigma_o)
    pos = ptysynth.spiral_positions(j, wl.pitch, 150.0, 128, ptysynth.stream(81, 3))
    cnt, probe = oracle.simulate(obj, wl.probe(), pos, wl.photons)
    cnt = ptysynth.poisson_counts(cnt, ptysynth.stream(81, 4))
    return obj, probe, pos, cnt, wl.photons


def test_network_input_matches_oracle():
    """The real-space input from counts and the probe (pty_cnn_input) against
    oracle.seed.network_input (float32 transforms: relative L2 1e-4)."""
    import torch
    from paper_2202_03144_amd.cnn import Net
    obj, probe, pos, cnt, photons = _seed_case(6)
    ref = oseed.network_input(cnt, c64(probe).astype(np.complex128))
    with Net(6, seed=0) as net:
        x = torch.empty((6, 128, 128, 2), dtype=torch.float32, device="cuda")
        net.input(torch.from_numpy(cnt).cuda(), torch.from_numpy(c64(probe)).cuda(), x)
        got = x.cpu().numpy()
    err = _rel(got, ref)
    print("input rel err", err)
    assert err <= 1e-4


@pytest.mark.parametrize("stride", [1, 3])
def test_seed_object_matches_oracle(stride):
    from paper_2202_03144_amd import Plan
    from paper_2202_03144_amd.cnn import Net
    obj, probe, pos, cnt, photons = _seed_case()
    flat = _params(21)
    j = len(pos)
    with Plan(128, 1, j, obj.shape) as pl, Net(4, seed=0) as net:
        net.set_params(flat)
        pl.load_patterns(cnt)
        pl.load_positions(pos)
        pl.set_probe(c64(probe))
        r = pl.seed_object(net, batch=4, stride=stride, fallback=False)   # ragged last batch at stride 1
        assert r["used_fallback"] is False
        got = pl.object()
    sel = np.arange(0, j, stride)
    # the kernels read the counts through A = sqrt(max(d, 0)) in float32
    a32 = np.sqrt(np.maximum(cnt, 0).astype(np.float32)).astype(np.float64)
    x = oseed.network_input(a32[sel] ** 2, c64(probe).astype(np.complex128))
    y, _ = unet.forward(_as_kernel_sees(flat), x)
    ref = oseed.average(y, pos[sel], *obj.shape)
    err = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
    print("seed rel err", err)
    assert err <= TOL_Y


def test_seed_fallback_and_model_error():
    from paper_2202_03144_amd import Plan
    from paper_2202_03144_amd.cnn import Net
    obj, probe, pos, cnt, photons = _seed_case(8)
    j = len(pos)
    with Plan(128, 1, j, obj.shape) as pl, Net(8, seed=5) as net:
        pl.load_patterns(cnt)
        pl.load_positions(pos)
        pl.set_probe(c64(probe))
        pl.seed_object(net, batch=8, fallback=False)
        seed_obj = pl.object()
        e_seed_direct = pl.model_error()
        r = pl.seed_object(net, batch=8, fallback=True)
        got = pl.object()
    amp = oracle.amplitude(cnt.astype(np.float64))
    pr = c64(probe).astype(np.complex128)
    e_flat_ref = oracle.model_error(np.ones(obj.shape), pr, amp, pos)
    e_seed_ref = oracle.model_error(seed_obj.astype(np.complex128), pr, amp, pos)
    assert abs(r["e_flat"] - e_flat_ref) <= 1e-5 * e_flat_ref
    assert abs(r["e_seed"] - e_seed_ref) <= 1e-5 * e_seed_ref
    assert abs(e_seed_direct - e_seed_ref) <= 1e-5 * e_seed_ref
    if r["used_fallback"]:
        assert r["e_seed"] > r["e_flat"] and np.all(got == 1.0)
    else:
        assert r["e_seed"] <= r["e_flat"] and np.array_equal(got, seed_obj)


def test_nrmse_and_history():
    from paper_2202_03144_amd import Plan
    obj, probe, pos, cnt, photons = _seed_case(12)
    j = len(pos)
    pr = c64(probe)
    with Plan(128, 1, j, obj.shape) as pl:
        pl.load_patterns(cnt)
        pl.load_positions(pos)
        pl.set_probe(pr)
        o0 = c64(np.ones(obj.shape) * (1 + 0.1j))
        pl.set_object(o0)
        pl.set_truth(c64(obj), 0.3)
        v0 = pl.nrmse()
        pl.iterate("lsqml", 3, probe_update_start=1 << 30, lsqml_batch=6)
        hist = pl.nrmse_history()
        v3 = pl.nrmse()
        last = pl.object()
        pl.set_truth(c64(obj), 0.0)          # every pixel
        v_all = pl.nrmse()
    mask = oracle.roi_mask(pr.astype(np.complex128), pos, *obj.shape)
    truth = c64(obj).astype(np.complex128)
    assert abs(v0 - oracle.nrmse(o0.astype(np.complex128), truth, mask)) <= 1e-5 * v0
    assert len(hist) == 3 and hist[-1] == v3
    assert abs(v3 - oracle.nrmse(last.astype(np.complex128), truth, mask)) <= 1e-5 * v3
    assert abs(v_all - oracle.nrmse(last.astype(np.complex128), truth, np.ones(obj.shape, bool))) <= 1e-5 * v_all


def test_full_size_inference_and_stitch():
    """The evaluation shape of the learned seed: 4,096 patterns in one batch
    (outputs sampled against the FP64 network) and 4,096 seeded patches
    stitched into a 1200 x 1200 object on the 4,096-point spiral (compared
    whole against the oracle's stitch)."""
    import torch
    from paper_2202_03144_amd import Plan
    from paper_2202_03144_amd.cnn import Net
    wl = ptysynth.workload(4)
    b = wl.j
    flat = _params(31)
    rng = np.random.default_rng(32)
    x = rng.uniform(0.0, 0.6, (b, 128, 128, 2)).astype(np.float32)
    with Net(b, seed=0) as net:
        net.set_params(flat)
        xt = torch.from_numpy(x).cuda()
        y = torch.empty((b, 64, 64, 2), dtype=torch.float32, device="cuda")
        net.forward(xt, y)
        yh = y.cpu().numpy()
    samples = [0, 1777, b - 1]
    ref, _ = unet.forward(_as_kernel_sees(flat), x[samples].astype(np.float64))
    err = _rel(yh[samples], ref)
    print("full-batch forward rel err", err)
    assert err <= TOL_Y
    # full-size stitch of seeded patches cut from an object, with random phase
    # offsets and 5% noise
    pos = wl.positions()
    obj = ptysynth.make_object(78, wl.h, wl.w, wl.sigma_o)
    t = oseed.placements(pos)
    pt = np.empty((b, 64, 64, 2), np.float32)
    for i, (ty, tx) in enumerate(t):
        o = obj[ty:ty + 64, tx:tx + 64] * np.exp(1j * rng.uniform(-np.pi, np.pi))
        o = o * (1 + 0.05 * rng.standard_normal(o.shape))
        pt[i, ..., 0] = np.abs(o)
        pt[i, ..., 1] = np.angle(o)
    with Plan(128, 1, b, (wl.h, wl.w)) as pl:
        pl.load_positions(pos)
        out = torch.empty((wl.h, wl.w), dtype=torch.complex64, device="cuda")
        pl.stitch(torch.from_numpy(pt).cuda(), out)
        got = out.cpu().numpy()
    ref_o, _ = oseed.stitch(pt.astype(np.float64), pos, wl.h, wl.w)
    err_o = float(np.linalg.norm(got - ref_o) / np.linalg.norm(ref_o))
    print("full-size stitch rel err", err_o)
    assert err_o <= 1e-4


def test_stitch_large_object_global_chain():
    """An object whose coarse chain grid does not fit in LDS (2,200 x 2,100:
    275 x 263 cells of 8 bytes) takes the global-memory chain."""
    import torch
    from paper_2202_03144_amd import Plan
    h, w = 2200, 2100
    rng = np.random.default_rng(41)
    pos = np.concatenate([ptysynth.spiral_positions(40, 6.0, 600.0, 128, ptysynth.stream(41, 3)),
                          ptysynth.spiral_positions(40, 6.0, 1500.0, 128, ptysynth.stream(42, 3))])
    obj = ptysynth.make_object(41, h, w, 3.0)
    t = oseed.placements(pos)
    p = np.empty((len(pos), 64, 64, 2), np.float32)
    for i, (ty, tx) in enumerate(t):
        o = obj[ty:ty + 64, tx:tx + 64] * np.exp(1j * rng.uniform(-np.pi, np.pi))
        p[i, ..., 0] = np.abs(o)
        p[i, ..., 1] = np.angle(o)
    with Plan(128, 1, len(pos), (h, w)) as pl:
        pl.load_positions(pos)
        out = torch.empty((h, w), dtype=torch.complex64, device="cuda")
        pl.stitch(torch.from_numpy(p).cuda(), out)
        got = out.cpu().numpy()
    ref, _ = oseed.stitch(p.astype(np.float64), pos, h, w)
    err = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
    print("global-chain stitch rel err", err)
    assert err <= 1e-5


def test_trained_network_seeds_better_than_the_flat_start():
    """What the trained network gains: trained on the GPU (forward model,
    Poisson draws, real-space inputs and targets all made by the library's
    kernels) for 300 Adam steps of 128 patterns from eight training objects,
    its stitched seed of a held-out object (the learned-initialiser workload's
    probe and dose, a 1,000-point spiral on a 600 x 600 object) is at most
    0.75 of the flat start's NRMSE (measured: see the printed line)."""
    import torch
    from paper_2202_03144_amd import Plan
    from paper_2202_03144_amd.cnn import Net
    from paper_2202_03144_amd.learned import train
    wl = ptysynth.workload(4)
    objs = [torch.from_numpy(ptysynth.make_object(1000 + i, 512, 512, wl.sigma_o).astype(np.complex64)).cuda()
            for i in range(8)]
    side = ptysynth.spiral_object_side(1000, wl.pitch, 128, 3.0)
    obj = ptysynth.make_object(9, side, side, wl.sigma_o).astype(np.complex64)
    pos = ptysynth.spiral_positions(1000, wl.pitch, side / 2.0, 128, ptysynth.stream(9, 3))
    with Net(256, seed=7) as net:
        losses = train(net, objs, wl.probe().astype(np.complex64), wl.photons, 300, 128, lr=1e-3,
                       lr_final=1e-4, seed=3)
        with Plan(128, 1, len(pos), (side, side)) as pl:
            lam = torch.empty((len(pos), 128, 128), dtype=torch.float32, device="cuda")
            cnt = torch.empty_like(lam)
            pl.load_positions(pos)
            pl.set_object(obj)
            pl.set_probe(wl.probe().astype(np.complex64))
            pl.simulate(wl.photons, out=lam)
            pl.poisson(lam, cnt, seed=9)
            pl.load_patterns(cnt)
            pl.set_object(np.ones((side, side), np.complex64))
            pl.set_truth(obj, 0.3)
            flat = pl.nrmse()
            r = pl.seed_object(net, batch=256, stride=1, fallback=False)
            seeded = pl.nrmse()
    print(f"[learned] loss {np.mean(losses[:10]):.5f} -> {np.mean(losses[-10:]):.5f}; "
          f"seed NRMSE {seeded:.4f} vs flat {flat:.4f} ({seeded / flat:.2f}x)", flush=True)
    assert seeded <= 0.75 * flat
