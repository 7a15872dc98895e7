#!/usr/bin/env python3
"""Throughput of the ptychographic reconstruction hot path on one MI355X.

Workload: 256 x 256 probe window, 3 incoherent modes, 2,500-point Fermat
spiral with +-0.5 px jitter (~70% overlap), 1700 x 1700 object, Poisson noise
at 1e8 photons per pattern; synthetic, seeded.  One step = one DM iteration
plus one LSQML iteration (5 groups of 500) over all 2,500 patterns, probe
updates on.  Value = pattern-iterations per second (2 x 2,500 per step).

Prints one JSON line.  --gpus N with N > 1 is refused: this build runs on one
GPU.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "pattern-iterations/s (256², 3 modes)"
PEAK_HBM_GBS = 8000.0        # MI355X HBM3E
PEAK_FP32_TFLOPS = 157.3     # MI355X FP32 vector (256 CUs x 2.4 GHz x 256 flop/clk, packed FMA)
PEAK_LDS_TBS = 78.6          # MI355X LDS (256 CUs x 2.4 GHz x 128 B/clk)


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def make_inputs(torch, photons=None):
    """Inputs of the 256 x 256, 3-mode, 2,500-position workload on the GPU: counts via the library's forward model + a seeded Poisson draw
    (``photons`` per pattern on average: the workload's own dose unless given)."""
    import dataclasses
    import ptysynth
    from paper_2202_03144_amd import Plan

    wl = ptysynth.workload(2)
    if photons is not None:
        wl = dataclasses.replace(wl, photons=float(photons))
    obj_true = wl.obj().astype(np.complex64)
    probe = wl.probe().astype(np.complex64)
    pos = wl.positions()
    expected = torch.empty((wl.j, wl.n, wl.n), dtype=torch.float32, device="cuda")
    with Plan(wl.n, wl.k, wl.j, (wl.h, wl.w)) as sim:
        sim.load_positions(pos)
        sim.set_object(obj_true)
        sim.set_probe(probe)
        sim.simulate(wl.photons, out=expected)
        probe = sim.probe()
    counts = ptysynth.poisson_counts(expected.cpu().numpy(), wl.noise_rng())
    del expected
    return wl, obj_true, probe, pos, torch.from_numpy(counts).cuda()


# Algorithmic HBM bytes per pattern of the Fourier-pass kernels at N, K (complex
# float32 = 8 B): the traffic the method's data dependencies force.  The chunk
# scratch between the passes and the per-pattern contribution planes are
# intermediates of this implementation and are not counted.
def algorithmic_bytes_per_pattern(plan, fam, n, k):
    nn = n * n
    table = {
        ("dm", "rows_fwd"): 8 * k * nn,      # exit waves psi read
        ("dm", "cols"): 4 * nn,              # measured moduli A read
        ("dm", "rows_inv"): 8 * k * nn,      # exit waves psi written
        ("lsqml", "rows_fwd"): 0,            # gathers only (object and probe stay in cache)
        ("lsqml", "cols"): 4 * nn,           # A read
        ("lsqml", "rows_inv"): 8 * k * nn,   # chi written
    }
    return table.get((plan, fam))


# Whole-iteration algorithmic bytes: DM reads psi twice (probe update, Fourier
# pass), writes it once and reads A; LSQML writes chi, reads it in the step-length
# sums, reads A; both add the object planes (DM ~40 B/px once, LSQML ~64 B/px per group).
def iteration_bytes(plan, n, k, j, h, w, groups):
    nn = n * n
    if plan == "dm":
        return j * nn * (4 + 24 * k) + 40 * h * w
    return j * nn * (4 + 16 * k) + 64 * h * w * groups


# HBM bytes measured by rocprofv3 FETCH_SIZE / WRITE_SIZE for full 64-pattern
# launches (profiles/dm_fourier_256x3_hbm_counters.md): read = 2.0 x FETCH_SIZE,
# written = 1.0 x WRITE_SIZE (factors from a plain copy of known size).  Valid
# only while the kernel sources hash to COUNTER_SRC_HASH.
COUNTER_SRC_HASH = "d7d195c9f63297d9"
COUNTER_SRCS = ["pty_fourier.hip", "pty_fft.hpp", "pty_geom.hpp", "pty_common.hpp"]
MEASURED_KIB = {  # (plan, family): (FETCH_SIZE KiB, WRITE_SIZE KiB, patterns per launch)
    ("dm", "rows_fwd"): (64185.7, 98304.0, 64),
    ("dm", "cols"): (65853.6, 98336.0, 64),
    ("dm", "rows_inv"): (66791.8, 131072.0, 64),
    ("lsqml", "rows_fwd"): (14428.8, 98304.0, 64),
    ("lsqml", "cols"): (65853.6, 98336.0, 64),
    ("lsqml", "rows_inv"): (50008.3, 131072.0, 64),
}


def kernel_src_hash():
    """Hash of what the Fourier kernels are compiled from: their sources and
    the part of the launcher header that defines their arguments."""
    import hashlib
    import re
    h = hashlib.sha256()
    for f in COUNTER_SRCS:
        with open(os.path.join(ROOT, "paper_2202_03144_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    with open(os.path.join(ROOT, "paper_2202_03144_amd", "csrc", "pty_kernels.hpp")) as fh:
        hdr = fh.read()
    h.update(hdr[:hdr.index("void launch_rows_fwd")].encode())
    return h.hexdigest()[:16]


# Algorithmic flops per pattern of a Fourier-pass kernel: 5 L log2 L per
# length-L line transform (N lines of length N per mode and direction, i.e.
# 5 N^2 log2 N per mode and one-dimensional pass), plus the pointwise work per
# pixel: bilinear gather 14 and exit wave 6 per mode (DM reflection +4 per
# mode); projection 4 per mode for the intensity, 8 for modulus, ratio and
# error, 2 per mode to scale; DM update 16 per mode (new exit wave and its
# contribution), stored chi's contribution 8 per mode.
def flops_per_pattern(plan, fam, n, k):
    nn = n * n
    line = 5.0 * nn * math.log2(n)
    if fam == "rows_fwd":
        return k * line + nn * (14 + 6 * k + (4 * k if plan == "dm" else 0))
    if fam == "cols":
        return 2 * k * line + nn * (6 * k + 8)
    return k * line + nn * ((14 + 16 * k) if plan == "dm" else 8 * k)


# Algorithmic LDS bytes per pattern: each line transform writes and reads its N
# values once through LDS for the exchange (16 N bytes per line).
def lds_bytes_per_pattern(fam, n, k):
    return (2 if fam == "cols" else 1) * k * 16 * n * n


KERNEL_NAMES = {
    ("dm", "rows_fwd"): "k_rows_fwd<256,3,DmReflect>",
    ("dm", "cols"): "k_cols<256,3,Project>",
    ("dm", "rows_inv"): "k_rows_inv<256,3,DmUpdate>",
    ("lsqml", "rows_fwd"): "k_rows_fwd<256,3,Plain>",
    ("lsqml", "cols"): "k_cols<256,3,Project>",
    ("lsqml", "rows_inv"): "k_rows_inv<256,3,StoreChi>",
}


def cpu_baseline(n_sample: int):
    """The FP64 oracle on a bounded sample of the same workload: one DM and one
    LSQML iteration over the first n_sample spiral positions."""
    import oracle
    import ptysynth

    wl = ptysynth.workload(2)
    obj_true = wl.obj()
    pos = wl.positions()[:n_sample]
    expected, probe = oracle.simulate(obj_true, wl.probe(), pos, wl.photons)
    counts = ptysynth.poisson_counts(expected, wl.noise_rng())
    amp = oracle.amplitude(counts.astype(np.float64))
    o0 = np.ones(obj_true.shape, np.complex128)
    t0 = time.perf_counter()
    psi = oracle.dm_init(o0, probe, pos)
    oracle.dm(o0, probe, psi, amp, pos, 1, start=0)
    t1 = time.perf_counter()
    oracle.lsqml(o0, probe, amp, pos, 1, start=0, batch=max(1, n_sample // 5))
    t2 = time.perf_counter()
    cores = len(os.sched_getaffinity(0))
    return {
        "value": 2 * n_sample / (t2 - t0),
        "unit": "pattern-iterations/s",
        "cores": cores,
        "kind": "oracle",
        "sample": (f"first {n_sample} of the 2,500 spiral positions (same object, probe and photon "
                   f"budget), one DM + one LSQML iteration in float64 NumPy/SciPy "
                   f"(scipy.fft workers={os.cpu_count()}); DM {t1 - t0:.1f} s, LSQML {t2 - t1:.1f} s"),
    }


def learned_leg(args, torch) -> dict:
    """Time to NRMSE <= 1e-2 with the learned seed vs the flat start (LSQML,
    fixed true probe) on the 128 x 128, 4,096-position spiral workload."""
    import ptysynth
    from paper_2202_03144_amd import Plan
    from paper_2202_03144_amd.cnn import Net
    from paper_2202_03144_amd.learned import time_to_nrmse, train

    wl = ptysynth.workload(4)
    stream = torch.cuda.Stream()
    torch.cuda.set_stream(stream)
    # held-out evaluation data: counts from the library's forward model and Poisson sampler
    obj_true = wl.obj().astype(np.complex64)
    pos = wl.positions()
    lam = torch.empty((wl.j, wl.n, wl.n), dtype=torch.float32, device="cuda")
    counts = torch.empty_like(lam)
    with Plan(wl.n, wl.k, wl.j, (wl.h, wl.w), stream=stream) as sim:
        sim.load_positions(pos)
        sim.set_object(obj_true)
        sim.set_probe(wl.probe().astype(np.complex64))
        sim.simulate(wl.photons, out=lam)
        sim.poisson(lam, counts, seed=4)
        probe = sim.probe()
    del lam
    # training objects: same generator and statistics, other seeds
    side = 1024
    objs = [torch.from_numpy(ptysynth.make_object(1000 + i, side, side, wl.sigma_o).astype(np.complex64)).cuda()
            for i in range(args.train_objects)]
    net = Net(args.infer_batch, seed=7, stream=stream)
    log(f"training: {args.train_steps} steps x {args.train_batch} patterns on {len(objs)} objects")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    losses = train(net, objs, wl.probe().astype(np.complex64), wl.photons, args.train_steps, args.train_batch,
                   lr=1e-3, lr_final=1e-4, seed=11, log_every=max(1, args.train_steps // 10), log=log)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    del objs
    # one full-batch inference, timed alone: the network's MFMA roofline
    xin = torch.rand((args.infer_batch, 128, 128, 2), device="cuda") * 0.6
    yout = torch.empty((args.infer_batch, 64, 64, 2), dtype=torch.float32, device="cuda")
    net.forward(xin, yout)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    for _ in range(3):
        net.forward(xin, yout)
    ev1.record(stream)
    stream.synchronize()
    infer_ms = ev0.elapsed_time(ev1) / 3
    infer_flop = 0.9576e9 * args.infer_batch       # 2 x MACs of the ten convolutions per pattern
    del xin, yout

    def arm(learned: bool, max_iter: int, stride: int = 1):
        pl = Plan(wl.n, wl.k, wl.j, (wl.h, wl.w), stream=stream)
        pl.load_patterns(counts)
        pl.load_positions(pos)
        pl.set_probe(probe)
        pl.set_object(np.ones((wl.h, wl.w), np.complex64))
        pl.set_truth(obj_true, 0.3)
        seed_ms, info, nrmse0 = 0.0, {}, pl.nrmse()
        if learned:
            pl.seed_object(net, batch=args.infer_batch, stride=stride)   # warm: allocations
            torch.cuda.synchronize()
            t = time.perf_counter()
            info = pl.seed_object(net, batch=args.infer_batch, stride=stride)
            torch.cuda.synchronize()
            seed_ms = (time.perf_counter() - t) * 1e3
            nrmse0 = pl.nrmse()
        hist, ms, hit = time_to_nrmse(pl, args.nrmse_target, max_iter, stream,
                                      probe_update_start=1 << 30, lsqml_batch=args.learned_lsqml_batch)
        pl.close()
        reach = {}
        for thr in (3e-2, 2e-2, 1.2e-2, args.nrmse_target):
            k = np.nonzero(hist <= thr)[0]
            reach[f"{thr:g}"] = None if not k.size else {"iterations": int(k[0]) + 1,
                                                          "ms": round(seed_ms + float(ms[k[0]]), 2)}
        res = {"nrmse_start": round(nrmse0, 5), "seed_ms": round(seed_ms, 2), "time_to": reach,
               "iterations_to_target": None if hit is None else hit + 1,
               "ms_to_target": None if hit is None else round(seed_ms + float(ms[hit]), 2),
               "lsqml_ms_per_iter": round(float(ms[-1]) / len(ms), 3),
               "nrmse_last": round(float(hist[-1]), 5), "iterations_run": len(ms),
               "nrmse_at": {str(i): round(float(hist[i - 1]), 5) for i in (1, 2, 5, 10, 20, 50, 100, 200, 400)
                            if i <= len(hist)}}
        if learned:
            res.update({"used_fallback": info["used_fallback"], "e_seed": round(info["e_seed"], 5),
                        "e_flat": round(info["e_flat"], 5)})
        return res

    log("plain arm")
    plain = arm(False, args.plain_iters)
    log(f"plain: {plain}")
    arms = {}
    for stride in sorted({int(v) for v in args.seed_strides.split(",")}):
        log(f"learned arm, every {stride}. pattern seeded")
        arms[stride] = arm(True, args.learned_iters, stride)
        arms[stride]["seed_stride"] = stride
        log(f"learned (stride {stride}): {arms[stride]}")
    net.close()
    best = min(arms, key=lambda k: arms[k]["ms_to_target"] or float("inf"))
    learned = arms[best]
    speed = None
    if learned["ms_to_target"] and plain["ms_to_target"]:
        speed = round(plain["ms_to_target"] / learned["ms_to_target"], 3)
    return {
        "metric": f"time to NRMSE {args.nrmse_target:g} (ms)",
        "value": learned["ms_to_target"], "unit": "ms", "n_gpus": 1, "higher_is_better": False,
        "vs_baseline": None, "dtype": "bf16 network, f32 reconstruction", "data": "synthetic",
        "config": {"workload": "128x128 probe (D 48), 1 mode fixed, 4,096-point Fermat spiral (c 8), "
                               f"1200x1200 object, Poisson 1e8 photons; LSQML groups of {args.learned_lsqml_batch}",
                   "n": wl.n, "positions": wl.j, "object": [wl.h, wl.w]},
        "learned": learned, "learned_arms": {str(k): v for k, v in arms.items()}, "plain": plain,
        "plain_over_learned": speed,
        "roofline": {"bound": "mfma", "kernel": f"network forward, batch {args.infer_batch}",
                     "achieved": round(infer_flop / (infer_ms * 1e-3) / 1e12, 1), "peak": 2500.0,
                     "unit": "TFLOP/s", "frac": round(infer_flop / (infer_ms * 1e-3) / 1e12 / 2500.0, 4),
                     "traffic": None, "ms": round(infer_ms, 3)},
        "training": {"patterns": args.train_steps * args.train_batch, "steps": args.train_steps,
                     "batch": args.train_batch, "seconds": round(train_s, 2),
                     "loss_first": round(float(np.mean(losses[:10])), 5),
                     "loss_last": round(float(np.mean(losses[-10:])), 5)},
    }


def batch_leg(args, torch) -> dict:
    """The batched-datasets workload: 64 LSQML reconstructions drawn with
    default_rng([5, 5]) -- N uniform in {64, 128, 256}, K uniform in {1, 2, 3},
    J log-uniform in [200, 10,000], photons log-uniform in [1e6, 1e9] -- with
    D = 84 N / 256, spiral pitch 14 N / 256, sigma_o = max(2, 4 N / 256), an
    8-pixel margin and Poisson counts (dataset i's streams default_rng([5, i,
    stream])).  Each dataset alone (eager, timed on its own: per-dataset
    throughput and roofline fraction), then all together with per-dataset
    streams and a captured graph per iteration, before and after autotuning
    (chunk and probe-sum slices)."""
    import ptysynth
    from paper_2202_03144_amd import Batch, Plan

    rng = np.random.default_rng([5, 5])
    specs = []
    for i in range(args.datasets):
        n = int(rng.choice([64, 128, 256]))
        k = int(rng.integers(1, 4))
        j = int(round(math.exp(rng.uniform(math.log(200), math.log(10000)))))
        ph = float(math.exp(rng.uniform(math.log(1e6), math.log(1e9))))
        specs.append((n, k, j, ph))
    log(f"building {len(specs)} datasets")
    datasets = []
    for i, (n, k, j, ph) in enumerate(specs):
        c = 14.0 * n / 256.0
        side = ptysynth.spiral_object_side(j, c, n, 8.0)
        obj = ptysynth.make_object(5, side, side, max(2.0, 4.0 * n / 256.0), i).astype(np.complex64)
        probe = ptysynth.make_probe(5, n, k, 84.0 * n / 256.0, max(1.0, 3.0 * n / 256),
                                    max(2.0, 12.0 * n / 256), 5.0, i).astype(np.complex64)
        pos = ptysynth.spiral_positions(j, c, side / 2.0, n, ptysynth.stream(5, 3, i))
        lam = torch.empty((j, n, n), dtype=torch.float32, device="cuda")
        cnt = torch.empty_like(lam)
        with Plan(n, k, j, (side, side)) as sim:
            sim.load_positions(pos)
            sim.set_object(obj)
            sim.set_probe(probe)
            sim.simulate(ph, out=lam)
            sim.poisson(lam, cnt, seed=(5 << 32) + (i << 8) + 4)
            probe = sim.probe()
        del lam
        datasets.append(dict(n=n, k=k, j=j, photons=ph, shape=(side, side), counts=cnt, pos=pos, probe=probe))
    batch = 512
    params = dict(probe_update_start=0, lsqml_batch=batch)
    iters = args.batch_iters

    def make_plan(d, stream):
        pl = Plan(d["n"], d["k"], d["j"], d["shape"], stream=stream)
        pl.load_patterns(d["counts"])
        pl.load_positions(d["pos"])
        pl.set_object(np.ones(d["shape"], np.complex64))
        pl.set_probe(d["probe"])
        return pl

    def roof_bytes(d):
        g = -(-d["j"] // batch)
        return d["j"] * d["n"] ** 2 * (4 + 16 * d["k"]) + 64 * d["shape"][0] * d["shape"][1] * g

    log(f"each dataset alone, {iters} iterations")
    per = []
    t_seq = 0.0
    for i, d in enumerate(datasets):
        pl = make_plan(d, None)
        pl.iterate("lsqml", 1, **params)
        pl.sync()
        t = time.perf_counter()
        pl.iterate("lsqml", iters, **params)
        pl.sync()
        dt = time.perf_counter() - t
        pl.close()
        t_seq += dt
        ms = dt * 1e3 / iters
        per.append({"n": d["n"], "k": d["k"], "j": d["j"], "photons": round(d["photons"]),
                    "ms_per_iter": round(ms, 3), "pit_per_s": round(d["j"] / (ms / 1e3), 1),
                    "roofline_frac": round(roof_bytes(d) / (ms / 1e3) / (PEAK_HBM_GBS * 1e9), 4)})
    pit = sum(d["j"] for d in datasets) * iters

    def run_batched(plans, tune_cache=None):
        with Batch(plans) as b:
            if tune_cache:
                t0 = time.perf_counter()
                b.autotune("lsqml", tune_cache, **params)
                tune_s = time.perf_counter() - t0
            else:
                tune_s = 0.0
            b.iterate("lsqml", 1, graph=True, **params)   # warm-up (buffers, graph capture)
            b.sync()
            t = time.perf_counter()
            b.iterate("lsqml", iters, graph=True, **params)
            b.sync()
            return time.perf_counter() - t, tune_s

    import tempfile
    cache = os.path.join(tempfile.mkdtemp(prefix="ptymi_tune_"), "tune.json")
    log("all datasets together, graph replay")
    plans = [make_plan(d, torch.cuda.Stream()) for d in datasets]
    t_b, _ = run_batched(plans)
    for pl in plans:
        pl.close()
    log("all datasets together, autotuned")
    plans = [make_plan(d, torch.cuda.Stream()) for d in datasets]
    t_bt, tune_s = run_batched(plans, cache)
    tuned = [pl.tuning() for pl in plans]
    for pl in plans:
        pl.close()
    for row, (ch, sl) in zip(per, tuned):
        row["tuned_chunk"], row["tuned_probe_slice"] = ch, sl
    # aggregates: per (N, K), and per decile of J over the 64 datasets
    def agg(rows):
        t = sum(r["j"] * iters / r["pit_per_s"] for r in rows)
        b = sum(roof_bytes(d) * iters for d, r in zip(datasets, per) if r in rows)
        return {"datasets": len(rows), "pit_per_s": round(sum(r["j"] * iters for r in rows) / t, 1),
                "roofline_frac": round(b / t / (PEAK_HBM_GBS * 1e9), 4)}
    by_nk = {f"n{n}_k{k}": agg([r for r in per if r["n"] == n and r["k"] == k])
             for n in (64, 128, 256) for k in (1, 2, 3) if any(r["n"] == n and r["k"] == k for r in per)}
    js = np.array([r["j"] for r in per])
    edges = np.quantile(js, np.linspace(0, 1, 11))
    by_decile = {}
    for q in range(10):
        lo, hi = edges[q], edges[q + 1]
        rows = [r for r in per if (lo <= r["j"] < hi) or (q == 9 and r["j"] == hi)]
        if rows:
            by_decile[f"d{q + 1} J {int(lo)}-{int(hi)}"] = agg(rows)
    by_nk_decile = {}
    for n in (64, 128, 256):
        for k in (1, 2, 3):
            for q in range(10):
                lo, hi = edges[q], edges[q + 1]
                rows = [r for r in per if r["n"] == n and r["k"] == k and ((lo <= r["j"] < hi) or (q == 9 and r["j"] == hi))]
                if rows:
                    by_nk_decile[f"n{n}_k{k}_d{q + 1}"] = agg(rows)
    total_bytes = sum(roof_bytes(d) for d in datasets) * iters
    out = {
        "sequential_pit_per_s": round(pit / t_seq, 1),
        "batched_graph_pit_per_s": round(pit / t_b, 1),
        "batched_graph_tuned_pit_per_s": round(pit / t_bt, 1),
        "batched_over_sequential": round(t_seq / t_b, 3),
        "batched_tuned_roofline_frac": round(total_bytes / t_bt / (PEAK_HBM_GBS * 1e9), 4),
        "autotune_s": round(tune_s, 2),
    }
    log(f"{out}")
    return {
        "metric": "pattern-iterations/s (64 uneven LSQML datasets)",
        "value": out["batched_graph_tuned_pit_per_s"], "unit": "pattern-iterations/s", "n_gpus": 1,
        "higher_is_better": True, "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"{len(datasets)} Fermat-spiral datasets drawn with default_rng([5, 5]): N in "
                               "{64, 128, 256}, K in {1, 2, 3}, J log-uniform 200-10,000, photons log-uniform "
                               f"1e6-1e9, Poisson counts; LSQML groups of {batch}, probe updates on; "
                               f"{iters} timed iterations each",
                   "pattern_iterations": pit},
        **out,
        "per_n_k": by_nk, "per_j_decile": by_decile, "per_n_k_j_decile": by_nk_decile, "per_dataset": per,
    }


def tiny_leg(args, torch) -> dict:
    """64 x 64 probe, 1 mode, 10 x 10 raster (100 positions), 160 x 160 object,
    Poisson 1e6: ePIE, DM and LSQML, 50 iterations each (probe updates from
    10), eager and (DM, LSQML) graph-replayed; the oracle timed beside."""
    import ptysynth
    import oracle
    from paper_2202_03144_amd import Plan

    wl = ptysynth.workload(1)
    obj = wl.obj()
    pos = wl.positions()
    expected, probe = oracle.simulate(obj, wl.probe(), pos, wl.photons)
    counts = ptysynth.poisson_counts(expected, wl.noise_rng())
    probe = probe.astype(np.complex64)
    iters = 50
    res = {}

    def run(algo, graph):
        pl = Plan(wl.n, wl.k, wl.j, (wl.h, wl.w))
        pl.load_patterns(counts)
        pl.load_positions(pos)
        pl.set_object(np.ones((wl.h, wl.w), np.complex64))
        pl.set_probe(probe)
        pl.iterate(algo, 1, graph=graph, probe_update_start=10)    # warm-up (buffers, capture)
        pl.sync()
        pl.set_object(np.ones((wl.h, wl.w), np.complex64))
        pl.set_probe(probe)
        t = time.perf_counter()
        pl.iterate(algo, iters, graph=graph, probe_update_start=10)
        pl.sync()
        dt = time.perf_counter() - t
        pl.close()
        return dt

    for algo in ("epie", "dm", "lsqml"):
        dt = run(algo, False)
        res[algo] = {"eager_pit_per_s": round(wl.j * iters / dt, 1), "eager_us_per_iter": round(dt / iters * 1e6, 1)}
        if algo != "epie":
            dg = run(algo, True)
            res[algo].update({"graph_pit_per_s": round(wl.j * iters / dg, 1),
                              "graph_us_per_iter": round(dg / iters * 1e6, 1)})
        log(f"{algo}: {res[algo]}")
    # the oracle, same inputs, 50 iterations each
    amp = oracle.amplitude(counts.astype(np.float64))
    o0 = np.ones((wl.h, wl.w), np.complex128)
    p0 = probe.astype(np.complex128)
    cpu = {}
    t = time.perf_counter()
    oracle.epie(o0, p0, amp, pos, iters, start=10)
    cpu["epie_s"] = round(time.perf_counter() - t, 2)
    t = time.perf_counter()
    oracle.dm(o0, p0, oracle.dm_init(o0, p0, pos), amp, pos, iters, start=10)
    cpu["dm_s"] = round(time.perf_counter() - t, 2)
    t = time.perf_counter()
    oracle.lsqml(o0, p0, amp, pos, iters, start=10)
    cpu["lsqml_s"] = round(time.perf_counter() - t, 2)
    cores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    return {
        "metric": "pattern-iterations/s (64², 1 mode, 100 positions)",
        "value": res["dm"]["graph_pit_per_s"], "unit": "pattern-iterations/s", "n_gpus": 1,
        "higher_is_better": True, "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "64x64 probe, 1 mode, 10x10 raster (8 px step), 160x160 object, Poisson 1e6; "
                               "50 iterations, probe updates from 10", "n": 64, "positions": 100},
        "algorithms": res,
        "cpu_baseline": {"kind": "oracle", "cores": cores, "seconds_for_50_iterations": cpu,
                         "epie_pit_per_s": round(wl.j * iters / cpu["epie_s"], 1),
                         "dm_pit_per_s": round(wl.j * iters / cpu["dm_s"], 1),
                         "lsqml_pit_per_s": round(wl.j * iters / cpu["lsqml_s"], 1)},
    }


def adjoint_leg(args, torch) -> dict:
    """Poisson-NLL forward and backward (object, probe and position
    gradients) on the 128 x 128, 4-mode, 1,000-position workload."""
    import ptysynth
    import oracle
    from paper_2202_03144_amd import Plan

    wl = ptysynth.workload(3)
    stream = torch.cuda.Stream()
    torch.cuda.set_stream(stream)
    obj_true = wl.obj().astype(np.complex64)
    pos = wl.positions()
    lam = torch.empty((wl.j, wl.n, wl.n), dtype=torch.float32, device="cuda")
    counts = torch.empty_like(lam)
    with Plan(wl.n, wl.k, wl.j, (wl.h, wl.w), stream=stream) as sim:
        sim.load_positions(pos)
        sim.set_object(obj_true)
        sim.set_probe(wl.probe().astype(np.complex64))
        sim.simulate(wl.photons, out=lam)
        sim.poisson(lam, counts, seed=3)
        probe = sim.probe()
    del lam
    rng = np.random.default_rng(3)
    o = torch.from_numpy((obj_true * (1 + 0.02 * rng.standard_normal(obj_true.shape))).astype(np.complex64)).cuda()
    p = torch.from_numpy(probe).cuda()
    g_o, g_p = torch.empty_like(o), torch.empty_like(p)
    g_r = torch.empty((wl.j, 2), dtype=torch.float32, device="cuda")
    pl = Plan(wl.n, wl.k, wl.j, (wl.h, wl.w), stream=stream)
    pl.load_patterns(counts)
    pl.load_positions(pos)
    for _ in range(2):
        pl.nll_forward(o, p)
        pl.nll_backward(o, p, 1.0, g_o, g_p, g_r)
    reps = 10
    e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(reps):
        pl.nll_forward(o, p)
    e1.record(stream)
    for _ in range(reps):
        pl.nll_backward(o, p, 1.0, g_o, g_p, g_r)
    e2.record(stream)
    stream.synchronize()
    ms_f = e0.elapsed_time(e1) / reps
    ms_b = e1.elapsed_time(e2) / reps
    pl.close()
    n2 = wl.n * wl.n
    fft_flop = 5.0 * n2 * np.log2(n2)               # one 2-D transform
    flop_f = wl.j * wl.k * fft_flop                   # K forward transforms per pattern
    flop_b = wl.j * 2 * wl.k * fft_flop               # recomputed forward + inverse
    achieved = flop_b / (ms_b * 1e-3) / 1e12
    # the oracle on a bounded sample of the same workload
    ns = args.adjoint_cpu_sample
    cnt_h = counts[:ns].cpu().numpy().astype(np.float64)
    t = time.perf_counter()
    oracle.nll_grad(o.cpu().numpy().astype(np.complex128), probe.astype(np.complex128), pos[:ns], cnt_h)
    cpu_s = time.perf_counter() - t
    cores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    return {
        "metric": "Poisson-NLL forward+backward (µs per pattern)",
        "value": round((ms_f + ms_b) * 1e3 / wl.j, 3), "unit": "us/pattern", "n_gpus": 1,
        "higher_is_better": False, "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "128x128 probe, 4 modes, 1,000 jittered spiral positions (c 7), 600x600 object, "
                               "Poisson 1e6; exit waves recomputed in the backward pass",
                   "n": wl.n, "modes": wl.k, "positions": wl.j},
        "forward_ms": round(ms_f, 4), "backward_ms": round(ms_b, 4),
        "roofline": {"bound": "alu", "kernel": "backward (all launches)", "achieved": round(achieved, 2),
                     "peak": 157.3, "unit": "TFLOP/s", "frac": round(achieved / 157.3, 4), "traffic": None,
                     "algorithmic_flop_per_pattern": 2 * wl.k * fft_flop},
        "cpu_baseline": {"value": round((cpu_s / ns) * 1e6, 1), "unit": "us/pattern", "cores": cores,
                         "kind": "oracle", "sample": f"first {ns} of the 1,000 positions, forward + gradients in FP64"},
    }




def listing1_leg(args, torch) -> dict:
    """The paper's script example: the sim512 command string (512 x 512 window,
    30 x 30 raster of 50 nm steps, 110 nm beam, known probe), simulated data,
    ePIE driven one step call at a time as in the script; DM and LSQML on the
    same data for comparison.  The oracle times one ePIE pass over a sample."""
    import oracle
    from paper_2202_03144_amd import command

    LISTING1 = command.make_command(command.SIM512)
    res = {}
    for algo in args.listing1_algos.split(","):
        pl, g, obj, probe = command.simulated_plan(LISTING1)
        pl.set_truth(obj, 0.3)
        prm = command.iteration_params(g)
        pl.iterate(algo, 0, **prm)
        pl.sync()
        iters = args.listing1_iters or g.iterations
        t = time.perf_counter()
        for _ in range(iters):
            pl.iterate(algo, 1, **prm)     # one step call per iteration, as in the script
        pl.sync()
        s = time.perf_counter() - t
        e, h = pl.errors(), pl.nrmse_history()
        pl.close()
        res[algo] = {"ms_per_iter": round(s * 1e3 / iters, 3),
                     "pattern_it_per_s": round(len(g.positions) * iters / s, 1),
                     "E_first": float(e[0]), "E_last": float(e[-1]),
                     "nrmse_first": round(float(h[0]), 5), "nrmse_last": round(float(h[-1]), 5)}
        log(f"{algo}: {res[algo]}")
    # the oracle: one ePIE pass over the first positions of the same data
    g = command.geometry(command.parse(LISTING1))
    obj = command.synthetic_object(g.obj_shape, 0)
    ns = args.listing1_cpu_sample
    pos = g.positions[:ns]
    cnt, pr = oracle.simulate(obj.astype(np.complex128), command.synthetic_probe(g.n, g.modes, g.beam_px), pos, 1e6)
    amp = oracle.amplitude(cnt)
    t = time.perf_counter()
    oracle.epie(np.ones(g.obj_shape, complex), pr, amp, pos, 1, start=1 << 30)
    cpu_s = time.perf_counter() - t
    cores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    return {"metric": "pattern-iterations/s (the paper's sim512 script, ePIE)",
            "value": res.get("epie", {}).get("pattern_it_per_s"), "unit": "pattern-iterations/s", "n_gpus": 1,
            "higher_is_better": True, "vs_baseline": None, "dtype": "f32", "data": "synthetic",
            "config": {"workload": "512x512 window, 1 mode, 30x30 raster (50 nm = 17.76 px steps), 110 nm "
                                   "(39.1 px) beam, 1029x1029 object, noise-free simulation at 1e6 photons; "
                                   "known probe; 100 iterations, one step call each (host-timed)",
                       "command": LISTING1},
            "runs": res,
            "cpu_baseline": {"value": round(ns / cpu_s, 2), "unit": "pattern-iterations/s", "cores": cores,
                             "kind": "oracle", "sample": f"one ePIE pass over the first {ns} of the 900 positions"}}


def blind_leg(args, torch) -> dict:
    """ePIE, LSQML and DM on the 64 x 64, one-mode, 10 x 10 raster workload
    started from an aperture guess (pty_guess_probe) instead of the probe,
    probe updates from the first iteration; NRMSE and E along the way."""
    import ptysynth
    import oracle
    from paper_2202_03144_amd import Plan

    wl = ptysynth.workload(1)
    obj_true = wl.obj()
    pos = wl.positions()
    expected, probe = oracle.simulate(obj_true, wl.probe(), pos, wl.photons)
    counts = ptysynth.poisson_counts(expected, wl.noise_rng())
    iters = args.blind_iters
    marks = [i for i in (10, 100, 300) if i <= iters]
    out = {}
    for start in ("disk26", "disk34", "true_probe"):
        for algo in ("epie", "lsqml", "dm"):
            pl = Plan(wl.n, wl.k, wl.j, (wl.h, wl.w))
            pl.load_patterns(counts)
            pl.load_positions(pos)
            pl.set_object(np.ones((wl.h, wl.w), np.complex64))
            if start == "true_probe":
                pl.set_probe(probe.astype(np.complex64))
            else:
                pl.guess_probe(float(start[4:]))
            pl.set_truth(obj_true.astype(np.complex64), 0.3)
            nr0 = pl.nrmse()
            pl.iterate(algo, iters, probe_update_start=0)
            h, e = pl.nrmse_history(), pl.errors()
            pl.close()
            out[f"{start}.{algo}"] = {"nrmse_start": round(nr0, 4),
                                      "nrmse_at": {str(i): round(float(h[i - 1]), 4) for i in marks},
                                      "e_at": {str(i): float(e[i - 1]) for i in marks}}
            log(f"{start} {algo}: {out[f'{start}.{algo}']}")
    return {"metric": "blind-start reconstructions (NRMSE)", "value": out["disk34.lsqml"]["nrmse_at"][str(marks[-1])],
            "unit": "NRMSE", "n_gpus": 1, "higher_is_better": False, "vs_baseline": None, "dtype": "f32",
            "data": "synthetic",
            "config": {"workload": "64x64 probe, 1 mode, 10x10 raster (8 px step), 160x160 object, Poisson 1e6; "
                                   f"probe updates from 0, {iters} iterations; starts: disks of 26 and 34 px, "
                                   "and the true probe"},
            "runs": out}


def positions_leg(args, torch) -> dict:
    """LSQML given the nominal (unjittered) spiral positions of the 256 x 256,
    3-mode, 2,500-position workload whose data were recorded at the jittered
    ones: with and without position refinement, NRMSE and position error
    against the truth, and the per-iteration cost of refining."""
    import dataclasses
    import ptysynth
    from paper_2202_03144_amd import Plan

    wl, obj_true, probe, pos_true, counts = make_inputs(torch)
    nominal = dataclasses.replace(wl, jitter=False).positions()
    stream = torch.cuda.Stream()
    torch.cuda.set_stream(stream)
    iters = args.position_iters
    base = dict(probe_update_start=wl.probe_start, lsqml_batch=500)

    def err(p):
        d = p - pos_true
        return float(np.sqrt(np.mean((d - d.mean(0)) ** 2)))

    def run(refine: bool):
        pl = Plan(wl.n, wl.k, wl.j, (wl.h, wl.w), stream=stream)
        pl.load_patterns(counts)
        pl.load_positions(nominal)
        pl.set_object(np.ones((wl.h, wl.w), np.complex64))
        pl.set_probe(probe)
        pl.set_truth(obj_true, 0.3)
        prm = dict(base, position_start=args.position_start) if refine else base
        pl.iterate("lsqml", 0, **prm)
        pl.sync()
        t = time.perf_counter()
        pl.iterate("lsqml", iters, **prm)
        pl.sync()
        ms = (time.perf_counter() - t) * 1e3 / iters
        h, e, p = pl.nrmse_history(), pl.errors(), pl.positions()
        # one more iteration with per-family kernel timing (event-bracketed)
        pl.set_timing(True)
        pl.iterate("lsqml", 1, **prm)
        fam = {k: round(v[0], 3) for k, v in pl.timing().items() if v[1]}
        pl.set_timing(False)
        pl.close()
        at = {str(i): round(float(h[i - 1]), 5) for i in (1, 5, 10, 20, 30, 50, 100) if i <= len(h)}
        return {"ms_per_iter": round(ms, 3), "nrmse_at": at, "e_last": float(e[-1]),
                "position_rms_error_px": round(err(p), 4), "kernel_ms_one_iteration": fam,
                "kernel_ms_total": round(sum(fam.values()), 3)}

    log("plain")
    plain = run(False)
    log(f"plain: {plain}")
    log("refined")
    refined = run(True)
    log(f"refined: {refined}")
    return {
        "metric": "LSQML with position refinement: NRMSE and position error from nominal positions",
        "value": refined["nrmse_at"][str(iters)], "unit": "NRMSE", "n_gpus": 1, "higher_is_better": False,
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "256x256 probe, 3 modes, 2,500-point Fermat spiral, 1700x1700 object, Poisson 1e8; "
                               "data at the jittered positions (+-0.5 px), solver given the unjittered ones; "
                               f"LSQML groups of 500, probe updates from {wl.probe_start}, refinement from "
                               f"{args.position_start}, {iters} iterations (host-timed, incl. the patch-list rebuild)",
                   "n": wl.n, "modes": wl.k, "positions": wl.j},
        "nominal_position_rms_error_px": round(err(nominal), 4),
        "plain": plain, "refined": refined,
        "refinement_cost": round(refined["ms_per_iter"] / plain["ms_per_iter"], 3),
    }


def strips_leg(args, torch) -> dict:
    """The 256 x 256, 3-mode, 2,500-position workload split by row into strips
    (one GPU's share each in a multi-GPU run), run one strip after another on
    this GPU with the halo and probe messages exchanged, against one context:
    time per iteration, each strip's share, and the bytes the exchange sends
    (what RCCL would carry over xGMI)."""
    from paper_2202_03144_amd import Plan
    from paper_2202_03144_amd.plan import Domains

    wl, obj_true, probe, pos, counts = make_inputs(torch)
    stream = torch.cuda.Stream()
    torch.cuda.set_stream(stream)
    o0 = np.ones((wl.h, wl.w), np.complex64)
    iters = args.strip_iters
    out = {}
    for algo, prm in (("dm", dict(probe_update_start=0)), ("lsqml", dict(probe_update_start=0, lsqml_batch=500))):
        pl = Plan(wl.n, wl.k, wl.j, (wl.h, wl.w), stream=stream)
        pl.load_patterns(counts)
        pl.load_positions(pos)
        pl.set_object(o0)
        pl.set_probe(probe)
        dd = Domains(wl.n, wl.k, pos, (wl.h, wl.w), args.strips, stream=stream)
        dd.load_patterns(counts)
        dd.set_object(o0)
        dd.set_probe(probe)
        res = {}
        for name, h in (("one_context", pl), ("strips", dd)):
            h.iterate(algo, 1, **prm)
            h.sync()
            t0 = time.perf_counter()
            h.iterate(algo, iters, **prm)
            h.sync()
            res[name] = (time.perf_counter() - t0) * 1e3 / iters
        h0, p0 = dd.traffic()
        dd.iterate(algo, 1, **prm)
        dd.sync()
        h1, p1 = dd.traffic()
        pl.iterate(algo, 1, **prm)
        info = [dd.strip(s) for s in range(args.strips)]
        ref = pl.object()
        rel = float(np.linalg.norm(dd.object() - ref) / np.linalg.norm(ref))
        # the same iterations of one context from a start perturbed by 1e-7
        # (relative, seeded): how far rounding-level differences grow
        rng = np.random.default_rng(11)
        o1 = (o0 * (1 + 1e-7 * rng.standard_normal(o0.shape))).astype(np.complex64)
        pl.set_object(o1)
        pl.set_probe(probe)
        pl.iterate(algo, iters + 2, **prm)
        pl.sync()
        sens = float(np.linalg.norm(pl.object() - ref) / np.linalg.norm(ref))
        pl.close()
        dd.close()
        halo_iter, probe_iter = h1 - h0, p1 - p0
        borders = max(1, args.strips - 1)
        out[algo] = {
            "ms_per_iter_one_context": round(res["one_context"], 3),
            "ms_per_iter_all_strips": round(res["strips"], 3),
            "ms_per_strip_share": round(res["strips"] / args.strips, 3),
            "halo_bytes_per_iter": halo_iter, "probe_message_bytes_per_iter": probe_iter,
            "halo_bytes_per_border_per_iter": halo_iter // borders,
            "strip_rows_held": [s["hi"] - s["lo"] for s in info],
            "strip_rows_owned": [s["own_hi"] - s["own_lo"] for s in info],
            "strip_positions": [s["positions"] for s in info],
            "iterations": iters + 2,
            "object_rel_strips_vs_one_context": rel,
            "object_rel_one_context_vs_1e-7_perturbed_start": sens,
        }
        log(f"{algo}: {out[algo]}")
    return {
        "metric": "strip decomposition on one GPU: ms per iteration and exchanged bytes",
        "value": out["dm"]["ms_per_strip_share"], "unit": "ms per strip share (DM)", "n_gpus": 1,
        "higher_is_better": False, "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"256x256 probe, 3 modes, 2,500-point Fermat spiral, 1700x1700 object, Poisson 1e8; "
                               f"{args.strips} row strips of equal position count, run one after another; "
                               f"{iters} iterations each of DM and LSQML (groups of 500), host-timed",
                   "n": wl.n, "modes": wl.k, "positions": wl.j, "strips": args.strips},
        **out,
    }


def poisson_leg(args, torch) -> dict:
    """LSQML on the 256 x 256, 3-mode, 2,500-position workload with the
    modulus-projection (amplitude) and the Poisson exit-wave updates, from a
    flat object with the true probe: per-iteration time, NRMSE, E and the
    Poisson likelihood of the result, and the per-family kernel times."""
    from paper_2202_03144_amd import Plan

    stream = torch.cuda.Stream()
    torch.cuda.set_stream(stream)
    iters = args.poisson_iters

    def run(likelihood: str):
        pl = Plan(wl.n, wl.k, wl.j, (wl.h, wl.w), stream=stream)
        pl.load_patterns(counts)
        pl.load_positions(pos)
        pl.set_object(np.ones((wl.h, wl.w), np.complex64))
        pl.set_probe(probe)
        pl.set_truth(obj_true, 0.3)
        prm = dict(base, likelihood=likelihood)
        pl.iterate("lsqml", 0, **prm)
        pl.sync()
        t = time.perf_counter()
        pl.iterate("lsqml", iters, **prm)
        pl.sync()
        ms = (time.perf_counter() - t) * 1e3 / iters
        h, e = pl.nrmse_history(), pl.errors()
        o = torch.from_numpy(pl.object()).to("cuda")
        p = torch.from_numpy(pl.probe()).to("cuda")
        nll = pl.nll_forward(o, p)
        pl.set_timing(True)
        pl.iterate("lsqml", 1, **prm)
        fam = {k: round(v[0], 3) for k, v in pl.timing().items() if v[1]}
        pl.set_timing(False)
        pl.close()
        at = {str(i): round(float(h[i - 1]), 5) for i in (1, 2, 5, 10, 20, 30, 50) if i <= len(h)}
        return {"ms_per_iter": round(ms, 3), "pattern_it_per_s": round(wl.j / (ms * 1e-3), 1), "nrmse_at": at,
                "e_at": {k: float(e[int(k) - 1]) for k in at}, "poisson_nll_last": nll,
                "kernel_ms_one_iteration": fam}

    doses = {}
    for photons in (None, args.poisson_low_dose):
        wl, obj_true, probe, pos, counts = make_inputs(torch, photons)
        base = dict(probe_update_start=wl.probe_start, lsqml_batch=500)
        out = {}
        for lk in ("amplitude", "poisson"):
            log(f"{wl.photons:g} photons, {lk}")
            out[lk] = run(lk)
            log(f"{lk}: {out[lk]}")
        out["poisson_cost"] = round(out["poisson"]["ms_per_iter"] / out["amplitude"]["ms_per_iter"], 3)
        doses[f"{wl.photons:g}"] = out
        del counts
    high = doses[next(iter(doses))]
    return {
        "metric": "LSQML with the Poisson exit-wave update: pattern-iterations/s and NRMSE",
        "value": high["poisson"]["pattern_it_per_s"], "unit": "pattern-iterations/s", "n_gpus": 1,
        "higher_is_better": True, "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "256x256 probe, 3 modes, 2,500-point jittered Fermat spiral, 1700x1700 object, "
                               f"Poisson noise at the workload's 1e8 photons per pattern and at "
                               f"{args.poisson_low_dose:g}; flat start, true probe, probe updates from "
                               f"{wl.probe_start}, LSQML groups of 500, {iters} iterations (host-timed)",
                   "n": wl.n, "modes": wl.k, "positions": wl.j},
        "by_photons": doses,
    }


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--cpu-sample", type=int, default=1200, help="positions in the oracle sample (0 = skip)")
    ap.add_argument("--no-timing-pass", action="store_true", help="skip the event-timed kernel pass")
    ap.add_argument("--learned", action="store_true",
                    help="instead: train the learned initialiser and time NRMSE 1e-2, learned vs flat start")
    ap.add_argument("--train-steps", type=int, default=800)
    ap.add_argument("--train-batch", type=int, default=256)
    ap.add_argument("--train-objects", type=int, default=8)
    ap.add_argument("--infer-batch", type=int, default=4096)
    ap.add_argument("--learned-iters", type=int, default=20)
    ap.add_argument("--plain-iters", type=int, default=200)
    ap.add_argument("--nrmse-target", type=float, default=1e-2)
    ap.add_argument("--seed-strides", default="2,4",
                    help="learned arms seeding every k-th pattern, for each k listed (coverage, not redundancy)")
    ap.add_argument("--learned-lsqml-batch", type=int, default=4096,
                    help="LSQML group size of both arms (512-position groups leave a noise floor of "
                         "NRMSE 1.05e-2 on this workload, above the target)")
    ap.add_argument("--batch", action="store_true",
                    help="instead: 64 uneven LSQML datasets, sequential vs batched with graphs and autotuning")
    ap.add_argument("--datasets", type=int, default=64)
    ap.add_argument("--adjoint", action="store_true",
                    help="instead: Poisson-NLL forward and backward on the 128x128x4, 1,000-position workload")
    ap.add_argument("--adjoint-cpu-sample", type=int, default=100)
    ap.add_argument("--tiny", action="store_true",
                    help="instead: the 64x64 one-mode raster workload, ePIE / DM / LSQML eager and graphed")
    ap.add_argument("--batch-iters", type=int, default=50)
    ap.add_argument("--listing1", action="store_true",
                    help="instead: the paper's sim512 script example (ePIE, with DM and LSQML beside it)")
    ap.add_argument("--listing1-cpu-sample", type=int, default=30)
    ap.add_argument("--listing1-iters", type=int, default=0,
                    help="iterations per algorithm (default: the command's 100; fewer for a profiled run)")
    ap.add_argument("--listing1-algos", default="epie,dm,lsqml")
    ap.add_argument("--blind", action="store_true",
                    help="instead: reconstructions of the 64x64 raster workload from an aperture guess")
    ap.add_argument("--blind-iters", type=int, default=300)
    ap.add_argument("--positions", action="store_true",
                    help="instead: LSQML from nominal positions with and without position refinement")
    ap.add_argument("--position-iters", type=int, default=30)
    ap.add_argument("--position-start", type=int, default=3)
    ap.add_argument("--strips", type=int, default=0,
                    help="instead: the production workload split into this many row strips (one GPU's share "
                         "each), against one context")
    ap.add_argument("--strip-iters", type=int, default=5)
    ap.add_argument("--poisson", action="store_true",
                    help="LSQML with the amplitude and the Poisson exit-wave updates on the production workload")
    ap.add_argument("--poisson-iters", type=int, default=30)
    ap.add_argument("--poisson-low-dose", type=float, default=1e5, help="photons per pattern of the low-dose arm")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); nothing was run.",
              file=sys.stderr)
        return 2
    import torch

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 1
    from paper_2202_03144_amd import Plan

    if args.learned:
        print(json.dumps(learned_leg(args, torch)), flush=True)
        return 0
    if args.batch:
        print(json.dumps(batch_leg(args, torch)), flush=True)
        return 0
    if args.adjoint:
        print(json.dumps(adjoint_leg(args, torch)), flush=True)
        return 0
    if args.tiny:
        print(json.dumps(tiny_leg(args, torch)), flush=True)
        return 0
    if args.positions:
        print(json.dumps(positions_leg(args, torch)), flush=True)
        return 0
    if args.blind:
        print(json.dumps(blind_leg(args, torch)), flush=True)
        return 0
    if args.poisson:
        print(json.dumps(poisson_leg(args, torch)), flush=True)
        return 0
    if args.strips:
        print(json.dumps(strips_leg(args, torch)), flush=True)
        return 0
    if args.listing1:
        print(json.dumps(listing1_leg(args, torch)), flush=True)
        return 0
    log("building the 256x256x3, 2,500-position inputs")
    wl, obj_true, probe, pos, counts = make_inputs(torch)
    # a plain device copy of known size (J x N x N float32 read + written); its
    # HBM counters calibrate the kernel counters in profiles/
    calib = counts.clone()
    torch.cuda.synchronize()
    del calib
    stream = torch.cuda.Stream()  # default priority; every kernel of both plans runs on it
    torch.cuda.set_stream(stream)
    plans = {}
    for algo in ("dm", "lsqml"):
        pl = Plan(wl.n, wl.k, wl.j, (wl.h, wl.w), stream=stream)
        pl.load_patterns(counts)
        pl.load_positions(pos)
        pl.set_object(np.ones((wl.h, wl.w), np.complex64))
        pl.set_probe(probe)
        plans[algo] = pl
    params = {"dm": dict(probe_update_start=0), "lsqml": dict(probe_update_start=0, lsqml_batch=500)}

    def step():
        for algo, pl in plans.items():
            pl.iterate(algo, 1, **params[algo])

    log(f"warmup {args.warmup}")
    for _ in range(args.warmup):
        step()
    for pl in plans.values():
        pl.sync()
    torch.cuda.synchronize()

    log(f"timed {args.steps} steps")
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2 * args.steps + 1)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev[0].record(stream)
    for s in range(args.steps):
        plans["dm"].iterate("dm", 1, **params["dm"])
        ev[2 * s + 1].record(stream)
        plans["lsqml"].iterate("lsqml", 1, **params["lsqml"])
        ev[2 * s + 2].record(stream)
    for pl in plans.values():
        pl.sync()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    dm_ms = sum(ev[2 * s].elapsed_time(ev[2 * s + 1]) for s in range(args.steps)) / args.steps
    lsq_ms = sum(ev[2 * s + 1].elapsed_time(ev[2 * s + 2]) for s in range(args.steps)) / args.steps
    ms_per_step = 1e3 * wall / args.steps
    value = 2 * wl.j / (ms_per_step / 1e3)
    errs = {a: pl.errors() for a, pl in plans.items()}
    for a, e in errs.items():
        if not np.all(np.isfinite(e)):
            print(f"non-finite error history in {a}", file=sys.stderr)
            return 1
    log(f"{ms_per_step:.2f} ms/step (DM {dm_ms:.2f} ms, LSQML {lsq_ms:.2f} ms)")

    roofline = None
    families = None
    kernel_roofs = None
    if not args.no_timing_pass:
        log("event-timed kernel pass")
        for pl in plans.values():
            pl.set_timing(True)
        for _ in range(args.steps):
            step()
        families = {}
        for algo, pl in plans.items():
            for fam, (ms, cnt) in pl.timing().items():
                if cnt:
                    families[f"{algo}.{fam}"] = {"ms_per_iter": ms / args.steps, "launches_per_iter": cnt / args.steps}
            pl.set_timing(False)
        # one entry per compiled kernel: the column pass is the same kernel in
        # DM and LSQML, so its launches are pooled
        kern = {}
        for (plan_name, fam), name in KERNEL_NAMES.items():
            f = families.get(f"{plan_name}.{fam}")
            if not f:
                continue
            e = kern.setdefault(name, {"fam": fam, "plan": plan_name, "ms_per_step": 0.0, "launches_per_step": 0.0,
                                       "traffic_key": (plan_name, fam), "plans": 0})
            e["plans"] += 1
            e["ms_per_step"] += f["ms_per_iter"]
            e["launches_per_step"] += f["launches_per_iter"]
        src_ok = kernel_src_hash() == COUNTER_SRC_HASH
        kernel_roofs = {}
        for name, e in kern.items():
            per_launch_ms = e["ms_per_step"] / e["launches_per_step"]
            ppl = e["plans"] * wl.j / e["launches_per_step"]   # every plan passes all J patterns
            b = algorithmic_bytes_per_pattern(e["plan"], e["fam"], wl.n, wl.k) * ppl
            fl = flops_per_pattern(e["plan"], e["fam"], wl.n, wl.k) * ppl
            lb = lds_bytes_per_pattern(e["fam"], wl.n, wl.k) * ppl
            t = {"hbm": b / (PEAK_HBM_GBS * 1e9), "alu": fl / (PEAK_FP32_TFLOPS * 1e12),
                 "lds": lb / (PEAK_LDS_TBS * 1e12)}
            bound = max(t, key=t.get)
            sec = per_launch_ms / 1e3
            if bound == "hbm":
                achieved, peak, unit = b / sec / 1e9, PEAK_HBM_GBS, "GB/s"
            elif bound == "alu":
                achieved, peak, unit = fl / sec / 1e12, PEAK_FP32_TFLOPS, "TFLOP/s"
            else:
                achieved, peak, unit = lb / sec / 1e12, PEAK_LDS_TBS, "TB/s"
            traffic = None
            if src_ok and e["traffic_key"] in MEASURED_KIB:
                fk, wk, npl = MEASURED_KIB[e["traffic_key"]]
                traffic = round((2.0 * fk + 1.0 * wk) * 1024 / npl * ppl)
            kernel_roofs[name] = {
                "bound": bound, "achieved": round(achieved, 2), "peak": peak, "unit": unit,
                "frac": round(t[bound] / sec, 4), "traffic": traffic,
                "hbm_frac": round(t["hbm"] / sec, 4), "alu_frac": round(t["alu"] / sec, 4),
                "lds_frac": round(t["lds"] / sec, 4),
                "algorithmic_bytes_per_launch": round(b), "flops_per_launch": round(fl),
                "lds_bytes_per_launch": round(lb), "avg_launch_ms": round(per_launch_ms, 4),
                "patterns_per_launch": round(ppl, 2), "ms_per_step": round(e["ms_per_step"], 3),
                "launches_per_step": e["launches_per_step"]}
        dom = max(kernel_roofs, key=lambda n: kernel_roofs[n]["ms_per_step"])
        roofline = dict(kernel_roofs[dom], kernel=dom)
        log(f"dominant kernel {dom}: {roofline}")
    groups = -(-wl.j // params["lsqml"]["lsqml_batch"])
    iteration = {}
    for plan_name, ms in (("dm", dm_ms), ("lsqml", lsq_ms)):
        b = iteration_bytes(plan_name, wl.n, wl.k, wl.j, wl.h, wl.w, groups)
        iteration[plan_name] = {"algorithmic_GB": round(b / 1e9, 3), "ms": round(ms, 3),
                                "achieved_GBs": round(b / (ms / 1e3) / 1e9, 1),
                                "frac": round(b / (ms / 1e3) / 1e9 / PEAK_HBM_GBS, 4)}

    cpu = None
    if args.cpu_sample > 0:
        log(f"cpu baseline on {args.cpu_sample} positions")
        cpu = cpu_baseline(args.cpu_sample)

    out = {
        "metric": METRIC,
        "value": round(value, 1),
        "unit": "pattern-iterations/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "256x256 probe, 3 modes, 2500-point jittered Fermat spiral, 1700x1700 object, "
                               "Poisson 1e8 photons; one DM + one LSQML (5x500) iteration per step",
                   "n": wl.n, "modes": wl.k, "positions": wl.j, "object": [wl.h, wl.w]},
        "dm_pattern_it_per_s": round(wl.j / (dm_ms / 1e3), 1),
        "lsqml_pattern_it_per_s": round(wl.j / (lsq_ms / 1e3), 1),
        "dm_ms_per_iter": round(dm_ms, 3),
        "lsqml_ms_per_iter": round(lsq_ms, 3),
        "roofline": roofline,
        "kernel_rooflines": kernel_roofs,
        "iteration_roofline": iteration,
        "kernel_families": families,
        "cpu_baseline": cpu,
    }
    for pl in plans.values():
        pl.close()
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
