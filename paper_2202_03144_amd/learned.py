"""Learned initialiser: training loop and seeded reconstruction (argument
marshalling and scheduling only; every step runs in the library's kernels).

Training data are made on the device: for a batch of random integer window
positions on a training object, the forward model gives the expected counts
(``Plan.simulate``), ``Plan.poisson`` draws the counts, ``Net.input`` forms the
network input (the real-space estimate from the counts and the probe) and
``Plan.training_targets`` the targets (amplitude and phase
relative to the mean phasor of the central 64 x 64 patch).
"""
from __future__ import annotations

import time

import numpy as np

from .cnn import Net
from .plan import Plan


def train(net: Net, objects, probe, photons: float, steps: int, batch: int, lr: float = 1e-3,
          seed: int = 0, objects_per_switch: int = 4, log_every: int = 0, log=print,
          lr_final: float | None = None) -> list:
    """Adam steps of `net` on freshly simulated batches; returns the losses.

    objects: a list of CUDA complex64 tensors (H, W), all of one shape, with
    H, W > 128; probe: (1, 128, 128) complex64, scaled on the first batch so
    that the mean pattern total equals `photons`.  The learning rate decays
    geometrically from lr to lr_final (default: constant).
    """
    import torch

    if batch > net.max_batch:
        raise ValueError("batch exceeds the network's max_batch")
    h, w = objects[0].shape
    rng = np.random.default_rng(seed)
    losses = []
    dev = objects[0].device
    lam = torch.empty((batch, 128, 128), dtype=torch.float32, device=dev)
    cnt = torch.empty_like(lam)
    x = torch.empty((batch, 128, 128, 2), dtype=torch.float32, device=dev)
    probe_dev = None
    tg = torch.empty((batch, 64, 64, 2), dtype=torch.float32, device=dev)
    t0 = time.perf_counter()
    with Plan(128, 1, batch, (h, w)) as pl:
        pl.set_probe(probe)
        scaled = False
        for s in range(steps):
            if s % objects_per_switch == 0:
                pl.set_object(objects[(s // objects_per_switch) % len(objects)])
            pos = np.stack([rng.integers(0, h - 128, batch), rng.integers(0, w - 128, batch)], axis=1)
            pl.load_positions(pos.astype(np.float64))
            pl.simulate(0.0 if scaled else photons, out=lam)
            if not scaled:
                probe_dev = torch.from_numpy(pl.probe()).to(dev)   # scaled to the photon budget
            scaled = True
            pl.poisson(lam, cnt, seed=(seed << 32) + s)
            net.input(cnt, probe_dev, x)
            pl.training_targets(tg)
            rate = lr if lr_final is None else lr * (lr_final / lr) ** (s / max(1, steps - 1))
            losses.append(net.train_step(x, tg, rate))
            if log_every and (s + 1) % log_every == 0:
                log(f"step {s + 1}/{steps} loss {np.mean(losses[-log_every:]):.5f} "
                    f"({time.perf_counter() - t0:.1f} s)")
    return losses


def time_to_nrmse(plan: Plan, target: float, max_iter: int, stream, **params):
    """Enqueues max_iter LSQML iterations with an event after each, then reads
    the per-iteration NRMSE (the plan needs a truth).

    Returns (per-iteration NRMSE, per-iteration elapsed ms since the first
    iteration was enqueued, index of the first iteration at or below `target`
    or None).  No host synchronisation happens between iterations.
    """
    import torch

    plan.iterate("lsqml", 0, **params)     # allocates the work buffers outside the timed span
    plan.sync()
    start = torch.cuda.Event(enable_timing=True)
    start.record(stream)
    evs = []
    for _ in range(max_iter):
        plan.iterate("lsqml", 1, **params)
        e = torch.cuda.Event(enable_timing=True)
        e.record(stream)
        evs.append(e)
    stream.synchronize()
    ms = np.array([start.elapsed_time(e) for e in evs])
    hist = plan.nrmse_history()[-max_iter:]
    hit = np.nonzero(hist <= target)[0]
    return hist, ms, (int(hit[0]) if hit.size else None)
