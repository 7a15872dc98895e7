"""Writes production_nrmse.json: the FP64 oracle's NRMSE (and amplitude error E)
after each of 100 DM and 100 LSQML iterations on the production workload:
256 x 256 probe with 3 modes, 2,500-point Fermat spiral with +-0.5 px jitter,
1700 x 1700 object, Poisson counts at 1e8 photons per pattern; start from
O = 1 and the true probe (float32-representable values), probe updates from
iteration 10, LSQML groups of 500 (5 interleaved groups).  NRMSE is the
invariant metric on the region where the true probe's illumination is at
least 0.3 of its maximum.

Only oracle/ and ptysynth/ are called.  Run from the repository root:
    python tests/golden/make_production_nrmse.py
(about 1.5 h on 8 cores; writes the JSON next to this file).
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import ptysynth  # noqa: E402

ITERS = 100
START = 10
BATCH = 500


def main():
    wl = ptysynth.workload(2)
    obj_true = wl.obj()
    pos = wl.positions()
    expected, probe = oracle.simulate(obj_true, wl.probe(), pos, wl.photons)
    counts = ptysynth.poisson_counts(expected, wl.noise_rng())
    del expected
    amp = oracle.amplitude(counts.astype(np.float64))
    del counts
    o0 = np.ones(obj_true.shape, np.complex64).astype(np.complex128)
    p0 = probe.astype(np.complex64).astype(np.complex128)
    truth = obj_true.astype(np.complex64).astype(np.complex128)
    mask = oracle.roi_mask(p0, pos, *obj_true.shape)
    out = {"workload": "256x256 probe, 3 modes, 2,500 spiral positions, 1700x1700 object, Poisson 1e8; "
                       f"O = 1, true probe, probe updates from {START}, LSQML groups of {BATCH}",
           "nrmse_start": oracle.nrmse(o0, truth, mask)}
    for algo in ("dm", "lsqml"):
        o, p = o0.copy(), p0.copy()
        psi = oracle.dm_init(o, p, pos) if algo == "dm" else None
        nr, es = [], []
        t0 = time.time()
        for t in range(ITERS):
            if algo == "dm":
                o, p, psi, e = oracle.dm(o, p, psi, amp, pos, 1, t0=t, start=START)
            else:
                o, p, e = oracle.lsqml(o, p, amp, pos, 1, t0=t, start=START, batch=BATCH)
            nr.append(oracle.nrmse(o, truth, mask))
            es.append(float(e[-1]))
            print(f"{algo} {t + 1}/{ITERS} nrmse {nr[-1]:.6f} E {es[-1]:.6g} ({time.time() - t0:.0f} s)",
                  flush=True)
        out[algo] = {"nrmse": nr, "E": es}
        del psi
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "production_nrmse.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print("wrote", path)


if __name__ == "__main__":
    main()
