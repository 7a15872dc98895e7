"""Writes sim512_epie.json: the FP64 oracle's ePIE run on the simulated
workload of the paper's script example (Sec. 3.2, Listing 1): a 512 x 512
window, a 30 x 30 raster of 50 nm steps, a 110 nm beam, wavelength
0.248 nm, 172 um detector pixels 1 m from the sample, a known probe (never
updated), 100 iterations from O = 1.  The data are the noise-free expected
counts (1e6 photons per pattern on average) of the seeded synthetic object
and probe that stand in for the paper's simulation images.

Geometry, written out here from those values (not from the library): the
object pixel is lambda z / (N dx_d); positions are the raster's top-left
corners from a 1-pixel margin; the object holds every patch.

Stored: E and the invariant NRMSE (region where the true probe's
illumination is at least 0.3 of its maximum) after every iteration, and a
summary of the positions.  Only oracle/ and ptysynth/ are called.  Run from
the repository root:
    python tests/golden/make_sim512_epie.py
(about 20 min on 8 cores).
"""
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import ptysynth  # noqa: E402

N = 512
WAVELENGTH = 2.4796837508399954e-10
DIST = 1.0
DET_PIXEL = 172e-6
BEAM = 110e-9
STEP = 50e-9
RASTER = 30
ITERS = 100
PHOTONS = 1e6


def geometry():
    dx = WAVELENGTH * DIST / (N * DET_PIXEL)
    s = STEP / dx
    yy, xx = np.meshgrid(1.0 + s * np.arange(RASTER), 1.0 + s * np.arange(RASTER), indexing="ij")
    pos = np.stack([yy.ravel(), xx.ravel()], axis=1)
    side = int(math.floor(pos.max())) + N + 2
    return dx, pos, (side, side)


def main():
    dx, pos, shape = geometry()
    obj_true = ptysynth.sim_object(shape, 0).astype(np.complex128)
    probe0 = ptysynth.sim_probe(N, 1, BEAM / dx).astype(np.complex128)
    counts, probe = oracle.simulate(obj_true, probe0, pos, PHOTONS)
    probe = probe.astype(np.complex64).astype(np.complex128)   # the start both sides can hold
    amp = oracle.amplitude(counts.astype(np.float32).astype(np.float64))
    del counts
    roi = oracle.roi_mask(probe, pos, *shape)
    obj = np.ones(shape, np.complex128)
    out = {"iterations": ITERS, "photons": PHOTONS, "object_shape": list(shape), "pixel_m": dx,
           "positions_sum": float(pos.sum()), "positions_first": pos[0].tolist(), "positions_last": pos[-1].tolist(),
           "E": [], "nrmse": []}
    t0 = time.time()
    for t in range(ITERS):
        obj, probe, e = oracle.epie(obj, probe, amp, pos, 1, t0=t, start=1 << 30)
        out["E"].append(float(e[0]))
        out["nrmse"].append(float(oracle.nrmse(obj, obj_true, roi)))
        print(f"it {t + 1}: E {e[0]:.4e} NRMSE {out['nrmse'][-1]:.5f} ({time.time() - t0:.0f} s)", flush=True)
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "sim512_epie.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
