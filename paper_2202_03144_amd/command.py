"""Command-string front end in the style of the paper's script example
(Sec. 3.2, Listing 1): ``-key=value`` tokens that describe the experiment in
physical units, turned into the pixel geometry the library works in, and the
simulation mode that builds a data set from them.

Keys (a leading program name and unknown ``-`` tokens are rejected, except
``jobID`` which only names the run):

=============  ==========================================================
``size``       detector window N (pixels)
``lambda``     wavelength (m)
``z``          sample-detector distance (m)
``dx_d``       detector pixel (m)
``beamSize``   probe diameter (m)
``scanDims``   raster rows,cols
``step``       raster step y,x (m)
``i``          iterations
``simulate``   1: build the data from a synthetic object and probe
``blind``      0: the probe is known (not updated); 1: start from an
               aperture guess of the beam size, probe updated throughout
``probeModes`` number of probe modes (default 1)
``jobID``      run name (kept, not used)
=============  ==========================================================

Far-field sampling gives the object-plane pixel dx = lambda z / (N dx_d).
Positions are the raster's top-left corners in object pixels, row-major,
from a 1-pixel margin; the object is just large enough to hold every patch.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

from ptysynth import sim_object as synthetic_object  # noqa: F401  (input ingredients)
from ptysynth import sim_probe as synthetic_probe  # noqa: F401

_FLOAT = {"lambda", "z", "dx_d", "beamSize"}
_INT = {"size", "i", "simulate", "blind", "probeModes"}
_PAIR = {"scanDims": int, "step": float}
_TEXT = {"jobID"}


# The simulated workload of the paper's script example (Sec. 3.2, Listing 1),
# as named values: a 512-pixel detector window, a 30 x 30 raster with 50 nm
# steps, a 110 nm beam, 5 keV photons (wavelength 0.248 nm), a detector of
# 172 um pixels 1 m from the sample, 100 iterations, simulated data from a
# known probe.
SIM512 = {
    "jobID": "sim512",
    "beamSize": 110e-9,
    "scanDims": (30, 30),
    "step": (50e-9, 50e-9),
    "i": 100,
    "size": 512,
    "lambda": 2.4796837508399954e-10,
    "dx_d": 172e-6,
    "z": 1.0,
    "simulate": 1,
    "blind": 0,
}


def make_command(opts: dict, program: str = "ptycho") -> str:
    """The ``-key=value`` command string of typed options (the inverse of
    :func:`parse`; pairs are written comma-separated)."""
    toks = [program] if program else []
    for k, v in opts.items():
        if k in _PAIR:
            v = ",".join(repr(_PAIR[k](x)) if _PAIR[k] is float else str(int(x)) for x in v)
        elif k in _FLOAT:
            v = repr(float(v))
        toks.append(f"-{k}={v}")
    return " ".join(toks)


def parse(cmd: str) -> dict:
    """``-key=value`` tokens to typed values (a first token without ``-`` is
    taken as the program name and skipped)."""
    toks = cmd.split()
    if toks and not toks[0].startswith("-"):
        toks = toks[1:]
    out = {}
    for t in toks:
        if not t.startswith("-") or "=" not in t:
            raise ValueError(f"not a -key=value token: {t!r}")
        k, v = t[1:].split("=", 1)
        if k in _FLOAT:
            out[k] = float(v)
        elif k in _INT:
            out[k] = int(v)
        elif k in _PAIR:
            parts = [_PAIR[k](x) for x in v.split(",")]
            if len(parts) != 2:
                raise ValueError(f"-{k} takes two comma-separated values")
            out[k] = tuple(parts)
        elif k in _TEXT:
            out[k] = v
        else:
            raise ValueError(f"unknown key -{k}")
    return out


@dataclasses.dataclass
class Geometry:
    n: int
    modes: int
    pixel: float                 # object-plane pixel (m)
    beam_px: float               # probe diameter (pixels)
    step_px: tuple               # raster step y, x (pixels)
    positions: np.ndarray        # (J, 2) top-left corners (pixels)
    obj_shape: tuple             # (H, W)
    iterations: int
    blind: bool


def geometry(opts: dict) -> Geometry:
    for k in ("size", "lambda", "z", "dx_d", "beamSize", "scanDims", "step"):
        if k not in opts:
            raise ValueError(f"missing -{k}")
    n = opts["size"]
    dx = opts["lambda"] * opts["z"] / (n * opts["dx_d"])
    sy, sx = (s / dx for s in opts["step"])
    rows, cols = opts["scanDims"]
    margin = 1.0
    yy, xx = np.meshgrid(margin + sy * np.arange(rows), margin + sx * np.arange(cols), indexing="ij")
    pos = np.stack([yy.ravel(), xx.ravel()], axis=1)
    h = int(math.floor(pos[:, 0].max())) + n + 2
    w = int(math.floor(pos[:, 1].max())) + n + 2
    return Geometry(n=n, modes=opts.get("probeModes", 1), pixel=dx, beam_px=opts["beamSize"] / dx,
                    step_px=(sy, sx), positions=pos, obj_shape=(h, w), iterations=opts.get("i", 100),
                    blind=bool(opts.get("blind", 0)))


def simulated_plan(cmd: str, photons: float = 1e6, seed: int = 0, device: int = 0, stream=None):
    """Simulation mode: the plan of the command with noise-free expected
    counts of a synthetic object and probe loaded (``photons`` per pattern on
    average), the object set to 1, and the probe set to the true one
    (``-blind=0``) or to the aperture guess of the beam size (``-blind=1``).
    Returns (plan, geometry, true object, true probe)."""
    import torch

    from .plan import Plan

    opts = parse(cmd)
    if opts.get("simulate", 0) != 1:
        raise ValueError("only the simulation mode (-simulate=1) builds its own data")
    g = geometry(opts)
    obj = synthetic_object(g.obj_shape, seed)
    probe0 = synthetic_probe(g.n, g.modes, g.beam_px)
    pl = Plan(g.n, g.modes, len(g.positions), g.obj_shape, device=device, stream=stream)
    pl.load_positions(g.positions)
    pl.set_object(obj)
    pl.set_probe(probe0)
    counts = torch.empty((len(g.positions), g.n, g.n), dtype=torch.float32, device=f"cuda:{device}")
    pl.simulate(photons, out=counts)
    probe = pl.probe()                 # scaled to the photon budget
    pl.load_patterns(counts)
    del counts
    pl.set_object(np.ones(g.obj_shape, np.complex64))
    if g.blind:
        pl.guess_probe(g.beam_px)
    else:
        pl.set_probe(probe)
    return pl, g, obj, probe


def iteration_params(g: Geometry) -> dict:
    """Known probe: never updated; blind start: updated from the first iteration."""
    return {"probe_update_start": 0 if g.blind else -1}
