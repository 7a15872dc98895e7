"""The command-string front end without a GPU: parsing and the geometry of the
paper's script example (Listing 1): dx = lambda z / (N dx_d) = 2.816 nm, a
110 nm beam is 39.06 px, a 50 nm step 17.76 px, 30 x 30 positions, every
patch inside the object."""
import math

import numpy as np
import pytest

from paper_2202_03144_amd import command

LISTING1 = command.make_command(command.SIM512)


def test_parse_listing1():
    o = command.parse(LISTING1)
    assert o["size"] == 512 and o["i"] == 100 and o["scanDims"] == (30, 30) and o["step"] == (50e-9, 50e-9)
    assert o["simulate"] == 1 and o["blind"] == 0 and o["jobID"] == "sim512"


@pytest.mark.parametrize("bad", ["-size", "-foo=1", "-scanDims=30", "size=512"])
def test_parse_rejects(bad):
    with pytest.raises(ValueError):
        command.parse("-size=512 " + bad)


def test_listing1_geometry():
    g = command.geometry(command.parse(LISTING1))
    dx = 2.4796837508399954e-10 * 1.0 / (512 * 172e-6)
    assert abs(g.pixel - dx) <= 1e-18 and abs(g.pixel - 2.8158e-9) <= 1e-12
    assert abs(g.beam_px - 110e-9 / dx) <= 1e-9 and abs(g.beam_px - 39.06) <= 0.01
    assert abs(g.step_px[0] - 50e-9 / dx) <= 1e-9 and abs(g.step_px[1] - 17.757) <= 1e-3
    assert g.positions.shape == (900, 2) and g.iterations == 100 and not g.blind
    # raster, row-major, 1-pixel margin; every patch inside the object
    assert np.allclose(g.positions[1] - g.positions[0], (0.0, g.step_px[1]))
    assert np.allclose(g.positions[30] - g.positions[0], (g.step_px[0], 0.0))
    h, w = g.obj_shape
    for y, x in g.positions:
        assert y >= 0 and x >= 0
        assert math.floor(y) + 512 + 1 <= h and math.floor(x) + 512 + 1 <= w


def test_synthetic_inputs():
    o = command.synthetic_object((64, 80), seed=3)
    assert o.shape == (64, 80) and o.dtype == np.complex64
    a = np.abs(o)
    assert a.min() >= 0.8 - 1e-6 and a.max() <= 1.0 + 1e-6
    assert np.abs(np.angle(o)).max() <= 0.5 + 1e-6
    p = command.synthetic_probe(64, 2, 20.0)
    assert abs(float(np.sum(np.abs(p) ** 2)) - 1.0) <= 1e-5
    c = 31.5
    u, v = np.meshgrid(np.arange(64) - c, np.arange(64) - c, indexing="ij")
    assert np.max(np.abs(p[:, u * u + v * v > 100.0])) == 0.0
