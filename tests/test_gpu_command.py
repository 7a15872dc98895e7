"""The paper's script example (Listing 1) end to end on the GPU through the
step API with a command string: the 512 x 512, 30 x 30-raster simulation,
ePIE steps with the known probe (E falls), and the blind variant."""
import numpy as np
import pytest

from paper_2202_03144_amd import command

pytestmark = pytest.mark.gpu

LISTING1 = command.make_command(command.SIM512)


def test_listing1_step_mode():
    from paper_2202_03144_amd import compat
    compat.epieinit(LISTING1)
    for _ in range(3):
        compat.epiestep()
    obj, probe = compat.epieresobj(), compat.epieresprobe()
    pl, params = compat._plan("epie")
    e = pl.errors()
    compat.epiepost()
    assert obj.shape == (1029, 1029) and probe.shape == (1, 512, 512)
    assert params["probe_update_start"] == -1
    assert len(e) == 3 and np.all(np.isfinite(e)) and e[2] < e[1] < e[0]


def test_listing1_blind_start():
    pl, g, obj, probe = command.simulated_plan(command.make_command({**command.SIM512, "blind": 1}))
    guess = pl.probe()
    pl.iterate("epie", 2, **command.iteration_params(g))
    e = pl.errors()
    assert np.all(np.isfinite(e)) and e[1] < e[0]
    assert not np.array_equal(pl.probe(), guess)       # the probe is being retrieved
    pl.close()
