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


def test_listing1_epie_matches_the_oracle_run():
    """The script example's ePIE run (known probe, 100 iterations from O = 1,
    noise-free counts) against the FP64 oracle's run on the same workload,
    stored in tests/golden/sim512_epie.json by make_sim512_epie.py (which
    calls only the oracle and the input ingredients): the first two
    iterations' error at 1e-4 and 1e-3 relative (ePIE is sequential, so float32
    rounding accumulates over the 900 positions of a pass) and the final NRMSE
    within 2%."""
    import json
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "sim512_epie.json")
    with open(path) as f:
        gold = json.load(f)
    pl, g, obj, probe = command.simulated_plan(LISTING1)
    assert list(g.obj_shape) == gold["object_shape"]
    assert abs(g.positions.sum() - gold["positions_sum"]) < 1e-6 * gold["positions_sum"]
    pl.set_truth(obj, 0.3)
    pl.iterate("epie", gold["iterations"], **command.iteration_params(g))
    e, h = pl.errors(), pl.nrmse_history()
    pl.close()
    print(f"\n[listing1] E {e[0]:.6e} / {gold['E'][0]:.6e}, {e[1]:.6e} / {gold['E'][1]:.6e}; "
          f"NRMSE {h[-1]:.6f} / {gold['nrmse'][-1]:.6f}", flush=True)
    assert abs(e[0] - gold["E"][0]) <= 1e-4 * gold["E"][0]
    assert abs(e[1] - gold["E"][1]) <= 1e-3 * gold["E"][1]
    assert abs(h[-1] - gold["nrmse"][-1]) <= 0.02 * gold["nrmse"][-1]
