"""C-ABI checks that need no GPU: the library loads, exports every symbol the
header declares, validates arguments before touching a device, and reports a
missing device as PTY_E_DEVICE."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_2202_03144_amd import _lib as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ptymi.h")


def _have_gpu():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


def header_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pty_[a-z_0-9]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = L.lib()
    syms = header_symbols()
    assert len(syms) >= 17
    for s in syms:
        assert hasattr(lib, s), s
    assert set(syms) == set(L.SIGNATURES), "binding and header disagree"


def test_iteration_flags_match_the_header():
    text = open(HEADER).read()
    flags = {m.group(1): int(m.group(2)) for m in re.finditer(r"#define PTY_ITER_(\w+) (\d+)u", text)}
    assert flags == {"GRAPH": L.ITER_GRAPH, "ORTHO_MODES": L.ITER_ORTHO_MODES, "POISSON": L.ITER_POISSON}
    assert len(set(flags.values())) == len(flags) and all(v & (v - 1) == 0 for v in flags.values())


def test_iterate_options_map_to_flags():
    from paper_2202_03144_amd.plan import _flags
    assert _flags(0, False, False, "amplitude") == 0
    assert _flags(0, True, True, "poisson") == L.ITER_GRAPH | L.ITER_ORTHO_MODES | L.ITER_POISSON
    assert _flags(L.ITER_GRAPH, False, False, "poisson") == L.ITER_GRAPH | L.ITER_POISSON
    with pytest.raises(ValueError):
        _flags(0, False, False, "gaussian")


def test_default_params():
    p = L.IterParams()
    assert L.lib().pty_default_params(C.byref(p)) == L.OK
    assert (p.alpha, p.beta, p.lsqml_batch, p.beta_obj, p.beta_probe) == (1.0, 1.0, 512, 1.0, 1.0)
    assert p.gamma_obj < 0 and p.gamma_probe < 0 and p.order_seed == 0 and p.chunk == 0
    assert p.position_start == -1 and p.position_max_shift == 0.5
    assert L.lib().pty_default_params(None) == L.E_INVALID


@pytest.mark.parametrize("field,value", [("n", 48), ("n", 1024), ("modes", 0), ("modes", 5), ("n_pos", 0),
                                         ("obj_h", 64), ("flags", 1), ("device", -1)])
def test_create_rejects_bad_plan_before_device(field, value):
    d = L.PlanDesc(64, 1, 10, 160, 160, 0, None, 0)
    setattr(d, field, value)
    out = C.c_void_p()
    assert L.lib().pty_create(C.byref(d), C.byref(out)) == L.E_INVALID
    assert out.value is None
    assert L.lib().pty_last_error(None)


def test_512_windows_take_at_most_two_modes():
    d = L.PlanDesc(512, 3, 10, 600, 600, 0, None, 0)
    out = C.c_void_p()
    assert L.lib().pty_create(C.byref(d), C.byref(out)) == L.E_INVALID
    assert b"512" in L.lib().pty_last_error(None)


def test_null_arguments_are_invalid():
    lib = L.lib()
    assert lib.pty_create(None, None) == L.E_INVALID
    for fn, args in [("pty_load_patterns", (None, None, 0)), ("pty_load_positions", (None, None)),
                     ("pty_set_object", (None, None, 0)), ("pty_set_probe", (None, None, 0)),
                     ("pty_iterate", (None, 1, 1, None)), ("pty_get_object", (None, None, 0)),
                     ("pty_get_probe", (None, None, 0)), ("pty_sync", (None,)),
                     ("pty_get_lsqml_steps", (None, None)), ("pty_get_exit_waves", (None, None, 0)),
                     ("pty_simulate", (None, 0.0, None, 0))]:
        assert getattr(lib, fn)(*args) == L.E_INVALID, fn
    n = C.c_int32()
    assert lib.pty_get_errors(None, None, 0, C.byref(n)) == L.E_INVALID
    assert lib.pty_mem_bytes(None, None) == L.E_INVALID
    sz = C.c_size_t()
    assert lib.pty_get_state(None, None, 0, C.byref(sz)) == L.E_INVALID
    assert lib.pty_set_state(None, None, 0) == L.E_INVALID
    assert lib.pty_get_positions(None, None) == L.E_INVALID
    assert lib.pty_set_mask(None, None) == L.E_INVALID
    assert lib.pty_guess_probe(None, 10.0) == L.E_INVALID
    lib.pty_destroy(None)  # NULL-safe


@pytest.mark.skipif(_have_gpu(), reason="checks the no-device path")
def test_create_without_device_reports_device_error():
    d = L.PlanDesc(64, 1, 10, 160, 160, 0, None, 0)
    out = C.c_void_p()
    assert L.lib().pty_create(C.byref(d), C.byref(out)) == L.E_DEVICE
    assert b"device" in L.lib().pty_last_error(None)
    from paper_2202_03144_amd import Plan, PtyError
    with pytest.raises(PtyError) as e:
        Plan(64, 1, 10, (160, 160))
    assert e.value.status == L.E_DEVICE


def test_product_path_does_not_import_oracle():
    pkg = os.path.join(ROOT, "paper_2202_03144_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".cpp", ".hip", ".hpp", ".h")):
                text = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in text and "from oracle" not in text, f
                # the seeded input ingredients (no reconstruction arithmetic) serve
                # only the command front end's simulation mode
                if f != "command.py":
                    assert "ptysynth" not in text, f
    text = open(os.path.join(ROOT, "ptysynth", "__init__.py")).read()
    assert "oracle" not in text.replace("the oracle", "") and "paper_2202_03144_amd" not in text


def test_domains_reject_bad_arguments_before_device():
    lib = L.lib()
    d = L.PlanDesc(64, 1, 4, 160, 160, 0, None, 0)
    yx = np.array([[0.0, 0.0], [10.0, 0.0], [20.0, 5.0], [30.0, 5.0]])
    ptr = yx.ctypes.data_as(C.c_void_p)
    out = C.c_void_p()
    assert lib.pty_domains_create(None, ptr, 2, C.byref(out)) == L.E_INVALID
    for strips in (0, 5, 17):   # none, more strips than positions, beyond the limit
        assert lib.pty_domains_create(C.byref(d), ptr, strips, C.byref(out)) == L.E_INVALID
        assert out.value is None
    bad = yx.copy()
    bad[1, 0] = 120.0           # patch past the object's last row
    assert lib.pty_domains_create(C.byref(d), bad.ctypes.data_as(C.c_void_p), 2, C.byref(out)) == L.E_INVALID
    assert b"past the object" in lib.pty_domains_last_error(None)
    assert lib.pty_domains_iterate(None, 1, 1, None) == L.E_INVALID
    assert lib.pty_domains_get_object(None, None, 0) == L.E_INVALID
    lib.pty_domains_destroy(None)
