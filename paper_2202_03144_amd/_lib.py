"""ctypes declarations of the C ABI in include/ptymi.h.

Loading fails loudly when the HIP library has not been built: there is no
fallback implementation.
"""
from __future__ import annotations

import ctypes as C
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libptymi.so")

OK, E_INVALID, E_STATE, E_NOMEM, E_DEVICE, E_NUMERIC, E_UNSUPPORTED = range(7)
STATUS_NAMES = {
    OK: "PTY_OK",
    E_INVALID: "PTY_E_INVALID",
    E_STATE: "PTY_E_STATE",
    E_NOMEM: "PTY_E_NOMEM",
    E_DEVICE: "PTY_E_DEVICE",
    E_NUMERIC: "PTY_E_NUMERIC",
    E_UNSUPPORTED: "PTY_E_UNSUPPORTED",
}
EPIE, DM, LSQML = 0, 1, 2


class PlanDesc(C.Structure):
    _fields_ = [
        ("n", C.c_int32),
        ("modes", C.c_int32),
        ("n_pos", C.c_int32),
        ("obj_h", C.c_int32),
        ("obj_w", C.c_int32),
        ("device", C.c_int32),
        ("stream", C.c_void_p),
        ("flags", C.c_uint32),
    ]


class IterParams(C.Structure):
    _fields_ = [
        ("alpha", C.c_float),
        ("beta", C.c_float),
        ("probe_update_start", C.c_int32),
        ("lsqml_batch", C.c_int32),
        ("gamma_obj", C.c_float),
        ("gamma_probe", C.c_float),
        ("beta_obj", C.c_float),
        ("beta_probe", C.c_float),
        ("order_seed", C.c_uint64),
        ("chunk", C.c_int32),
        ("flags", C.c_uint32),
        ("position_start", C.c_int32),
        ("position_max_shift", C.c_float),
    ]


# name -> (restype, argtypes); every symbol declared in include/ptymi.h
SIGNATURES = {
    "pty_default_params": (C.c_int, [C.POINTER(IterParams)]),
    "pty_create": (C.c_int, [C.POINTER(PlanDesc), C.POINTER(C.c_void_p)]),
    "pty_load_patterns": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int]),
    "pty_load_positions": (C.c_int, [C.c_void_p, C.c_void_p]),
    "pty_set_object": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int]),
    "pty_set_probe": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int]),
    "pty_iterate": (C.c_int, [C.c_void_p, C.c_int, C.c_int32, C.POINTER(IterParams)]),
    "pty_get_object": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int]),
    "pty_get_probe": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int]),
    "pty_get_errors": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int32, C.POINTER(C.c_int32)]),
    "pty_get_lsqml_steps": (C.c_int, [C.c_void_p, C.c_void_p]),
    "pty_get_exit_waves": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int]),
    "pty_mem_bytes": (C.c_int, [C.c_void_p, C.POINTER(C.c_size_t)]),
    "pty_set_mask": (C.c_int, [C.c_void_p, C.c_void_p]),
    "pty_guess_probe": (C.c_int, [C.c_void_p, C.c_double]),
    "pty_get_positions": (C.c_int, [C.c_void_p, C.c_void_p]),
    "pty_get_state": (C.c_int, [C.c_void_p, C.c_void_p, C.c_size_t, C.POINTER(C.c_size_t)]),
    "pty_set_state": (C.c_int, [C.c_void_p, C.c_void_p, C.c_size_t]),
    "pty_sync": (C.c_int, [C.c_void_p]),
    "pty_destroy": (None, [C.c_void_p]),
    "pty_last_error": (C.c_char_p, [C.c_void_p]),
    "pty_simulate": (C.c_int, [C.c_void_p, C.c_double, C.c_void_p, C.c_int]),
    "pty_set_timing": (C.c_int, [C.c_void_p, C.c_int]),
    "pty_get_timing": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32]),
    "pty_nll_forward": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(C.c_double)]),
    "pty_nll_backward": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_float, C.c_void_p,
                                   C.c_void_p, C.c_void_p, C.POINTER(C.c_double)]),
    "pty_nll_forward_noalloc": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32,
                                          C.c_void_p]),
    "pty_domains_create": (C.c_int, [C.POINTER(PlanDesc), C.c_void_p, C.c_int32, C.POINTER(C.c_void_p)]),
    "pty_domains_load_patterns": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int]),
    "pty_domains_set_object": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int]),
    "pty_domains_set_probe": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int]),
    "pty_domains_iterate": (C.c_int, [C.c_void_p, C.c_int, C.c_int32, C.POINTER(IterParams)]),
    "pty_domains_get_object": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int]),
    "pty_domains_get_probe": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int]),
    "pty_domains_get_errors": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int32, C.POINTER(C.c_int32)]),
    "pty_domains_strip": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p]),
    "pty_domains_traffic": (C.c_int, [C.c_void_p, C.POINTER(C.c_uint64), C.POINTER(C.c_uint64)]),
    "pty_domains_sync": (C.c_int, [C.c_void_p]),
    "pty_domains_destroy": (None, [C.c_void_p]),
    "pty_domains_last_error": (C.c_char_p, [C.c_void_p]),
    "pty_get_tuning": (C.c_int, [C.c_void_p, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]),
    "pty_batch_autotune": (C.c_int, [C.c_void_p, C.c_int, C.POINTER(IterParams), C.c_char_p]),
    "pty_model_error": (C.c_int, [C.c_void_p, C.POINTER(C.c_double)]),
    "pty_set_truth": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int, C.c_float]),
    "pty_nrmse": (C.c_int, [C.c_void_p, C.POINTER(C.c_double)]),
    "pty_get_nrmse": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int32, C.POINTER(C.c_int32)]),
    "pty_cnn_create": (C.c_int, [C.c_int32, C.c_void_p, C.c_int32, C.c_uint64, C.POINTER(C.c_void_p)]),
    "pty_cnn_destroy": (None, [C.c_void_p]),
    "pty_cnn_last_error": (C.c_char_p, [C.c_void_p]),
    "pty_cnn_num_params": (C.c_int, [C.c_void_p, C.POINTER(C.c_int64)]),
    "pty_cnn_get_params": (C.c_int, [C.c_void_p, C.c_void_p]),
    "pty_cnn_set_params": (C.c_int, [C.c_void_p, C.c_void_p]),
    "pty_cnn_forward": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p]),
    "pty_cnn_grad": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p,
                               C.POINTER(C.c_double)]),
    "pty_cnn_train_step": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.c_float,
                                     C.POINTER(C.c_double)]),
    "pty_cnn_input": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p]),
    "pty_poisson": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_size_t, C.c_uint64]),
    "pty_training_targets": (C.c_int, [C.c_void_p, C.c_void_p]),
    "pty_stitch": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "pty_seed_object": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int32, C.c_int32, C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    "pty_batch_create": (C.c_int, [C.POINTER(C.c_void_p), C.c_int32, C.POINTER(C.c_void_p)]),
    "pty_batch_iterate": (C.c_int, [C.c_void_p, C.c_int, C.c_int32, C.POINTER(IterParams)]),
    "pty_batch_sync": (C.c_int, [C.c_void_p]),
    "pty_batch_destroy": (None, [C.c_void_p]),
    "pty_batch_last_error": (C.c_char_p, [C.c_void_p]),
    "pty_autotune": (C.c_int, [C.c_void_p, C.c_int, C.POINTER(IterParams), C.c_char_p, C.POINTER(C.c_int32)]),
}

ITER_GRAPH = 1
ITER_ORTHO_MODES = 2
ITER_POISSON = 4

TIMING_FAMILIES = ["rows_fwd", "cols", "rows_inv", "obj_gather", "probe_acc", "probe_finish_apply",
                   "lsq_steps", "epie_update", "other"]

_lib = None


def lib() -> C.CDLL:
    """The loaded library (raises if it has not been built).

    PyTorch for ROCm ships its own HIP runtime with the same SONAME
    (libamdhip64.so.7).  Importing torch first lets the dynamic linker satisfy
    the library's dependency with that already-loaded runtime, so the process
    holds one HIP runtime and torch's device pointers and streams are valid
    here; without torch the system runtime is used.
    """
    global _lib
    if _lib is None:
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is missing: build it with `python -m paper_2202_03144_amd.build` "
                "(there is no CPU fallback)")
        handle = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(handle, name)
            fn.restype = res
            fn.argtypes = args
        _lib = handle
    return _lib


class PtyError(RuntimeError):
    """A non-OK status from the library."""

    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status
