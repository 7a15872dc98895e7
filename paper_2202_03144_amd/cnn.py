"""Python front end of the learned initialiser's network (pty_cnn_* in
include/ptymi.h): argument marshalling only; the network runs in the HIP
kernels of libptymi.so."""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import _lib as L
from ._lib import PtyError
from .plan import _is_torch, _ptr

IN_SIZE = 128
IN_CH = 2
OUT_SIZE = 64


class Net:
    """U-Net on one GPU with buffers for batches of up to ``max_batch``."""

    def __init__(self, max_batch: int, seed: int = 0, device: int = 0, stream=None):
        self._lib = L.lib()
        if stream is not None and hasattr(stream, "cuda_stream"):
            stream = stream.cuda_stream
        out = C.c_void_p()
        st = self._lib.pty_cnn_create(int(device), C.c_void_p(stream) if stream else None, int(max_batch),
                                      int(seed) & ((1 << 64) - 1), C.byref(out))
        if st != L.OK:
            raise PtyError(st, self._lib.pty_cnn_last_error(None).decode())
        self._net = out
        self.max_batch = int(max_batch)
        n = C.c_int64()
        self._check(self._lib.pty_cnn_num_params(self._net, C.byref(n)))
        self.num_params = int(n.value)

    def _check(self, st: int) -> None:
        if st != L.OK:
            raise PtyError(st, self._lib.pty_cnn_last_error(self._net).decode())

    def _live(self):
        if self._net is None:
            raise PtyError(L.E_STATE, "network is closed")
        return self._net

    @staticmethod
    def _dev(x, shape, name):
        if not (_is_torch(x) and x.is_cuda):
            raise TypeError(f"{name} must be a CUDA tensor")
        if not x.is_contiguous():
            raise ValueError(f"{name} must be contiguous")
        ptr, _, _ = _ptr(x, np.float32, shape)
        return ptr

    def params(self) -> np.ndarray:
        out = np.empty(self.num_params, dtype=np.float32)
        self._check(self._lib.pty_cnn_get_params(self._live(), out.ctypes.data_as(C.c_void_p)))
        return out

    def set_params(self, flat) -> None:
        a = np.ascontiguousarray(flat, dtype=np.float32)
        if a.shape != (self.num_params,):
            raise ValueError(f"expected {self.num_params} parameters, got shape {a.shape}")
        self._check(self._lib.pty_cnn_set_params(self._live(), a.ctypes.data_as(C.c_void_p)))

    def forward(self, x, out):
        b = x.shape[0]
        self._check(self._lib.pty_cnn_forward(self._live(), self._dev(x, (b, IN_SIZE, IN_SIZE, IN_CH), "x"), b,
                                              self._dev(out, (b, OUT_SIZE, OUT_SIZE, 2), "out")))
        return out

    def grad(self, x, target):
        """(loss, gradient as a float32 NumPy vector); parameters unchanged."""
        b = x.shape[0]
        g = np.empty(self.num_params, dtype=np.float32)
        loss = C.c_double()
        self._check(self._lib.pty_cnn_grad(self._live(), self._dev(x, (b, IN_SIZE, IN_SIZE, IN_CH), "x"),
                                           self._dev(target, (b, OUT_SIZE, OUT_SIZE, 2), "target"), b,
                                           g.ctypes.data_as(C.c_void_p), C.byref(loss)))
        return loss.value, g

    def train_step(self, x, target, lr: float) -> float:
        b = x.shape[0]
        loss = C.c_double()
        self._check(self._lib.pty_cnn_train_step(self._live(), self._dev(x, (b, IN_SIZE, IN_SIZE, IN_CH), "x"),
                                                 self._dev(target, (b, OUT_SIZE, OUT_SIZE, 2), "target"), b,
                                                 float(lr), C.byref(loss)))
        return loss.value

    def input(self, counts, probe, out):
        """Network input (B, 128, 128, 2) from centred counts (B, 128, 128) and the
        probe (1, 128, 128) complex64, all CUDA tensors (see pty_cnn_input)."""
        b = counts.shape[0]
        if not (_is_torch(probe) and probe.is_cuda):
            raise TypeError("probe must be a CUDA tensor")
        pp, _, _ = _ptr(probe, np.complex64, (1, IN_SIZE, IN_SIZE))
        self._check(self._lib.pty_cnn_input(self._live(), self._dev(counts, (b, IN_SIZE, IN_SIZE), "counts"), b,
                                            pp, self._dev(out, (b, IN_SIZE, IN_SIZE, IN_CH), "out")))
        return out

    def close(self) -> None:
        if getattr(self, "_net", None) is not None:
            self._lib.pty_cnn_destroy(self._net)
            self._net = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
