"""Python front end of the ptymi C ABI (argument marshalling only).

Every step of a reconstruction runs in the HIP kernels behind
``include/ptymi.h``; this module converts NumPy arrays or torch tensors into
pointers and status codes into exceptions.  torch is used only for device
memory and the current HIP stream.
"""
from __future__ import annotations

import ctypes as C
from typing import Optional

import numpy as np

from . import _lib as L
from ._lib import PtyError

ALGOS = {"epie": L.EPIE, "dm": L.DM, "lsqml": L.LSQML}


def _flags(flags: int, graph: bool, ortho_modes: bool, likelihood: str) -> int:
    if likelihood not in ("amplitude", "poisson"):
        raise ValueError(f"likelihood must be 'amplitude' or 'poisson', not {likelihood!r}")
    return (int(flags) | (L.ITER_GRAPH if graph else 0) | (L.ITER_ORTHO_MODES if ortho_modes else 0)
            | (L.ITER_POISSON if likelihood == "poisson" else 0))


def _is_torch(x) -> bool:
    return type(x).__module__.startswith("torch")


def _ptr(x, dtype, shape):
    """(pointer, on_device, keepalive) for a NumPy array or torch tensor of the given layout."""
    if _is_torch(x):
        import torch

        want = {np.float32: torch.float32, np.float64: torch.float64, np.complex64: torch.complex64}[dtype]
        if tuple(x.shape) != tuple(shape):
            raise ValueError(f"expected shape {tuple(shape)}, got {tuple(x.shape)}")
        if x.dtype != want:
            raise ValueError(f"expected dtype {want}, got {x.dtype}")
        if x.is_cuda:
            x = x.contiguous()
            return C.c_void_p(x.data_ptr()), 1, x
        x = x.detach().contiguous().numpy()
    a = np.ascontiguousarray(x, dtype=dtype)
    if a.shape != tuple(shape):
        raise ValueError(f"expected shape {tuple(shape)}, got {a.shape}")
    return a.ctypes.data_as(C.c_void_p), 0, a


class Plan:
    """One reconstruction context on one GPU.

    Parameters mirror ``pty_plan_desc``: window ``n``, ``modes``, positions
    ``n_pos``, object shape ``(H, W)``.  ``stream``: a HIP stream handle (an
    int, or a ``torch.cuda.Stream``); None lets the library own its stream.
    """

    def __init__(self, n: int, modes: int, n_pos: int, obj_shape, device: int = 0, stream=None):
        self._lib = L.lib()
        if stream is not None and hasattr(stream, "cuda_stream"):
            stream = stream.cuda_stream
        desc = L.PlanDesc(int(n), int(modes), int(n_pos), int(obj_shape[0]), int(obj_shape[1]),
                          int(device), C.c_void_p(stream) if stream else None, 0)
        out = C.c_void_p()
        st = self._lib.pty_create(C.byref(desc), C.byref(out))
        if st != L.OK:
            raise PtyError(st, self._lib.pty_last_error(None).decode())
        self._ctx = out
        self.n, self.modes, self.n_pos = int(n), int(modes), int(n_pos)
        self.obj_shape = (int(obj_shape[0]), int(obj_shape[1]))

    # -- helpers -----------------------------------------------------------
    def _check(self, st: int) -> None:
        if st != L.OK:
            raise PtyError(st, self._lib.pty_last_error(self._ctx).decode())

    def _live(self):
        if self._ctx is None:
            raise PtyError(L.E_STATE, "plan is closed")
        return self._ctx

    @staticmethod
    def default_params(**overrides) -> L.IterParams:
        p = L.IterParams()
        L.lib().pty_default_params(C.byref(p))
        for k, v in overrides.items():
            if not hasattr(p, k):
                raise TypeError(f"unknown iteration parameter {k!r}")
            setattr(p, k, v)
        return p

    # -- inputs ------------------------------------------------------------
    def load_patterns(self, counts) -> None:
        """Photon counts (J, N, N) float32, zero frequency at (N/2, N/2)."""
        ptr, dev, keep = _ptr(counts, np.float32, (self.n_pos, self.n, self.n))
        self._check(self._lib.pty_load_patterns(self._live(), ptr, dev))
        del keep

    def load_positions(self, yx) -> None:
        """Top-left corners (J, 2) float64 in object pixels."""
        ptr, _, keep = _ptr(yx, np.float64, (self.n_pos, 2))
        self._check(self._lib.pty_load_positions(self._live(), ptr))
        del keep

    def set_object(self, obj) -> None:
        ptr, dev, keep = _ptr(obj, np.complex64, self.obj_shape)
        self._check(self._lib.pty_set_object(self._live(), ptr, dev))
        del keep

    def set_probe(self, probe) -> None:
        ptr, dev, keep = _ptr(probe, np.complex64, (self.modes, self.n, self.n))
        self._check(self._lib.pty_set_probe(self._live(), ptr, dev))
        del keep

    # -- iteration ---------------------------------------------------------
    def iterate(self, algo, n_iter: int = 1, graph: bool = False, ortho_modes: bool = False,
                likelihood: str = "amplitude", **params) -> None:
        """Enqueue ``n_iter`` iterations of 'epie', 'dm' or 'lsqml' (asynchronous).

        graph=True replays captured iterations (PTY_ITER_GRAPH; DM and LSQML);
        ortho_modes=True orthogonalises the probe modes after every iteration
        that updated the probe (PTY_ITER_ORTHO_MODES); likelihood='poisson'
        takes LSQML's exit-wave update from the Poisson likelihood
        (PTY_ITER_POISSON) instead of the modulus projection ('amplitude')."""
        a = ALGOS[algo] if isinstance(algo, str) else int(algo)
        params["flags"] = _flags(params.get("flags", 0), graph, ortho_modes, likelihood)
        p = self.default_params(**params)
        self._check(self._lib.pty_iterate(self._live(), a, int(n_iter), C.byref(p)))

    def autotune(self, algo, cache_path: Optional[str] = None, **params) -> int:
        """Choose the Fourier-pass chunk by timing (see pty_autotune); returns it."""
        a = ALGOS[algo] if isinstance(algo, str) else int(algo)
        p = self.default_params(**params)
        out = C.c_int32()
        self._check(self._lib.pty_autotune(self._live(), a, C.byref(p),
                                           cache_path.encode() if cache_path else None, C.byref(out)))
        return int(out.value)

    def tuning(self) -> tuple:
        """(chunk, probe-sum slice size) chosen by autotune; 0 = the default rule."""
        ch, sl = C.c_int32(), C.c_int32()
        self._check(self._lib.pty_get_tuning(self._live(), C.byref(ch), C.byref(sl)))
        return int(ch.value), int(sl.value)

    def sync(self) -> None:
        self._check(self._lib.pty_sync(self._live()))

    # -- outputs -----------------------------------------------------------
    def _get(self, fn, shape, dtype, out):
        if out is not None:
            ptr, dev, keep = _ptr(out, dtype, shape)
            self._check(fn(self._live(), ptr, dev))
            if dev == 0 and _is_torch(out):
                out.copy_(__import__("torch").from_numpy(keep))
            return out
        a = np.empty(shape, dtype=dtype)
        self._check(fn(self._live(), a.ctypes.data_as(C.c_void_p), 0))
        return a

    def object(self, out=None):
        return self._get(self._lib.pty_get_object, self.obj_shape, np.complex64, out)

    def probe(self, out=None):
        return self._get(self._lib.pty_get_probe, (self.modes, self.n, self.n), np.complex64, out)

    def exit_waves(self, out=None):
        return self._get(self._lib.pty_get_exit_waves, (self.n_pos, self.modes, self.n, self.n),
                         np.complex64, out)

    def errors(self) -> np.ndarray:
        """Amplitude error E of every iteration so far (float64)."""
        cap = 1 << 16
        buf = np.empty(cap, dtype=np.float64)
        n = C.c_int32()
        self._check(self._lib.pty_get_errors(self._live(), buf.ctypes.data_as(C.c_void_p), cap, C.byref(n)))
        return buf[: n.value].copy()

    def guess_probe(self, diameter: float) -> None:
        """Blind start: the probe becomes an aperture guess of the given
        diameter (pixels), scaled to the loaded patterns (pty_guess_probe)."""
        self._check(self._lib.pty_guess_probe(self._live(), float(diameter)))

    def positions(self) -> np.ndarray:
        """Current scan positions (J, 2) float64: as loaded, or as refined."""
        out = np.empty((self.n_pos, 2), dtype=np.float64)
        self._check(self._lib.pty_get_positions(self._live(), out.ctypes.data_as(C.c_void_p)))
        return out

    def set_mask(self, mask) -> None:
        """Detector mask (N x N, centred like the counts, nonzero = measured);
        None measures every pixel again."""
        if mask is None:
            self._check(self._lib.pty_set_mask(self._live(), None))
            return
        m = np.ascontiguousarray(np.asarray(mask) != 0, dtype=np.uint8)
        if m.shape != (self.n, self.n):
            raise ValueError(f"mask must be {self.n} x {self.n}")
        self._check(self._lib.pty_set_mask(self._live(), m.ctypes.data_as(C.c_void_p)))

    def state(self) -> bytes:
        """Checkpoint of what object and probe do not carry (iteration
        counter, error and NRMSE histories, current DM exit waves), for
        `set_state` on a plan of the same shape."""
        n = C.c_size_t()
        self._check(self._lib.pty_get_state(self._live(), None, 0, C.byref(n)))
        buf = np.empty(n.value, dtype=np.uint8)
        self._check(self._lib.pty_get_state(self._live(), buf.ctypes.data_as(C.c_void_p), n.value, C.byref(n)))
        return buf.tobytes()

    def set_state(self, blob: bytes) -> None:
        """Restores a checkpoint from `state`; call after set_object / set_probe."""
        buf = np.frombuffer(blob, dtype=np.uint8)
        self._check(self._lib.pty_set_state(self._live(), buf.ctypes.data_as(C.c_void_p), buf.size))

    def lsqml_steps(self) -> np.ndarray:
        out = np.empty((self.n_pos, 2), dtype=np.float32)
        self._check(self._lib.pty_get_lsqml_steps(self._live(), out.ctypes.data_as(C.c_void_p)))
        return out

    def simulate(self, photons: float = 0.0, out=None):
        """Expected counts (J, N, N), centred; rescales the probe if photons > 0."""
        shape = (self.n_pos, self.n, self.n)
        if out is not None:
            ptr, dev, keep = _ptr(out, np.float32, shape)
            self._check(self._lib.pty_simulate(self._live(), float(photons), ptr, dev))
            return out
        a = np.empty(shape, dtype=np.float32)
        self._check(self._lib.pty_simulate(self._live(), float(photons), a.ctypes.data_as(C.c_void_p), 0))
        return a

    def _dev(self, x, dtype, shape, name):
        """Device pointer of a CUDA tensor with the given layout (adjoint inputs/outputs)."""
        if x is None:
            return None
        if not (_is_torch(x) and x.is_cuda):
            raise TypeError(f"{name} must be a CUDA tensor")
        ptr, _, _ = _ptr(x, dtype, shape)
        if not x.is_contiguous():
            raise ValueError(f"{name} must be contiguous")
        return ptr

    def nll_forward(self, obj, probe, positions=None) -> float:
        """Poisson NLL of the loaded counts for (obj, probe) given as CUDA complex64 tensors;
        ``positions``: (J, 2) float32 CUDA tensor of top-left corners, or None for the loaded ones."""
        loss = C.c_double()
        self._check(self._lib.pty_nll_forward(
            self._live(), self._dev(obj, np.complex64, self.obj_shape, "obj"),
            self._dev(probe, np.complex64, (self.modes, self.n, self.n), "probe"),
            self._dev(positions, np.float32, (self.n_pos, 2), "positions"), C.byref(loss)))
        return loss.value

    def nll_backward(self, obj, probe, grad_out: float = 1.0, g_obj=None, g_probe=None, g_pos=None,
                     positions=None) -> float:
        """Writes grad_out times the NLL gradients into the given CUDA tensors (any may be None);
        ``positions`` as in :meth:`nll_forward`."""
        loss = C.c_double()
        self._check(self._lib.pty_nll_backward(
            self._live(), self._dev(obj, np.complex64, self.obj_shape, "obj"),
            self._dev(probe, np.complex64, (self.modes, self.n, self.n), "probe"),
            self._dev(positions, np.float32, (self.n_pos, 2), "positions"), float(grad_out),
            self._dev(g_obj, np.complex64, self.obj_shape, "g_obj"),
            self._dev(g_probe, np.complex64, (self.modes, self.n, self.n), "g_probe"),
            self._dev(g_pos, np.float32, (self.n_pos, 2), "g_pos"), C.byref(loss)))
        return loss.value

    # -- evaluation and the learned seed --------------------------------------
    def model_error(self) -> float:
        """Amplitude error E of the current object and probe (state unchanged)."""
        v = C.c_double()
        self._check(self._lib.pty_model_error(self._live(), C.byref(v)))
        return v.value

    def set_truth(self, truth, roi_frac: float = 0.3) -> None:
        """Record the NRMSE against `truth` after every iteration (None: stop)."""
        if truth is None:
            self._check(self._lib.pty_set_truth(self._live(), None, 0, 0.0))
            return
        ptr, dev, keep = _ptr(truth, np.complex64, self.obj_shape)
        self._check(self._lib.pty_set_truth(self._live(), ptr, dev, float(roi_frac)))

    def nrmse(self) -> float:
        v = C.c_double()
        self._check(self._lib.pty_nrmse(self._live(), C.byref(v)))
        return v.value

    def nrmse_history(self) -> np.ndarray:
        cap = 1 << 16
        buf = np.empty(cap, dtype=np.float64)
        n = C.c_int32()
        self._check(self._lib.pty_get_nrmse(self._live(), buf.ctypes.data_as(C.c_void_p), cap, C.byref(n)))
        return buf[: n.value].copy()

    def stitch(self, patches, out=None):
        """Stitch (J, 64, 64, 2) amplitude/phase patches (CUDA float32) into an
        object; into `out` (CUDA complex64) if given, else into the plan's object."""
        pp = self._dev(patches, np.float32, (self.n_pos, 64, 64, 2), "patches")
        po = self._dev(out, np.complex64, self.obj_shape, "out")
        self._check(self._lib.pty_stitch(self._live(), pp, po))
        return out

    def seed_object(self, net, batch: int = 4096, stride: int = 1, fallback: bool = True) -> dict:
        """Learned seed of the object from every stride-th loaded pattern (see pty_seed_object)."""
        used = C.c_int32()
        es = C.c_double(float("nan"))
        ef = C.c_double(float("nan"))
        self._check(self._lib.pty_seed_object(self._live(), net._live(), int(batch), int(stride),
                                              1 if fallback else 0, C.byref(used), C.byref(es), C.byref(ef)))
        return {"used_fallback": bool(used.value), "e_seed": es.value, "e_flat": ef.value}

    def training_targets(self, out):
        """Network targets (J, 64, 64, 2) of every (integer) window, into a CUDA tensor."""
        self._check(self._lib.pty_training_targets(
            self._live(), self._dev(out, np.float32, (self.n_pos, self.n // 2, self.n // 2, 2), "out")))
        return out

    def poisson(self, lam, out, seed: int) -> None:
        """out ~ Poisson(lam) elementwise (CUDA float32 tensors of equal shape)."""
        if tuple(lam.shape) != tuple(out.shape):
            raise ValueError("lam and out shapes differ")
        n = int(np.prod(lam.shape))
        self._check(self._lib.pty_poisson(self._live(), self._dev(lam, np.float32, lam.shape, "lam"),
                                          self._dev(out, np.float32, out.shape, "out"), n,
                                          int(seed) & ((1 << 64) - 1)))

    def set_timing(self, enable: bool = True) -> None:
        """Clear the per-family kernel times and enable (or disable) event timing."""
        self._check(self._lib.pty_set_timing(self._live(), 1 if enable else 0))

    def timing(self) -> dict:
        """{family: (milliseconds, launches)} accumulated since set_timing(True)."""
        nf = len(L.TIMING_FAMILIES)
        ms = np.zeros(nf, dtype=np.float64)
        cnt = np.zeros(nf, dtype=np.int64)
        self._check(self._lib.pty_get_timing(self._live(), ms.ctypes.data_as(C.c_void_p),
                                             cnt.ctypes.data_as(C.c_void_p), nf))
        return {f: (float(ms[i]), int(cnt[i])) for i, f in enumerate(L.TIMING_FAMILIES)}

    def mem_bytes(self) -> int:
        v = C.c_size_t()
        self._check(self._lib.pty_mem_bytes(self._live(), C.byref(v)))
        return int(v.value)

    def close(self) -> None:
        if getattr(self, "_ctx", None) is not None:
            self._lib.pty_destroy(self._ctx)
            self._ctx = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Several plans iterated together, each on its own stream (pty_batch_*)."""

    def __init__(self, plans):
        self._lib = L.lib()
        self.plans = list(plans)
        arr = (C.c_void_p * len(self.plans))(*[pl._live().value for pl in self.plans])
        out = C.c_void_p()
        st = self._lib.pty_batch_create(arr, len(self.plans), C.byref(out))
        if st != L.OK:
            raise PtyError(st, self._lib.pty_batch_last_error(None).decode())
        self._b = out

    def _check(self, st: int) -> None:
        if st != L.OK:
            raise PtyError(st, self._lib.pty_batch_last_error(self._b).decode())

    def iterate(self, algo, n_iter: int = 1, graph: bool = False, ortho_modes: bool = False,
                likelihood: str = "amplitude", **params) -> None:
        a = ALGOS[algo] if isinstance(algo, str) else int(algo)
        params["flags"] = _flags(params.get("flags", 0), graph, ortho_modes, likelihood)
        p = Plan.default_params(**params)
        self._check(self._lib.pty_batch_iterate(self._b, a, int(n_iter), C.byref(p)))

    def autotune(self, algo, cache_path: Optional[str] = None, **params) -> None:
        """pty_autotune on every plan of the batch (see Plan.autotune)."""
        a = ALGOS[algo] if isinstance(algo, str) else int(algo)
        p = Plan.default_params(**params)
        self._check(self._lib.pty_batch_autotune(self._b, a, C.byref(p),
                                                 cache_path.encode() if cache_path else None))

    def sync(self) -> None:
        self._check(self._lib.pty_batch_sync(self._b))

    def close(self) -> None:
        if getattr(self, "_b", None) is not None:
            self._lib.pty_batch_destroy(self._b)
            self._b = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def reconstruct(algo: str, counts, positions, obj, probe, n_iter: int, device: int = 0, **params):
    """Whole-mode reconstruction (Sec. 3.2: run without returning between
    iterations); returns (object, probe, errors) as NumPy arrays."""
    counts_shape = tuple(counts.shape)
    with Plan(counts_shape[-1], probe.shape[0], counts_shape[0], obj.shape, device=device) as pl:
        pl.load_patterns(counts)
        pl.load_positions(positions)
        pl.set_object(obj)
        pl.set_probe(probe)
        pl.iterate(algo, n_iter, **params)
        return pl.object(), pl.probe(), pl.errors()


class Domains:
    """One scan split by row into strips, each a context of its own, with the
    object-row halos and the probe sums exchanged between them
    (pty_domains_*; DM and LSQML)."""

    def __init__(self, n: int, modes: int, positions, obj_shape, strips: int, device: int = 0, stream=None):
        self._lib = L.lib()
        if stream is not None and hasattr(stream, "cuda_stream"):
            stream = stream.cuda_stream
        yx = np.ascontiguousarray(positions, dtype=np.float64)
        if yx.ndim != 2 or yx.shape[1] != 2:
            raise ValueError("positions must be (J, 2)")
        desc = L.PlanDesc(int(n), int(modes), int(yx.shape[0]), int(obj_shape[0]), int(obj_shape[1]),
                          int(device), C.c_void_p(stream) if stream else None, 0)
        out = C.c_void_p()
        st = self._lib.pty_domains_create(C.byref(desc), yx.ctypes.data_as(C.c_void_p), int(strips), C.byref(out))
        if st != L.OK:
            raise PtyError(st, self._lib.pty_domains_last_error(None).decode())
        self._d = out
        self.n, self.modes, self.n_pos, self.strips = int(n), int(modes), int(yx.shape[0]), int(strips)
        self.obj_shape = (int(obj_shape[0]), int(obj_shape[1]))

    def _check(self, st: int) -> None:
        if st != L.OK:
            raise PtyError(st, self._lib.pty_domains_last_error(self._d).decode())

    def _live(self):
        if self._d is None:
            raise PtyError(L.E_STATE, "domains are closed")
        return self._d

    def load_patterns(self, counts) -> None:
        ptr, dev, keep = _ptr(counts, np.float32, (self.n_pos, self.n, self.n))
        self._check(self._lib.pty_domains_load_patterns(self._live(), ptr, dev))
        del keep

    def set_object(self, obj) -> None:
        ptr, dev, keep = _ptr(obj, np.complex64, self.obj_shape)
        self._check(self._lib.pty_domains_set_object(self._live(), ptr, dev))
        del keep

    def set_probe(self, probe) -> None:
        ptr, dev, keep = _ptr(probe, np.complex64, (self.modes, self.n, self.n))
        self._check(self._lib.pty_domains_set_probe(self._live(), ptr, dev))
        del keep

    def iterate(self, algo, n_iter: int = 1, **params) -> None:
        a = ALGOS[algo] if isinstance(algo, str) else int(algo)
        p = Plan.default_params(**params)
        self._check(self._lib.pty_domains_iterate(self._live(), a, int(n_iter), C.byref(p)))

    def object(self) -> np.ndarray:
        a = np.empty(self.obj_shape, dtype=np.complex64)
        self._check(self._lib.pty_domains_get_object(self._live(), a.ctypes.data_as(C.c_void_p), 0))
        return a

    def probe(self) -> np.ndarray:
        a = np.empty((self.modes, self.n, self.n), dtype=np.complex64)
        self._check(self._lib.pty_domains_get_probe(self._live(), a.ctypes.data_as(C.c_void_p), 0))
        return a

    def errors(self) -> np.ndarray:
        cap = 1 << 16
        buf = np.empty(cap, dtype=np.float64)
        n = C.c_int32()
        self._check(self._lib.pty_domains_get_errors(self._live(), buf.ctypes.data_as(C.c_void_p), cap,
                                                     C.byref(n)))
        return buf[: n.value].copy()

    def strip(self, s: int) -> dict:
        """Rows held [lo, hi), rows owned [own_lo, own_hi) and positions of strip s."""
        info = (C.c_int32 * 5)()
        self._check(self._lib.pty_domains_strip(self._live(), int(s), info))
        return {"lo": info[0], "hi": info[1], "own_lo": info[2], "own_hi": info[3], "positions": info[4]}

    def traffic(self) -> tuple:
        """(halo bytes, probe-message bytes) sent so far."""
        h, p = C.c_uint64(), C.c_uint64()
        self._check(self._lib.pty_domains_traffic(self._live(), C.byref(h), C.byref(p)))
        return int(h.value), int(p.value)

    def sync(self) -> None:
        self._check(self._lib.pty_domains_sync(self._live()))

    def close(self) -> None:
        if getattr(self, "_d", None) is not None:
            self._lib.pty_domains_destroy(self._d)
            self._d = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        self.close()
