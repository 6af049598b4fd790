"""ctypes binding of libmagpie.so (C ABI declared in include/magpie.h).

Argument marshalling only: every step of the solver runs in the HIP library.
NumPy arrays are passed as host pointers; torch tensors that live on a GPU
are passed as device pointers (``data_ptr()``), which the library reads in
stream order on the context's stream.
"""

from __future__ import annotations

import ctypes
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "lib", "libmagpie.so")

MAGPIE_OK = 0
ERRORS = {
    -1: "INVALID_ARG", -2: "BAD_STATE", -3: "OOM", -4: "HIP", -5: "NUMERIC", -6: "UNSUPPORTED",
}
C64, C128 = 0, 1
UPDATE_PROBE = 0x1
GRAPH = 0x2
PHASE_RECYCLE = 0x4
PROBE_ALTERNATE = 0x8
PERSISTENT = 0x10
W_F32, W_BF16 = 0, 1
COARSE_C64, COARSE_C128, COARSE_LOGPOLAR = 0, 1, 2

_lib = None


class MagpieError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code
        self.name = ERRORS.get(code, str(code))


def _bind(lib):
    vp, i, d, u32, u64 = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_uint32, ctypes.c_uint64
    sig = {
        "magpie_last_error": (ctypes.c_char_p, []),
        "magpie_create": (i, [ctypes.POINTER(vp), i, i, i, i, d, i, vp]),
        "magpie_destroy": (i, [vp]),
        "magpie_set_probe": (i, [vp, vp, i, i]),
        "magpie_set_regularization": (i, [vp, d, vp]),
        "magpie_set_positions": (i, [vp, i, vp]),
        "magpie_load_intensities": (i, [vp, vp, i, i]),
        "magpie_set_object": (i, [vp, vp, i, i]),
        "magpie_run_epochs": (i, [vp, i, i, u64, vp]),
        "magpie_run_minibatch": (i, [vp, i, vp]),
        "magpie_run_epochs_noalloc": (i, [vp, i, i, u64]),
        "magpie_objective": (i, [vp, ctypes.POINTER(d), ctypes.POINTER(d)]),
        "magpie_get_step_phi": (i, [vp, vp]),
        "magpie_get_object": (i, [vp, vp, i, i]),
        "magpie_get_probe": (i, [vp, vp, i, i]),
        "magpie_sync": (i, [vp]),
        "magpie_set_flags": (i, [vp, u32, d]),
        "magpie_forward_model": (i, [vp, vp, i, vp, i]),
        "magpie_permutation": (i, [u64, u64, i, vp]),
        "magpie_get_epoch_index": (i, [vp, ctypes.POINTER(u64)]),
        "magpie_set_epoch_index": (i, [vp, u64]),
        "magpie_set_timing": (i, [vp, i]),
        "magpie_list_plans": (i, [i, vp, i]),
        "magpie_get_launch_times": (i, [vp, i, vp, vp, i]),
        "magpie_set_tuning": (i, [vp, i, i]),
        "magpie_get_tuning": (i, [vp, ctypes.POINTER(i), ctypes.POINTER(i)]),
        "magpie_autotune": (i, [vp, i, i, ctypes.POINTER(d), ctypes.POINTER(d)]),
        "magpie_autotune_batch": (i, [vp, vp, i, i, ctypes.POINTER(ctypes.c_int32), vp]),
        "magpie_run_epochs_multi": (i, [ctypes.POINTER(vp), i, i, ctypes.POINTER(i), u64]),
        "magpie_get_timing": (i, [vp, ctypes.POINTER(d), ctypes.POINTER(d), ctypes.POINTER(ctypes.c_int64),
                                  ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64)]),
        # learned start (include/magpie_learned.h)
        "magpie_cnn_create": (i, [ctypes.POINTER(vp), i, i, i, i, i, i, vp]),
        "magpie_cnn_destroy": (i, [vp]),
        "magpie_cnn_num_params": (i, [vp, ctypes.POINTER(ctypes.c_int64)]),
        "magpie_cnn_set_params": (i, [vp, vp, i]),
        "magpie_cnn_get_params": (i, [vp, vp, i]),
        "magpie_cnn_get_grads": (i, [vp, vp, i]),
        "magpie_cnn_forward": (i, [vp, vp, vp, i, i]),
        "magpie_cnn_loss": (i, [vp, vp, vp, i, i, i, ctypes.POINTER(d)]),
        "magpie_cnn_backward": (i, [vp, vp, i, i]),
        "magpie_cnn_adam_step": (i, [vp, ctypes.c_float, ctypes.c_float, ctypes.c_float, ctypes.c_float]),
        "magpie_cnn_sync": (i, [vp]),
        "magpie_input_map": (i, [vp, i, vp, i]),
        "magpie_set_object_from_coarse": (i, [vp, vp, i, i, i]),
        "magpie_restrict_object": (i, [vp, i, i, i, vp, vp]),
        "magpie_learned_start": (i, [vp, vp, ctypes.POINTER(d), ctypes.POINTER(d), ctypes.POINTER(i)]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


def load_library(path: str | None = None):
    """Load the built HIP library; raises if it is missing (there is no fallback)."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise RuntimeError(f"libmagpie.so not built at {p}; run `python -m paper_2504_10118_amd.build`")
    # One HIP runtime per process: torch ships its own libamdhip64 under the same
    # soname, so loading torch's libraries first lets the library bind to that copy
    # (loading ours first would make torch load a second runtime that cannot
    # initialise the GPU).  Importing torch does not touch the GPU.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = _bind(ctypes.CDLL(p))
    if path is None:
        _lib = lib
    return lib


def _check(rc: int):
    if rc != MAGPIE_OK:
        raise MagpieError(rc, _lib.magpie_last_error().decode())


def _is_torch(x):
    return type(x).__module__.startswith("torch")


def _ptr(x, dtype, shape=None):
    """(pointer, on_device, keepalive) for a numpy array or torch tensor."""
    if _is_torch(x):
        import torch
        tdt = {np.complex64: torch.complex64, np.complex128: torch.complex128,
               np.float32: torch.float32, np.float64: torch.float64, np.int32: torch.int32}[dtype]
        if x.is_cuda:
            if x.dtype != tdt or not x.is_contiguous():
                raise ValueError(f"device tensor must be contiguous {tdt}")
            if shape is not None and tuple(x.shape) != tuple(shape):
                raise ValueError(f"expected shape {shape}, got {tuple(x.shape)}")
            return ctypes.c_void_p(x.data_ptr()), 1, x
        x = x.detach().numpy()
    a = np.ascontiguousarray(x, dtype=dtype)
    if shape is not None and a.shape != tuple(shape):
        raise ValueError(f"expected shape {shape}, got {a.shape}")
    return a.ctypes.data_as(ctypes.c_void_p), 0, a


def permutation(seed: int, epoch: int, n: int) -> np.ndarray:
    """The library's splitmix64 Fisher-Yates permutation for (seed, epoch)."""
    lib = load_library()
    out = np.empty(n, dtype=np.int32)
    _check(lib.magpie_permutation(seed, epoch, n, out.ctypes.data_as(ctypes.c_void_p)))
    return out


def list_plans(m: int) -> list[int]:
    """Compiled FFT plans of the step kernel for probe side m (threads per 1-D transform), default first."""
    lib = load_library()
    buf = (ctypes.c_int32 * 8)()
    n = lib.magpie_list_plans(m, ctypes.cast(buf, ctypes.c_void_p), 8)
    if n < 0:
        _check(n)
    return [buf[i] for i in range(n)]


def run_epochs_multi(contexts, n_epochs: int, batch, seed: int = 0):
    """Advance several independent reconstructions together (one launch per plan / tile group per round)."""
    lib = load_library()
    cs = list(contexts)
    if isinstance(batch, int):
        batch = [batch] * len(cs)
    hs = (ctypes.c_void_p * len(cs))(*[c._h.value for c in cs])
    bs = (ctypes.c_int * len(cs))(*[int(b) for b in batch])
    _check(lib.magpie_run_epochs_multi(hs, len(cs), n_epochs, bs, seed))


class Magpie:
    """One reconstruction context (object n_rows x n_cols, probe m x m, L grids)."""

    def __init__(self, n_rows: int, n_cols: int, m: int, levels: int, alpha: float,
                 device: int = 0, stream=None):
        self.lib = load_library()
        self.n_rows, self.n_cols, self.m, self.levels = n_rows, n_cols, m, levels
        self.n_pos = 0
        h = ctypes.c_void_p()
        st = ctypes.c_void_p(stream) if stream is not None else None
        _check(self.lib.magpie_create(ctypes.byref(h), n_rows, n_cols, m, levels, float(alpha), device, st))
        self._h = h

    # -- lifetime
    def close(self):
        if getattr(self, "_h", None):
            self.lib.magpie_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # -- inputs
    def set_probe(self, probe):
        dt = np.complex128 if getattr(probe, "dtype", None) in (np.complex128, "complex128") or \
            str(getattr(probe, "dtype", "")) == "torch.complex128" else np.complex64
        p, dev, keep = _ptr(probe, dt, (self.m, self.m))
        _check(self.lib.magpie_set_probe(self._h, p, C128 if dt is np.complex128 else C64, dev))

    def set_regularization(self, alpha: float = 0.0, u=None):
        if u is None:
            _check(self.lib.magpie_set_regularization(self._h, float(alpha), None))
        else:
            a = np.ascontiguousarray(u, dtype=np.float64).reshape(self.m, self.m)
            _check(self.lib.magpie_set_regularization(self._h, float(alpha), a.ctypes.data_as(ctypes.c_void_p)))

    def set_positions(self, offsets):
        a = np.ascontiguousarray(offsets, dtype=np.int32)
        if a.ndim != 2 or a.shape[1] != 2:
            raise ValueError("offsets must be [N, 2]")
        _check(self.lib.magpie_set_positions(self._h, a.shape[0], a.ctypes.data_as(ctypes.c_void_p)))
        self.n_pos = a.shape[0]

    def load_intensities(self, d, is_sqrt: bool = False):
        p, dev, keep = _ptr(d, np.float32, (self.n_pos, self.m, self.m))
        _check(self.lib.magpie_load_intensities(self._h, p, int(bool(is_sqrt)), dev))
        self._keep_d = keep if dev else None

    def set_object(self, z):
        dt = np.complex128 if str(getattr(z, "dtype", "")) in ("complex128", "torch.complex128") else np.complex64
        p, dev, keep = _ptr(z, dt, (self.n_rows, self.n_cols))
        _check(self.lib.magpie_set_object(self._h, p, C128 if dt is np.complex128 else C64, dev))
        self._keep_z = keep if dev else None

    def set_flags(self, flags: int, beta: float = 0.0):
        _check(self.lib.magpie_set_flags(self._h, flags, float(beta)))

    # -- solver
    def run_epochs(self, n_epochs: int, batch: int, seed: int = 0, order=None):
        if order is None:
            _check(self.lib.magpie_run_epochs(self._h, n_epochs, batch, seed, None))
        else:
            o = np.ascontiguousarray(order, dtype=np.int32).reshape(n_epochs, self.n_pos)
            _check(self.lib.magpie_run_epochs(self._h, n_epochs, batch, seed, o.ctypes.data_as(ctypes.c_void_p)))

    def run_epochs_noalloc(self, n_epochs: int, batch: int, seed: int = 0):
        """run_epochs with the library's permutations, taking no device allocation (fixed scratch)."""
        _check(self.lib.magpie_run_epochs_noalloc(self._h, n_epochs, batch, seed))

    def run_minibatch(self, positions):
        """One minibatch step over exactly these (distinct) positions; the epoch counter is kept."""
        a = np.ascontiguousarray(positions, dtype=np.int32).ravel()
        _check(self.lib.magpie_run_minibatch(self._h, int(a.size), a.ctypes.data_as(ctypes.c_void_p)))

    def objective(self):
        phi, st = ctypes.c_double(), ctypes.c_double()
        _check(self.lib.magpie_objective(self._h, ctypes.byref(phi), ctypes.byref(st)))
        return phi.value, st.value

    def step_phi(self):
        out = np.empty(self.n_pos, dtype=np.float64)
        _check(self.lib.magpie_get_step_phi(self._h, out.ctypes.data_as(ctypes.c_void_p)))
        return out

    def sync(self):
        _check(self.lib.magpie_sync(self._h))

    @property
    def epoch_index(self) -> int:
        v = ctypes.c_uint64()
        _check(self.lib.magpie_get_epoch_index(self._h, ctypes.byref(v)))
        return v.value

    @epoch_index.setter
    def epoch_index(self, value: int):
        _check(self.lib.magpie_set_epoch_index(self._h, int(value)))

    def set_timing(self, enable: bool = True):
        _check(self.lib.magpie_set_timing(self._h, int(bool(enable))))

    def get_timing(self) -> dict:
        """Summed HIP-event times of the kernels launched since the last read (ms)."""
        sm, am = ctypes.c_double(), ctypes.c_double()
        sl, al, pos = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        _check(self.lib.magpie_get_timing(self._h, ctypes.byref(sm), ctypes.byref(am), ctypes.byref(sl),
                                          ctypes.byref(al), ctypes.byref(pos)))
        return {"step_ms": sm.value, "accum_ms": am.value, "step_launches": sl.value,
                "accum_launches": al.value, "positions": pos.value}

    def launch_times(self, kind: int):
        """(durations in us, positions) of the recorded launches of the step (0) or
        accumulation (1) kernel since timing was last read; does not reset them."""
        n = self.lib.magpie_get_launch_times(self._h, kind, None, None, 0)
        if n < 0:
            _check(n)
        us = np.empty(n, dtype=np.float64)
        pos = np.empty(n, dtype=np.int32)
        if n:
            _check(min(0, self.lib.magpie_get_launch_times(self._h, kind, us.ctypes.data_as(ctypes.c_void_p),
                                                           pos.ctypes.data_as(ctypes.c_void_p), n)))
        return us, pos

    def set_tuning(self, threads_per_transform: int = 0, tile_rows: int = 0):
        _check(self.lib.magpie_set_tuning(self._h, threads_per_transform, tile_rows))

    def get_tuning(self):
        rb, th = ctypes.c_int(), ctypes.c_int()
        _check(self.lib.magpie_get_tuning(self._h, ctypes.byref(rb), ctypes.byref(th)))
        return rb.value, th.value

    def autotune(self, batch: int, trial_epochs: int = 3):
        """Pick the fastest FFT plan and tile height on this context's data; returns (plan, tile, step_us, acc_us)."""
        su, au = ctypes.c_double(), ctypes.c_double()
        _check(self.lib.magpie_autotune(self._h, batch, trial_epochs, ctypes.byref(su), ctypes.byref(au)))
        rb, th = self.get_tuning()
        return rb, th, su.value, au.value

    def autotune_batch(self, candidates, trial_epochs: int = 3):
        """Pick the minibatch size with the fastest objective decrease from the current state;
        returns (best, rates) with rates[i] the objective decrease per second of candidates[i]."""
        c = np.ascontiguousarray(candidates, dtype=np.int32)
        rates = np.zeros(len(c), dtype=np.float64)
        best = ctypes.c_int32()
        _check(self.lib.magpie_autotune_batch(self._h, c.ctypes.data_as(ctypes.c_void_p), len(c), trial_epochs,
                                              ctypes.byref(best), rates.ctypes.data_as(ctypes.c_void_p)))
        return int(best.value), rates

    # -- outputs
    def get_object(self, out=None, dtype=np.complex64):
        if out is None:
            out = np.empty((self.n_rows, self.n_cols), dtype=dtype)
        dt = np.complex128 if str(out.dtype) in ("complex128", "torch.complex128") else np.complex64
        if _is_torch(out) and out.is_cuda:
            _check(self.lib.magpie_get_object(self._h, ctypes.c_void_p(out.data_ptr()),
                                              C128 if dt is np.complex128 else C64, 1))
            return out
        _check(self.lib.magpie_get_object(self._h, out.ctypes.data_as(ctypes.c_void_p),
                                          C128 if dt is np.complex128 else C64, 0))
        return out

    def get_probe(self, dtype=np.complex64):
        out = np.empty((self.m, self.m), dtype=dtype)
        _check(self.lib.magpie_get_probe(self._h, out.ctypes.data_as(ctypes.c_void_p),
                                         C128 if dtype is np.complex128 else C64, 0))
        return out

    # -- learned start
    def input_map(self, side: int, out=None):
        """Network input map [4, side, side] (float32) from this context's intensities."""
        if out is not None and _is_torch(out) and out.is_cuda:
            _check(self.lib.magpie_input_map(self._h, side, ctypes.c_void_p(out.data_ptr()), 1))
            return out
        res = np.empty((4, side, side), dtype=np.float32)
        _check(self.lib.magpie_input_map(self._h, side, res.ctypes.data_as(ctypes.c_void_p), 0))
        return res

    def set_object_from_coarse(self, coarse, fmt: int = COARSE_C64):
        """Object <- coarse object copied into f x f blocks (f = object side / coarse side)."""
        if fmt == COARSE_LOGPOLAR:
            p, dev, keep = _ptr(coarse, np.float32)
            side = int(coarse.shape[-1])
        else:
            p, dev, keep = _ptr(coarse, np.complex128 if fmt == COARSE_C128 else np.complex64)
            side = int(coarse.shape[-1])
        _check(self.lib.magpie_set_object_from_coarse(self._h, p, side, fmt, dev))

    def learned_start(self, net: "CNN"):
        """Learned start with the flat-start fallback; returns (used, phi_learned, phi_flat)."""
        pl, pf, used = ctypes.c_double(), ctypes.c_double(), ctypes.c_int()
        _check(self.lib.magpie_learned_start(self._h, net._h, ctypes.byref(pl), ctypes.byref(pf), ctypes.byref(used)))
        return bool(used.value), pl.value, pf.value

    def forward_model(self, z, out=None):
        p, dev, keep = _ptr(z, np.complex64, (self.n_rows, self.n_cols))
        if out is not None and _is_torch(out) and out.is_cuda:
            _check(self.lib.magpie_forward_model(self._h, p, dev, ctypes.c_void_p(out.data_ptr()), 1))
            return out
        res = np.empty((self.n_pos, self.m, self.m), dtype=np.float32)
        _check(self.lib.magpie_forward_model(self._h, p, dev, res.ctypes.data_as(ctypes.c_void_p), 0))
        return res


def restrict_object(z, times: int, out=None, stream=None):
    """Whole-object restriction (f x f block means, f = 2**times) of a complex64 device tensor."""
    import torch
    if not (_is_torch(z) and z.is_cuda and z.dtype == torch.complex64 and z.is_contiguous()):
        raise ValueError("z must be a contiguous complex64 device tensor")
    lib = load_library()
    nr, nc = int(z.shape[-2]), int(z.shape[-1])
    f = 1 << times
    lead = tuple(z.shape[:-2])
    if out is None:
        out = torch.empty(lead + (nr // f, nc // f), dtype=torch.complex64, device=z.device)
    st = ctypes.c_void_p(stream if stream is not None else torch.cuda.current_stream(z.device).cuda_stream)
    zz = z.reshape(-1, nr, nc)
    oo = out.reshape(-1, nr // f, nc // f)
    for b in range(zz.shape[0]):
        _check(lib.magpie_restrict_object(ctypes.c_void_p(zz[b].data_ptr()), nr, nc, times,
                                          ctypes.c_void_p(oo[b].data_ptr()), st))
    return out


class CNN:
    """Coarse-object network of the learned start (5 conv layers, width 32, FP32 or BF16 weights)."""

    def __init__(self, in_ch: int = 4, side: int = 64, max_batch: int = 32, weight_dtype: int = W_F32,
                 device: int = 0, stream=None):
        self.lib = load_library()
        self.in_ch, self.side, self.max_batch = in_ch, side, max_batch
        h = ctypes.c_void_p()
        st = ctypes.c_void_p(stream) if stream is not None else None
        _check(self.lib.magpie_cnn_create(ctypes.byref(h), in_ch, 32, side, max_batch, weight_dtype, device, st))
        self._h = h
        n = ctypes.c_int64()
        _check(self.lib.magpie_cnn_num_params(self._h, ctypes.byref(n)))
        self.n_params = n.value

    def close(self):
        if getattr(self, "_h", None):
            self.lib.magpie_cnn_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_params(self, params):
        p, dev, keep = _ptr(params, np.float32, (self.n_params,))
        _check(self.lib.magpie_cnn_set_params(self._h, p, dev))
        self._keep_p = keep if dev else None

    def get_params(self) -> np.ndarray:
        out = np.empty(self.n_params, dtype=np.float32)
        _check(self.lib.magpie_cnn_get_params(self._h, out.ctypes.data_as(ctypes.c_void_p), 0))
        return out

    def get_grads(self) -> np.ndarray:
        out = np.empty(self.n_params, dtype=np.float32)
        _check(self.lib.magpie_cnn_get_grads(self._h, out.ctypes.data_as(ctypes.c_void_p), 0))
        return out

    def forward(self, x, out=None):
        nb = int(x.shape[0])
        s2 = 2 * self.side
        p, dev, keep = _ptr(x, np.float32, (nb, self.in_ch, self.side, self.side))
        if dev:
            if out is None:
                _check(self.lib.magpie_cnn_forward(self._h, p, None, nb, 1))
                return None
            _check(self.lib.magpie_cnn_forward(self._h, p, ctypes.c_void_p(out.data_ptr()), nb, 1))
            return out
        res = np.empty((nb, 2, s2, s2), dtype=np.float32)
        _check(self.lib.magpie_cnn_forward(self._h, p, res.ctypes.data_as(ctypes.c_void_p), nb, 0))
        return res

    def loss(self, target, mask, align_phase: bool = False) -> float:
        nb = int(target.shape[0])
        s2 = 2 * self.side
        pt, dev, kt = _ptr(target, np.complex64, (nb, s2, s2))
        pm, devm, km = _ptr(mask, np.float32, (s2, s2))
        if dev != devm:
            raise ValueError("target and mask must both be host arrays or both device tensors")
        out = ctypes.c_double()
        _check(self.lib.magpie_cnn_loss(self._h, pt, pm, nb, int(bool(align_phase)), dev, ctypes.byref(out)))
        return out.value

    def backward(self, dy=None, nbatch=None):
        if dy is None:
            _check(self.lib.magpie_cnn_backward(self._h, None, int(nbatch), 0))
            return
        nb = int(dy.shape[0])
        s2 = 2 * self.side
        p, dev, keep = _ptr(dy, np.float32, (nb, 2, s2, s2))
        _check(self.lib.magpie_cnn_backward(self._h, p, nb, dev))

    def adam_step(self, lr: float = 1e-3, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8):
        _check(self.lib.magpie_cnn_adam_step(self._h, lr, beta1, beta2, eps))

    def sync(self):
        _check(self.lib.magpie_cnn_sync(self._h))
