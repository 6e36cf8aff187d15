"""Python binding of the gfx950 Super Smoother period search (``libssgpu.so``).

Argument marshalling only: every step of the search runs in the HIP library
behind the C ABI of ``include/ssgpu.h``.  PyTorch supplies device memory and
the stream; tensors are passed as raw device pointers.  Importing this module
does not touch the GPU; the first call loads the library and fails loudly if
it has not been built (``python -m paper_2111_07396_amd.build``).
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libssgpu.so")

SS_OK = 0
SS_ERR_INVALID_ARG, SS_ERR_HIP, SS_ERR_OOM, SS_ERR_UNSUPPORTED = -1, -2, -3, -4
SS_ERR_INVARIANT = -5
SS_FLAG_CHECK_INVARIANTS, SS_FLAG_CHECK_SELFTEST = 1, 2
SS_FP64, SS_FP32C = 0, 1
SS_METHOD_SS, SS_METHOD_SSSP, SS_METHOD_SSSP_GV = 0, 1, 2
OBJ_OK, OBJ_TOO_FEW, OBJ_BAD_ERR, OBJ_NONFINITE, OBJ_CONST_MAG = 0, 1, 2, 3, 4
OBJ_TOO_LONG, OBJ_BAD_RANGE = 5, 6
MAX_POINTS = 4096

EXPORTED = ("ss_params_default", "ss_ctx_create", "ss_ctx_destroy", "ss_periodogram",
            "sssp_periodogram", "ss_best_period", "ss_num_shapes", "ss_shape_info",
            "ss_ctx_set_shape", "ss_ctx_set_tile", "ss_ctx_set_timing", "ss_ctx_trial_kernel_ms",
            "ss_last_error", "ss_version", "ss_bin_table", "ss_enc_num_params", "ss_enc_forward",
            "ss_enc_train_grad", "ss_adam_step", "ss_refine_best_period",
            "ss_learned_best_period", "ss_bin_scores", "ss_method_periodogram",
            "ss_pdm_periodogram", "ss_model_create", "ss_model_destroy", "ss_model_info",
            "ss_model_save", "ss_model_load", "ss_model_file_write", "ss_model_file_read",
            "ss_train_step", "ss_best_period_learned", "ss_model_copy_params",
            "ss_shared_periodogram", "ss_shared_best_period", "ss_plan_batches",
            "ss_periodogram_batched", "ss_best_period_noalloc", "ss_ctx_set_concurrency",
            "ss_ctx_check_counts")
ENC_PARAMS = 145536
ENC_BINS = 1024


def shapes():
    """[(nw, ppl), ...] trial-group shapes built into the library."""
    lib = load_library()
    out = []
    for i in range(lib.ss_num_shapes()):
        nw, ppl = ctypes.c_int32(), ctypes.c_int32()
        lib.ss_shape_info(i, ctypes.byref(nw), ctypes.byref(ppl))
        out.append((nw.value, ppl.value))
    return out


class SSError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"ssgpu error {code}: {msg}")
        self.code = code


class _Grid(ctypes.Structure):
    _fields_ = [("f_min", ctypes.c_double), ("f_max", ctypes.c_double),
                ("n_freq", ctypes.c_int64)]


class _Params(ctypes.Structure):
    _fields_ = [("span_min", ctypes.c_double), ("span_mid", ctypes.c_double),
                ("span_max", ctypes.c_double), ("alpha", ctypes.c_double),
                ("fixed_span", ctypes.c_double), ("precision", ctypes.c_int32),
                ("flags", ctypes.c_int32)]


class _SharedCatalog(ctypes.Structure):
    _fields_ = [("n_obj", ctypes.c_int64), ("n_points", ctypes.c_int64),
                ("t", ctypes.c_void_p), ("y", ctypes.c_void_p), ("e", ctypes.c_void_p)]


class _Catalog(ctypes.Structure):
    _fields_ = [("n_obj", ctypes.c_int64), ("n_points", ctypes.c_int64),
                ("offsets", ctypes.c_void_p),
                ("t", ctypes.c_void_p), ("y", ctypes.c_void_p), ("e", ctypes.c_void_p)]


_lib = None
_SINK = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64, ctypes.c_void_p,
                         ctypes.c_void_p)


def load_library(path: str = LIB_PATH):
    """Loads libssgpu.so (raises if it is missing: there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is not built; run `python -m paper_2111_07396_amd.build`")
    lib = ctypes.CDLL(path)
    vp, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32
    lib.ss_params_default.argtypes = [ctypes.POINTER(_Params)]
    lib.ss_params_default.restype = None
    lib.ss_ctx_create.argtypes = [ctypes.c_int, ctypes.POINTER(vp)]
    lib.ss_ctx_create.restype = ctypes.c_int
    lib.ss_ctx_destroy.argtypes = [vp]
    lib.ss_ctx_destroy.restype = None
    for name in ("ss_periodogram", "sssp_periodogram"):
        f = getattr(lib, name)
        f.argtypes = [vp, ctypes.POINTER(_Catalog), ctypes.POINTER(_Grid), ctypes.POINTER(_Params),
                      vp, vp, vp]
        f.restype = ctypes.c_int
    lib.ss_method_periodogram.argtypes = [vp, i32, ctypes.POINTER(_Catalog),
                                          ctypes.POINTER(_Grid), ctypes.POINTER(_Params), vp,
                                          vp, vp]
    lib.ss_method_periodogram.restype = ctypes.c_int
    lib.ss_pdm_periodogram.argtypes = [vp, i32, ctypes.POINTER(_Catalog), ctypes.POINTER(_Grid),
                                       ctypes.POINTER(_Params), i32, vp, vp, vp, vp]
    lib.ss_pdm_periodogram.restype = ctypes.c_int
    lib.ss_best_period.argtypes = [vp, i32, ctypes.POINTER(_Catalog), ctypes.POINTER(_Grid),
                                   ctypes.POINTER(_Params), vp, vp, vp, vp, vp]
    lib.ss_best_period.restype = ctypes.c_int
    lib.ss_best_period_noalloc.argtypes = lib.ss_best_period.argtypes
    lib.ss_best_period_noalloc.restype = ctypes.c_int
    lib.ss_num_shapes.argtypes = []
    lib.ss_num_shapes.restype = ctypes.c_int
    lib.ss_shape_info.argtypes = [ctypes.c_int, ctypes.POINTER(i32), ctypes.POINTER(i32)]
    lib.ss_shape_info.restype = ctypes.c_int
    lib.ss_ctx_set_shape.argtypes = [vp, i32, i32, i32]
    lib.ss_ctx_set_shape.restype = ctypes.c_int
    lib.ss_ctx_set_concurrency.argtypes = [vp, i32]
    lib.ss_ctx_set_concurrency.restype = ctypes.c_int
    lib.ss_ctx_set_tile.argtypes = [vp, i32]
    lib.ss_ctx_set_tile.restype = ctypes.c_int
    lib.ss_ctx_set_timing.argtypes = [vp, ctypes.c_int]
    lib.ss_ctx_set_timing.restype = ctypes.c_int
    lib.ss_ctx_trial_kernel_ms.argtypes = [vp, ctypes.POINTER(ctypes.c_double),
                                           ctypes.POINTER(ctypes.c_int32)]
    lib.ss_ctx_trial_kernel_ms.restype = ctypes.c_int
    lib.ss_ctx_check_counts.argtypes = [vp, ctypes.POINTER(ctypes.c_int64)]
    lib.ss_ctx_check_counts.restype = ctypes.c_int
    lib.ss_last_error.argtypes = []
    lib.ss_last_error.restype = ctypes.c_char_p
    lib.ss_version.argtypes = []
    lib.ss_version.restype = ctypes.c_int
    lib.ss_bin_table.argtypes = [ctypes.POINTER(_Grid), vp]
    lib.ss_bin_table.restype = ctypes.c_int
    lib.ss_enc_num_params.argtypes = []
    lib.ss_enc_num_params.restype = ctypes.c_int
    lib.ss_enc_forward.argtypes = [vp, ctypes.POINTER(_Catalog), ctypes.POINTER(_Grid), vp, vp,
                                   vp, vp, vp]
    lib.ss_enc_forward.restype = ctypes.c_int
    lib.ss_enc_train_grad.argtypes = [vp, ctypes.POINTER(_Catalog), ctypes.POINTER(_Grid), vp,
                                      vp, vp, vp, vp, vp]
    lib.ss_enc_train_grad.restype = ctypes.c_int
    lib.ss_adam_step.argtypes = [vp, vp, vp, vp, i64, i32, ctypes.c_float, ctypes.c_float,
                                 ctypes.c_float, ctypes.c_float, vp]
    lib.ss_adam_step.restype = ctypes.c_int
    lib.ss_refine_best_period.argtypes = [vp, i32, ctypes.POINTER(_Catalog),
                                          ctypes.POINTER(_Grid), ctypes.POINTER(_Params), vp,
                                          i32, i32, i32, vp, vp, vp, vp, vp]
    lib.ss_refine_best_period.restype = ctypes.c_int
    lib.ss_learned_best_period.argtypes = [vp, i32, ctypes.POINTER(_Catalog),
                                           ctypes.POINTER(_Grid), ctypes.POINTER(_Params), vp,
                                           ctypes.c_float, i32, i32, i32, vp, vp, vp, vp, vp]
    lib.ss_learned_best_period.restype = ctypes.c_int
    lib.ss_bin_scores.argtypes = [vp, ctypes.POINTER(_Catalog), ctypes.POINTER(_Grid), vp, vp,
                                  vp]
    lib.ss_bin_scores.restype = ctypes.c_int
    lib.ss_shared_periodogram.argtypes = [vp, i32, ctypes.POINTER(_SharedCatalog),
                                          ctypes.POINTER(_Grid), ctypes.POINTER(_Params), vp, vp,
                                          vp]
    lib.ss_shared_periodogram.restype = ctypes.c_int
    lib.ss_shared_best_period.argtypes = [vp, i32, ctypes.POINTER(_SharedCatalog),
                                          ctypes.POINTER(_Grid), ctypes.POINTER(_Params), vp, vp,
                                          vp, vp, vp]
    lib.ss_shared_best_period.restype = ctypes.c_int
    lib.ss_plan_batches.argtypes = [vp, i64, i64, ctypes.POINTER(_Grid), i32, i32,
                                    ctypes.c_double, i64, ctypes.POINTER(i64),
                                    ctypes.POINTER(i64)]
    lib.ss_plan_batches.restype = ctypes.c_int
    lib.ss_periodogram_batched.argtypes = [vp, i32, ctypes.POINTER(_Catalog),
                                           ctypes.POINTER(_Grid), ctypes.POINTER(_Params), vp,
                                           i64, _SINK, vp, vp, vp]
    lib.ss_periodogram_batched.restype = ctypes.c_int
    fp = ctypes.POINTER(ctypes.c_float)
    lib.ss_model_create.argtypes = [vp, ctypes.POINTER(_Grid), fp, ctypes.POINTER(vp)]
    lib.ss_model_create.restype = ctypes.c_int
    lib.ss_model_destroy.argtypes = [vp]
    lib.ss_model_destroy.restype = None
    lib.ss_model_info.argtypes = [vp, ctypes.POINTER(_Grid), ctypes.POINTER(i32),
                                  ctypes.POINTER(vp)]
    lib.ss_model_info.restype = ctypes.c_int
    lib.ss_model_save.argtypes = [vp, ctypes.c_char_p]
    lib.ss_model_save.restype = ctypes.c_int
    lib.ss_model_load.argtypes = [vp, ctypes.c_char_p, ctypes.POINTER(vp)]
    lib.ss_model_load.restype = ctypes.c_int
    lib.ss_model_file_write.argtypes = [ctypes.c_char_p, ctypes.POINTER(_Grid), i32, fp, fp, fp]
    lib.ss_model_file_write.restype = ctypes.c_int
    lib.ss_model_file_read.argtypes = [ctypes.c_char_p, ctypes.POINTER(_Grid),
                                       ctypes.POINTER(i32), fp, fp, fp]
    lib.ss_model_file_read.restype = ctypes.c_int
    lib.ss_model_copy_params.argtypes = [vp, vp, vp]
    lib.ss_model_copy_params.restype = ctypes.c_int
    lib.ss_train_step.argtypes = [vp, vp, ctypes.POINTER(_Catalog), vp, ctypes.c_float, vp, vp,
                                  vp]
    lib.ss_train_step.restype = ctypes.c_int
    lib.ss_best_period_learned.argtypes = [vp, vp, i32, ctypes.POINTER(_Catalog),
                                           ctypes.POINTER(_Grid), ctypes.POINTER(_Params),
                                           ctypes.c_float, i32, i32, i32, vp, vp, vp, vp, vp]
    lib.ss_best_period_learned.restype = ctypes.c_int
    _lib = lib
    return lib


def _check(rc: int):
    if rc != SS_OK:
        raise SSError(rc, _lib.ss_last_error().decode())


@dataclass
class Params:
    span_min: float = 0.05
    span_mid: float = 0.2
    span_max: float = 0.5
    alpha: float = 9.0
    fixed_span: float = 0.0
    precision: int = SS_FP64
    flags: int = 0

    def _c(self) -> _Params:
        return _Params(self.span_min, self.span_mid, self.span_max, self.alpha, self.fixed_span,
                       self.precision, self.flags)


@dataclass
class DeviceCatalog:
    """A catalog resident in device memory (CSR, float64)."""
    offsets: torch.Tensor  # int64 [n_obj + 1]
    t: torch.Tensor
    y: torch.Tensor
    e: torch.Tensor

    @property
    def n_obj(self) -> int:
        return int(self.offsets.numel() - 1)

    @staticmethod
    def from_numpy(offsets, t, y, e, device="cuda") -> "DeviceCatalog":
        def tt(a, dt):
            return torch.as_tensor(a, dtype=dt).to(device).contiguous()
        return DeviceCatalog(tt(offsets, torch.int64), tt(t, torch.float64),
                             tt(y, torch.float64), tt(e, torch.float64))

    def _c(self) -> _Catalog:
        for a, dt in ((self.offsets, torch.int64), (self.t, torch.float64),
                      (self.y, torch.float64), (self.e, torch.float64)):
            if a.dtype != dt or not a.is_cuda or not a.is_contiguous():
                raise ValueError("catalog tensors must be contiguous CUDA tensors "
                                 "(offsets int64; t, y, e float64)")
        if not (self.t.numel() == self.y.numel() == self.e.numel()):
            raise ValueError("t, y and e must have the same length")
        return _Catalog(self.n_obj, self.t.numel(), self.offsets.data_ptr(), self.t.data_ptr(),
                        self.y.data_ptr(), self.e.data_ptr())


@dataclass
class SharedCatalog:
    """Light curves observed at one set of times (device, float64): t [n],
    y and e [n_obj, n]."""
    t: torch.Tensor
    y: torch.Tensor
    e: torch.Tensor

    @property
    def n_obj(self) -> int:
        return int(self.y.shape[0])

    @staticmethod
    def from_numpy(t, y, e, device="cuda") -> "SharedCatalog":
        def tt(a):
            return torch.as_tensor(a, dtype=torch.float64).to(device).contiguous()
        return SharedCatalog(tt(t), tt(y), tt(e))

    def _c(self) -> _SharedCatalog:
        n = self.t.numel()
        for a in (self.t, self.y, self.e):
            if a.dtype != torch.float64 or not a.is_cuda or not a.is_contiguous():
                raise ValueError("shared catalog tensors must be contiguous CUDA float64")
        if self.y.dim() != 2 or self.y.shape != self.e.shape or self.y.shape[1] != n:
            raise ValueError("y and e must be [n_obj, n] with n = len(t)")
        return _SharedCatalog(self.n_obj, n, self.t.data_ptr(), self.y.data_ptr(),
                              self.e.data_ptr())


def bin_table(grid):
    """First grid index of each of the 1024 log bins, plus n_freq (host int64[1025])."""
    import numpy as np
    lib = load_library()
    out = np.zeros(ENC_BINS + 1, dtype=np.int64)
    g = _Grid(float(grid[0]), float(grid[1]), int(grid[2]))
    _check(lib.ss_bin_table(ctypes.byref(g), ctypes.c_void_p(out.ctypes.data)))
    return out


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def _f32_dev(t, n, what):
    if t.dtype != torch.float32 or not t.is_cuda or not t.is_contiguous() or t.numel() != n:
        raise ValueError(f"{what} must be a contiguous CUDA float32 tensor of {n} elements")


def adam_step(params, grad, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
    """One in-place Adam step on FP32 device tensors (step counts from 1)."""
    n = params.numel()
    for t, w in ((params, "params"), (grad, "grad"), (m, "m"), (v, "v")):
        _f32_dev(t, n, w)
    load_library()
    _check(_lib.ss_adam_step(_ptr(params), _ptr(grad), _ptr(m), _ptr(v), n, int(step),
                             float(lr), float(beta1), float(beta2), float(eps),
                             _stream_ptr(stream)))


def _stream_ptr(stream):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


class Context:
    """Owns an ss_ctx (workspace) on one device."""

    def __init__(self, device: int = 0):
        lib = load_library()
        self._h = ctypes.c_void_p()
        _check(lib.ss_ctx_create(device, ctypes.byref(self._h)))
        self.device = device

    def close(self):
        if self._h:
            _lib.ss_ctx_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_shape(self, n_max: int, nw: int, ppl: int):
        """Objects with n <= n_max run on trial groups of nw waves x ppl points per thread
        (nw = 0 clears every rule)."""
        _check(_lib.ss_ctx_set_shape(self._h, int(n_max), int(nw), int(ppl)))

    def set_concurrency(self, enable: bool = True):
        """Run a call's size classes concurrently (forked streams) or serially."""
        _check(_lib.ss_ctx_set_concurrency(self._h, int(bool(enable))))

    def set_tile(self, tile_f: int):
        """Trial frequencies per work item (0 = automatic)."""
        _check(_lib.ss_ctx_set_tile(self._h, int(tile_f)))

    def set_timing(self, enable: bool = True):
        """Record HIP events around the fused trial-kernel launches of each call."""
        _check(_lib.ss_ctx_set_timing(self._h, int(bool(enable))))

    def trial_kernel_ms(self):
        """(milliseconds, launches) of the trial kernels of the last call."""
        ms = ctypes.c_double(0.0)
        n = ctypes.c_int32(0)
        _check(_lib.ss_ctx_trial_kernel_ms(self._h, ctypes.byref(ms), ctypes.byref(n)))
        return ms.value, n.value

    def check_counts(self):
        """(trials, keys out of order, windows with W <= 0) of the last call made
        with SS_FLAG_CHECK_INVARIANTS on this context."""
        out = (ctypes.c_int64 * 3)()
        _check(_lib.ss_ctx_check_counts(self._h, out))
        return tuple(int(v) for v in out)

    def _pgram(self, fn, cat: DeviceCatalog, grid, params: Params, out=None, status=None,
               stream=None):
        n_obj = cat.n_obj
        dt = torch.float64 if params.precision == SS_FP64 else torch.float32
        dev = cat.offsets.device
        if out is None:
            out = torch.empty((n_obj, int(grid[2])), dtype=dt, device=dev)
        if status is None:
            status = torch.empty(n_obj, dtype=torch.int32, device=dev)
        g = _Grid(float(grid[0]), float(grid[1]), int(grid[2]))
        c = cat._c()
        p = params._c()
        _check(fn(self._h, ctypes.byref(c), ctypes.byref(g), ctypes.byref(p),
                  ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(status.data_ptr()),
                  _stream_ptr(stream)))
        return out, status

    def ss_periodogram(self, cat, grid, params=None, out=None, status=None, stream=None):
        """P[o, k] of the Super Smoother (Listing 1) on grid (fmin, fmax, n_freq)."""
        return self._pgram(_lib.ss_periodogram, cat, grid, params or Params(), out, status,
                           stream)

    def sssp_periodogram(self, cat, grid, params=None, out=None, status=None, stream=None):
        """P[o, k] of the single-pass generalized-validation variant (Sec. 3)."""
        return self._pgram(_lib.sssp_periodogram, cat, grid, params or Params(), out, status,
                           stream)

    def method_periodogram(self, method, cat, grid, params=None, out=None, status=None,
                           stream=None):
        """P[o, k] of any method (SS_METHOD_SS, _SSSP or _SSSP_GV)."""
        m = int(method)
        return self._pgram(lambda *a: _lib.ss_method_periodogram(a[0], m, *a[1:]), cat, grid,
                           params or Params(), out, status, stream)

    def pdm_periodogram(self, method, cat, grid, n_bins=0, params=None, stream=None):
        """(P of the method, phase-dispersion score, status) from one fold and sort per trial."""
        params = params or Params()
        n_obj = cat.n_obj
        dt = torch.float64 if params.precision == SS_FP64 else torch.float32
        dev = cat.offsets.device
        pg = torch.empty((n_obj, int(grid[2])), dtype=dt, device=dev)
        pd = torch.empty((n_obj, int(grid[2])), dtype=dt, device=dev)
        st = torch.empty(n_obj, dtype=torch.int32, device=dev)
        g = _Grid(float(grid[0]), float(grid[1]), int(grid[2]))
        c = cat._c()
        p = params._c()
        _check(_lib.ss_pdm_periodogram(self._h, int(method), ctypes.byref(c), ctypes.byref(g),
                                       ctypes.byref(p), int(n_bins), _ptr(pg), _ptr(pd), _ptr(st),
                                       _stream_ptr(stream)))
        return pg, pd, st

    def ss_best_period(self, method, cat, grid, params=None, out=None, stream=None):
        """(best_idx int64, best_period f64, best_power f64, status int32) per object."""
        params = params or Params()
        n_obj = cat.n_obj
        dev = cat.offsets.device
        if out is None:
            out = (torch.empty(n_obj, dtype=torch.int64, device=dev),
                   torch.empty(n_obj, dtype=torch.float64, device=dev),
                   torch.empty(n_obj, dtype=torch.float64, device=dev),
                   torch.empty(n_obj, dtype=torch.int32, device=dev))
        bi, bp, bw, st = out
        g = _Grid(float(grid[0]), float(grid[1]), int(grid[2]))
        c = cat._c()
        p = params._c()
        _check(_lib.ss_best_period(self._h, int(method), ctypes.byref(c), ctypes.byref(g),
                                   ctypes.byref(p), ctypes.c_void_p(bi.data_ptr()),
                                   ctypes.c_void_p(bp.data_ptr()), ctypes.c_void_p(bw.data_ptr()),
                                   ctypes.c_void_p(st.data_ptr()), _stream_ptr(stream)))
        return bi, bp, bw, st

    def plan_batches(self, n_obj, n_points, grid, precision=SS_FP64, want_pgram=True,
                     beta=0.75, mem_bytes=0):
        """(objects per batch, number of batches) from the memory model of
        ss_plan_batches (Eq. 1 of Sec. 4.1 on the periodogram footprint)."""
        g = _Grid(float(grid[0]), float(grid[1]), int(grid[2]))
        per = ctypes.c_int64(0)
        nb = ctypes.c_int64(0)
        _check(_lib.ss_plan_batches(self._h, int(n_obj), int(n_points), ctypes.byref(g),
                                    int(precision), int(bool(want_pgram)), float(beta),
                                    int(mem_bytes), ctypes.byref(per), ctypes.byref(nb)))
        return per.value, nb.value

    def periodogram_batched(self, method, cat: DeviceCatalog, grid, params=None, beta=0.75,
                            mem_bytes=0, sink=None, stream=None):
        """Periodogram in object batches planned by plan_batches.  Each batch is
        computed into one reused device chunk; `sink(lo, hi, chunk_rows, status)`
        receives it (default: gather into host arrays, returned as
        (pgram [n_obj, n_freq] numpy, status numpy, n_batches))."""
        import numpy as np
        params = params or Params()
        n_obj = cat.n_obj
        per, nb = self.plan_batches(n_obj, cat.t.numel(), grid, params.precision, True, beta,
                                    mem_bytes)
        dt = torch.float64 if params.precision == SS_FP64 else torch.float32
        dev = cat.offsets.device
        chunk = torch.empty((max(per, 1), int(grid[2])), dtype=dt, device=dev)
        status = torch.empty(n_obj, dtype=torch.int32, device=dev)
        host = None
        if sink is None:
            host = np.empty((n_obj, int(grid[2])), dtype=np.float64 if dt == torch.float64
                            else np.float32)

            def sink(lo, hi, rows, st):
                host[lo:hi] = rows.cpu().numpy()

        def _cb(user, lo, hi, ptr, st_ptr):
            sink(lo, hi, chunk[:hi - lo], status[lo:hi])

        cb = _SINK(_cb)
        g = _Grid(float(grid[0]), float(grid[1]), int(grid[2]))
        c = cat._c()
        p = params._c()
        _check(_lib.ss_periodogram_batched(self._h, int(method), ctypes.byref(c),
                                           ctypes.byref(g), ctypes.byref(p), _ptr(chunk),
                                           int(per), cb, None, _ptr(status),
                                           _stream_ptr(stream)))
        return host, status.cpu().numpy(), nb

    def shared_periodogram(self, method, cat: SharedCatalog, grid, params=None, stream=None):
        """(P [n_obj, n_freq], status) of objects that share their times."""
        params = params or Params()
        dt = torch.float64 if params.precision == SS_FP64 else torch.float32
        dev = cat.t.device
        pg = torch.empty((cat.n_obj, int(grid[2])), dtype=dt, device=dev)
        st = torch.empty(cat.n_obj, dtype=torch.int32, device=dev)
        g = _Grid(float(grid[0]), float(grid[1]), int(grid[2]))
        c = cat._c()
        p = params._c()
        _check(_lib.ss_shared_periodogram(self._h, int(method), ctypes.byref(c), ctypes.byref(g),
                                          ctypes.byref(p), _ptr(pg), _ptr(st),
                                          _stream_ptr(stream)))
        return pg, st

    def shared_best_period(self, method, cat: SharedCatalog, grid, params=None, out=None,
                           stream=None):
        """(best_idx, best_period, best_power, status) of objects that share their times."""
        params = params or Params()
        bi, bp, bw, st = self._best_out(cat.n_obj, cat.t.device, out)
        g = _Grid(float(grid[0]), float(grid[1]), int(grid[2]))
        c = cat._c()
        p = params._c()
        _check(_lib.ss_shared_best_period(self._h, int(method), ctypes.byref(c), ctypes.byref(g),
                                          ctypes.byref(p), _ptr(bi), _ptr(bp), _ptr(bw), _ptr(st),
                                          _stream_ptr(stream)))
        return bi, bp, bw, st

    def ss_best_period_noalloc(self, method, cat, grid, params=None, out=None, stream=None):
        """ss_best_period in the library's fixed device region (no allocation
        by the library; the outputs are allocated here unless `out` is given)."""
        params = params or Params()
        bi, bp, bw, st = self._best_out(cat.n_obj, cat.offsets.device, out)
        g = _Grid(float(grid[0]), float(grid[1]), int(grid[2]))
        c = cat._c()
        p = params._c()
        _check(_lib.ss_best_period_noalloc(self._h, int(method), ctypes.byref(c),
                                           ctypes.byref(g), ctypes.byref(p), _ptr(bi), _ptr(bp),
                                           _ptr(bw), _ptr(st), _stream_ptr(stream)))
        return bi, bp, bw, st

    def _best_out(self, n_obj, dev, out):
        if out is None:
            out = (torch.empty(n_obj, dtype=torch.int64, device=dev),
                   torch.empty(n_obj, dtype=torch.float64, device=dev),
                   torch.empty(n_obj, dtype=torch.float64, device=dev),
                   torch.empty(n_obj, dtype=torch.int32, device=dev))
        return out

    def enc_forward(self, cat, grid, enc_params, stream=None):
        """(emb [n_obj,128], logits [n_obj,1024], status) of the set encoder."""
        n_obj = cat.n_obj
        dev = cat.offsets.device
        _f32_dev(enc_params, ENC_PARAMS, "enc_params")
        emb = torch.empty((n_obj, 128), dtype=torch.float32, device=dev)
        logits = torch.empty((n_obj, ENC_BINS), dtype=torch.float32, device=dev)
        st = torch.empty(n_obj, dtype=torch.int32, device=dev)
        g = _Grid(float(grid[0]), float(grid[1]), int(grid[2]))
        c = cat._c()
        _check(_lib.ss_enc_forward(self._h, ctypes.byref(c), ctypes.byref(g), _ptr(enc_params),
                                   _ptr(emb), _ptr(logits), _ptr(st), _stream_ptr(stream)))
        return emb, logits, st

    def enc_train_grad(self, cat, grid, enc_params, labels, grad=None, loss=None, stream=None):
        """(grad [ENC_PARAMS], loss [1], status) of the mean cross-entropy."""
        n_obj = cat.n_obj
        dev = cat.offsets.device
        _f32_dev(enc_params, ENC_PARAMS, "enc_params")
        if labels.dtype != torch.int32 or not labels.is_cuda or labels.numel() != n_obj:
            raise ValueError("labels must be a CUDA int32 tensor of n_obj elements")
        labels = labels.contiguous()
        if grad is None:
            grad = torch.empty(ENC_PARAMS, dtype=torch.float32, device=dev)
        if loss is None:
            loss = torch.empty(1, dtype=torch.float32, device=dev)
        st = torch.empty(n_obj, dtype=torch.int32, device=dev)
        g = _Grid(float(grid[0]), float(grid[1]), int(grid[2]))
        c = cat._c()
        _check(_lib.ss_enc_train_grad(self._h, ctypes.byref(c), ctypes.byref(g),
                                      _ptr(enc_params), _ptr(labels), _ptr(grad), _ptr(loss),
                                      _ptr(st), _stream_ptr(stream)))
        return grad, loss, st

    def refine_best_period(self, method, cat, grid, logits, top_k=16, margin=1, full_below=0,
                           params=None, out=None, stream=None):
        """Exact search over the fine-grid frequencies of each object's top bins."""
        params = params or Params()
        n_obj = cat.n_obj
        _f32_dev(logits, n_obj * ENC_BINS, "logits")
        bi, bp, bw, st = self._best_out(n_obj, cat.offsets.device, out)
        g = _Grid(float(grid[0]), float(grid[1]), int(grid[2]))
        c = cat._c()
        p = params._c()
        _check(_lib.ss_refine_best_period(self._h, int(method), ctypes.byref(c), ctypes.byref(g),
                                          ctypes.byref(p), _ptr(logits), int(top_k), int(margin),
                                          int(full_below), _ptr(bi), _ptr(bp), _ptr(bw), _ptr(st),
                                          _stream_ptr(stream)))
        return bi, bp, bw, st

    def bin_scores(self, cat, grid, stream=None):
        """(scores [n_obj, 1024], status): the cheap exact-grid proposal score per log bin."""
        n_obj = cat.n_obj
        dev = cat.offsets.device
        sc = torch.empty((n_obj, ENC_BINS), dtype=torch.float32, device=dev)
        st = torch.empty(n_obj, dtype=torch.int32, device=dev)
        g = _Grid(float(grid[0]), float(grid[1]), int(grid[2]))
        c = cat._c()
        _check(_lib.ss_bin_scores(self._h, ctypes.byref(c), ctypes.byref(g), _ptr(sc), _ptr(st),
                                  _stream_ptr(stream)))
        return sc, st

    def learned_best_period(self, method, cat, grid, enc_params=None, gamma=0.0, top_k=16,
                            margin=1, full_below=0, params=None, out=None, stream=None):
        """Proposal (encoder logits + gamma x bin scores) + exact refine in one call."""
        params = params or Params()
        n_obj = cat.n_obj
        if enc_params is not None:
            _f32_dev(enc_params, ENC_PARAMS, "enc_params")
        bi, bp, bw, st = self._best_out(n_obj, cat.offsets.device, out)
        g = _Grid(float(grid[0]), float(grid[1]), int(grid[2]))
        c = cat._c()
        p = params._c()
        ep = _ptr(enc_params) if enc_params is not None else ctypes.c_void_p(None)
        _check(_lib.ss_learned_best_period(self._h, int(method), ctypes.byref(c),
                                           ctypes.byref(g), ctypes.byref(p), ep, float(gamma),
                                           int(top_k), int(margin), int(full_below), _ptr(bi),
                                           _ptr(bp), _ptr(bw), _ptr(st), _stream_ptr(stream)))
        return bi, bp, bw, st


def _f32_host(a, what):
    import numpy as np
    a = np.ascontiguousarray(a, dtype=np.float32)
    if a.size != ENC_PARAMS:
        raise ValueError(f"{what} must hold {ENC_PARAMS} floats")
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_float))


def model_file_write(path, grid, step, params, adam_m, adam_v):
    """Writes a model file from host arrays (no device needed)."""
    lib = load_library()
    g = _Grid(float(grid[0]), float(grid[1]), int(grid[2]))
    keep = [_f32_host(a, w) for a, w in ((params, "params"), (adam_m, "adam_m"),
                                         (adam_v, "adam_v"))]
    _check(lib.ss_model_file_write(os.fsencode(path), ctypes.byref(g), int(step),
                                   *[k[1] for k in keep]))


def model_file_read(path):
    """(grid, step, params, adam_m, adam_v) from a model file, on the host."""
    import numpy as np
    lib = load_library()
    g = _Grid()
    st = ctypes.c_int32(0)
    arrs = [np.empty(ENC_PARAMS, dtype=np.float32) for _ in range(3)]
    ptrs = [a.ctypes.data_as(ctypes.POINTER(ctypes.c_float)) for a in arrs]
    _check(lib.ss_model_file_read(os.fsencode(path), ctypes.byref(g), ctypes.byref(st), *ptrs))
    return (g.f_min, g.f_max, g.n_freq), st.value, arrs[0], arrs[1], arrs[2]


class Model:
    """An ss_model: encoder parameters, Adam state and the grid they belong to."""

    def __init__(self, handle):
        self._h = handle

    @staticmethod
    def create(ctx: "Context", grid, params) -> "Model":
        lib = load_library()
        g = _Grid(float(grid[0]), float(grid[1]), int(grid[2]))
        a, ap = _f32_host(params, "params")
        h = ctypes.c_void_p()
        _check(lib.ss_model_create(ctx._h, ctypes.byref(g), ap, ctypes.byref(h)))
        return Model(h)

    @staticmethod
    def load(ctx: "Context", path) -> "Model":
        lib = load_library()
        h = ctypes.c_void_p()
        _check(lib.ss_model_load(ctx._h, os.fsencode(path), ctypes.byref(h)))
        return Model(h)

    def save(self, path):
        _check(_lib.ss_model_save(self._h, os.fsencode(path)))

    def info(self):
        """(grid, step, device pointer of the parameters)."""
        g = _Grid()
        st = ctypes.c_int32(0)
        p = ctypes.c_void_p()
        _check(_lib.ss_model_info(self._h, ctypes.byref(g), ctypes.byref(st), ctypes.byref(p)))
        return (g.f_min, g.f_max, g.n_freq), st.value, p.value

    def params(self, device="cuda", stream=None) -> torch.Tensor:
        """A copy of the current parameters as a float32 device tensor."""
        out = torch.empty(ENC_PARAMS, dtype=torch.float32, device=device)
        _check(_lib.ss_model_copy_params(self._h, _ptr(out), _stream_ptr(stream)))
        return out

    def close(self):
        if self._h:
            _lib.ss_model_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def train_step(self, ctx: "Context", batch: DeviceCatalog, labels: torch.Tensor, lr: float,
                   loss: torch.Tensor | None = None, stream=None):
        """Gradient of the batch plus one Adam step; returns the loss tensor [1]."""
        n_obj = batch.n_obj
        if labels.dtype != torch.int32 or not labels.is_cuda or labels.numel() != n_obj:
            raise ValueError("labels must be a CUDA int32 tensor of n_obj elements")
        labels = labels.contiguous()
        dev = batch.offsets.device
        if loss is None:
            loss = torch.empty(1, dtype=torch.float32, device=dev)
        st = torch.empty(n_obj, dtype=torch.int32, device=dev)
        c = batch._c()
        _check(_lib.ss_train_step(ctx._h, self._h, ctypes.byref(c), _ptr(labels),
                                  float(lr), _ptr(loss), _ptr(st), _stream_ptr(stream)))
        return loss

    def best_period(self, ctx: "Context", method, cat: DeviceCatalog, grid, gamma=0.0, top_k=16,
                    margin=1, full_below=0, params=None, out=None, stream=None):
        """Search-and-refine with this model (ss_best_period_learned)."""
        params = params or Params()
        bi, bp, bw, st = ctx._best_out(cat.n_obj, cat.offsets.device, out)
        g = _Grid(float(grid[0]), float(grid[1]), int(grid[2]))
        c = cat._c()
        p = params._c()
        _check(_lib.ss_best_period_learned(ctx._h, self._h, int(method), ctypes.byref(c),
                                           ctypes.byref(g), ctypes.byref(p), float(gamma),
                                           int(top_k), int(margin), int(full_below), _ptr(bi),
                                           _ptr(bp), _ptr(bw), _ptr(st), _stream_ptr(stream)))
        return bi, bp, bw, st
