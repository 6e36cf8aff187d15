"""ctypes wrapper around the FP64 CPU oracle (``ss_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and the
CPU-baseline leg of the benchmark.  The product path (the HIP library and its
Python binding) never imports this package.

Every function takes and returns NumPy float64 / int64 arrays.  The C source
documents which passage of the paper each function follows.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libss_oracle.so")

STATUS_OK, STATUS_TOO_FEW, STATUS_BAD_ERR, STATUS_NONFINITE, STATUS_CONST_MAG = 0, 1, 2, 3, 4
SS, SSSP, SSSP2 = 0, 1, 2
DEFAULT_SPANS = (0.05, 0.2, 0.5)

_dp = ctypes.POINTER(ctypes.c_double)
_lp = ctypes.POINTER(ctypes.c_int64)
_ip = ctypes.POINTER(ctypes.c_int32)
_lib = None


def build() -> None:
    """Compile the oracle shared library (gcc, FP64, OpenMP)."""
    subprocess.check_call(["sh", os.path.join(_HERE, "build.sh")])


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        build()
    lib = ctypes.CDLL(_LIB_PATH)
    lib.ora_prep.restype = ctypes.c_int
    lib.ora_prep.argtypes = [ctypes.c_int64, _dp, _dp, _dp, _dp, _dp, _dp, _dp]
    lib.ora_freq.restype = ctypes.c_double
    lib.ora_freq.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_int64, ctypes.c_int64]
    lib.ora_grid_nfreq.restype = ctypes.c_int64
    lib.ora_grid_nfreq.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_double]
    lib.ora_fold.restype = None
    lib.ora_fold.argtypes = [ctypes.c_int64, _dp, ctypes.c_double, _dp]
    lib.ora_argsort.restype = None
    lib.ora_argsort.argtypes = [ctypes.c_int64, _dp, _lp]
    lib.ora_halfwidth.restype = ctypes.c_int
    lib.ora_halfwidth.argtypes = [ctypes.c_int, ctypes.c_double]
    lib.ora_smooth.restype = None
    lib.ora_smooth.argtypes = [ctypes.c_int, _dp, _dp, _dp, ctypes.c_double, ctypes.c_int,
                               ctypes.c_int, ctypes.c_double, _dp, _dp, _dp]
    lib.ora_supsmu.restype = None
    lib.ora_supsmu.argtypes = [ctypes.c_int, _dp, _dp, _dp, ctypes.c_int, _dp, ctypes.c_double,
                               ctypes.c_double, _dp]
    lib.ora_sssp.restype = ctypes.c_double
    lib.ora_sssp.argtypes = [ctypes.c_int, _dp, _dp, _dp, ctypes.c_int, _dp, ctypes.c_int,
                             ctypes.c_double, _dp, _dp, ctypes.POINTER(ctypes.c_int)]
    lib.ora_pdm.restype = ctypes.c_double
    lib.ora_pdm.argtypes = [ctypes.c_int, _dp, _dp, _dp, ctypes.c_double, ctypes.c_double,
                            ctypes.c_double, ctypes.c_int]
    lib.ora_sssp2.restype = ctypes.c_double
    lib.ora_sssp2.argtypes = [ctypes.c_int, _dp, _dp, _dp, ctypes.c_int, _dp, ctypes.c_double,
                              ctypes.c_double]
    lib.ora_trial.restype = ctypes.c_double
    lib.ora_trial.argtypes = [ctypes.c_int, ctypes.c_int, _dp, _dp, _dp, ctypes.c_double,
                              ctypes.c_double, ctypes.c_int, _dp, ctypes.c_double, ctypes.c_double]
    lib.ora_num_threads.restype = ctypes.c_int
    lib.ora_num_threads.argtypes = []
    lib.ora_periodogram.restype = None
    lib.ora_periodogram.argtypes = [ctypes.c_int, ctypes.c_int64, _lp, _dp, _dp, _dp,
                                    ctypes.c_double, ctypes.c_double, ctypes.c_int64, _lp,
                                    ctypes.c_int64, _dp, ctypes.c_double, ctypes.c_double,
                                    _dp, _ip]
    lib.ora_best.restype = ctypes.c_int64
    lib.ora_best.argtypes = [ctypes.c_int64, _dp]
    _lib = lib
    return lib


def _d(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(_dp)


def _l(a):
    a = np.ascontiguousarray(a, dtype=np.int64)
    return a, a.ctypes.data_as(_lp)


def num_threads() -> int:
    return int(_load().ora_num_threads())


def prep(t, y, e):
    """Returns (status, tt, w, ybar, chi0)."""
    lib = _load()
    t, tp = _d(t)
    y, yp = _d(y)
    e, ep = _d(e)
    n = t.size
    tt, ttp = _d(np.zeros(n))
    w, wp = _d(np.zeros(n))
    yb = ctypes.c_double(0.0)
    c0 = ctypes.c_double(0.0)
    st = lib.ora_prep(n, tp, yp, ep, ttp, wp, ctypes.byref(yb), ctypes.byref(c0))
    return int(st), tt, w, yb.value, c0.value


def freq(fmin, fmax, n_freq, k) -> float:
    return float(_load().ora_freq(fmin, fmax, n_freq, k))


def grid_nfreq(t_extent_max, fmin, fmax) -> int:
    return int(_load().ora_grid_nfreq(t_extent_max, fmin, fmax))


def fold(tt, f):
    tt, tp = _d(tt)
    out, op = _d(np.zeros(tt.size))
    _load().ora_fold(tt.size, tp, f, op)
    return out


def argsort(key):
    key, kp = _d(key)
    perm, pp = _l(np.zeros(key.size, dtype=np.int64))
    _load().ora_argsort(key.size, kp, pp)
    return perm


def halfwidth(n, span) -> int:
    return int(_load().ora_halfwidth(n, span))


def smooth(x, v, w, span, periodic=True, cv=True, vsmlsq=0.0):
    """Returns (s, r, lev) of the running-line smoother on sorted x."""
    x, xp = _d(x)
    v, vp = _d(v)
    w, wp = _d(w)
    n = x.size
    s, sp = _d(np.zeros(n))
    r, rp = _d(np.zeros(n))
    lev, lp = _d(np.zeros(n))
    _load().ora_smooth(n, xp, vp, wp, span, int(bool(periodic)), int(bool(cv)), vsmlsq, sp, rp, lp)
    return s, r, lev


def supsmu(x, y, w, spans=DEFAULT_SPANS, alpha=9.0, fixed_span=0.0, periodic=True):
    x, xp = _d(x)
    y, yp = _d(y)
    w, wp = _d(w)
    sp_, spp = _d(np.asarray(spans, dtype=np.float64))
    smo, op = _d(np.zeros(x.size))
    _load().ora_supsmu(x.size, xp, yp, wp, 2 if periodic else 1, spp, alpha, fixed_span, op)
    return smo


def sssp(x, y, w, spans=DEFAULT_SPANS, fixed_span=0.0, periodic=True):
    """Returns (chi2, rss[K], tr[K], kbest)."""
    x, xp = _d(x)
    y, yp = _d(y)
    w, wp = _d(w)
    sp_, spp = _d(np.asarray(spans, dtype=np.float64))
    K = len(spans)
    rss, rp = _d(np.zeros(K))
    tr, tp = _d(np.zeros(K))
    kb = ctypes.c_int(0)
    chi2 = _load().ora_sssp(x.size, xp, yp, wp, 2 if periodic else 1, spp, K, fixed_span, rp, tp,
                            ctypes.byref(kb))
    return float(chi2), rss, tr, kb.value


def pdm_bins(n, n_bins=0):
    """Phase bins of the dispersion score: n_bins, or clamp(n // 5, 4, 32) when 0."""
    return int(n_bins) if n_bins > 0 else min(32, max(4, n // 5))


def pdm_periodogram(offsets, t, y, e, fmin, fmax, n_freq, n_bins=0, ks=None):
    """Phase-dispersion score of every object at every (selected) grid
    frequency; NaN rows for objects with a bad status."""
    lib = _load()
    offsets = np.asarray(offsets, dtype=np.int64)
    n_obj = offsets.size - 1
    kk = np.arange(n_freq) if ks is None else np.asarray(ks, dtype=np.int64)
    out = np.full((n_obj, kk.size), np.nan)
    for o in range(n_obj):
        a, b = offsets[o], offsets[o + 1]
        st, tt, w, ybar, chi0 = prep(t[a:b], y[a:b], e[a:b])
        if st != 0:
            continue
        ttp = tt.ctypes.data_as(_dp)
        yy = np.ascontiguousarray(y[a:b], dtype=np.float64)
        yp = yy.ctypes.data_as(_dp)
        wp = w.ctypes.data_as(_dp)
        B = pdm_bins(b - a, n_bins)
        for i, k in enumerate(kk):
            out[o, i] = lib.ora_pdm(int(b - a), ttp, yp, wp, ybar, chi0,
                                    freq(fmin, fmax, n_freq, int(k)), B)
    return out


def sssp2(x, y, w, spans=DEFAULT_SPANS, alpha=9.0, fixed_span=0.0, periodic=True):
    """chi^2 of the second single-pass reading (per-point span choice by the
    un-smoothed GV residual, bass, blend)."""
    x, xp = _d(x)
    y, yp = _d(y)
    w, wp = _d(w)
    sp_, spp = _d(np.asarray(spans, dtype=np.float64))
    return float(_load().ora_sssp2(x.size, xp, yp, wp, 2 if periodic else 1, spp, alpha,
                                   fixed_span))


def trial(method, tt, y, w, chi0, f, spans=DEFAULT_SPANS, alpha=9.0, fixed_span=0.0,
          periodic=True):
    tt, ttp = _d(tt)
    y, yp = _d(y)
    w, wp = _d(w)
    sp_, spp = _d(np.asarray(spans, dtype=np.float64))
    return float(_load().ora_trial(method, tt.size, ttp, yp, wp, chi0, f, 2 if periodic else 1,
                                   spp, alpha, fixed_span))


def periodogram(method, offsets, t, y, e, fmin, fmax, n_freq, ks=None, spans=DEFAULT_SPANS,
                alpha=9.0, fixed_span=0.0):
    """P[o, i] for every object o and every selected frequency index (all when
    ks is None).  Returns (pgram[n_obj, nk], status[n_obj])."""
    lib = _load()
    offsets, op = _l(offsets)
    t, tp = _d(t)
    y, yp = _d(y)
    e, ep = _d(e)
    n_obj = offsets.size - 1
    if ks is None:
        nk, kp = n_freq, None
    else:
        ks, kp = _l(ks)
        nk = ks.size
    sp_, spp = _d(np.asarray(spans, dtype=np.float64))
    pg, pgp = _d(np.zeros(n_obj * nk))
    st = np.zeros(n_obj, dtype=np.int32)
    lib.ora_periodogram(method, n_obj, op, tp, yp, ep, fmin, fmax, n_freq, kp, nk, spp, alpha,
                        fixed_span, pgp, st.ctypes.data_as(_ip))
    return pg.reshape(n_obj, nk), st


def best(p) -> int:
    p, pp = _d(p)
    return int(_load().ora_best(p.size, pp))
