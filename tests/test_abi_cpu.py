"""Host-side checks of the C-ABI library (no GPU needed): it loads, exports
every function include/ssgpu.h declares, and rejects bad arguments before
touching a device."""
import ctypes
import os
import re

import pytest

import paper_2111_07396_amd as ssg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    src = open(os.path.join(ROOT, "include", "ssgpu.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\**\s*([a-z_][a-z0-9_]*)\s*\(",
                       src, flags=re.M)
    return sorted(set(names))


def test_library_exports_every_declared_symbol():
    lib = ssg.load_library()
    names = _declared_functions()
    assert set(ssg.EXPORTED) <= set(names)
    for n in names:
        assert hasattr(lib, n), n


def test_version_and_defaults():
    lib = ssg.load_library()
    assert lib.ss_version() == 140
    p = ssg._Params()
    lib.ss_params_default(ctypes.byref(p))
    assert (p.span_min, p.span_mid, p.span_max, p.alpha, p.fixed_span, p.precision) == \
        (0.05, 0.2, 0.5, 9.0, 0.0, ssg.SS_FP64)


def test_null_arguments_rejected_without_device():
    lib = ssg.load_library()
    g = ssg._Grid(0.1, 10.0, 100)
    p = ssg._Params()
    lib.ss_params_default(ctypes.byref(p))
    c = ssg._Catalog(1, 10, None, None, None, None)
    rc = lib.ss_periodogram(None, ctypes.byref(c), ctypes.byref(g), ctypes.byref(p), None, None,
                            None)
    assert rc == ssg.SS_ERR_INVALID_ARG
    assert b"null" in lib.ss_last_error()
    rc = lib.ss_best_period(None, 0, ctypes.byref(c), ctypes.byref(g), ctypes.byref(p), None,
                            None, None, None, None)
    assert rc == ssg.SS_ERR_INVALID_ARG
    out = ctypes.c_void_p()
    assert lib.ss_ctx_create(0, None) == ssg.SS_ERR_INVALID_ARG
