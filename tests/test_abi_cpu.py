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
    src = re.sub(r"typedef[^;]*;", "", src)  # type names, function-pointer types
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
    assert lib.ss_version() == 151
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


# ----------------------------------------------------------------- model file (host only)

def _model_arrays(seed=0):
    import numpy as np
    rng = np.random.default_rng(seed)
    return [rng.normal(0, s, ssg.ENC_PARAMS).astype(np.float32) for s in (0.1, 1e-3, 1e-6)]


def test_model_file_round_trip(tmp_path):
    import json
    import struct

    import numpy as np
    p, m, v = _model_arrays()
    grid = (0.05, 20.0, 50000)
    path = str(tmp_path / "enc.ssm")
    ssg.model_file_write(path, grid, 1234, p, m, v)
    g2, step, p2, m2, v2 = ssg.model_file_read(path)
    assert g2 == grid and step == 1234
    for a, b in ((p, p2), (m, m2), (v, v2)):
        assert np.array_equal(a.view(np.uint32), b.view(np.uint32))  # bit for bit
    raw = open(path, "rb").read()
    assert raw[:8] == b"SSGPUMDL"
    fmt, jlen = struct.unpack_from("<II", raw, 8)
    assert fmt == 1
    hdr = 8 + 4 + 4 + 8 + 4 + 4 * 3 + 8 * 2 + 8 + 8
    meta = json.loads(raw[hdr:hdr + jlen].decode())
    assert meta["n_params"] == ssg.ENC_PARAMS and meta["step"] == 1234
    assert meta["grid"] == {"f_min": 0.05, "f_max": 20.0, "n_freq": 50000}
    assert len(meta["feature_freqs"]) == 32 and meta["bins"] == ssg.ENC_BINS
    assert abs(meta["feature_freqs"][0] - 0.05) < 1e-15 and meta["feature_freqs"][-1] == 20.0
    (off,) = struct.unpack_from("<Q", raw, hdr - 8)
    assert off % 64 == 0 and len(raw) == off + 3 * 4 * ssg.ENC_PARAMS


def test_model_file_rejects_bad_files(tmp_path):
    p, m, v = _model_arrays(1)
    good = str(tmp_path / "good.ssm")
    ssg.model_file_write(good, (0.1, 10.0, 2000), 0, p, m, v)
    raw = open(good, "rb").read()
    cases = {
        "short": raw[:20],
        "magic": b"XSGPUMDL" + raw[8:],
        "truncated": raw[:-4],
        "version": raw[:8] + (7).to_bytes(4, "little") + raw[12:],
    }
    for name, data in cases.items():
        path = str(tmp_path / (name + ".ssm"))
        open(path, "wb").write(data)
        with pytest.raises(ssg.SSError) as ei:
            ssg.model_file_read(path)
        want = ssg.SS_ERR_UNSUPPORTED if name == "version" else ssg.SS_ERR_INVALID_ARG
        assert ei.value.code == want, name
    with pytest.raises(ssg.SSError):
        ssg.model_file_read(str(tmp_path / "missing.ssm"))
    with pytest.raises(ssg.SSError):
        ssg.model_file_write(str(tmp_path / "bad_grid.ssm"), (1.0, 0.5, 10), 0, p, m, v)


def test_plan_batches_rejects_bad_arguments_without_device():
    lib = ssg.load_library()
    g = ssg._Grid(0.1, 10.0, 100)
    per = ctypes.c_int64()
    nb = ctypes.c_int64()
    assert lib.ss_plan_batches(None, 10, 100, ctypes.byref(g), 0, 1, 0.75, 1 << 20,
                               ctypes.byref(per), ctypes.byref(nb)) == ssg.SS_ERR_INVALID_ARG
