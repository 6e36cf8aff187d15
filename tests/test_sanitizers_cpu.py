"""AddressSanitizer and UndefinedBehaviorSanitizer builds, on the CPU:
the oracle (every entry point, edge cases: too few points, a bad error bar,
a NaN magnitude, constant magnitude, repeated times) and the host side of
the runtime library (the entry points that need no GPU: argument checks and
their messages, the shape and bin tables, the model file format with
truncated, foreign and missing files).  Leak detection is on.  Skipped when
the compilers or their sanitizer runtimes are missing."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = os.path.join(ROOT, "tests", "sanitize")
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
           UBSAN_OPTIONS="print_stacktrace=1")


def _run(cmd, **kw):
    return subprocess.run(cmd, capture_output=True, text=True, timeout=600, **kw)


def _clean(r):
    text = r.stdout + r.stderr
    assert r.returncode == 0, text[-4000:]
    assert "AddressSanitizer" not in text and "runtime error" not in text, text[-4000:]
    assert "LeakSanitizer" not in text, text[-4000:]


def test_oracle_under_asan_and_ubsan(tmp_path):
    if not shutil.which("gcc"):
        pytest.skip("gcc not found")
    exe = str(tmp_path / "oracle_san")
    r = _run(["gcc", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
              "-fno-omit-frame-pointer", "-g", "-O1", "-std=c11", "-ffp-contract=off", "-o", exe,
              os.path.join(ROOT, "oracle", "ss_oracle.c"), os.path.join(SAN, "oracle_main.c"),
              "-lm"])
    if r.returncode != 0 and "asan" in (r.stderr + r.stdout).lower():
        pytest.skip("no sanitizer runtime for gcc")
    assert r.returncode == 0, r.stderr
    out = _run([exe], env=ENV)
    _clean(out)
    assert "oracle checksum" in out.stdout


def test_runtime_host_code_under_asan_and_ubsan(tmp_path):
    hipcc = shutil.which("hipcc")
    build = os.path.join(ROOT, "paper_2111_07396_amd", "_build")
    others = [os.path.join(build, n + ".o")
              for n in ("binscore", "encoder", "prep_reduce", "trial_f32c", "trial_f64")]
    if not hipcc or not all(os.path.exists(o) for o in others):
        pytest.skip("hipcc or the library objects (build() first) are missing")
    from paper_2111_07396_amd import build as b
    api = str(tmp_path / "api_san.o")
    # host code instrumented (the device code of the same file is untouched)
    san = []
    for f in ("-fsanitize=address", "-fsanitize=undefined", "-fno-sanitize-recover=all",
              "-fno-omit-frame-pointer"):
        san += ["-Xarch_host", f]
    flags = [f for f in b.FLAGS if f != "-O3"] + ["-O1", "-g"]
    r = _run([hipcc] + flags + san + ["-c", os.path.join(ROOT, "paper_2111_07396_amd", "csrc",
                                                         "api.hip"), "-o", api])
    assert r.returncode == 0, r.stderr[-4000:]
    exe = str(tmp_path / "runtime_san")
    r = _run([hipcc, "--offload-arch=" + b.ARCH, "-g", "-fsanitize=address,undefined",
              "-fno-sanitize-recover=all", "-x", "c", "-I", os.path.join(ROOT, "include"),
              os.path.join(SAN, "runtime_main.c"), "-x", "none", api] + others + ["-o", exe])
    assert r.returncode == 0, r.stderr[-4000:]
    out = _run([exe, str(tmp_path)], env=ENV)
    _clean(out)
    assert "0 failure(s)" in out.stdout
