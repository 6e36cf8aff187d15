"""The trial kernels' own source run on the CPU, one thread per lane
(tests/native/lds_race_check.cpp with the HIP stand-in of tests/native/emu),
under ThreadSanitizer: for shapes 1x1 .. 4x2 and 2x4, the three methods (plus
a fixed span) in FP64 and the compensated-FP32 policy on the 256-point
shapes, no LDS access of one lane may go unordered against another lane's
write to the same word, and the periodograms must match the CPU oracle at the GPU parity
bar.  A planted unordered access (no barrier between a write and another
wavefront's read) must be reported, and the same with a barrier must not."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
NATIVE = os.path.join(ROOT, "tests", "native")


@pytest.fixture(scope="module")
def race_exe(tmp_path_factory):
    if not (shutil.which("gcc") and shutil.which("g++")):
        pytest.skip("gcc/g++ not found")
    d = tmp_path_factory.mktemp("race")
    ora = str(d / "oracle_tsan.o")
    exe = str(d / "lds_race_check")
    r = subprocess.run(["gcc", "-O1", "-g", "-fsanitize=thread", "-std=c11", "-ffp-contract=off",
                        "-c", os.path.join(ROOT, "oracle", "ss_oracle.c"), "-o", ora],
                       capture_output=True, text=True, timeout=600)
    if r.returncode != 0 and "tsan" in (r.stdout + r.stderr).lower():
        pytest.skip("no ThreadSanitizer runtime")
    assert r.returncode == 0, r.stderr[-3000:]
    r = subprocess.run(["g++", "-std=c++20", "-O1", "-g", "-fsanitize=thread", "-ffp-contract=off",
                        "-Wno-attributes", "-Wno-unknown-pragmas", "-I", os.path.join(NATIVE, "emu"),
                        "-I", os.path.join(ROOT, "paper_2111_07396_amd", "csrc"),
                        os.path.join(NATIVE, "lds_race_check.cpp"), ora, "-o", exe, "-pthread",
                        "-lm"], capture_output=True, text=True, timeout=900)
    assert r.returncode == 0, r.stderr[-3000:]
    return exe


def _run(exe, *args):
    return subprocess.run([exe] + list(args), capture_output=True, text=True, timeout=1800,
                          env=dict(os.environ, TSAN_OPTIONS="halt_on_error=0"))


def test_planted_race_is_reported(race_exe):
    bad = _run(race_exe, "plant", "0")
    assert bad.returncode != 0 and "WARNING: ThreadSanitizer: data race" in bad.stderr
    good = _run(race_exe, "plant", "1")
    assert good.returncode == 0 and "ThreadSanitizer" not in good.stderr, good.stderr[-3000:]


def test_trial_kernels_have_no_unordered_lds_access(race_exe):
    r = _run(race_exe)
    assert "ThreadSanitizer" not in r.stderr, r.stderr[-6000:]
    assert r.returncode == 0, r.stdout[-3000:]
    assert "over tolerance: 0" in r.stdout, r.stdout[-3000:]
