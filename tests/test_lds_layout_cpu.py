"""Host-side bounds check of the trial kernels' LDS regions and indices
(tests/native/lds_layout_check.cpp, built host-only against the kernels'
own header): every built shape, method, span set, fixed span and light-curve
length; the regions must not overlap and every prefix slot, scratch array,
sort array and exchange slot the kernels reach must lie inside its region."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_lds_layout_bounds(tmp_path):
    hipcc = shutil.which("hipcc")
    if not hipcc:
        pytest.skip("hipcc not found")
    exe = str(tmp_path / "lds_layout_check")
    r = subprocess.run([hipcc, "-std=c++17", "--cuda-host-only", "-O1", "-I",
                        os.path.join(ROOT, "paper_2111_07396_amd", "csrc"), "-x", "hip",
                        os.path.join(ROOT, "tests", "native", "lds_layout_check.cpp"), "-o", exe],
                       capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-4000:]
    out = subprocess.run([exe], capture_output=True, text=True, timeout=600)
    assert out.returncode == 0, out.stdout[-4000:]
    assert " 0 failures" in out.stdout, out.stdout
