"""Host checks of the kernels' index helpers (no GPU needed).

The fused kernel divides element indices by launch-constant divisors with the
multiply-high/add/shift method of Granlund and Montgomery (1994).  This test
compiles the library's own header into a host program and compares the
division with the exact quotient over many divisors and numerators up to 2^31,
and checks that the XCD block order is a bijection grouping each XCD's blocks.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "native", "fastdiv_check.cpp")


def _hipcc():
    for cand in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    return None


def test_index_helpers(tmp_path):
    hipcc = _hipcc()
    if hipcc is None:
        pytest.skip("hipcc not available")
    exe = str(tmp_path / "fastdiv_check")
    inc = ["-I", os.path.join(ROOT, "include"), "-I", os.path.join(ROOT, "paper_1712_09999_amd", "csrc")]
    r = subprocess.run([hipcc, "-O2", "-std=c++17", "-x", "hip", "--offload-arch=gfx950", *inc, SRC,
                        "-o", exe], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    out = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert out.returncode == 0, out.stdout + out.stderr
    assert "divisors" in out.stdout and "mismatches 0\n" in out.stdout
    assert "xcd orders mismatches 0" in out.stdout
