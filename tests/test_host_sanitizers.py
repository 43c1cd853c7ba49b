"""The host code of the runtime (validation, footprint, argument and error
paths of every entry point) built under AddressSanitizer and
UndefinedBehaviorSanitizer and driven by tests/native/abi_host_check.cpp.

Only the host side is instrumented (each -fsanitize= follows -Xarch_host; the
device code of runtime.hip is built as usual) and no call in the driver
reaches the device, so this runs on a machine without a GPU.  The kernel
sources are linked in uninstrumented, as the library itself links them."""

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1712_09999_amd", "csrc")
DRIVER = os.path.join(ROOT, "tests", "native", "abi_host_check.cpp")


def _hipcc():
    for cand in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    return None


def test_runtime_host_paths_under_asan_ubsan(tmp_path):
    hipcc = _hipcc()
    if hipcc is None:
        pytest.skip("hipcc not available")
    inc = ["-I", os.path.join(ROOT, "include"), "-I", CSRC]
    common = ["--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC",
              "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", *inc]
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer"]
    objs = []
    jobs = []
    built = os.path.join(ROOT, "paper_1712_09999_amd", "_build")
    headers = [os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hpp")]
    headers.append(os.path.join(ROOT, "include", "pasd.h"))
    newest_header = max(os.path.getmtime(h) for h in headers)
    for src in sorted(os.listdir(CSRC)):
        if not src.endswith(".hip"):
            continue
        path = os.path.join(CSRC, src)
        prebuilt = os.path.join(built, src.replace(".hip", ".o"))
        if (src != "runtime.hip" and os.path.exists(prebuilt)
                and os.path.getmtime(prebuilt) >= max(os.path.getmtime(path), newest_header)):
            objs.append(prebuilt)  # the library's own, current object of a kernel source
            continue
        obj = str(tmp_path / src.replace(".hip", ".o"))
        flags = common + (san if src == "runtime.hip" else [])
        jobs.append(subprocess.Popen([hipcc, *flags, "-c", path, "-o", obj],
                                     stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True))
        objs.append(obj)
    drv = str(tmp_path / "drv.o")
    jobs.append(subprocess.Popen([hipcc, *common, *san, "-x", "hip", "-c", DRIVER, "-o", drv],
                                 stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True))
    for j in jobs:
        out, err = j.communicate(timeout=600)
        assert j.returncode == 0, err
    exe = str(tmp_path / "abi_host_check")
    r = subprocess.run([hipcc, "--offload-arch=gfx950", *san, drv, *objs, "-o", exe],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1", HIP_VISIBLE_DEVICES="")
    out = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    print(out.stdout[-2000:], out.stderr[-4000:])
    assert out.returncode == 0, out.stdout + out.stderr
    assert "host checks ok" in out.stdout
    assert "runtime error" not in out.stderr and "AddressSanitizer" not in out.stderr
