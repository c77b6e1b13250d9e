"""The library's host code under AddressSanitizer, on the CPU.

Every source is compiled with AddressSanitizer on its host pass (the device
code is built as usual but never runs) and linked with ``tests/host_check/host_check.cpp``, which
drives the C ABI through the paths that need no kernel: options validation
and workspace layouts over a grid of settings, NULL and out-of-range
arguments, the profiler counters, and the builds' error paths (on a machine
without a GPU every device call fails and the context is released).  An
out-of-bounds access, use after free or double free on those paths fails the
test with the sanitizer's report.
"""
import os
import shutil
import subprocess
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1503_03467_amd", "csrc")


def _hipcc():
    exe = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    return exe if os.path.exists(exe) else None


def test_host_logic_under_address_sanitizer(tmp_path):
    hipcc = _hipcc()
    if hipcc is None:
        pytest.skip("hipcc not available")
    from paper_1503_03467_amd.build import SOURCES
    # sanitizer flags apply to the host pass only (each one after -Xarch_host)
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fno-omit-frame-pointer"]
    # device code is compiled too (the host objects refer to it) but never runs
    common = ["-Xarch_host", "-O1", "-Xarch_host", "-g", "-Xarch_device", "-O1", "-std=c++17", "-fPIC",
              "--offload-arch=gfx950", "-I", os.path.join(ROOT, "include"), "-w"]

    def compile_one(src):
        obj = str(tmp_path / (os.path.splitext(os.path.basename(src))[0] + ".o"))
        r = subprocess.run([hipcc, *common, *san, "-c", src, "-o", obj], capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-4000:]
        return obj

    srcs = [os.path.join(CSRC, s) for s in SOURCES] + [os.path.join(ROOT, "tests", "host_check", "host_check.cpp")]
    with ThreadPoolExecutor(max_workers=8) as ex:
        objs = list(ex.map(compile_one, srcs))
    exe = str(tmp_path / "host_check")
    r = subprocess.run([hipcc, "--offload-arch=gfx950", "-Xarch_host", "-fsanitize=address", *objs, "-o", exe,
                        "-pthread"], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0:halt_on_error=1",
               HIP_VISIBLE_DEVICES=os.environ.get("HIP_VISIBLE_DEVICES", ""))
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    print(r.stdout[-2000:])
    assert "AddressSanitizer" not in r.stderr, r.stderr[-6000:]
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-4000:])
