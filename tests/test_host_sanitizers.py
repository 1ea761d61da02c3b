"""The library's host code under AddressSanitizer and UndefinedBehaviorSanitizer.

fnls_api.hip is compiled with the sanitizers on its host side (hipcc
-Xarch_host -fsanitize=..., the device code unchanged) and linked into
tests/host/abi_host_check.cpp, which replaces the kernel launchers by stubs
and drives every path of the C ABI that needs no GPU: option defaults, status
strings, workspace layout arithmetic over valid and invalid sizes, every
rejection of fnls_check_assemble (with full, truncated and absent message
buffers), the status acceptance rule across the 32-bit wrap, NULL contexts
and batches, and context creation without a device.  The run must print OK
with no sanitizer report (leak detection on).  The paths that need a GPU
(launch sequencing, staging ring, graph cache) run in the GPU tests.
"""
import os
import shutil
import subprocess

import pytest

from paper_2410_03643_amd import build

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def hipcc():
    return os.environ.get("HIPCC") or shutil.which("hipcc") or (
        "/opt/rocm/bin/hipcc" if os.path.exists("/opt/rocm/bin/hipcc") else None)


@pytest.mark.skipif(hipcc() is None, reason="hipcc not available")
def test_host_code_is_clean_under_sanitizers(tmp_path):
    cc = hipcc()
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined"]
    common = ["--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fno-omit-frame-pointer",
              "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
              "-I", os.path.join(ROOT, "include"), "-I", os.path.join(ROOT, "paper_2410_03643_amd", "csrc")]
    api_o = str(tmp_path / "api.o")
    chk_o = str(tmp_path / "check.o")
    exe = str(tmp_path / "abi_host_check")
    subprocess.run([cc, *common, *san, "-fPIC", "-c",
                    os.path.join(ROOT, "paper_2410_03643_amd", "csrc", "fnls_api.hip"), "-o", api_o],
                   check=True, capture_output=True)
    subprocess.run([cc, *common, *san, "-c", os.path.join(ROOT, "tests", "host", "abi_host_check.cpp"),
                    "-o", chk_o], check=True, capture_output=True)
    subprocess.run([cc, "--offload-arch=gfx950", *san, chk_o, api_o, "-o", exe, *build.LINK_LIBS],
                   check=True, capture_output=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    print(r.stdout[-2000:], r.stderr[-4000:])
    assert r.returncode == 0, r.stderr[-4000:]
    assert r.stdout.startswith("OK ")
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr
