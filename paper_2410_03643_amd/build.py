"""Build libfnls.so (HIP, gfx950) in-tree with hipcc.

Usage: python -m paper_2410_03643_amd.build  (or __graft_entry__.build()).
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libfnls.so")
SOURCES = ["fnls_pass64.hip", "fnls_pass32.hip", "fnls_kernels.hip", "fnls_api.hip"]
ARCH = os.environ.get("FNLS_OFFLOAD_ARCH", "gfx950")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
# the host trace ranges (roctx) resolve against the ROCm profiler SDK's library
LINK_LIBS = ["-L" + os.path.join(ROCM, "lib"), "-Wl,-rpath," + os.path.join(ROCM, "lib"),
             "-lrocprofiler-sdk-roctx"]


def hipcc() -> str:
    cand = os.environ.get("HIPCC") or shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    return cand


def build(verbose: bool = False, extra_flags=()) -> str:
    """Compile every HIP source into libfnls.so (always recompiles)."""
    objs = []
    flags = ["--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC",
             # packed FP32 instructions stay disabled: some of their forms have
             # given wrong results on MI355X with no error
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-I", os.path.join(ROOT, "include"), "-I", CSRC, *extra_flags]
    procs = []
    for src in SOURCES:   # the translation units compile in parallel
        obj = os.path.join(CSRC, src.replace(".hip", ".o"))
        cmd = [hipcc(), *flags, "-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((subprocess.Popen(cmd), cmd))
        objs.append(obj)
    failed = [cmd for p, cmd in procs if p.wait() != 0]
    if failed:
        raise subprocess.CalledProcessError(1, failed[0])
    tmp = LIB + ".tmp"
    cmd = [hipcc(), "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp, *objs, *LINK_LIBS]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    check_kernels(tmp)
    os.replace(tmp, LIB)
    for o in objs:
        os.remove(o)
    return LIB


def _section(lib: str, name: str) -> bytes:
    out = lib + name.replace(".", "_") + ".bin"
    subprocess.run(["objcopy", "-O", "binary", "--only-section=" + name, lib, out], check=True)
    with open(out, "rb") as fh:
        data = fh.read()
    os.remove(out)
    return data


def check_kernels(lib: str) -> int:
    """Every kernel the host code registers (its mangled name among the host
    strings) must be present in the device code objects: a source edited
    while the host and device passes of one file compiled gives a library
    that aborts at the first launch of the missing kernel."""
    import re
    host = _section(lib, ".rodata")
    dev = _section(lib, ".hip_fatbin")
    names = set(re.findall(rb"_ZN4fnls[0-9A-Za-z_]+", host))
    kernels = [k for k in names if re.match(rb"_ZN4fnls[0-9]+k_", k)]
    missing = [k.decode() for k in kernels if k not in dev]
    if missing:
        raise RuntimeError("kernels registered by the host but absent from the device code: %s" % missing[:5])
    return len(kernels)


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
