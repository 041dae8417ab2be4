"""Build the HIP library ``libmpg.so`` for gfx950 in-tree.

Usage: ``python -m paper_2210_08052_amd.build`` (or ``build()`` from Python).
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libmpg.so")
SOURCES = ["mpg_dp_k1.hip", "mpg_dp_k2.hip", "mpg_dp_k4.hip", "mpg_dp_p1.hip", "mpg_dp_p2.hip",
           "mpg_dp16.hip", "mpg_chain.hip", "mpg_kernels.hip", "mpg_lib.cpp"]
ARCH = os.environ.get("MPG_OFFLOAD_ARCH", "gfx950")

# Packed-FP32 instructions are disabled for all device code.  The DP kernels
# unroll their 64-step chunks completely (#pragma unroll); the default size
# limit on pragma-requested unrolling would leave the wider variants rolled.
DEVICE_FLAGS = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                "-mllvm", "-pragma-unroll-threshold=1000000"]


def _hipcc() -> str:
    for c in ("/opt/rocm/bin/hipcc", "hipcc"):
        if os.path.exists(c) or c == "hipcc":
            return c
    raise RuntimeError("hipcc not found")


def build(verbose: bool = False, extra=None, out: str | None = None) -> str:
    """Compile every source into one shared library (always recompiles).
    ``extra``: more compiler flags (e.g. -D tuning macros); ``out``: write the
    library there instead of the in-tree libmpg.so (variant builds)."""
    objs, procs = [], []
    lib = out or LIB
    build_dir = os.path.join(HERE, "_build") if out is None else out + ".objs"
    os.makedirs(build_dir, exist_ok=True)
    for src in SOURCES:
        obj = os.path.join(build_dir, src + ".o")
        cmd = [_hipcc(), "-c", "-fPIC", "-O3", "-std=c++17", "--offload-arch=" + ARCH,
               "-Wall", "-Wno-unused-function", "-Wno-unused-variable", "-Wno-unused-result"]
        if src.endswith(".hip"):
            cmd += DEVICE_FLAGS + ["-x", "hip"]
        cmd += list(extra or []) + [os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((src, subprocess.Popen(cmd)))
        objs.append(obj)
    for src, pr in procs:
        if pr.wait() != 0:
            raise RuntimeError("compiling %s failed" % src)
    tmp = lib + ".tmp%d" % os.getpid()
    cmd = [_hipcc(), "-shared", "-fPIC", "--offload-arch=" + ARCH, "-o", tmp] + objs + [
        "-lpthread"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, lib)
    return lib


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
    print(LIB)
