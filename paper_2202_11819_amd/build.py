"""Build libj3d.so (HIP for gfx950 + C++ host engine) in-tree.

Usage: python -m paper_2202_11819_amd.build   (or build() from Python)

Every file is compiled with -ffp-contract=off: the update must round each
addition and the final multiplication separately to match the paper's
readings bit for bit.  Packed FP32 instructions are disabled for all device
code.
"""
from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libj3d.so")
ROOT = os.path.dirname(PKG)

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

COMMON = ["-O3", "-std=c++17", "-fPIC", "-ffp-contract=off", "-Wall", "-Wextra",
          "-Wno-unused-parameter", f"-I{os.path.join(ROOT, 'include')}", f"-I{CSRC}"]
DEVICE = [f"--offload-arch={ARCH}", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]

KERNEL_SOURCES = ["j3d_kernels.hip", "j3d_twostep.hip", "j3d_noalloc.hip"]
HOST_SOURCES = ["j3d_plan.cpp", "j3d_solver.cpp", "j3d_pool.cpp"]


def _run(cmd):
    print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)


def _stale(obj: str, src: str) -> bool:
    """True unless obj is newer than its source and every header."""
    if not os.path.exists(obj):
        return True
    deps = [src] + [os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hpp")]
    deps.append(os.path.join(ROOT, "include", "j3d.h"))
    return any(os.path.getmtime(d) > os.path.getmtime(obj) for d in deps)


def build(verbose_resources: bool = False, incremental: bool = False) -> str:
    """Compile every source (incremental: only those older than their object) and link libj3d.so."""
    os.makedirs(BUILD, exist_ok=True)
    objs = []
    for src in KERNEL_SOURCES:
        obj = os.path.join(BUILD, src + ".o")
        extra = ["-Rpass-analysis=kernel-resource-usage"] if verbose_resources else []
        if not incremental or _stale(obj, os.path.join(CSRC, src)):
            _run([HIPCC, "-x", "hip", *COMMON, *DEVICE, *extra, "-c", os.path.join(CSRC, src), "-o", obj])
        objs.append(obj)
    for src in HOST_SOURCES:
        obj = os.path.join(BUILD, src + ".o")
        if not incremental or _stale(obj, os.path.join(CSRC, src)):
            _run([HIPCC, "-x", "c++", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include", *COMMON, "-c",
                  os.path.join(CSRC, src), "-o", obj])
        objs.append(obj)
    tmp = LIB + ".tmp"
    _run([HIPCC, "-shared", f"--offload-arch={ARCH}", "-fPIC", *objs, "-o", tmp])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose_resources="-v" in sys.argv, incremental="--incremental" in sys.argv)
