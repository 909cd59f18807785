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

KERNEL_SOURCES = ["j3d_kernels.hip", "j3d_twostep.hip"]
HOST_SOURCES = ["j3d_plan.cpp", "j3d_solver.cpp", "j3d_pool.cpp"]


def _run(cmd):
    print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)


def build(verbose_resources: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    objs = []
    for src in KERNEL_SOURCES:
        obj = os.path.join(BUILD, src + ".o")
        extra = ["-Rpass-analysis=kernel-resource-usage"] if verbose_resources else []
        _run([HIPCC, "-x", "hip", *COMMON, *DEVICE, *extra, "-c", os.path.join(CSRC, src), "-o", obj])
        objs.append(obj)
    for src in HOST_SOURCES:
        obj = os.path.join(BUILD, src + ".o")
        _run([HIPCC, "-x", "c++", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include", *COMMON, "-c", os.path.join(CSRC, src),
              "-o", obj])
        objs.append(obj)
    tmp = LIB + ".tmp"
    _run([HIPCC, "-shared", f"--offload-arch={ARCH}", "-fPIC", *objs, "-o", tmp])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose_resources="-v" in sys.argv)
