"""Build libfrbx.so in-tree with hipcc for gfx950.

    python -m paper_1801_02391_amd.build

Compiles the HIP kernels and the host side of the library and links them
into paper_1801_02391_amd/libfrbx.so.  Every build recompiles from source.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "libfrbx.so")

ARCH = "gfx950"
# Packed FP32 instructions are kept out of every device code object.
DEVICE_FLAGS = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
# Matrix-core results go straight to VGPRs (no accumulator read-back).
KERNEL_FLAGS = ["-mllvm", "-amdgpu-mfma-vgpr-form=true"]
COMMON = ["-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
          f"--offload-arch={ARCH}"]


def _hipcc():
    h = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(h):
        raise RuntimeError("hipcc not found")
    return h


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError(f"build step failed: {' '.join(cmd[:3])} ...")
    return r


def build(verbose: bool = True) -> str:
    os.makedirs(BUILD, exist_ok=True)
    hipcc = _hipcc()
    objs = []
    k_obj = os.path.join(BUILD, "frbx_kernels.o")
    _run([hipcc, "-c", "-O3", *COMMON, *DEVICE_FLAGS, *KERNEL_FLAGS,
          os.path.join(CSRC, "frbx_kernels.hip"), "-o", k_obj], verbose)
    objs.append(k_obj)
    h_obj = os.path.join(BUILD, "frbx_host.o")
    # float64 tables must not be contracted into FMAs: keep Eq. 2 rounding
    # bit-identical to a plain evaluation of the formula.
    _run([hipcc, "-c", "-O2", "-ffp-contract=off", *COMMON, *DEVICE_FLAGS,
          os.path.join(CSRC, "frbx_host.cpp"), "-o", h_obj], verbose)
    objs.append(h_obj)
    tmp = LIB + ".tmp"
    _run([hipcc, "-shared", f"--offload-arch={ARCH}", "-fPIC", *objs, "-o", tmp], verbose)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-q" not in sys.argv)
    print(LIB)
