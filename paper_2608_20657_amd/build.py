"""Build libheom.so in-tree for gfx950.

Host table builder: g++ (C++17, -ffp-contract=off so table coefficients are
the unfused expressions written in the source). Kernels and the C ABI: hipcc
for gfx950, with packed-FP32 instructions disabled.
"""
from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INC = os.path.join(ROOT, "include")
BUILD = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libheom.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

HIP_FLAGS = ["--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-I", INC, "-I", CSRC]
HOST_FLAGS = ["-O2", "-std=c++17", "-fPIC", "-ffp-contract=off", "-I", INC, "-I", CSRC,
              "-Wall", "-Wextra", "-Wno-unused-parameter"]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("build step failed: " + " ".join(cmd))
    return r


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    tables_o = os.path.join(BUILD, "tables.o")
    device_o = os.path.join(BUILD, "device.o")
    recon_o = os.path.join(BUILD, "reconstruct.o")
    _run(["g++"] + HOST_FLAGS + ["-c", os.path.join(CSRC, "tables.cpp"), "-o", tables_o], verbose)
    _run([HIPCC] + HIP_FLAGS + ["-c", os.path.join(CSRC, "device.hip"), "-o", device_o], verbose)
    _run([HIPCC] + HIP_FLAGS + ["-c", os.path.join(CSRC, "reconstruct.hip"), "-o", recon_o], verbose)
    tmp = LIB + ".tmp"
    _run([HIPCC, "--offload-arch=" + ARCH, "-shared", "-fPIC", tables_o, device_o, recon_o, "-o", tmp], verbose)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
