"""Builds libmb4.so (the MB4 HIP kernels and their C ABI) for gfx950.

``python -m paper_2003_04345_amd._build`` or ``build_library()`` regenerates
mb4_constants.h from its exact derivation and compiles with hipcc in place,
next to this file.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(PKG, "csrc")
ROOT = os.path.dirname(PKG)
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libmb4.so")
SOURCES = ["mb4_kernels.hip", "mb4_spectral.hip", "mb4_runtime.hip", "mb4_engine.hip",
           "mb4_ensemble.hip", "mb4_server.hip", "mb4_noalloc.hip"]
ARCH = "gfx950"


def hipcc() -> str:
    for cand in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def compile_command(out: str = LIB) -> list[str]:
    return [
        hipcc(), f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-shared",
        "-fvisibility=hidden", "-ffp-contract=on",
        # no packed FP32 instructions anywhere in the device code
        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
        "-Wall", "-Wno-unused-function",
        f"-I{INCLUDE}", f"-I{CSRC}",
        *[os.path.join(CSRC, s) for s in SOURCES],
        "-o", out,
    ]


def build_library(verbose: bool = False) -> str:
    gen = os.path.join(CSRC, "gen_constants.py")
    subprocess.run([sys.executable, gen], check=True)
    tmp = LIB + ".tmp"
    cmd = compile_command(tmp)
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build_library(verbose=True))
