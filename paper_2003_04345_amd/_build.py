"""Builds libmb4.so (the MB4 HIP kernels and their C ABI) for gfx950.

``python -m paper_2003_04345_amd._build`` or ``build_library()`` regenerates
mb4_constants.h from its exact derivation and compiles with hipcc in place,
next to this file.
"""
from __future__ import annotations

import concurrent.futures
import os
import shutil
import subprocess
import sys
import tempfile

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


# Extra flags of single sources.  mb4_kernels.hip holds the persistent
# ensemble kernel (k_member_run), whose loops over tiles run whole tile
# bodies; machine-level loop-invariant code motion hoists their constants
# and addresses out of those loops, where they stay live and spill (about 30
# VGPRs, against 8 without it).  The file's per-phase kernels have no such
# loops and compile to the same instructions either way.
EXTRA_FLAGS = {"mb4_kernels.hip": ["-mllvm", "-disable-machine-licm"]}


def common_flags() -> list[str]:
    return [
        f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
        "-fvisibility=hidden", "-ffp-contract=on",
        # no packed FP32 instructions anywhere in the device code
        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
        "-Wall", "-Wno-unused-function",
        f"-I{INCLUDE}", f"-I{CSRC}",
    ]


def compile_commands(out: str, objdir: str) -> list[list[str]]:
    """One hipcc -c per source (each with its extra flags), then the link."""
    cmds, objs = [], []
    for src in SOURCES:
        obj = os.path.join(objdir, os.path.splitext(src)[0] + ".o")
        cmds.append([hipcc(), *common_flags(), *EXTRA_FLAGS.get(src, []), "-c",
                     os.path.join(CSRC, src), "-o", obj])
        objs.append(obj)
    cmds.append([hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", out])
    return cmds


def build_library(verbose: bool = False) -> str:
    gen = os.path.join(CSRC, "gen_constants.py")
    subprocess.run([sys.executable, gen], check=True)
    tmp = LIB + ".tmp"
    with tempfile.TemporaryDirectory(prefix="_build_obj_", dir=PKG) as objdir:
        cmds = compile_commands(tmp, objdir)
        if verbose:
            for c in cmds:
                print(" ".join(c), flush=True)
        workers = max(1, min(len(cmds) - 1, os.cpu_count() or 1, 8))
        with concurrent.futures.ThreadPoolExecutor(workers) as pool:
            for f in [pool.submit(subprocess.run, c, check=True) for c in cmds[:-1]]:
                f.result()
        subprocess.run(cmds[-1], check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build_library(verbose=True))
