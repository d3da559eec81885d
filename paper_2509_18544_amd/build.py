"""Build the HIP library libsfft.so for gfx950 in-tree (hipcc, no JIT).

Usage: python -m paper_2509_18544_amd.build  (or call build()).
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIBDIR = os.path.join(HERE, "_lib")
LIB = os.path.join(LIBDIR, "libsfft.so")
SOURCES = ("sfft.hip", "mlp.hip", "render.hip", "align.hip")

ARCH = "gfx950"
FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "-shared",
    f"--offload-arch={ARCH}",
    # no packed FP32 instructions anywhere in the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-result",
    # keep the correlation kernel's per-rotation accumulate blocks apart: sunk
    # into one block they need a register rotation per residue (more VALU
    # instructions and 256 instead of 205 VGPRs)
    "-mllvm", "-simplifycfg-sink-common=false",
]


# roctx ranges around the ABI calls and stages (shown by rocprofv3 --marker-trace)
LIBS = ["-lrocprofiler-sdk-roctx"]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found: the gfx950 HIP library cannot be built")


def build(verbose: bool = False) -> str:
    os.makedirs(LIBDIR, exist_ok=True)
    tmp = LIB + ".tmp"
    cmd = [hipcc(), *FLAGS, *(os.path.join(CSRC, f) for f in SOURCES), *LIBS, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed building libsfft.so")
    if verbose and res.stderr.strip():
        sys.stderr.write(res.stderr)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
