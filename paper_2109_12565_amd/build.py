"""Build the HIP library ``libtlb.so`` for gfx950 in-tree.

``python -m paper_2109_12565_amd.build`` (or ``__graft_entry__.build()``)
compiles ``csrc/tlb.hip`` with hipcc into ``paper_2109_12565_amd/lib/``.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = os.path.join(HERE, "csrc", "tlb.hip")
PROBE_SRC = os.path.join(HERE, "csrc", "hbm_probe.hip")
LIBDIR = os.path.join(HERE, "lib")
LIB = os.path.join(LIBDIR, "libtlb.so")
PROBE = os.path.join(LIBDIR, "hbm_probe")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
COMMON = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    # keep the compiler from forming packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall",
    "-Wno-unused-function",
    "-I", os.path.join(ROOT, "include"),
]
FLAGS = COMMON + ["-fPIC", "-shared"]


def build(verbose: bool = False) -> str:
    os.makedirs(LIBDIR, exist_ok=True)
    tmp = LIB + ".tmp"
    cmd = [HIPCC, *FLAGS, SRC, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    # HBM bandwidth probe (practical ceiling for the roofline)
    cmd = [HIPCC, *COMMON, PROBE_SRC, "-o", PROBE + ".tmp"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(PROBE + ".tmp", PROBE)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
    print(LIB)
