"""Build the HIP library ``libtlb.so`` (and the HBM probe) for gfx950 in-tree.

``python -m paper_2109_12565_amd.build`` (or ``__graft_entry__.build()``)
compiles the C ABI (``csrc/tlb.hip``), the adjoint launches
(``csrc/adjoint.hip``) and one translation unit per storage type
(``csrc/launch_*.hip``) in parallel with hipcc, links them into
``paper_2109_12565_amd/lib/libtlb.so``, and builds ``lib/hbm_probe``.
"""
from __future__ import annotations

import glob
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIBDIR = os.path.join(HERE, "lib")
OBJDIR = os.path.join(LIBDIR, "obj")
LIB = os.path.join(LIBDIR, "libtlb.so")
PROBE_SRC = os.path.join(CSRC, "hbm_probe.hip")
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


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)


def build(verbose: bool = False, jobs: int = 0) -> str:
    os.makedirs(OBJDIR, exist_ok=True)
    sources = ([os.path.join(CSRC, "tlb.hip"), os.path.join(CSRC, "adjoint.hip")] +
               sorted(glob.glob(os.path.join(CSRC, "launch_*.hip"))))
    objects = [os.path.join(OBJDIR, os.path.basename(s)[:-4] + ".o") for s in sources]
    jobs = jobs or min(len(sources), os.cpu_count() or 1, 16)
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        list(ex.map(lambda so: _run([HIPCC, *COMMON, "-fPIC", "-c", so[0], "-o", so[1]], verbose),
                    zip(sources, objects)))
    _run([HIPCC, "--offload-arch=gfx950", "-shared", *objects, "-o", LIB + ".tmp"], verbose)
    os.replace(LIB + ".tmp", LIB)
    # HBM bandwidth probe (practical ceiling for the roofline)
    _run([HIPCC, *COMMON, PROBE_SRC, "-o", PROBE + ".tmp"], verbose)
    os.replace(PROBE + ".tmp", PROBE)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
    print(LIB)
