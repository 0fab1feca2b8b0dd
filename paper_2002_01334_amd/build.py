"""Build liblpbfmm.so (HIP for gfx950 + host C++) in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "liblpbfmm.so")

# (the longest compiles first; the orbit orders and the fixed-KB products are
# split over several translation units so that they compile in parallel)
HIP_SOURCES = ["lpb_m2l_orbit_d.hip", "lpb_m2l_orbit_c.hip", "lpb_m2l_orbit_b.hip", "lpb_m2l_orbit_a.hip",
               "lpb_m2l_tile_kb32.hip", "lpb_m2l_tile_kb64.hip", "lpb_m2l_tile.hip", "lpb_eval.hip",
               "lpb_p2m_l2p.hip", "lpb_opgen.hip", "lpb_tree_dev.hip", "lpb_adaptive.hip"]
CXX_SOURCES = ["lpb_plan.cpp", "lpb_capi.cpp"]
ARCH = "gfx950"
# packed FP32 instructions are disabled for all device code
DEVICE_FLAGS = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
COMMON = ["-O3", "-fPIC", "-std=c++17", "-Wall", "-Wno-unused-function", f"-I{os.path.join(HERE, '..', 'include')}"]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)


def build(verbose: bool = False, jobs: int = 8) -> str:
    os.makedirs(BUILD, exist_ok=True)
    procs = []
    objs = []
    for src in HIP_SOURCES:
        obj = os.path.join(BUILD, src + ".o")
        cmd = ["hipcc", "-c", f"--offload-arch={ARCH}", *DEVICE_FLAGS, *COMMON, os.path.join(CSRC, src), "-o", obj]
        objs.append(obj)
        procs.append(cmd)
    for src in CXX_SOURCES:
        obj = os.path.join(BUILD, src + ".o")
        cmd = ["hipcc", "-c", f"--offload-arch={ARCH}", *DEVICE_FLAGS, *COMMON, os.path.join(CSRC, src), "-o", obj]
        objs.append(obj)
        procs.append(cmd)
    running = []
    for cmd in procs:
        if verbose:
            print(" ".join(cmd), flush=True)
        running.append(subprocess.Popen(cmd))
        if len(running) >= jobs:
            if running.pop(0).wait() != 0:
                raise RuntimeError("hipcc failed")
    for p in running:
        if p.wait() != 0:
            raise RuntimeError("hipcc failed")
    tmp = LIB + ".tmp"
    _run(["hipcc", "-shared", "-fPIC", f"--offload-arch={ARCH}", *objs, "-o", tmp], verbose)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
