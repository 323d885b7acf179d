"""Build librcb.so (HIP, gfx950) in-tree with hipcc.

The build, walk and neighbour kernels are compiled with -ffp-contract=off:
their canonical sums and predicates must round exactly like their
definitions. The interaction kernels (gravity, VJP) allow multiply-add
contraction. Packed FP32 instructions are disabled everywhere.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
OBJ = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "librcb.so")
ARCH = os.environ.get("RCB_OFFLOAD_ARCH", "gfx950")

SOURCES = ["rcb_api.hip", "k_build.hip", "k_scan.hip", "k_walk.hip", "k_neigh.hip", "k_grav.hip",
           "k_vjp.hip", "k_sort.hip"]
CONTRACT = {"k_grav.hip": "-ffp-contract=fast", "k_vjp.hip": "-ffp-contract=fast"}
FLAGS = ["-O3", "-fPIC", "-std=c++17", f"--offload-arch={ARCH}",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-Wall", "-Wno-unused-result",
         "-I", INCLUDE, "-I", CSRC]


def _compile(src: str) -> str:
    obj = os.path.join(OBJ, src.replace(".hip", ".o"))
    cmd = ["hipcc", "-c", *FLAGS, CONTRACT.get(src, "-ffp-contract=off"), "-o", obj,
           os.path.join(CSRC, src)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr}")
    return obj


def build(verbose: bool = True) -> str:
    os.makedirs(OBJ, exist_ok=True)
    with ThreadPoolExecutor(max_workers=min(8, len(SOURCES))) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = ["hipcc", "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + r.stderr)
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build()
    sys.exit(0)
