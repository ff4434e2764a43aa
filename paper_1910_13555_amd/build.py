"""Build libbsm.so for gfx950 in-tree with hipcc (no JIT, no torch extension).

Sources: csrc/bsm_symbolic.hip (norms, symbolic phase), csrc/bsm_numeric.hip
(numeric kernel), csrc/bsm_backward.hip (gradient product lists) and csrc/bsm_api.cpp (host
planner and the C ABI of include/bsm.h).
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libbsm.so")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
         # packed fp32 instructions stay off: some of their forms have given
         # wrong results on this hardware now and then, without an error
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-function", "-Wno-unused-result",
         "-I", os.path.join(ROOT, "include")]

SOURCES = ["bsm_scan.hip", "bsm_symbolic.hip", "bsm_numeric.hip", "bsm_numeric_rm.hip", "bsm_numeric_rmb.hip", "bsm_numeric_gen.hip", "bsm_split.hip", "bsm_order.hip", "bsm_steps.hip",
           "bsm_backward.hip", "bsm_remap.hip", "bsm_noalloc.hip",
           "bsm_api.cpp", "bsm_tensor.cpp", "bsm_batch.cpp", "bsm_check.cpp", "bsm_ops.hip", "bsm_ops_api.cpp"]


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC, *FLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stdout}\n{r.stderr}")
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    with ThreadPoolExecutor(len(SOURCES)) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
