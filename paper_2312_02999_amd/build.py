"""Build libpdipc.so (HIP, gfx950) in-tree with hipcc.

Usage: python -m paper_2312_02999_amd.build   (or build() from Python)
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libpdipc.so")
ARCH = os.environ.get("PDIPC_ARCH", "gfx950")

SOURCES = ["k_local.hip", "k_util.hip", "k_contact.hip", "k_barrier.hip", "k_factor.hip", "k_dense.hip",
           "k_cinv.hip", "k_adjoint.hip", "k_variants.hip", "k_noalloc.hip", "solver.cpp", "host_factor.cpp"]

# Packed FP32 instructions are disabled for every device pass.
DEVICE_FLAGS = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
COMMON = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-Wno-unused-result",
          "-I", os.path.join(HERE, "..", "include")]
# Sources whose floating point decides a discrete result (constraint-set
# membership, the closest feature of a pair): every product and sum rounded on
# its own, so that the decision follows the written formula bit for bit.
NO_CONTRACT = {"k_contact.hip", "k_barrier.hip"}


def _hipcc() -> str:
    for p in ("/opt/rocm/bin/hipcc", "hipcc"):
        if os.path.exists(p) or p == "hipcc":
            return p
    return "hipcc"


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    path = os.path.join(CSRC, src)
    if src.endswith(".hip"):
        extra = ["-ffp-contract=off"] if src in NO_CONTRACT else []
        cmd = [_hipcc(), "-x", "hip", *COMMON, *DEVICE_FLAGS, *extra, "-c", path, "-o", obj]
    else:
        cmd = [_hipcc(), *COMMON, "-c", path, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return obj


def build(verbose: bool = True) -> str:
    os.makedirs(BUILD, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 4)) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB + ".tmp"
    cmd = [_hipcc(), "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}")
    return LIB


if __name__ == "__main__":
    build()
    sys.exit(0)
