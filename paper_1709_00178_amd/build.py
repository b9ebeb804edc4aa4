"""Build libpyrit.so (host plan + gfx950 HIP kernels) in-tree with hipcc.

Usage: python -m paper_1709_00178_amd.build [-v]
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libpyrit.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

SOURCES = [
    "plan.cpp",
    "serve.cpp",
    "device_api.hip",
    "batch.hip",
    "batch_host.cpp",
    "transpose.hip",
    "plain_ring0.hip",
    "plain_ring1.hip",
    "plain_ring2.hip",
    "plain_ring3.hip",
    "plain_ring4.hip",
    "plain_ring5.hip",
    "plain_ring6.hip",
    "plain_ring7.hip",
]

COMMON = ["-O3", "-fPIC", "-std=c++17", "-Wall", f"-I{os.path.join(HERE, '..', 'include')}"]
# Packed-FP32 instructions stay disabled in every device compile.
# The two LLVM options keep the small fields' fused coefficient bodies (a
# tree of wave-uniform branches on the coefficient's bits, 2^w leaves per
# output) in registers: without them the CFG structurizer turns each uniform
# if/else into a linear flow that keeps every accumulator's old value alive
# beside its new one (twice the VGPRs), and common-code sinking merges leaf
# bodies into one indexed by a PHI of array indices (arrays in scratch).
# Branches that are not wave-uniform are structurized as before.  The third
# option turns off GVN's memory-dependence queries, which took most of the
# compile time of those large bodies (minutes per kernel) and changed no
# instruction of the generated code.
HIP_FLAGS = [f"--offload-arch={ARCH}", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-fgpu-flush-denormals-to-zero", "-munsafe-fp-atomics",
             "-mllvm", "-structurizecfg-skip-uniform-regions=true",
             "-mllvm", "-simplifycfg-sink-common=false",
             "-mllvm", "-enable-gvn-memdep=false"]


def _compile(src: str, verbose: bool) -> str:
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    path = os.path.join(CSRC, src)
    if src.endswith(".hip"):
        cmd = [HIPCC, "-x", "hip", *HIP_FLAGS, *COMMON, "-c", path, "-o", obj]
    else:
        cmd = [HIPCC, "-x", "c++", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include", *COMMON,
               "-c", path, "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {src}\n{r.stdout}\n{r.stderr}")
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    workers = min(len(SOURCES), max(1, min(8, os.cpu_count() or 1)))
    with cf.ThreadPoolExecutor(workers) as ex:
        objs = list(ex.map(lambda s: _compile(s, verbose), SOURCES))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
