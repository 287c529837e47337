"""Compile the HIP C-ABI library ``librpy.so`` for gfx950 (in-tree).

Every HIP source is compiled with ``-Xclang -target-feature -Xclang
-packed-fp32-ops`` so that hipcc never emits packed FP32 instructions.
"""
from __future__ import annotations

import glob
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "librpy.so")
INCLUDE = os.path.join(os.path.dirname(HERE), "include")

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-Wall",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]
# Per-file additions.  The block-product and W-tile kernels keep their MFMA
# accumulators in ordinary VGPRs: with the default heuristic the loop-carried
# FP64 accumulators are copied to and from AGPRs around every MFMA batch.
FILE_FLAGS = {
    "rpy_block.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form"],
    "rpy_grad.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form"],
}


def _run(cmd):
    print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)


def build(jobs: int = 4) -> str:
    """Compile each .hip to an object in parallel, then link librpy.so."""
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")))
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    objs, procs = [], []
    for src in srcs:
        obj = os.path.join(objdir, os.path.basename(src) + ".o")
        objs.append(obj)
        extra = FILE_FLAGS.get(os.path.basename(src), [])
        cmd = [hipcc, *HIPCC_FLAGS, *extra, "-I", INCLUDE, "-c", src, "-o", obj]
        print(" ".join(cmd), flush=True)
        procs.append(subprocess.Popen(cmd))
        if len(procs) >= jobs:
            if procs.pop(0).wait() != 0:
                raise RuntimeError("hipcc failed")
    for p in procs:
        if p.wait() != 0:
            raise RuntimeError("hipcc failed")
    tmp = LIB + ".tmp"
    _run([hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(int(sys.argv[1]) if len(sys.argv) > 1 else 4)
