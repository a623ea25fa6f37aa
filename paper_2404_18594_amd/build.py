"""Build the gfx950 shared library libcdtwa.so in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libcdtwa.so")
SOURCES = ["csrc/host.cpp", "csrc/host_mlp.cpp", "csrc/host_batch.cpp", "csrc/kernels_generic.hip",
           "csrc/kernels_big.hip", "csrc/kernels_batch.hip", "csrc/kernels_dense.hip", "csrc/kernels_spin.hip",
           "csrc/kernels_spin_fused.hip", "csrc/kernels_fused.hip", "csrc/kernels_plaq.hip",
           "csrc/kernels_mlp.hip", "csrc/noalloc.hip", "csrc/kernels_traj.hip"]
FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950",
    # packed FP32 math disabled: plain FP32 VALU instructions only
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]


def build(verbose: bool = False, jobs: int = 4) -> str:
    """Compile every source to an object in parallel, then link."""
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    procs, objs = [], []
    for src in SOURCES:
        obj = os.path.join(objdir, os.path.basename(src) + ".o")
        objs.append(obj)
        lang = ["-x", "hip"] if src.endswith(".hip") else []
        cmd = ["hipcc", *FLAGS, "-c", *lang, os.path.join(HERE, src), "-o", obj,
               "-I", os.path.join(ROOT, "include")]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append(subprocess.Popen(cmd))
        if len(procs) >= jobs:
            for p in procs:
                if p.wait() != 0:
                    raise RuntimeError("hipcc failed")
            procs = []
    for p in procs:
        if p.wait() != 0:
            raise RuntimeError("hipcc failed")
    tmp = LIB + f".tmp{os.getpid()}"
    subprocess.run(["hipcc", "-shared", "-fPIC", "--offload-arch=gfx950", *objs, "-o", tmp], check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
    print(LIB)
