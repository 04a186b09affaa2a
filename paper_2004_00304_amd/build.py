"""Build the gfx950 HIP library liblbmpcd.so in-tree with hipcc.

Flags: IEEE arithmetic without FMA contraction (-ffp-contract=off; explicit
fma() only where the method's update uses one), no packed FP32 ops, native
FP64 atomics (the workspace is ordinary coarse-grained device memory).
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "liblbmpcd.so")
SOURCES = ["api.hip", "kernels_lb.hip", "kernels_mpcd.hip", "kernels_mpcd_ce.hip", "kernels_mpcd_det.hip",
           "kernels_util.hip", "kernels_mlp.hip"]
ARCH = os.environ.get("LBMPCD_ARCH", "gfx950")

FLAGS = [
    "-O3", "-std=c++17", f"--offload-arch={ARCH}", "-fPIC",
    "-ffp-contract=off", "-fno-fast-math", "-munsafe-fp-atomics",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-result",
]
PER_FILE: dict[str, list[str]] = {}


def build(force: bool = True, verbose: bool = False) -> str:
    if not force and os.path.exists(LIB):
        return LIB
    os.makedirs(OBJ, exist_ok=True)
    procs, objs = [], []
    for src in SOURCES:
        obj = os.path.join(OBJ, src.replace(".hip", ".o"))
        cmd = ["hipcc", *FLAGS, *PER_FILE.get(src, []), "-c", "-o", obj, os.path.join(CSRC, src)]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((src, subprocess.Popen(cmd)))
        objs.append(obj)
    failed = [src for src, pr in procs if pr.wait() != 0]
    if failed:
        raise RuntimeError(f"hipcc failed for {', '.join(failed)}")
    tmp = LIB + ".tmp"
    cmd = ["hipcc", f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    print(LIB)
    sys.exit(0)
