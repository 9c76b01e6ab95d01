"""Builds libgridenv.so (the gfx950 kernels and the C-ABI) in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libgridenv.so")
SOURCES = [os.path.join(CSRC, "kernels.hip"), os.path.join(CSRC, "render.hip"),
           os.path.join(CSRC, "runtime.cpp"), os.path.join(CSRC, "server.cpp"),
           os.path.join(CSRC, "static_rollout.cpp"), os.path.join(CSRC, "probe.hip")]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # the reward is three separately rounded fp32 operations: no contraction
    "-ffp-contract=off",
    # no packed fp32 instructions anywhere in device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


def build(verbose: bool = False) -> str:
    tmp = LIB + ".tmp"
    cmd = [HIPCC, *FLAGS]
    for src in SOURCES:
        cmd += ["-x", "hip", src]
    cmd += ["-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
