"""Build the HIP library libfv3.so in-tree for gfx950 (hipcc)."""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libfv3.so")
SOURCES = ["grid.cpp", "abi.cpp", "kernels.hip", "ensemble.cpp", "correction.hip", "mlp.hip", "remap.hip"]
# Packed FP32 instructions are disabled for all device code.
HIPFLAGS = ["-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC", "-Wall",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def build(verbose: bool = False, jobs: int = 4) -> str:
    objs = []
    procs = []
    for src in SOURCES:
        obj = os.path.join(CSRC, src + ".o")
        cmd = ["hipcc", "-c"] + HIPFLAGS + ["-o", obj, os.path.join(CSRC, src)]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((cmd, subprocess.Popen(cmd)))
        objs.append(obj)
    for cmd, p in procs:
        if p.wait() != 0:
            raise RuntimeError("compile failed: " + " ".join(cmd))
    # link to a temporary name and rename, so a reader never sees a partial file
    tmp = LIB + ".tmp"
    link = ["hipcc", "-shared", "--offload-arch=gfx950", "-fPIC", "-o", tmp] + objs
    if verbose:
        print(" ".join(link), flush=True)
    subprocess.run(link, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
