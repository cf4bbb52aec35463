"""Compiles librg.so (the HIP library behind include/rg.h) for gfx950, in-tree."""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "librg.so")
SOURCES = ["build.hip", "trace.hip", "render.hip", "serve.hip", "post.hip"]
ARCH = "gfx950"

FLAGS = [
    "--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC", "-shared",
    # keep float arithmetic scalar: packed fp32 forms are not used
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # wave-uniform branches stay plain scalar branches: structurizing them as
    # if they were divergent makes the values they select between meet in
    # joins that cost a register copy per value
    "-mllvm", "-structurizecfg-skip-uniform-regions=true",
    "-Wno-unused-command-line-argument",
]


def build(verbose: bool = False) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    tmp = LIB + ".tmp"
    cmd = [hipcc] + FLAGS + [os.path.join(CSRC, s) for s in SOURCES] + ["-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + res.stdout[-4000:] + res.stderr[-8000:])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
