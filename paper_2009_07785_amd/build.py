"""Builds the gfx950 propagation library (libprop.so) in-tree with hipcc."""
from __future__ import annotations

import os
import shutil
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libprop.so")
SOURCES = ["prop_kernels.hip", "prop_batch.hip", "prop_static.hip", "prop_host.cpp",
           "prop_layout_host.cpp", "prop_serve.cpp"]
ARCH = "gfx950"


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found; the HIP library cannot be built")


def build(verbose: bool = False) -> str:
    """Compile every source of the library for gfx950; returns the .so path."""
    tmp = LIB + ".tmp"
    cmd = [
        hipcc(), f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-shared",
        "-ffp-contract=off", "-fno-fast-math",
        # keep the per-step register arrays as scalars: promoting them to one
        # vector register tuple makes every guarded step copy the whole tuple
        "-mllvm", "-amdgpu-promote-alloca-to-vector-limit=1",
        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
        "-Wall", "-Wno-unused-function", "-pthread",
        "-I", os.path.join(os.path.dirname(HERE), "include"),
        *[os.path.join(CSRC, s) for s in SOURCES],
        "-o", tmp,
    ]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"hipcc failed ({res.returncode}):\n{res.stderr[-6000:]}")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
