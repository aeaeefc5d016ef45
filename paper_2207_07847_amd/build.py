"""Build liblapgpu.so (HIP for gfx950 + host setup) in-tree.

    python -m paper_2207_07847_amd.build
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "liblapgpu.so")
ARCH = os.environ.get("LAPGPU_ARCH", "gfx950")

# Packed FP32 instructions stay off on this target (see the design notes).
# Kernel arguments are preloaded into SGPRs (up to 16 dwords): a kernel's
# first loads then do not wait for a load of its own arguments.  The
# compiler keeps a prologue that loads them for firmware without preload.
HIP_FLAGS = ["-O3", "-std=c++17", f"--offload-arch={ARCH}", "-fPIC",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-mllvm", "-amdgpu-kernarg-preload-count=16",
             "-Wall", "-Wno-unused-result"]


def _hipcc():
    for cand in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def build(verbose: bool = False) -> str:
    os.makedirs(os.path.join(HERE, "_build"), exist_ok=True)
    obj = os.path.join(HERE, "_build", "setup.o")
    cmd1 = ["g++", "-O3", "-std=c++17", "-fPIC", "-Wall", "-c", "-I", INCLUDE, "-I", CSRC,
            os.path.join(CSRC, "setup.cpp"), "-o", obj]
    hobj = os.path.join(HERE, "_build", "lap.o")
    cmd2 = [_hipcc(), *HIP_FLAGS, "-c", "-I", INCLUDE, "-I", CSRC,
            os.path.join(CSRC, "lap.hip"), "-o", hobj]
    tmp = LIB + ".tmp"
    cmd3 = [_hipcc(), f"--offload-arch={ARCH}", "-shared", hobj, obj, "-o", tmp]
    for cmd in (cmd1, cmd2, cmd3):
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
