"""Build libddmgnn.so (HIP for gfx950) in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libddmgnn.so")
SOURCES = [os.path.join(HERE, "csrc", f) for f in
           ("kernels.hip", "dss_mfma.hip", "train.hip", "runtime.cpp", "server.cpp")]
# plain host C++ (no HIP): compiled for the host only, then linked in
HOST_SOURCES = [os.path.join(HERE, "csrc", f) for f in ("setup.cpp",)]
HOST_FLAGS = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function"]

HIP_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # keep the compiler from emitting packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


def build(verbose: bool = False) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    cxx = os.environ.get("HOST_CXX", "/opt/rocm/llvm/bin/amdclang++")
    inc = ["-I", os.path.join(ROOT, "include"), "-I", os.path.join(HERE, "csrc")]
    objs = []
    for src in HOST_SOURCES:
        obj = LIB + "." + os.path.splitext(os.path.basename(src))[0] + ".o"
        cmd = [cxx, *HOST_FLAGS, *inc, "-c", src, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.check_call(cmd)
        objs.append(obj)
    # "-x none": objects after the HIP sources are linked, not compiled
    cmd = [hipcc, *HIP_FLAGS, *inc, "-o", LIB + ".tmp", *SOURCES, "-x", "none", *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    for obj in objs:
        os.remove(obj)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
