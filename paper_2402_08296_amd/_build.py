"""Build libddmgnn.so (HIP for gfx950) in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libddmgnn.so")
SOURCES = [os.path.join(HERE, "csrc", f) for f in
           ("kernels.hip", "dss_mfma.hip", "train.hip", "noalloc.hip", "factor.hip", "overlap.hip", "runtime.cpp", "server.cpp")]
# plain host C++ (no HIP): compiled for the host only, then linked in
HOST_SOURCES = [os.path.join(HERE, "csrc", f) for f in ("setup.cpp",)]
HOST_FLAGS = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function"]

HIP_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # keep the compiler from emitting packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


def _obj(src: str) -> str:
    return LIB + "." + os.path.splitext(os.path.basename(src))[0] + ".o"


def build(verbose: bool = False) -> str:
    """Compiles every translation unit to an object in parallel (each HIP source
    holds its own device code, none calls another's), then links the library."""
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    cxx = os.environ.get("HOST_CXX", "/opt/rocm/llvm/bin/amdclang++")
    inc = ["-I", os.path.join(ROOT, "include"), "-I", os.path.join(HERE, "csrc")]
    cmds = [[cxx, *HOST_FLAGS, *inc, "-c", s, "-o", _obj(s)] for s in HOST_SOURCES]
    cmds += [[hipcc, *HIP_FLAGS, *inc, "-c", s, "-o", _obj(s)] for s in SOURCES]

    def run(cmd):
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.check_call(cmd)

    objs = [c[-1] for c in cmds]
    try:
        with ThreadPoolExecutor(max_workers=min(len(cmds), os.cpu_count() or 1)) as ex:
            list(ex.map(run, cmds))
        run([hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", LIB + ".tmp", *objs])
    finally:
        for obj in objs:
            if os.path.exists(obj):
                os.remove(obj)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
