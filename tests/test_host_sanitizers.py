"""Host setup code built with AddressSanitizer and UBSan (CPU only, no GPU).

The driver (sanitize_setup_driver.cpp) runs validation, overlap expansion, the
local graphs, the coarse operator and its inverse and the local inverses of a
small generated problem; any out-of-bounds access, leak or undefined behaviour
aborts it.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

import workload as W
from tests._cases import host_problem

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CXX = "/opt/rocm/llvm/bin/amdclang++"


@pytest.mark.skipif(not os.path.exists(CXX), reason="amdclang++ not available")
def test_setup_under_address_and_ub_sanitizers(tmp_path):
    p = W.make_problem(12, 2500, 5, 0.3)
    hp = host_problem(p)
    arrays = {"xy": hp.xy, "val": hp.val, "b": hp.b, "u0": hp.u0, "weights": hp.weights, "tri": hp.tri,
              "rowptr": hp.rowptr, "col": hp.col, "sub_nodes": hp.sub_nodes, "part": p.part.astype(np.int32),
              "dirichlet": hp.dirichlet, "sub_ptr": hp.sub_ptr, "meta": np.array([p.n_parts, 2], np.int64)}
    for name, a in arrays.items():
        np.ascontiguousarray(a).tofile(str(tmp_path / name))
    exe = str(tmp_path / "driver")
    src = os.path.join(ROOT, "paper_2402_08296_amd", "csrc")
    cmd = [CXX, "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-I", os.path.join(ROOT, "include"), "-I", src,
           os.path.join(HERE, "sanitize_setup_driver.cpp"), os.path.join(src, "setup.cpp"), "-o", exe, "-lpthread"]
    subprocess.check_call(cmd)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe, str(tmp_path)], capture_output=True, text=True, timeout=600, env=env)
    print(r.stdout, r.stderr[-2000:])
    assert r.returncode == 0 and r.stdout.startswith("OK"), r.stderr[-2000:]
    shutil.rmtree(tmp_path, ignore_errors=True)
