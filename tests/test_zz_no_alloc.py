"""The allocation-free dot product (ddmgnn_dot_noalloc) against ddmgnn_dot.

Both run the solver's two-kernel reduction (per-workgroup partial sums, then
one workgroup sums them in workgroup order), so the results agree bit for bit;
both are also held to the reordered-FP64 bar against numpy. Two calls in a
row, the second on a smaller input, check that the shared static scratch
carries nothing from one call into the next.
"""
import ctypes

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_2402_08296_amd as dg  # noqa: E402

pytestmark = pytest.mark.gpu


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, np.float64)).cuda()


@pytest.mark.timeout(120)
def test_dot_noalloc_matches_dot():
    ctx = dg.Context()
    out = torch.full((1,), np.nan, dtype=torch.float64, device="cuda")
    for n in (262_144 * 3 + 17, 1000, 1, 0):
        print(f"[gpu] dot_noalloc n={n}", flush=True)
        rng = np.random.default_rng(n)
        a, b = rng.standard_normal(n), rng.standard_normal(n)
        x, y = _dev(a), _dev(b)
        ref = ctx.dot(x, y)
        out.fill_(np.nan)
        ctx.dot_noalloc(x, y, out)
        torch.cuda.synchronize()
        got = float(out.cpu()[0])
        assert got == ref, (n, got, ref)
        assert abs(got - float(a @ b)) <= 1e-13 * float(np.abs(a) @ np.abs(b))


@pytest.mark.timeout(120)
def test_dot_noalloc_refuses_oversized_n():
    ctx = dg.Context()
    x = _dev(np.ones(4))
    out = torch.zeros(1, dtype=torch.float64, device="cuda")
    p = ctypes.c_void_p
    rc = dg.lib().ddmgnn_dot_noalloc(ctx.h, 2**31, p(x.data_ptr()), p(x.data_ptr()), p(out.data_ptr()))
    assert rc == -1  # DDMGNN_E_INVALID
    assert b"DDMGNN_NOALLOC_DOT_MAX_N" in dg.lib().ddmgnn_last_error()
    assert dg.lib().ddmgnn_dot_noalloc(ctx.h, -1, p(x.data_ptr()), p(x.data_ptr()), p(out.data_ptr())) == -1
