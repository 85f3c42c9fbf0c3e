"""The Python binding refuses buffers whose length differs from what the library
would read or write, before any device call (the C ABI takes bare pointers).

Runs on the CPU: the checks come before the device check, so CPU tensors of a
wrong length raise ValueError, and the methods are called on stand-in objects
that carry only the sizes (no library handle is ever used)."""
from types import SimpleNamespace

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_2402_08296_amd as dg  # noqa: E402
from tests._cases import small_problem  # noqa: E402


def _fake_problem(n=10, K=2, sub_ptr=(0, 6, 10)):
    hp = SimpleNamespace(sub_ptr=np.array(sub_ptr, np.int64))
    return SimpleNamespace(n=n, K=K, sum_k=int(sub_ptr[-1]), hp=hp, h=None, ctx=SimpleNamespace(h=None))


def f64(n):
    return torch.zeros(n, dtype=torch.float64)


def f32(n):
    return torch.zeros(n, dtype=torch.float32)


def test_dev_checks_length_dtype_and_device():
    with pytest.raises(ValueError, match="expected 5 values"):
        dg._dev(f64(4), n=5, what="u")
    with pytest.raises(TypeError, match="float64"):
        dg._dev(f32(5), n=5)
    with pytest.raises(TypeError, match="contiguous"):
        dg._dev(f64(10)[::2], n=5)
    with pytest.raises(TypeError, match="device"):
        dg._dev(f64(5), n=5)  # right length, but host memory
    with pytest.raises(TypeError):
        dg._dev(np.zeros(5), n=5)


@pytest.mark.parametrize("call", [
    lambda P: dg.Problem.solve(P, f64(9)),
    lambda P: dg.Problem.apply(P, f64(10), f64(11)),
    lambda P: dg.Problem.apply(P, f64(9), f64(10)),
    lambda P: dg.Problem.time_apply_stages(P, f64(10), f64(9)),
    lambda P: dg.Problem.spmv(P, f64(10), f64(12)),
    lambda P: dg.Problem.dss_forward(P, f64(9), f64(10)),
    lambda P: dg.Problem.dss_forward(P, f64(10), f64(11)),
    lambda P: dg.Problem.dss_forward_sub(P, 1, f64(6), f64(4)),   # sub-mesh 1 holds 4 nodes
    lambda P: dg.Problem.dss_forward_sub(P, 2, f64(4), f64(4)),   # no sub-mesh 2
    lambda P: dg.Problem.dss_forward_sub(P, -1, f64(6), f64(6)),
    lambda P: dg.Problem.train_rhs(P, f64(10), f32(9)),
    lambda P: dg.Problem.train_rhs(P, f64(11), f32(10)),
])
def test_problem_methods_refuse_wrong_lengths(call):
    with pytest.raises(ValueError):
        call(_fake_problem())


def test_apply_refuses_aliased_buffers(monkeypatch):
    monkeypatch.setattr(dg, "_devs", lambda *specs: [None] * len(specs))
    buf = f64(20)
    with pytest.raises(ValueError, match="alias"):
        dg.Problem.apply(_fake_problem(), buf[:10], buf[5:15])
    with pytest.raises(ValueError, match="alias"):
        dg.Problem.spmv(_fake_problem(), buf[:10], buf[:10])


def test_train_grad_refuses_bad_samples():
    P = _fake_problem()
    nt = dg.n_theta(30, 10)
    assert nt == 37530  # Table II, (kbar, d) = (30, 10)
    ok = dict(theta=f32(nt), c=f32(10), grad=f32(nt))
    with pytest.raises(ValueError, match="range"):
        dg.Problem.train_grad(P, subs=[0, 2], c_off=[0, 0], **ok)
    with pytest.raises(ValueError, match="outside"):
        dg.Problem.train_grad(P, subs=[0, 1], c_off=[0, 7], **ok)   # 7 + 4 > 10
    with pytest.raises(ValueError, match="outside"):
        dg.Problem.train_grad(P, subs=[0], c_off=[-1], **ok)
    with pytest.raises(ValueError, match="differ"):
        dg.Problem.train_grad(P, subs=[0, 1], c_off=[0], **ok)
    with pytest.raises(ValueError, match="theta"):
        dg.Problem.train_grad(P, subs=[0], c_off=[0], theta=f32(nt - 1), c=f32(10), grad=f32(nt))
    with pytest.raises(ValueError, match="grad"):
        dg.Problem.train_grad(P, subs=[0], c_off=[0], theta=f32(nt), c=f32(10), grad=f32(nt + 1))


def test_adam_dot_and_batch_refuse_wrong_lengths():
    ctx = SimpleNamespace(h=None)
    with pytest.raises(ValueError, match="m"):
        dg.adam_step(ctx, f32(5), f32(5), f32(4), f32(5), 1.0, 1)
    with pytest.raises(ValueError, match="y"):
        dg.Context.dot(ctx, f64(5), f64(6))
    P = _fake_problem()
    with pytest.raises(ValueError, match="u_outs"):
        dg.solve_batch(ctx, [P, P], [f64(10), f64(11)])
    with pytest.raises(ValueError, match="one output"):
        dg.solve_batch(ctx, [P, P], [f64(10)])


def test_host_problem_shapes_checked():
    _, hp = small_problem(seed=3, n=400, parts=2)
    fields = dict(xy=hp.xy, tri=hp.tri, dirichlet=hp.dirichlet, rowptr=hp.rowptr, col=hp.col, val=hp.val,
                  b=hp.b, u0=hp.u0, sub_ptr=hp.sub_ptr, sub_nodes=hp.sub_nodes, weights=hp.weights)
    dg.HostProblem(**fields)  # consistent
    for name, bad in [("b", hp.b[:-1]), ("u0", hp.u0[:-1]), ("dirichlet", hp.dirichlet[1:]),
                      ("rowptr", hp.rowptr[:-1]), ("col", hp.col[:-1]), ("val", hp.val[:-1]),
                      ("tri", hp.tri.ravel()[:-1]), ("weights", hp.weights[:-1]), ("sub_nodes", hp.sub_nodes[1:]),
                      ("xy", hp.xy.ravel())]:
        with pytest.raises(ValueError):
            dg.HostProblem(**{**fields, name: bad})
