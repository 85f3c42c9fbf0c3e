"""GPU: launch schedules (the autotuner's choices) against the default schedule.

The DSS workgroup size is a pure schedule: each tile is computed the same way
whichever workgroup runs it, and the restriction sums follow one fixed order,
so the bar is bitwise equality. The vector-kernel workgroup count reorders the
Krylov reductions, so a solve under another count is held to the solve bars of
test_gpu_parity.py (converged, true residual, iterations close to the default's).
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_2402_08296_amd as dg  # noqa: E402
import workload as W  # noqa: E402
from tests._cases import oracle_problem  # noqa: E402

pytestmark = pytest.mark.gpu

SMOOTHER = W.smoother_theta(omega=0.15, out_scale=1.7)


@pytest.fixture(scope="module")
def ctx():
    print("[gpu] creating context", flush=True)
    return dg.Context()


@pytest.fixture(scope="module")
def mixed():
    # sub-meshes of uneven size: some fit two workgroups per compute unit, some do not
    p = W.make_problem(31, 12000, 18, 0.45)  # sub-meshes of 470..1613 nodes
    return p, oracle_problem(p)


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, np.float64)).cuda()


def test_small_workgroups_keep_every_bit(ctx, mixed):
    print("[gpu] DSS schedule split", flush=True)
    p, hp = mixed
    k = np.diff(hp.sub_ptr)
    print(f"[gpu]   sub-mesh sizes {k.min()}..{k.max()}", flush=True)
    prob = dg.Problem(ctx, hp, dg.Model(ctx, SMOOTHER))
    r = np.random.default_rng(9).standard_normal(p.n)
    r[p.mesh.dirichlet == 1] = 0
    o = dg.default_opts(precision="bf16")
    outs = []
    for lds in (0, 48 * 1024, 79 * 1024):
        prob.set_tuning(small_lds=lds)
        assert prob.tuning().small_lds == lds
        z = torch.empty(p.n, dtype=torch.float64, device="cuda")
        prob.apply(_dev(r), z, o)
        outs.append((z, [t.clone() for t in prob.intermediates()]))
    for z, inter in outs[1:]:
        assert torch.equal(z, outs[0][0])
        for a, b in zip(inter, outs[0][1]):
            assert torch.equal(a, b)
    u1 = torch.empty(p.n, dtype=torch.float64, device="cuda")
    u2 = torch.empty_like(u1)
    prob.set_tuning(small_lds=0)
    s1 = prob.solve(u1, dg.default_opts(precision="bf16", rtol=1e-6))
    prob.set_tuning(small_lds=79 * 1024)
    s2 = prob.solve(u2, dg.default_opts(precision="bf16", rtol=1e-6))
    assert s1.converged and s1.iterations == s2.iterations and torch.equal(u1, u2)


def test_vector_workgroups_and_autotune(ctx, mixed):
    print("[gpu] vec_blocks / autotune", flush=True)
    p, hp = mixed
    prob = dg.Problem(ctx, hp, dg.Model(ctx, SMOOTHER))
    u = torch.empty(p.n, dtype=torch.float64, device="cuda")
    base = prob.solve(u, dg.default_opts(precision="fp64", rtol=1e-8))
    prob.set_tuning(vec_blocks=8)
    st = prob.solve(u, dg.default_opts(precision="fp64", rtol=1e-8))
    print(f"[gpu]   iterations default={base.iterations} vec_blocks=8: {st.iterations}", flush=True)
    assert st.converged and abs(st.iterations - base.iterations) <= 1 and st.true_rel_residual <= 2e-8
    t, ms = prob.autotune(dg.default_opts(precision="bf16"), 8)
    print(f"[gpu]   autotune -> {t.as_dict()} {ms:.3f} ms/iteration", flush=True)
    assert ms > 0 and prob.tuning().as_dict() == t.as_dict()
    assert t.small_lds in (0, 48 * 1024, 64 * 1024, 79 * 1024) and t.vec_blocks in (0, 256, 512, 1024)
    st = prob.solve(u, dg.default_opts(precision="bf16", rtol=1e-6))
    assert st.converged and st.true_rel_residual <= 1.5e-6
    with pytest.raises(dg.DDMGNNError):
        prob.set_tuning(small_lds=200_000)
    with pytest.raises(dg.DDMGNNError):
        prob.set_tuning(vec_blocks=12)


def test_forked_schedule_in_batches_and_stage_timing(ctx, mixed):
    """Problems with the split schedule (two DSS launches on two streams) solved in one
    batch give the bits of their solo solves under the default schedule; the stage
    timer leaves z = M(r) and reports positive times."""
    print("[gpu] forked schedule in a batch / stage timing", flush=True)
    p, hp = mixed
    q = W.make_problem(32, 9000, 14, 0.45)
    hq = oracle_problem(q)
    model = dg.Model(ctx, SMOOTHER)
    o = dg.default_opts(precision="bf16", rtol=1e-6)
    solo = []
    for pp, hh in ((p, hp), (q, hq)):
        prob = dg.Problem(ctx, hh, model)
        u = torch.empty(pp.n, dtype=torch.float64, device="cuda")
        st = prob.solve(u, o)
        solo.append((u.cpu().numpy(), st.iterations))
    probs = [dg.Problem(ctx, hh, model) for hh in (hp, hq)]
    for pr in probs:
        pr.set_tuning(small_lds=79 * 1024)
    outs = [torch.empty(pp.n, dtype=torch.float64, device="cuda") for pp in (p, q)]
    sts = dg.solve_batch(ctx, probs, outs, o)
    for (u, it), ub, st in zip(solo, outs, sts):
        assert st.converged and st.iterations == it and np.array_equal(ub.cpu().numpy(), u)
    r = np.random.default_rng(5).standard_normal(p.n)
    r[p.mesh.dirichlet == 1] = 0
    z1 = torch.empty(p.n, dtype=torch.float64, device="cuda")
    z2 = torch.empty_like(z1)
    probs[0].apply(_dev(r), z1, o)
    t_local, t_coarse, t_glue = probs[0].time_apply_stages(_dev(r), z2, o, reps=3)
    print(f"[gpu]   stages {t_local:.3f} {t_coarse:.3f} {t_glue:.3f} ms", flush=True)
    assert t_local > 0 and t_coarse > 0 and t_glue > 0
    assert torch.equal(z1, z2)
