"""GPU: several problems solved together (one launch per kernel) and the
serving loop, against each problem solved alone.

A problem's arithmetic does not depend on the other members of its batch
(its reductions run over its own workgroups in a fixed order, its DSS
workgroups see only its own sub-meshes), so the bar is bitwise equality of
the solutions and equal iteration counts. The solo solves themselves are
pinned to the oracle in test_gpu_parity.py.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_2402_08296_amd as dg  # noqa: E402
import workload as W  # noqa: E402
from tests._cases import oracle_problem  # noqa: E402

pytestmark = pytest.mark.gpu

SMOOTHER = W.smoother_theta(omega=0.15, out_scale=1.7)
# sizes spanning one to several vector workgroups per problem, one single-sub-mesh problem
SPECS = [(201, 3000, 4), (202, 9000, 12), (203, 700, 1), (204, 5000, 7)]


@pytest.fixture(scope="module")
def ctx():
    print("[gpu] creating context", flush=True)
    return dg.Context()


@pytest.fixture(scope="module")
def mix():
    out = []
    for seed, n, parts in SPECS:
        p = W.make_problem(seed, n, parts, 0.2)
        out.append((p, oracle_problem(p)))
    return out


def _solo(ctx, model, mix, opts):
    res = []
    for p, hp in mix:
        prob = dg.Problem(ctx, hp, model)
        u = torch.empty(p.n, dtype=torch.float64, device="cuda")
        st = prob.solve(u, opts, check=False)
        res.append((u.cpu().numpy(), st.iterations, st.status))
    return res


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16"])
def test_batch_equals_solo(ctx, mix, prec):
    print(f"[gpu] batch vs solo {prec}", flush=True)
    model = dg.Model(ctx, SMOOTHER)
    opts = dg.default_opts(precision=prec, rtol=1e-6, max_it=3000)
    solo = _solo(ctx, model, mix, opts)
    probs = [dg.Problem(ctx, hp, model) for _, hp in mix]
    outs = [torch.empty(p.n, dtype=torch.float64, device="cuda") for p, _ in mix]
    for rep in range(2):  # second call replays the cached batch and graph
        sts = dg.solve_batch(ctx, probs, outs, opts)
        for i, ((u, it, status), ub, st) in enumerate(zip(solo, outs, sts)):
            print(f"[gpu]   rep {rep} problem {i}: iterations solo={it} batch={st.iterations}", flush=True)
            assert status == 0 and st.status == 0 and st.converged
            assert st.iterations == it
            assert np.array_equal(ub.cpu().numpy(), u), (rep, i)
    # each member's solution checked outside the library: scipy residual and direct solve
    import scipy.sparse.linalg as spl
    for (p, _), ub in zip(mix, outs):
        A = p.A.to_scipy()
        ug = ub.cpu().numpy()
        res = np.linalg.norm(p.b - A @ ug) / np.linalg.norm(p.b - A @ p.u0)
        ud = spl.spsolve(A.tocsc(), p.b)
        err = np.linalg.norm(ug - ud) / np.linalg.norm(ud)
        print(f"[gpu]   N={p.n}: scipy residual {res:.2e}, L2 vs direct {err:.2e}", flush=True)
        assert res <= 1e-6 and err <= 1e-4


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_wide_and_narrow_dss_forms_agree(ctx, prec):
    """A solve whose launches hold fewer sub-meshes than the device has compute units runs
    the 1024-thread VALU DSS form; 33 copies of the same problem in one batch (264
    sub-meshes) run the 512-thread form. Both forms sum the restriction norms over the same
    virtual threads, so every copy equals the solo solve bit for bit."""
    print(f"[gpu] wide vs narrow DSS form {prec}", flush=True)
    p = W.config_problem("c1", 0)
    hp = oracle_problem(p)
    assert hp.K * 33 >= 256 > hp.K
    model = dg.Model(ctx, SMOOTHER)
    opts = dg.default_opts(precision=prec, rtol=1e-8, max_it=500)
    (u, it, status), = _solo(ctx, model, [(p, hp)], opts)
    probs = [dg.Problem(ctx, hp, model) for _ in range(33)]
    outs = [torch.empty(p.n, dtype=torch.float64, device="cuda") for _ in probs]
    sts = dg.solve_batch(ctx, probs, outs, opts)
    print(f"[gpu]   solo {it} iterations, batch {[st.iterations for st in sts][:3]}...", flush=True)
    assert status == 0
    for st, ub in zip(sts, outs):
        assert st.converged and st.iterations == it and np.array_equal(ub.cpu().numpy(), u)


def test_batch_lu_equals_solo(ctx, mix):
    """DDM-LU (exact local solves) batched: same bits and iterations as solo; the
    one-sub-mesh problem with its exact local solve converges at once."""
    print("[gpu] batch vs solo DDM-LU", flush=True)
    model = dg.Model(ctx, SMOOTHER)
    opts = dg.default_opts(krylov=dg.PCG, local_solver=dg.LOCAL_LU, prolong=dg.PROLONG_UNWEIGHTED,
                           precision="fp64", rtol=1e-8, max_it=500)
    solo = _solo(ctx, model, mix, opts)
    probs = [dg.Problem(ctx, hp, model) for _, hp in mix]
    outs = [torch.empty(p.n, dtype=torch.float64, device="cuda") for p, _ in mix]
    sts = dg.solve_batch(ctx, probs, outs, opts)
    for i, ((u, it, status), ub, st) in enumerate(zip(solo, outs, sts)):
        print(f"[gpu]   problem {i}: iterations solo={it} batch={st.iterations} kernel={st.dss_kernel}", flush=True)
        assert status == 0 and st.status == 0 and st.converged and st.dss_kernel == 3
        assert st.iterations == it
        assert np.array_equal(ub.cpu().numpy(), u), i
    one = [i for i, spec in enumerate(SPECS) if spec[2] == 1][0]
    assert sts[one].iterations <= 2
    # the inverses are held on the device: sum k_i^2 doubles more than before
    hp = mix[1][1]
    k = np.diff(hp.sub_ptr).astype(np.int64)
    assert probs[1].device_bytes() >= int((k * k).sum()) * 8


def test_batch_fgmres_equals_solo(ctx, mix):
    """FGMRES(8) batched: restarts at different iterations per problem, same bits as solo."""
    print("[gpu] batch vs solo FGMRES", flush=True)
    model = dg.Model(ctx, SMOOTHER)
    opts = dg.default_opts(krylov=dg.FGMRES, restart=8, precision="fp32", rtol=1e-7, max_it=800)
    solo = _solo(ctx, model, mix, opts)
    probs = [dg.Problem(ctx, hp, model) for _, hp in mix]
    outs = [torch.empty(p.n, dtype=torch.float64, device="cuda") for p, _ in mix]
    sts = dg.solve_batch(ctx, probs, outs, opts)
    for i, ((u, it, status), ub, st) in enumerate(zip(solo, outs, sts)):
        print(f"[gpu]   problem {i}: iterations solo={it} batch={st.iterations}", flush=True)
        assert status == 0 and st.status == 0 and st.converged
        assert st.iterations == it
        assert np.array_equal(ub.cpu().numpy(), u), i


def test_batch_order_and_eager(ctx, mix):
    """Member order and eager launches do not change any member's result."""
    print("[gpu] batch order / eager", flush=True)
    model = dg.Model(ctx, SMOOTHER)
    opts = dg.default_opts(precision="fp32", rtol=1e-6, max_it=3000, m_max=2)
    solo = _solo(ctx, model, mix, opts)
    probs = [dg.Problem(ctx, hp, model) for _, hp in mix]
    order = [2, 0, 3, 1]
    outs = [torch.empty(mix[i][0].n, dtype=torch.float64, device="cuda") for i in order]
    for graph in (1, 0):
        sts = dg.solve_batch(ctx, [probs[i] for i in order], outs,
                             dg.default_opts(precision="fp32", rtol=1e-6, max_it=3000, m_max=2, graph=graph,
                                             check_every=5))
        for j, i in enumerate(order):
            assert sts[j].iterations == solo[i][1]
            assert np.array_equal(outs[j].cpu().numpy(), solo[i][0]), (graph, i)


def test_batch_masks_and_status(ctx, mix):
    """A member with a zero initial residual and one that hits max_it leave the others untouched."""
    print("[gpu] batch masks", flush=True)
    model = dg.Model(ctx, SMOOTHER)
    p0, hp0 = mix[0]
    zero = dg.HostProblem(hp0.xy, hp0.tri, hp0.dirichlet, hp0.rowptr, hp0.col, hp0.val,
                          p0.A.to_scipy() @ p0.u0, p0.u0, hp0.sub_ptr, hp0.sub_nodes, hp0.weights)
    opts = dg.default_opts(precision="fp32", rtol=1e-6, max_it=3000)
    solo = _solo(ctx, model, mix[1:2], opts)
    probs = [dg.Problem(ctx, zero, model), dg.Problem(ctx, mix[1][1], model)]
    outs = [torch.empty(p0.n, dtype=torch.float64, device="cuda"),
            torch.empty(mix[1][0].n, dtype=torch.float64, device="cuda")]
    sts = dg.solve_batch(ctx, probs, outs, opts)
    assert sts[0].iterations == 0 and sts[0].converged
    assert np.array_equal(outs[0].cpu().numpy(), p0.u0)
    assert sts[1].iterations == solo[0][1] and np.array_equal(outs[1].cpu().numpy(), solo[0][0])
    # max_it reached: per-problem status, the call reports the first failure
    sts = dg.solve_batch(ctx, probs, outs, dg.default_opts(precision="fp32", rtol=1e-12, max_it=7), check=False)
    assert sts[0].status == 0 and sts[1].status == -6 and sts[1].iterations == 7
    with pytest.raises(dg.DDMGNNError):
        dg.solve_batch(ctx, probs, outs, dg.default_opts(precision="fp32", rtol=1e-12, max_it=7))


def test_batch_rejects_mixed_models_and_duplicates(ctx, mix):
    print("[gpu] batch argument checks", flush=True)
    m1, m2 = dg.Model(ctx, SMOOTHER), dg.Model(ctx, SMOOTHER)
    a, b = dg.Problem(ctx, mix[0][1], m1), dg.Problem(ctx, mix[2][1], m2)
    outs = [torch.empty(mix[0][0].n, dtype=torch.float64, device="cuda"),
            torch.empty(mix[2][0].n, dtype=torch.float64, device="cuda")]
    with pytest.raises(dg.DDMGNNError):
        dg.solve_batch(ctx, [a, b], outs)
    with pytest.raises(dg.DDMGNNError):
        dg.solve_batch(ctx, [a, a], [outs[0], outs[0]])


def test_server_matches_solo(ctx, mix):
    """Continuous batching with admissions and retirements mid-solve gives the solo results."""
    print("[gpu] server", flush=True)
    model = dg.Model(ctx, SMOOTHER)
    opts = dg.default_opts(precision="bf16", rtol=1e-6, max_it=3000, check_every=4)
    opts64 = dg.default_opts(precision="fp64", rtol=1e-6, max_it=3000, check_every=4)
    solo = _solo(ctx, model, mix, opts)
    solo64 = _solo(ctx, model, mix[:1], opts64)
    torch.cuda.synchronize()
    bytes_each = [dg.Problem(ctx, hp, model).device_bytes() for _, hp in mix]
    sctx = dg.Context(torch.cuda.Stream())
    # room for about two problems at a time: later ones are admitted as earlier ones retire
    srv = dg.Server(sctx, model, hbm_budget=int(sorted(bytes_each)[-1] + sorted(bytes_each)[-2]), max_active=3,
                    setup_threads=2)
    tickets = [srv.submit(hp, opts) for _, hp in mix]
    t64 = srv.submit(mix[0][1], opts64)  # different structure: waits for the bf16 group to drain
    tickets += [srv.submit(hp, opts) for _, hp in mix[:2]]
    srv.drain()
    for k, t in enumerate(tickets):
        rc, st, u = srv.poll(t)
        i = k % len(mix)
        print(f"[gpu]   ticket {t}: rc={rc} iterations={st.iterations} solo={solo[i][1]} "
              f"latency={st.latency_ms:.1f} ms", flush=True)
        assert rc == 0 and st.converged and st.iterations == solo[i][1]
        assert np.array_equal(u, solo[i][0])
        assert st.latency_ms > 0
    rc, st, u = srv.poll(t64)
    assert rc == 0 and st.iterations == solo64[0][1] and np.array_equal(u, solo64[0][0])
    with pytest.raises(KeyError):
        srv.poll(t64)
    srv.close()


def test_server_lu_and_gnn_groups(ctx, mix):
    """DDM-LU requests (inverses built by the setup workers), DDM-GNN FCG and FGMRES
    requests in one stream: each group batches on its own (eager chunks), results equal
    the solo solves (graph replay)."""
    print("[gpu] server DDM-LU / DDM-GNN", flush=True)
    model = dg.Model(ctx, SMOOTHER)
    lu = dg.default_opts(krylov=dg.PCG, local_solver=dg.LOCAL_LU, prolong=dg.PROLONG_UNWEIGHTED,
                         precision="fp64", rtol=1e-8, max_it=500, check_every=4)
    gnn = dg.default_opts(precision="fp32", rtol=1e-6, max_it=3000, check_every=4)
    solo_lu = _solo(ctx, model, mix, lu)
    solo_gnn = _solo(ctx, model, mix[:2], gnn)
    torch.cuda.synchronize()
    sctx = dg.Context(torch.cuda.Stream())
    srv = dg.Server(sctx, model, hbm_budget=8 << 30, max_active=4, setup_threads=2)
    fg = dg.default_opts(krylov=dg.FGMRES, restart=10, precision="fp32", rtol=1e-7, max_it=800, check_every=4)
    solo_fg = _solo(ctx, model, mix[1:3], fg)
    t_lu = [srv.submit(hp, lu) for _, hp in mix]
    t_gnn = [srv.submit(hp, gnn) for _, hp in mix[:2]]
    t_fg = [srv.submit(hp, fg) for _, hp in mix[1:3]]
    srv.drain()
    for tickets, solo in ((t_lu, solo_lu), (t_gnn, solo_gnn), (t_fg, solo_fg)):
        for t, (u0, it, _) in zip(tickets, solo):
            rc, st, u = srv.poll(t)
            print(f"[gpu]   ticket {t}: rc={rc} iterations={st.iterations} solo={it}", flush=True)
            assert rc == 0 and st.converged and st.iterations == it
            assert np.array_equal(u, u0)
    srv.close()


def test_server_budget_and_invalid(ctx, mix):
    print("[gpu] server budget / invalid", flush=True)
    model = dg.Model(ctx, SMOOTHER)
    sctx = dg.Context(torch.cuda.Stream())
    srv = dg.Server(sctx, model, hbm_budget=1 << 20, max_active=4)
    t_big = srv.submit(mix[1][1])
    hp = mix[0][1]
    bad_val = hp.val.copy()
    # break the symmetry of one off-diagonal entry: the setup validation rejects it
    row = int(np.flatnonzero(np.diff(hp.rowptr) > 1)[0])
    for e in range(hp.rowptr[row], hp.rowptr[row + 1]):
        if hp.col[e] != row:
            bad_val[e] += 1.0
            break
    bad = dg.HostProblem(hp.xy, hp.tri, hp.dirichlet, hp.rowptr, hp.col, bad_val, hp.b, hp.u0, hp.sub_ptr,
                         hp.sub_nodes, hp.weights)
    t_bad = srv.submit(bad)
    srv.drain()
    rc, st, _ = srv.poll(t_big)
    assert rc == -8 and st.status == -8
    rc, st, _ = srv.poll(t_bad)
    assert rc == -1
    srv.close()


def test_server_admission_failure_beside_running_chunks(ctx, mix):
    """A request whose coarse matrix is singular (two identical sub-meshes) fails with
    E_NOT_SPD when the server forms its coarse level on the upload stream, while the
    requests admitted around it iterate; they still finish with their solo bits."""
    print("[gpu] server admission failure", flush=True)
    model = dg.Model(ctx, SMOOTHER)
    opts = dg.default_opts(precision="bf16", rtol=1e-6, max_it=3000, check_every=4)
    solo = _solo(ctx, model, mix, opts)
    hp = mix[1][1]
    sp = np.concatenate([hp.sub_ptr, [hp.sub_ptr[-1] + hp.sub_ptr[1]]])
    sn = np.concatenate([hp.sub_nodes, hp.sub_nodes[:hp.sub_ptr[1]]])
    w = np.concatenate([hp.weights, hp.weights[:hp.sub_ptr[1]]])
    w[:hp.sub_ptr[1]] *= 0.5
    w[hp.sub_ptr[-1]:] *= 0.5
    singular = dg.HostProblem(hp.xy, hp.tri, hp.dirichlet, hp.rowptr, hp.col, hp.val, hp.b, hp.u0, sp, sn, w)
    sctx = dg.Context(torch.cuda.Stream())
    srv = dg.Server(sctx, model, hbm_budget=1 << 34, max_active=8, setup_threads=2)
    tickets = [srv.submit(h, opts) for _, h in mix[:2]]
    t_bad = srv.submit(singular, opts)
    tickets += [srv.submit(h, opts) for _, h in mix[2:]]
    srv.drain()
    rc, st, _ = srv.poll(t_bad)
    print(f"[gpu]   singular request: rc={rc}", flush=True)
    assert rc == -4 and st.status == -4
    for i, t in enumerate(tickets):
        rc, st, u = srv.poll(t)
        assert rc == 0 and st.converged and st.iterations == solo[i][1]
        assert np.array_equal(u, solo[i][0])
    srv.close()
