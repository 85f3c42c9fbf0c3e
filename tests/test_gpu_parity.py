"""GPU parity: the HIP path through the C ABI against the CPU FP64 oracle.

Tolerances:
  * SpMV, dots, FP64 DSS and FP64 applies: reordering of FP64 sums only,
    relative 1e-12 (DSS) / 1e-13 (linear algebra) of the largest magnitude.
  * FP32 DSS: one FP32 rounding per operation over 30 blocks; relative 3e-5
    of the largest output magnitude (measured errors are ~1e-6).
  * BF16 DSS (matrix-core kernel): twice the error of a float64 model of the
    kernel's roundings (bf16 operands, FP16 projections and message sums;
    tests/_bf16_model.py) against the oracle, relative to the largest output
    magnitude.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_2402_08296_amd as dg  # noqa: E402
import workload as W  # noqa: E402
from oracle import decomp as dc, dss, krylov as kr, schwarz as sw  # noqa: E402
from tests import _bf16_model as bm  # noqa: E402
from tests._cases import oracle_problem, small_problem  # noqa: E402

pytestmark = pytest.mark.gpu

XAVIER = W.xavier_theta(W.THETA_SEED)
SMOOTHER = W.smoother_theta(omega=0.15, out_scale=1.7)


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, np.float64)).cuda()


@pytest.fixture(scope="module")
def ctx():
    print("[gpu] creating context", flush=True)
    return dg.Context()


@pytest.fixture(scope="module")
def c1(ctx):
    p = W.config_problem("c1", 0)
    hp = oracle_problem(p)
    return p, hp


def _oracle_M(p, hp, theta, prolong="pou", coarse=True):
    dec = dc.Decomposition(p.n, hp.sub_ptr, hp.sub_nodes, hp.weights)
    return sw.DDMGNN(p.A.to_scipy(), p.mesh.xy, p.mesh.tri, p.mesh.dirichlet, dec, theta, prolong=prolong,
                     coarse=coarse)


def test_spmv_and_dot(ctx):
    print("[gpu] spmv/dot", flush=True)
    p, hp = small_problem(seed=11, n=3000, parts=5)
    prob = dg.Problem(ctx, hp, dg.Model(ctx, XAVIER))
    x = np.random.default_rng(0).standard_normal(p.n)
    y = torch.empty(p.n, dtype=torch.float64, device="cuda")
    prob.spmv(_dev(x), y)
    ref = p.A.to_scipy() @ x
    scale = np.abs(p.A.to_scipy()) @ np.abs(x)
    assert np.all(np.abs(y.cpu().numpy() - ref) <= 1e-14 * scale + 1e-300)
    for n in [0, 1, 63, 64, 65, 1000, 262_145]:
        a = np.random.default_rng(n).standard_normal(n)
        b = np.random.default_rng(n + 1).standard_normal(n)
        got = ctx.dot(_dev(a), _dev(b))
        assert abs(got - float(a @ b)) <= 1e-13 * max(1.0, float(np.abs(a) @ np.abs(b)))
        assert got == ctx.dot(_dev(a), _dev(b))  # deterministic


def _c_of(hp, r):
    """Per-slot normalised restrictions c_i = R_i r / |R_i r| of a residual r."""
    c = np.empty(hp.sub_nodes.size)
    for i in range(hp.K):
        ri = r[hp.sub_nodes[hp.sub_ptr[i]:hp.sub_ptr[i + 1]]]
        c[hp.sub_ptr[i]:hp.sub_ptr[i + 1]] = ri / np.linalg.norm(ri)
    return c


def _c_inputs(p, hp, seed):
    """Per-slot normalised restrictions c_i = R_i r / |R_i r| of a random residual."""
    r = np.random.default_rng(seed).standard_normal(p.n)
    r[p.mesh.dirichlet == 1] = 0
    c = np.empty(hp.sub_nodes.size)
    for i in range(hp.K):
        sl = slice(hp.sub_ptr[i], hp.sub_ptr[i + 1])
        ri = r[hp.sub_nodes[sl]]
        c[sl] = ri / np.linalg.norm(ri)
    return c


def _graphs(p, hp):
    return [dc.local_graph(hp.sub_nodes[hp.sub_ptr[i]:hp.sub_ptr[i + 1]], p.mesh.tri, p.mesh.xy, p.mesh.dirichlet)
            for i in range(hp.K)]


def _slices(hp, c):
    return [c[hp.sub_ptr[i]:hp.sub_ptr[i + 1]] for i in range(hp.K)]


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("fp32", 3e-5), ("bf16", None)])
@pytest.mark.parametrize("theta_name", ["xavier", "smoother"])
def test_dss_forward_all_subdomains(ctx, c1, prec, tol, theta_name):
    print(f"[gpu] dss_forward {prec} {theta_name}", flush=True)
    p, hp = c1
    theta = XAVIER if theta_name == "xavier" else SMOOTHER
    prob = dg.Problem(ctx, hp, dg.Model(ctx, theta))
    c = _c_inputs(p, hp, 1)
    out = torch.empty(hp.sub_nodes.size, dtype=torch.float64, device="cuda")
    prob.dss_forward(_dev(c), out, prec)
    got = out.cpu().numpy()
    blocks = dss.unpack(theta, 30, 10)
    graphs = _graphs(p, hp)
    worst = 0.0
    for i, g in enumerate(graphs):
        sl = slice(hp.sub_ptr[i], hp.sub_ptr[i + 1])
        ref = dss.forward(blocks, g, c[sl], 1e-3, 10)
        err = np.abs(got[sl] - ref).max() / np.abs(ref).max()
        worst = max(worst, err)
    if tol is None:
        tol = bm.tolerance(blocks, graphs, _slices(hp, c), 1e-3, 10)
    print(f"[gpu]   worst relative error {worst:.3e} (bar {tol:.3e})", flush=True)
    assert worst <= tol


@pytest.mark.parametrize("kbar,d", [(5, 5), (10, 20), (20, 10), (10, 5)])
@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("fp32", 3e-5), ("bf16", 3e-5)])
def test_dss_forward_widths(ctx, c1, kbar, d, prec, tol):
    """(kbar, d) variants of DSS_theta (Table II sweep): Xavier weights of each size against
    the oracle. BF16 runs the matrix-core kernel at d = 10 and at d = 5 (embedded in width 10
    with zero weights, hence the rounding model's bar); d = 20 takes the FP32 kernel (hence the
    FP32 bar)."""
    print(f"[gpu] dss_forward kbar={kbar} d={d} {prec}", flush=True)
    p, hp = c1
    theta = W.xavier_theta(7, kbar, d)
    prob = dg.Problem(ctx, hp, dg.Model(ctx, theta, kbar=kbar, d=d))
    c = _c_inputs(p, hp, 3)
    out = torch.empty(hp.sub_nodes.size, dtype=torch.float64, device="cuda")
    prob.dss_forward(_dev(c), out, prec)
    got = out.cpu().numpy()
    blocks = dss.unpack(theta, kbar, d)
    graphs = _graphs(p, hp)
    worst = 0.0
    for i, g in enumerate(graphs):
        sl = slice(hp.sub_ptr[i], hp.sub_ptr[i + 1])
        ref = dss.forward(blocks, g, c[sl], 1e-3, d)
        worst = max(worst, np.abs(got[sl] - ref).max() / np.abs(ref).max())
    if prec == "bf16" and d <= 10:
        tol = bm.tolerance(blocks, graphs, _slices(hp, c), 1e-3, d)
    print(f"[gpu]   worst relative error {worst:.3e} (bar {tol:.3e})", flush=True)
    assert worst <= tol


@pytest.mark.parametrize("d", [5, 20])
def test_solve_widths_match_oracle(ctx, c1, d):
    """FCG with a constructed smoother of latent width d: FP64 iterations equal the oracle's;
    a BF16 request runs the matrix-core kernel at d = 5 (kernel id 2) and the FP32 VALU
    kernel at d = 20 (kernel id 1)."""
    print(f"[gpu] solve d={d}", flush=True)
    p, hp = c1
    theta = W.smoother_theta(kbar=10, d=d, omega=0.15, out_scale=1.7)
    prob = dg.Problem(ctx, hp, dg.Model(ctx, theta, kbar=10, d=d))
    u = torch.empty(p.n, dtype=torch.float64, device="cuda")
    st = prob.solve(u, dg.default_opts(precision="fp64", rtol=1e-8, max_it=1000))
    dec = dc.Decomposition(p.n, hp.sub_ptr, hp.sub_nodes, hp.weights)
    M = sw.DDMGNN(p.A.to_scipy(), p.mesh.xy, p.mesh.tri, p.mesh.dirichlet, dec, theta, kbar=10, d=d)
    ref = kr.fcg(p.A.to_scipy(), p.b, p.u0, M, 1e-8, max_it=1000)
    print(f"[gpu]   iterations gpu={st.iterations} oracle={ref.iterations}", flush=True)
    assert ref.converged and st.converged and abs(st.iterations - ref.iterations) <= 1
    st = prob.solve(u, dg.default_opts(precision="bf16", rtol=1e-6, max_it=1000))
    print(f"[gpu]   bf16: iterations {st.iterations} kernel {st.dss_kernel} true residual "
          f"{st.true_rel_residual:.2e}", flush=True)
    assert st.converged and st.true_rel_residual <= 1.5e-6 and st.dss_kernel == (2 if d == 5 else 1)


def test_model_rejects_bad_sizes(ctx):
    with pytest.raises(dg.DDMGNNError):
        dg.Model(ctx, W.xavier_theta(7, 5, 10), kbar=5, d=7)
    with pytest.raises(dg.DDMGNNError):
        dg.Model(ctx, W.xavier_theta(7, 5, 10), kbar=6, d=10)


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("fp32", 3e-5), ("bf16", None)])
@pytest.mark.parametrize("prolong", [dg.PROLONG_POU, dg.PROLONG_UNWEIGHTED])
def test_apply_and_intermediates(ctx, c1, prec, tol, prolong):
    print(f"[gpu] apply {prec} prolong={prolong}", flush=True)
    p, hp = c1
    prob = dg.Problem(ctx, hp, dg.Model(ctx, XAVIER))
    r = np.random.default_rng(2).standard_normal(p.n)
    r[p.mesh.dirichlet == 1] = 0
    z = torch.empty(p.n, dtype=torch.float64, device="cuda")
    opts = dg.default_opts(precision=prec, prolong=prolong)
    prob.apply(_dev(r), z, opts)
    s, y0, y, loc = [t.cpu().numpy() for t in prob.intermediates()]
    M = _oracle_M(p, hp, XAVIER, "pou" if prolong == dg.PROLONG_POU else "unweighted")
    ref_z = M(r)
    # a5: restriction norms and coarse restriction
    for i in range(hp.K):
        ri = r[hp.sub_nodes[hp.sub_ptr[i]:hp.sub_ptr[i + 1]]]
        assert abs(s[i] - np.linalg.norm(ri)) <= 1e-14 * np.linalg.norm(ri)
    ref_y0 = M.coarse.Z.T @ r
    assert np.abs(y0 - ref_y0).max() <= 1e-13 * np.abs(r).max() * 100
    # a6: coarse solve
    ref_y = np.linalg.solve(M.coarse.A0, y0)
    assert np.abs(y - ref_y).max() <= 1e-10 * np.abs(ref_y).max()
    # a7: local terms s_i r~_i
    if tol is None:
        tol = bm.tolerance(dss.unpack(XAVIER, 30, 10), _graphs(p, hp), _slices(hp, _c_of(hp, r)), 1e-3, 10)
    worst = 0.0
    for i in range(hp.K):
        sl = slice(hp.sub_ptr[i], hp.sub_ptr[i + 1])
        si, rt = M.local(i, r)
        worst = max(worst, np.abs(loc[sl] - si * rt).max() / np.abs(si * rt).max())
    print(f"[gpu]   local terms worst relative error {worst:.3e}", flush=True)
    assert worst <= tol
    # a8: glued z
    zg = z.cpu().numpy()
    assert np.all(zg[p.mesh.dirichlet == 1] == 0)
    assert np.abs(zg - ref_z).max() <= max(tol, 1e-10) * np.abs(ref_z).max()


def test_apply_deterministic_and_homogeneous(ctx, c1):
    print("[gpu] apply determinism", flush=True)
    p, hp = c1
    prob = dg.Problem(ctx, hp, dg.Model(ctx, XAVIER))
    r = np.random.default_rng(3).standard_normal(p.n)
    r[p.mesh.dirichlet == 1] = 0
    z1 = torch.empty(p.n, dtype=torch.float64, device="cuda")
    z2 = torch.empty_like(z1)
    z3 = torch.empty_like(z1)
    for prec in ("fp64", "fp32", "bf16"):
        o = dg.default_opts(precision=prec)
        prob.apply(_dev(r), z1, o)
        prob.apply(_dev(r), z2, o)
        prob.apply(_dev(8.0 * r), z3, o)
        assert torch.equal(z1, z2)
        assert torch.equal(z3, 8.0 * z1)


def test_zero_residual_subdomain(ctx, c1):
    """A sub-mesh with R_i r = 0 contributes nothing (s_i = 0 branch)."""
    p, hp = c1
    prob = dg.Problem(ctx, hp, dg.Model(ctx, XAVIER))
    r = np.zeros(p.n)
    only0 = np.setdiff1d(hp.sub_nodes[:hp.sub_ptr[1]], hp.sub_nodes[hp.sub_ptr[1]:])
    only0 = only0[p.mesh.dirichlet[only0] == 0]
    r[only0[:10]] = 1.0
    z = torch.empty(p.n, dtype=torch.float64, device="cuda")
    prob.apply(_dev(r), z, dg.default_opts(precision="fp64"))
    s, _, _, loc = [t.cpu().numpy() for t in prob.intermediates()]
    assert s[0] > 0 and np.all(s[1:] == 0)
    assert np.all(loc[hp.sub_ptr[1]:] == 0)
    ref = _oracle_M(p, hp, XAVIER)(r)
    assert np.abs(z.cpu().numpy() - ref).max() <= 1e-10 * np.abs(ref).max()


def test_solve_fp64_matches_oracle(ctx, c1):
    print("[gpu] solve fp64", flush=True)
    p, hp = c1
    prob = dg.Problem(ctx, hp, dg.Model(ctx, SMOOTHER))
    u = torch.empty(p.n, dtype=torch.float64, device="cuda")
    st = prob.solve(u, dg.default_opts(precision="fp64", rtol=1e-10))
    ref = kr.fcg(p.A.to_scipy(), p.b, p.u0, _oracle_M(p, hp, SMOOTHER), 1e-10, max_it=2000)
    print(f"[gpu]   iterations gpu={st.iterations} oracle={ref.iterations} "
          f"true_rel={st.true_rel_residual:.2e}", flush=True)
    assert st.converged and abs(st.iterations - ref.iterations) <= 1
    assert st.true_rel_residual <= 2e-10
    ug = u.cpu().numpy()
    assert np.linalg.norm(ug - ref.u) / np.linalg.norm(ref.u) <= 1e-6
    import scipy.sparse.linalg as spl
    ud = spl.spsolve(p.A.to_scipy().tocsc(), p.b)
    assert np.linalg.norm(ug - ud) / np.linalg.norm(ud) <= 1e-6


def _host_rel_res(p, u):
    A = p.A.to_scipy()
    return np.linalg.norm(p.b - A @ u) / np.linalg.norm(p.b - A @ p.u0)


def test_solve_fp32_converges_to_tolerance(ctx, c1):
    print("[gpu] solve fp32", flush=True)
    p, hp = c1
    prob = dg.Problem(ctx, hp, dg.Model(ctx, SMOOTHER))
    u = torch.empty(p.n, dtype=torch.float64, device="cuda")
    st = prob.solve(u, dg.default_opts(precision="fp32", rtol=1e-6))
    ref = kr.fcg(p.A.to_scipy(), p.b, p.u0, _oracle_M(p, hp, SMOOTHER), 1e-6, max_it=2000)
    res = _host_rel_res(p, u.cpu().numpy())
    print(f"[gpu]   iterations gpu={st.iterations} oracle={ref.iterations} scipy residual {res:.2e}", flush=True)
    assert st.converged and res <= 1e-6
    assert abs(st.iterations - ref.iterations) <= max(2, 0.1 * ref.iterations)


def test_solve_bf16_converges_to_tolerance(ctx, c1):
    print("[gpu] solve bf16", flush=True)
    p, hp = c1
    prob = dg.Problem(ctx, hp, dg.Model(ctx, SMOOTHER))
    u = torch.empty(p.n, dtype=torch.float64, device="cuda")
    st = prob.solve(u, dg.default_opts(precision="bf16", rtol=1e-6, max_it=2000))
    ref = kr.fcg(p.A.to_scipy(), p.b, p.u0, _oracle_M(p, hp, SMOOTHER), 1e-6, max_it=2000)
    res = _host_rel_res(p, u.cpu().numpy())
    print(f"[gpu]   iterations gpu={st.iterations} oracle={ref.iterations} scipy residual {res:.2e}", flush=True)
    assert st.converged and res <= 1e-6
    assert st.iterations <= 1.5 * ref.iterations + 5


@pytest.fixture(scope="module")
def c1_tight(c1):
    """The oracle's FCG (FP64 DSS) to rtol 1e-10 on c1, and scipy's direct solve."""
    import scipy.sparse.linalg as spl
    p, hp = c1
    ref = kr.fcg(p.A.to_scipy(), p.b, p.u0, _oracle_M(p, hp, SMOOTHER), 1e-10, max_it=3000)
    ud = spl.spsolve(p.A.to_scipy().tocsc(), p.b)
    assert ref.converged
    return ref, ud


@pytest.mark.timeout(300)
@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_mixed_precision_solution_matches_oracle(ctx, c1, c1_tight, prec):
    """Solution parity for the mixed-precision forms: both sides solved to rtol 1e-10, the
    GPU's u within 1e-6 relative L2 of the oracle's FCG solution and of the direct solve
    (the preconditioner's precision changes the path, not the solution)."""
    print(f"[gpu] solve {prec} rtol 1e-10 against the oracle", flush=True)
    p, hp = c1
    ref, ud = c1_tight
    prob = dg.Problem(ctx, hp, dg.Model(ctx, SMOOTHER))
    u = torch.empty(p.n, dtype=torch.float64, device="cuda")
    for m in (1, 4):
        st = prob.solve(u, dg.default_opts(precision=prec, rtol=1e-10, m_max=m, max_it=3000))
        ug = u.cpu().numpy()
        e_orc = np.linalg.norm(ug - ref.u) / np.linalg.norm(ref.u)
        e_dir = np.linalg.norm(ug - ud) / np.linalg.norm(ud)
        print(f"[gpu]   FCG({m}) iterations gpu={st.iterations} oracle={ref.iterations} L2 vs oracle {e_orc:.2e} "
              f"vs direct {e_dir:.2e}", flush=True)
        assert st.converged and _host_rel_res(p, ug) <= 2e-10
        assert e_orc <= 1e-6 and e_dir <= 1e-6


def test_graph_replay_matches_eager(ctx, c1):
    """Chunks of iterations replayed as a captured graph give the eager result, bit for bit."""
    print("[gpu] graph replay", flush=True)
    p, hp = c1
    prob = dg.Problem(ctx, hp, dg.Model(ctx, SMOOTHER))
    ue = torch.empty(p.n, dtype=torch.float64, device="cuda")
    ug = torch.empty_like(ue)
    z = torch.empty_like(ue)
    r = _dev(np.random.default_rng(9).standard_normal(p.n))
    for prec in ("fp32", "bf16"):
        st_e = prob.solve(ue, dg.default_opts(precision=prec, graph=0, check_every=4))
        for rep in range(3):
            st_g = prob.solve(ug, dg.default_opts(precision=prec, graph=1, check_every=4))
            assert st_g.iterations == st_e.iterations and torch.equal(ug, ue), (prec, rep)
            prob.apply(r, z, dg.default_opts(precision=prec))  # eager work between replays
            torch.cuda.synchronize()


def test_krylov_modes(ctx, c1):
    print("[gpu] cg/pcg", flush=True)
    p, hp = c1
    A = p.A.to_scipy()
    prob = dg.Problem(ctx, hp, dg.Model(ctx, SMOOTHER))
    u = torch.empty(p.n, dtype=torch.float64, device="cuda")
    st = prob.solve(u, dg.default_opts(krylov=dg.CG, rtol=1e-6))
    ref = kr.cg(A, p.b, p.u0, 1e-6)
    assert st.converged and abs(st.iterations - ref.iterations) <= 1
    # Algorithm 1 needs a symmetric positive definite M: unweighted glue and a
    # Richardson step with omega * lambda_max(L) < 2 give one.
    spd = W.smoother_theta(omega=0.08)
    prob_spd = dg.Problem(ctx, hp, dg.Model(ctx, spd))
    st = prob_spd.solve(u, dg.default_opts(krylov=dg.PCG, precision="fp64", rtol=1e-8,
                                           prolong=dg.PROLONG_UNWEIGHTED, max_it=500))
    ref = kr.pcg(A, p.b, p.u0, _oracle_M(p, hp, spd, prolong="unweighted"), 1e-8, max_it=500)
    assert ref.converged and st.converged and abs(st.iterations - ref.iterations) <= 1
    for m in (3, 4):  # 4: the largest ring of kept directions
        st = prob.solve(u, dg.default_opts(m_max=m, precision="fp64", rtol=1e-8))
        ref = kr.fcg(A, p.b, p.u0, _oracle_M(p, hp, SMOOTHER), 1e-8, m_max=m)
        assert st.converged and abs(st.iterations - ref.iterations) <= 1, m
        assert np.linalg.norm(u.cpu().numpy() - ref.u) <= 1e-6 * np.linalg.norm(ref.u)


@pytest.mark.parametrize("prolong", [dg.PROLONG_UNWEIGHTED, dg.PROLONG_POU])
def test_lu_apply_matches_oracle(ctx, c1, prolong):
    """DDM-LU (eq. (7)): exact local solves, coarse solve and glue, FP64 throughout."""
    print(f"[gpu] DDM-LU apply prolong={prolong}", flush=True)
    p, hp = c1
    prob = dg.Problem(ctx, hp, dg.Model(ctx, XAVIER))
    r = np.random.default_rng(4).standard_normal(p.n)
    r[p.mesh.dirichlet == 1] = 0
    z = torch.empty(p.n, dtype=torch.float64, device="cuda")
    prob.apply(_dev(r), z, dg.default_opts(local_solver=dg.LOCAL_LU, prolong=prolong))
    s, _, _, loc = [t.cpu().numpy() for t in prob.intermediates()]
    dec = dc.Decomposition(p.n, hp.sub_ptr, hp.sub_nodes, hp.weights)
    M = sw.DDMLU(p.A.to_scipy(), p.mesh.dirichlet, dec,
                 prolong="pou" if prolong == dg.PROLONG_POU else "unweighted")
    import scipy.linalg as sla
    worst = 0.0
    for i in range(hp.K):
        sl = slice(hp.sub_ptr[i], hp.sub_ptr[i + 1])
        ri = r[hp.sub_nodes[sl]]
        assert abs(s[i] - np.linalg.norm(ri)) <= 1e-14 * np.linalg.norm(ri)
        ref = sla.cho_solve(M.factors[i], ri)
        worst = max(worst, np.abs(loc[sl] - ref).max() / np.abs(ref).max())
    print(f"[gpu]   local solves worst relative error {worst:.3e}", flush=True)
    assert worst <= 1e-10
    zg = z.cpu().numpy()
    ref_z = M(r)
    assert np.all(zg[p.mesh.dirichlet == 1] == 0)
    assert np.abs(zg - ref_z).max() <= 1e-10 * np.abs(ref_z).max()
    z2 = torch.empty_like(z)
    prob.apply(_dev(r), z2, dg.default_opts(local_solver=dg.LOCAL_LU, prolong=prolong))
    assert torch.equal(z, z2)


@pytest.mark.parametrize("krylov", [dg.PCG, dg.FCG])
def test_lu_solve_matches_oracle(ctx, c1, krylov):
    print(f"[gpu] DDM-LU solve krylov={krylov}", flush=True)
    p, hp = c1
    A = p.A.to_scipy()
    prob = dg.Problem(ctx, hp, dg.Model(ctx, SMOOTHER))
    u = torch.empty(p.n, dtype=torch.float64, device="cuda")
    st = prob.solve(u, dg.default_opts(krylov=krylov, local_solver=dg.LOCAL_LU, precision="fp64",
                                       prolong=dg.PROLONG_UNWEIGHTED, rtol=1e-10, max_it=500))
    dec = dc.Decomposition(p.n, hp.sub_ptr, hp.sub_nodes, hp.weights)
    M = sw.DDMLU(A, p.mesh.dirichlet, dec, prolong="unweighted")
    solve = kr.pcg if krylov == dg.PCG else kr.fcg
    ref = solve(A, p.b, p.u0, M, 1e-10, max_it=500)
    print(f"[gpu]   iterations gpu={st.iterations} oracle={ref.iterations} kernel={st.dss_kernel}", flush=True)
    assert st.dss_kernel == 3
    assert ref.converged and st.converged and abs(st.iterations - ref.iterations) <= 1
    assert st.true_rel_residual <= 2e-10
    ug = u.cpu().numpy()
    assert np.linalg.norm(ug - ref.u) / np.linalg.norm(ref.u) <= 1e-8


@pytest.mark.parametrize("restart,local", [(30, dg.LOCAL_GNN), (5, dg.LOCAL_GNN), (30, dg.LOCAL_LU)])
def test_fgmres_solve_matches_oracle(ctx, c1, restart, local):
    """Restarted flexible GMRES on the GPU (classical Gram-Schmidt run twice) against the
    oracle's (modified Gram-Schmidt): the same iterate up to rounding, so iteration counts
    within 2 and solutions within 1e-8 of each other at rtol 1e-10."""
    print(f"[gpu] FGMRES({restart}) local={local}", flush=True)
    p, hp = c1
    A = p.A.to_scipy()
    prob = dg.Problem(ctx, hp, dg.Model(ctx, SMOOTHER))
    u = torch.empty(p.n, dtype=torch.float64, device="cuda")
    st = prob.solve(u, dg.default_opts(krylov=dg.FGMRES, restart=restart, local_solver=local, precision="fp64",
                                       rtol=1e-10, max_it=600))
    dec = dc.Decomposition(p.n, hp.sub_ptr, hp.sub_nodes, hp.weights)
    if local == dg.LOCAL_LU:
        M = sw.DDMLU(A, p.mesh.dirichlet, dec, prolong="pou")
    else:
        M = _oracle_M(p, hp, SMOOTHER)
    ref = kr.fgmres(A, p.b, p.u0, M, 1e-10, max_it=600, restart=restart)
    print(f"[gpu]   iterations gpu={st.iterations} oracle={ref.iterations} rel={st.rel_residual:.2e} "
          f"true={st.true_rel_residual:.2e}", flush=True)
    assert ref.converged and st.converged and abs(st.iterations - ref.iterations) <= 2
    assert st.true_rel_residual <= 2e-10
    ug = u.cpu().numpy()
    assert np.linalg.norm(ug - ref.u) / np.linalg.norm(ref.u) <= 1e-8


def test_fgmres_bf16_and_graph_replay(ctx, c1):
    """FGMRES with the BF16 DSS converges; a second solve (graph replay) repeats it bit for bit."""
    print("[gpu] FGMRES bf16", flush=True)
    p, hp = c1
    prob = dg.Problem(ctx, hp, dg.Model(ctx, SMOOTHER))
    u1 = torch.empty(p.n, dtype=torch.float64, device="cuda")
    u2 = torch.empty_like(u1)
    o = dg.default_opts(krylov=dg.FGMRES, restart=20, precision="bf16", rtol=1e-6, max_it=600)
    s1 = prob.solve(u1, o)
    s2 = prob.solve(u2, o)
    print(f"[gpu]   iterations {s1.iterations} true_rel={s1.true_rel_residual:.2e}", flush=True)
    assert s1.converged and s1.true_rel_residual <= 1.5e-6
    assert s1.iterations == s2.iterations and torch.equal(u1, u2)
    eager = prob.solve(u2, dg.default_opts(krylov=dg.FGMRES, restart=20, precision="bf16", rtol=1e-6,
                                           max_it=600, graph=0))
    assert eager.iterations == s1.iterations and torch.equal(u1, u2)


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16"])
def test_dss_forward_sub_matches_full(ctx, c1, prec):
    """The one-sub-mesh forward entry gives the bits of the full forward's slice."""
    print(f"[gpu] dss_forward_sub {prec}", flush=True)
    p, hp = c1
    prob = dg.Problem(ctx, hp, dg.Model(ctx, XAVIER))
    c = _c_inputs(p, hp, 4)
    full = torch.empty(hp.sub_nodes.size, dtype=torch.float64, device="cuda")
    prob.dss_forward(_dev(c), full, prec)
    for i in (0, hp.K // 2, hp.K - 1):
        sl = slice(hp.sub_ptr[i], hp.sub_ptr[i + 1])
        one = torch.empty(sl.stop - sl.start, dtype=torch.float64, device="cuda")
        prob.dss_forward_sub(i, _dev(c[sl]), one, prec)
        assert torch.equal(one, full[sl])
    with pytest.raises((dg.DDMGNNError, ValueError)):
        prob.dss_forward_sub(hp.K, _dev(c[:10]), one, prec)


def test_problem_from_device_arrays(ctx, c1):
    """A descriptor of device pointers (mem_kind = DEVICE) builds the same problem as the
    host one: same sizes, bitwise equal solves."""
    print("[gpu] problem from device arrays", flush=True)
    import ctypes
    p, hp = c1
    model = dg.Model(ctx, SMOOTHER)
    keep = {}

    def dptr(name, a):
        t = torch.from_numpy(np.ascontiguousarray(a)).cuda()
        keep[name] = t
        return ctypes.c_void_p(t.data_ptr())

    d = dg.ProblemDesc(hp.n, dptr("xy", hp.xy), hp.tri.size // 3, dptr("tri", hp.tri), dptr("dir", hp.dirichlet),
                       dptr("rp", hp.rowptr), dptr("col", hp.col), dptr("val", hp.val), dptr("b", hp.b),
                       dptr("u0", hp.u0), hp.K, dptr("sp", hp.sub_ptr), dptr("sn", hp.sub_nodes),
                       dptr("w", hp.weights), dg.MEM_DEVICE)
    torch.cuda.synchronize()
    pd = dg.Problem(ctx, hp, model, desc=d)
    ph = dg.Problem(ctx, hp, model)
    assert (pd.n, pd.nnz, pd.K, pd.sum_k, pd.n_edges) == (ph.n, ph.nnz, ph.K, ph.sum_k, ph.n_edges)
    u1 = torch.empty(p.n, dtype=torch.float64, device="cuda")
    u2 = torch.empty_like(u1)
    o = dg.default_opts(precision="fp32", rtol=1e-6)
    s1, s2 = pd.solve(u1, o), ph.solve(u2, o)
    assert s1.converged and s1.iterations == s2.iterations and torch.equal(u1, u2)


def test_xavier_history_matches_oracle(ctx, c1):
    """The seeded (untrained) model stagnates; the GPU recurrence tracks the oracle's."""
    print("[gpu] xavier history", flush=True)
    p, hp = c1
    prob = dg.Problem(ctx, hp, dg.Model(ctx, XAVIER))
    u = torch.empty(p.n, dtype=torch.float64, device="cuda")
    st = prob.solve(u, dg.default_opts(precision="fp64", max_it=15), check=False)
    ref = kr.fcg(p.A.to_scipy(), p.b, p.u0, _oracle_M(p, hp, XAVIER), 1e-6, max_it=15)
    assert st.status == -6 and st.iterations == 15
    assert abs(st.rel_residual - ref.history[-1]) <= 1e-8 * ref.history[-1]
    assert np.linalg.norm(u.cpu().numpy() - ref.u) <= 1e-8 * np.linalg.norm(ref.u)


def test_zero_rhs_and_large_subdomain(ctx):
    print("[gpu] edge cases", flush=True)
    # a single sub-mesh close to the size limit exercises the global-Q FP64 path
    p = W.make_problem(31, 1900, 1)
    hp = oracle_problem(p, delta=0)
    assert hp.sub_ptr[1] <= 2048
    prob = dg.Problem(ctx, hp, dg.Model(ctx, XAVIER))
    c = _c_inputs(p, hp, 5)
    blocks = dss.unpack(XAVIER, 30, 10)
    g = dc.local_graph(hp.sub_nodes, p.mesh.tri, p.mesh.xy, p.mesh.dirichlet)
    ref = dss.forward(blocks, g, c, 1e-3, 10)
    out = torch.empty(hp.sub_nodes.size, dtype=torch.float64, device="cuda")
    bf16_bar = bm.tolerance(blocks, [g], [c], 1e-3, 10)
    for prec, tol in (("fp64", 1e-12), ("fp32", 3e-5), ("bf16", bf16_bar)):
        prob.dss_forward(_dev(c), out, prec)
        err = np.abs(out.cpu().numpy() - ref).max() / np.abs(ref).max()
        print(f"[gpu]   k={hp.sub_ptr[1]} {prec} relative error {err:.3e}", flush=True)
        assert err <= tol
    # b = A u0: the initial residual is zero, nothing to do
    hp0 = dg.HostProblem(hp.xy, hp.tri, hp.dirichlet, hp.rowptr, hp.col, hp.val, p.A.to_scipy() @ p.u0, p.u0,
                         hp.sub_ptr, hp.sub_nodes, hp.weights)
    prob0 = dg.Problem(ctx, hp0, dg.Model(ctx, XAVIER))
    u = torch.empty(p.n, dtype=torch.float64, device="cuda")
    st = prob0.solve(u)
    assert st.converged and st.iterations == 0
    assert torch.equal(u.cpu(), torch.from_numpy(p.u0))


def test_failure_statuses_forced_by_data(ctx, c1):
    """E_NONFINITE and E_BREAKDOWN, forced from the inputs (every kernel runs to its end):
    a right-hand side of 1e200 (finite, so validation accepts it) makes |r_0|^2 overflow;
    all-zero weights without the coarse level give z = 0, so <p, A p> = 0. In both cases
    u is the last finite iterate, u_0."""
    print("[gpu] failure statuses", flush=True)
    p, hp = c1
    u = torch.empty(p.n, dtype=torch.float64, device="cuda")
    hb = dg.HostProblem(hp.xy, hp.tri, hp.dirichlet, hp.rowptr, hp.col, hp.val, p.b * 1e200, p.u0,
                        hp.sub_ptr, hp.sub_nodes, hp.weights)
    prob = dg.Problem(ctx, hb, dg.Model(ctx, SMOOTHER))
    st = prob.solve(u, dg.default_opts(precision="fp32", max_it=50), check=False)
    print(f"[gpu]   huge rhs: status {st.status} iterations {st.iterations}", flush=True)
    assert st.status == -7 and not st.converged and st.iterations == 0  # DDMGNN_E_NONFINITE
    assert torch.equal(u.cpu(), torch.from_numpy(p.u0))
    zero = np.zeros_like(W.xavier_theta(9))
    prob0 = dg.Problem(ctx, hp, dg.Model(ctx, zero))
    st = prob0.solve(u, dg.default_opts(precision="fp64", coarse=0, max_it=50), check=False)
    print(f"[gpu]   zero preconditioner: status {st.status} iterations {st.iterations}", flush=True)
    assert st.status == -5 and st.iterations == 0  # DDMGNN_E_BREAKDOWN
    assert torch.equal(u.cpu(), torch.from_numpy(p.u0))
