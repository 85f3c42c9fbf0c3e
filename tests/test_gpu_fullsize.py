"""GPU parity at a size where the vector kernels take their full-size paths.

A ~300k-node problem from the generator (500 parts, the c3 partition jitter):
at the default 1024 workgroups per problem each vector-kernel workgroup walks
two 256-row groups, and with 64 workgroups about eighteen, so the row mapping
that every Krylov kernel shares is exercised as at c3. The decomposition is
the oracle's own (oracle.decomp.decompose), not the library's. Every check is
made on the host against something outside the library: scipy's residual and
direct solve for the solutions, and the oracle's DDM-GNN apply (Sec. III.A
steps 1-3) element by element for one preconditioner apply.

A separate small problem with dense rows (a clique added to the stiffness
matrix) drives the SpMV through its row-by-row path for row groups whose
nonzeros exceed the LDS chunk.
"""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spl

torch = pytest.importorskip("torch")

import paper_2402_08296_amd as dg  # noqa: E402
import workload as W  # noqa: E402
from oracle import decomp as dc, dss, schwarz as sw  # noqa: E402
from tests import _bf16_model as bm  # noqa: E402

pytestmark = pytest.mark.gpu

SMOOTHER = W.smoother_theta(omega=0.15, out_scale=1.7)
BIG = (4242, 300_000, 500, W.CONFIGS["c3"]["jitter"])


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, np.float64)).cuda()


def _host_problem(p, dec):
    return dg.HostProblem(p.mesh.xy, p.mesh.tri, p.mesh.dirichlet, p.A.rowptr, p.A.col, p.A.val, p.b, p.u0,
                          dec.sub_ptr, dec.sub_nodes, dec.weights)


@pytest.fixture(scope="module")
def ctx():
    print("[gpu] creating context", flush=True)
    return dg.Context()


@pytest.fixture(scope="module")
def big():
    print(f"[gpu] full-size problem {BIG}", flush=True)
    p = W.make_problem(*BIG)
    dec = dc.decompose(p.n, p.mesh.tri, p.mesh.dirichlet, p.part, p.n_parts, 2)
    A = p.A.to_scipy()
    ud = spl.spsolve(A.tocsc(), p.b)
    print(f"[gpu]   N={p.n} K={dec.K} sum_k={dec.sub_nodes.size} max k={np.diff(dec.sub_ptr).max()}", flush=True)
    return p, dec, A, ud


@pytest.fixture(scope="module")
def big_prob(ctx, big):
    p, dec, _, _ = big
    model = dg.Model(ctx, SMOOTHER)
    return dg.Problem(ctx, _host_problem(p, dec), model), model


def _rel_res(A, b, u, u0):
    return np.linalg.norm(b - A @ u) / np.linalg.norm(b - A @ u0)


@pytest.mark.timeout(300)
def test_fullsize_spmv_and_dot(ctx, big, big_prob):
    p, _, A, _ = big
    prob, _ = big_prob
    assert prob.n > 256 * 1024  # several row groups per workgroup at the default count
    x = np.random.default_rng(0).standard_normal(p.n)
    ref = A @ x
    scale = abs(A) @ np.abs(x)
    y = torch.empty(p.n, dtype=torch.float64, device="cuda")
    for vb in (0, 64, 8):
        prob.set_tuning(vec_blocks=vb)
        print(f"[gpu] spmv N={p.n} vec_blocks={vb}", flush=True)
        y.fill_(np.nan)
        prob.spmv(_dev(x), y)
        assert np.all(np.abs(y.cpu().numpy() - ref) <= 1e-14 * scale)
    prob.set_tuning()
    for n in (p.n, 262_144 * 3 + 17):
        a = np.random.default_rng(n).standard_normal(n)
        b = np.random.default_rng(n + 1).standard_normal(n)
        got = ctx.dot(_dev(a), _dev(b))
        assert abs(got - float(a @ b)) <= 1e-13 * float(np.abs(a) @ np.abs(b))
        assert got == ctx.dot(_dev(a), _dev(b))


@pytest.mark.timeout(600)
def test_fullsize_apply_matches_oracle(ctx, big, big_prob):
    """One apply at full size against the oracle's DDM-GNN, node by node (s_i, y0, y,
    every local term s_i r~_i, and z), for the FP64 and BF16 DSS."""
    p, dec, A, _ = big
    prob, _ = big_prob
    r = p.b - A @ p.u0
    print("[gpu] oracle apply at full size (CPU)", flush=True)
    M = sw.DDMGNN(A, p.mesh.xy, p.mesh.tri, p.mesh.dirichlet, dec, SMOOTHER)
    loc_ref = np.zeros(dec.sub_nodes.size)
    s_ref = np.zeros(dec.K)
    for i in range(dec.K):
        s_ref[i], rt = M.local(i, r)
        loc_ref[dec.sub_ptr[i]:dec.sub_ptr[i + 1]] = s_ref[i] * rt
    z_ref = M(r)
    y0_ref = M.coarse.Z.T @ r
    y_ref = np.linalg.solve(M.coarse.A0, y0_ref)
    graphs, cs = [], []
    for i in range(0, dec.K, 4):  # the model's bar from every fourth sub-mesh (about 19 s of CPU)
        nodes = dec.sub_nodes[dec.sub_ptr[i]:dec.sub_ptr[i + 1]]
        graphs.append(dc.local_graph(nodes, p.mesh.tri, p.mesh.xy, p.mesh.dirichlet))
        cs.append(r[nodes] / np.linalg.norm(r[nodes]))
    print("[gpu] rounding model of the BF16 kernel (CPU)", flush=True)
    bf16_bar = bm.tolerance(dss.unpack(SMOOTHER, 30, 10), graphs, cs, 1e-3, 10)
    z = torch.empty(p.n, dtype=torch.float64, device="cuda")
    for prec, tol in (("fp64", 1e-12), ("bf16", bf16_bar)):
        print(f"[gpu] apply {prec} N={p.n}", flush=True)
        prob.apply(_dev(r), z, dg.default_opts(precision=prec))
        s, y0, y, loc = [t.cpu().numpy() for t in prob.intermediates()]
        assert np.abs(s - s_ref).max() <= 1e-13 * s_ref.max()
        assert np.abs(y0 - y0_ref).max() <= 1e-12 * np.abs(y0_ref).max()
        assert np.abs(y - y_ref).max() <= 1e-9 * np.abs(y_ref).max()
        worst = 0.0
        for i in range(dec.K):
            sl = slice(dec.sub_ptr[i], dec.sub_ptr[i + 1])
            worst = max(worst, np.abs(loc[sl] - loc_ref[sl]).max() / np.abs(loc_ref[sl]).max())
        zg = z.cpu().numpy()
        zerr = np.abs(zg - z_ref).max() / np.abs(z_ref).max()
        print(f"[gpu]   worst local term error {worst:.2e}, z error {zerr:.2e}", flush=True)
        assert worst <= tol and zerr <= max(tol, 1e-11)
        assert np.all(zg[p.mesh.dirichlet == 1] == 0)


@pytest.mark.timeout(300)
@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16"])
def test_fullsize_solve_checked_on_host(ctx, big, big_prob, prec):
    """Solves to rtol 1e-10 (default schedule and 64 vector workgroups): the true residual
    recomputed by scipy and the relative L2 distance to scipy's direct solve are both
    at most 1e-6 (the solution-parity bar); a solve to the headline rtol 1e-6 leaves a
    scipy residual of at most 1e-6."""
    p, _, A, ud = big
    prob, _ = big_prob
    u = torch.empty(p.n, dtype=torch.float64, device="cuda")
    for vb in (0, 64):
        prob.set_tuning(vec_blocks=vb)
        print(f"[gpu] solve {prec} rtol 1e-10 vec_blocks={vb}", flush=True)
        st = prob.solve(u, dg.default_opts(precision=prec, rtol=1e-10, m_max=4, max_it=3000))
        ug = u.cpu().numpy()
        res = _rel_res(A, p.b, ug, p.u0)
        err = np.linalg.norm(ug - ud) / np.linalg.norm(ud)
        print(f"[gpu]   iterations {st.iterations}, scipy residual {res:.2e}, L2 vs direct {err:.2e}", flush=True)
        assert st.converged and res <= 1e-9 and err <= 1e-6
    prob.set_tuning()
    st = prob.solve(u, dg.default_opts(precision=prec, rtol=1e-6, m_max=4, max_it=3000))
    ug = u.cpu().numpy()
    res = _rel_res(A, p.b, ug, p.u0)
    err = np.linalg.norm(ug - ud) / np.linalg.norm(ud)
    print(f"[gpu]   rtol 1e-6: iterations {st.iterations}, scipy residual {res:.2e}, L2 vs direct {err:.2e}",
          flush=True)
    assert st.converged and res <= 1e-6


def _dense_row_problem():
    """A small generated problem whose stiffness matrix gets a clique Laplacian
    eps * sum_{i<j in S} (e_i - e_j)(e_i - e_j)^T over 300 free nodes S: symmetric,
    still positive definite, and the row groups holding S exceed the SpMV's LDS chunk
    (2048 nonzeros per 256 rows)."""
    p = W.make_problem(21, 3000, 5, 0.0)
    A = p.A.to_scipy().tocsr()
    free = np.flatnonzero(p.mesh.dirichlet == 0)
    S = np.sort(np.random.default_rng(1).choice(free[:600], 300, replace=False))
    eps = 0.05
    C = sp.csr_matrix((np.full(S.size * S.size, -eps), (np.repeat(S, S.size), np.tile(S, S.size))),
                      shape=A.shape).tolil()
    C[S, S] = 0.0
    C = C.tocsr()
    C = C + sp.diags(-np.asarray(C.sum(axis=1)).ravel())
    A2 = (A + C).tocsr()
    A2.sum_duplicates()
    A2.sort_indices()
    return p, A2, S


@pytest.mark.timeout(300)
def test_spmv_long_row_groups_and_solve(ctx):
    p, A2, S = _dense_row_problem()
    rowptr = A2.indptr.astype(np.int32)
    assert max(rowptr[min(g + 256, p.n)] - rowptr[g] for g in range(0, p.n, 256)) > 2048
    dec = dc.decompose(p.n, p.mesh.tri, p.mesh.dirichlet, p.part, p.n_parts, 2)
    hp = dg.HostProblem(p.mesh.xy, p.mesh.tri, p.mesh.dirichlet, rowptr, A2.indices, A2.data, p.b, p.u0,
                        dec.sub_ptr, dec.sub_nodes, dec.weights)
    prob = dg.Problem(ctx, hp, dg.Model(ctx, SMOOTHER))
    x = np.random.default_rng(2).standard_normal(p.n)
    y = torch.empty(p.n, dtype=torch.float64, device="cuda")
    print("[gpu] spmv with dense row groups", flush=True)
    prob.spmv(_dev(x), y)
    assert np.all(np.abs(y.cpu().numpy() - A2 @ x) <= 1e-14 * (abs(A2) @ np.abs(x)))
    u = torch.empty(p.n, dtype=torch.float64, device="cuda")
    st = prob.solve(u, dg.default_opts(precision="fp64", rtol=1e-10, max_it=3000))
    ud = spl.spsolve(A2.tocsc(), p.b)
    ug = u.cpu().numpy()
    err = np.linalg.norm(ug - ud) / np.linalg.norm(ud)
    print(f"[gpu]   iterations {st.iterations}, L2 vs direct {err:.2e}", flush=True)
    assert st.converged and _rel_res(A2, p.b, ug, p.u0) <= 1e-9 and err <= 1e-6
