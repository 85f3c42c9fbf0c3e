"""Setup on the device against independent host computations.

* Overlap expansion and partition-of-unity weights (Sec. II.A, overlap of
  Sec. IV.A): bit-exact against the oracle's decomposition (oracle.decomp).
* Coarse level (Sec. III.A step 1): the device forms R_0 A R_0^T and inverts
  it by blocked Gauss-Jordan; the coarse solve y = A_0^{-1} y0 of an apply is
  compared with numpy's solve of the oracle's A_0, on problems whose K spans
  many pivot blocks and tiles of the inversion.
* DDM-LU local solvers (eq. (7)): the device assembles and inverts every
  R_i A R_i^T; the local terms of an apply are compared with numpy's solve of
  the oracle's local matrices.
The tolerances are those of an explicitly formed inverse of order m applied
to a vector against a direct solve: m * eps * kappa relative to the largest
entry.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_2402_08296_amd as dg  # noqa: E402
import workload as W  # noqa: E402
from oracle import decomp as dc, schwarz as sw  # noqa: E402
from tests._cases import oracle_problem  # noqa: E402

pytestmark = pytest.mark.gpu

SMOOTHER = W.smoother_theta(omega=0.15, out_scale=1.7)


@pytest.fixture(scope="module")
def ctx():
    print("[gpu] creating context", flush=True)
    return dg.Context()


def _i32(a):
    return torch.from_numpy(np.ascontiguousarray(a, np.int32)).cuda()


@pytest.mark.timeout(300)
@pytest.mark.parametrize("seed,n,parts,delta", [(1, 2500, 5, 2), (2, 4000, 9, 1), (3, 3000, 4, 4), (4, 6000, 12, 0),
                                                (5, 100_000, 150, 2)])
def test_overlap_expansion_on_device_bitexact(ctx, seed, n, parts, delta):
    p = W.make_problem(seed, n, parts, 0.3)
    print(f"[gpu] device overlap N={p.n} parts={parts} delta={delta}", flush=True)
    sp, nodes, w = ctx.expand_overlap_device(p.n, _i32(p.mesh.tri), _i32(p.part),
                                             torch.from_numpy(p.mesh.dirichlet.astype(np.uint8)).cuda(), parts, delta)
    dec = dc.decompose(p.n, p.mesh.tri, p.mesh.dirichlet, p.part, parts, delta)
    assert np.array_equal(sp, dec.sub_ptr)
    assert np.array_equal(nodes.cpu().numpy(), dec.sub_nodes)
    assert np.array_equal(w.cpu().numpy(), dec.weights)


def test_overlap_expansion_refuses_bad_ids(ctx):
    p = W.make_problem(1, 2000, 4, 0.3)
    bad = p.part.copy()
    bad[7] = 4
    with pytest.raises(dg.DDMGNNError, match="part id"):
        ctx.expand_overlap_device(p.n, _i32(p.mesh.tri), _i32(bad),
                                  torch.from_numpy(p.mesh.dirichlet.astype(np.uint8)).cuda(), 4, 2)
    tri = p.mesh.tri.copy()
    tri[3, 1] = p.n
    with pytest.raises(dg.DDMGNNError, match="triangle"):
        ctx.expand_overlap_device(p.n, _i32(tri), _i32(p.part),
                                  torch.from_numpy(p.mesh.dirichlet.astype(np.uint8)).cuda(), 4, 2)


@pytest.mark.timeout(300)
@pytest.mark.parametrize("seed,n,parts,delta", [(11, 20_000, 40, 2), (12, 120_000, 700, 2), (15, 6000, 240, 4)])
def test_coarse_level_formed_on_device(ctx, seed, n, parts, delta):
    """y = A_0^{-1} R_0 r of one apply against numpy's solve of the oracle's A_0 (K = 40 and
    700: one and eleven pivot blocks of 64, up to 121 tiles of 64 x 64 per step). The third
    problem (small parts, overlap 4) has rows of A_0 with more than 32 nonzero columns, which
    the assembly sums on one thread, beside rows summed by whole workgroups."""
    p = W.make_problem(seed, n, parts, 0.3)
    hp = oracle_problem(p, delta=delta)
    print(f"[gpu] device coarse level N={p.n} K={hp.K}", flush=True)
    prob = dg.Problem(ctx, hp, dg.Model(ctx, SMOOTHER))
    A = p.A.to_scipy()
    dec = dc.Decomposition(p.n, hp.sub_ptr, hp.sub_nodes, hp.weights)
    co = sw.Coarse(A, dec)
    if delta == 4:
        assert (np.count_nonzero(co.A0, axis=1) > 32).any() and (np.count_nonzero(co.A0, axis=1) <= 32).any()
    r = p.b - A @ p.u0
    z = torch.empty(p.n, dtype=torch.float64, device="cuda")
    prob.apply(torch.from_numpy(r).cuda(), z, dg.default_opts(precision="fp64"))
    _, y0, y, _ = [t.cpu().numpy() for t in prob.intermediates()]
    y0_ref = co.Z.T @ r
    y_ref = np.linalg.solve(co.A0, y0_ref)
    err = np.abs(y - y_ref).max() / np.abs(y_ref).max()
    cond = np.linalg.cond(co.A0)
    print(f"[gpu]   coarse solve relative error {err:.2e} (cond(A_0) {cond:.1e})", flush=True)
    assert np.abs(y0 - y0_ref).max() <= 1e-12 * np.abs(y0_ref).max()
    assert err <= hp.K * np.finfo(float).eps * cond  # an inverse of order K against a direct solve


@pytest.mark.timeout(300)
def test_singular_coarse_refused_on_device(ctx):
    """Two identical sub-meshes make R_0 A R_0^T singular: problem creation reports E_NOT_SPD."""
    p = W.make_problem(13, 1800, 4, 0.2)
    hp = oracle_problem(p)
    sp = np.concatenate([hp.sub_ptr, [hp.sub_ptr[-1] + hp.sub_ptr[1]]])
    sn = np.concatenate([hp.sub_nodes, hp.sub_nodes[:hp.sub_ptr[1]]])
    w = np.concatenate([hp.weights, hp.weights[:hp.sub_ptr[1]]])
    w[:hp.sub_ptr[1]] *= 0.5
    w[hp.sub_ptr[-1]:] *= 0.5
    hp2 = dg.HostProblem(hp.xy, hp.tri, hp.dirichlet, hp.rowptr, hp.col, hp.val, hp.b, hp.u0, sp, sn, w)
    with pytest.raises(dg.DDMGNNError) as ei:
        dg.Problem(ctx, hp2, dg.Model(ctx, SMOOTHER))
    assert ei.value.code == -4


@pytest.mark.timeout(300)
def test_local_inverses_formed_on_device(ctx):
    """Local terms of a DDM-LU apply (the device inverses times R_i r) against numpy's solve
    of each R_i A R_i^T (every seventh sub-mesh; sub-meshes of 219 to 6102 nodes, up to 96
    pivot blocks of 64 in one batch)."""
    p = W.make_problem(14, 60_000, 60, 0.5)
    hp = oracle_problem(p)
    ks = np.diff(hp.sub_ptr)
    print(f"[gpu] device local inverses K={hp.K} k in [{ks.min()}, {ks.max()}]", flush=True)
    prob = dg.Problem(ctx, hp, dg.Model(ctx, SMOOTHER))
    A = p.A.to_scipy().tocsr()
    r = p.b - A @ p.u0
    z = torch.empty(p.n, dtype=torch.float64, device="cuda")
    prob.apply(torch.from_numpy(r).cuda(), z, dg.default_opts(local_solver=dg.LOCAL_LU,
                                                              prolong=dg.PROLONG_UNWEIGHTED))
    loc = prob.intermediates()[3].cpu().numpy()
    worst = 0.0
    for i in range(0, hp.K, 7):
        idx = hp.sub_nodes[hp.sub_ptr[i]:hp.sub_ptr[i + 1]]
        Ai = A[idx][:, idx].toarray()
        ref = np.linalg.solve(Ai, r[idx])
        err = np.abs(loc[hp.sub_ptr[i]:hp.sub_ptr[i + 1]] - ref).max() / np.abs(ref).max()
        worst = max(worst, err / (idx.size * np.finfo(float).eps * np.linalg.cond(Ai)))
    print(f"[gpu]   worst local error in units of k eps kappa: {worst:.2e}", flush=True)
    assert worst <= 1.0
