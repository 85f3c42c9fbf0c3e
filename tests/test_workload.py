"""Pins of the seeded input generator: mesh, P1 assembly, partition, weights."""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spl

import workload as W


def test_generator_deterministic():
    a = W.make_problem(3, 3000, 4, 0.2)
    b = W.make_problem(3, 3000, 4, 0.2)
    assert a.mesh.xy.tobytes() == b.mesh.xy.tobytes()
    assert a.mesh.tri.tobytes() == b.mesh.tri.tobytes()
    assert a.A.val.tobytes() == b.A.val.tobytes()
    assert a.b.tobytes() == b.b.tobytes()
    assert a.part.tobytes() == b.part.tobytes()
    c = W.make_problem(4, 3000, 4, 0.2)
    assert c.mesh.xy.shape != a.mesh.xy.shape or c.mesh.xy.tobytes() != a.mesh.xy.tobytes()


def test_mesh_is_valid_triangulation():
    m = W.make_mesh(7, 2000)
    p = m.xy[m.tri]
    det = (p[:, 1, 0] - p[:, 0, 0]) * (p[:, 2, 1] - p[:, 0, 1]) - \
          (p[:, 2, 0] - p[:, 0, 0]) * (p[:, 1, 1] - p[:, 0, 1])
    assert (det > 0).all()
    # Euler characteristic of a disc: V - E + F = 1
    t = m.tri.astype(np.int64)
    e = np.concatenate([t[:, [0, 1]], t[:, [1, 2]], t[:, [2, 0]]])
    e = np.unique(np.sort(e, 1), axis=0)
    assert m.n - e.shape[0] + t.shape[0] == 1
    # boundary edges (one triangle) carry only Dirichlet nodes, and every
    # Dirichlet node is on a boundary edge
    ed = np.sort(np.concatenate([t[:, [0, 1]], t[:, [1, 2]], t[:, [2, 0]]]), 1)
    u, cnt = np.unique(ed, axis=0, return_counts=True)
    bnodes = np.unique(u[cnt == 1])
    assert set(bnodes.tolist()) == set(np.flatnonzero(m.dirichlet).tolist())
    # all nodes used
    assert np.unique(t).size == m.n


def test_mesh_is_delaunay():
    m = W.make_mesh(11, 600)
    xy = m.xy
    for tr in m.tri:
        a, b, c = xy[tr]
        # circumcircle by brute force
        M = np.array([[b[0] - a[0], b[1] - a[1]], [c[0] - a[0], c[1] - a[1]]])
        rhs = 0.5 * np.array([b @ b - a @ a, c @ c - a @ a])
        cc = np.linalg.solve(M, rhs)
        r2 = ((a - cc) ** 2).sum()
        d2 = ((xy - cc) ** 2).sum(1)
        d2[tr] = np.inf
        assert (d2 >= r2 * (1 - 1e-9)).all()


def test_node_count_near_target():
    for target in [5000, 20000]:
        m = W.make_mesh(0, target)
        assert 0.85 * target < m.n < 1.15 * target


def _stiffness(mesh, eliminate):
    f_mid = np.zeros((mesh.tri.shape[0], 3))
    g = np.zeros(mesh.n)
    return W.assemble(mesh, f_mid, g, eliminate)


def test_stiffness_symmetric_and_kernel():
    m = W.make_mesh(5, 3000)
    A, _ = _stiffness(m, eliminate=False)
    As = A.to_scipy()
    assert abs(As - As.T).max() == 0.0
    assert np.abs(As @ np.ones(m.n)).max() < 1e-13
    # rows are sorted, diagonal present
    for i in range(0, m.n, 97):
        cols = A.col[A.rowptr[i]:A.rowptr[i + 1]]
        assert (np.diff(cols) > 0).all() and i in cols


def test_delaunay_interior_offdiagonals_nonpositive():
    m = W.make_mesh(6, 3000)
    A, _ = _stiffness(m, eliminate=False)
    As = A.to_scipy().tocoo()
    t = m.tri.astype(np.int64)
    ed = np.sort(np.concatenate([t[:, [0, 1]], t[:, [1, 2]], t[:, [2, 0]]]), 1)
    u, cnt = np.unique(ed, axis=0, return_counts=True)
    interior = {tuple(x) for x in u[cnt == 2]}
    for i, j, v in zip(As.row, As.col, As.data):
        if i < j and (i, j) in interior:
            assert v <= 1e-14


def test_eliminated_system_spd_and_identity_rows():
    p = W.make_problem(2, 1500, 2)
    A = p.A.to_scipy().toarray()
    np.linalg.cholesky(A)
    for i in np.flatnonzero(p.mesh.dirichlet):
        row = A[i].copy()
        assert row[i] == 1.0
        row[i] = 0
        assert not row.any() and not A[:, i][np.arange(p.n) != i].any()
        assert p.b[i] == p.u0[i]
    r0 = p.b - p.A.to_scipy() @ p.u0
    assert np.all(r0[p.mesh.dirichlet == 1] == 0.0)


def test_patch_test_linear_solution_exact():
    """f = 0 and linear g: the P1 solution equals g at every node."""
    m = W.make_mesh(9, 2500)
    g = 0.7 * m.xy[:, 0] - 1.3 * m.xy[:, 1] + 0.25
    A, b = W.assemble(m, np.zeros((m.tri.shape[0], 3)), g, eliminate=True)
    u = spl.spsolve(A.to_scipy().tocsc(), b)
    assert np.abs(u - g).max() < 1e-12


@pytest.mark.slow
def test_manufactured_solution_second_order():
    """u = sin(a x) cos(b y): nodal L2 error falls as h^2 when h halves on the same domain."""
    errs = []
    h0 = W.ELEMENT_SIZE * 4
    for k in range(3):
        h = h0 / 2 ** k
        m = W.make_mesh(21, 1500 * 4 ** k, h)
        R = m.R
        a, bb = np.pi / R, 0.5 * np.pi / R
        u_ex = lambda x, y: np.sin(a * x) * np.cos(bb * y)
        f = lambda x, y: (a * a + bb * bb) * np.sin(a * x) * np.cos(bb * y)
        mid = W.edge_midpoints(m)
        A, b = W.assemble(m, f(mid[..., 0], mid[..., 1]), u_ex(m.xy[:, 0], m.xy[:, 1]), True)
        u = spl.spsolve(A.to_scipy().tocsc(), b)
        e = u - u_ex(m.xy[:, 0], m.xy[:, 1])
        errs.append(np.sqrt(np.mean(e ** 2)))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert (rates > 1.7).all() and (rates < 2.5).all(), (errs, rates)


def test_partition_exact_count_and_cover():
    p = W.make_problem(1, 8000, 11, 0.3)
    cnt = np.bincount(p.part, minlength=11)
    assert cnt.size == 11 and (cnt > 0).all() and cnt.sum() == p.n
    q = W.make_problem(1, 8000, 8, 0.0)
    cnt = np.bincount(q.part)
    assert cnt.max() - cnt.min() <= 2


def test_xavier_theta_layout_and_bounds():
    th = W.xavier_theta(42, 30, 10).astype(np.float64)
    assert th.size == 30 * (11 * 100 + 150 + 1)
    d = 10
    pos = 0
    for _ in range(30):
        for fan_in, fan_out in [(23, 10), (23, 10), (31, 10), (10, 1)]:
            a1 = np.sqrt(6.0 / (fan_in + d))
            W1 = th[pos:pos + d * fan_in]; pos += d * fan_in
            assert np.abs(W1).max() <= a1 and np.abs(W1).max() > 0.5 * a1
            assert not th[pos:pos + d].any(); pos += d
            a2 = np.sqrt(6.0 / (d + fan_out))
            W2 = th[pos:pos + fan_out * d]; pos += fan_out * d
            assert np.abs(W2).max() <= a2
            assert not th[pos:pos + fan_out].any(); pos += fan_out
    assert pos == th.size


def test_splitmix64_reference_outputs():
    """The published splitmix64 generator from state 0 starts 0xe220a8397b1dcdaf,
    0x6e789e6aa1b965f4, 0x06c45d188009454f."""
    assert [int(x) for x in W.splitmix64(0, 3)] == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]
    # counter-based: a later output depends only on the seed and its index
    assert int(W.splitmix64(5, 10)[7]) == int(W.splitmix64(5 + 7 * 0x9E3779B97F4A7C15 % 2**64, 1)[0])
