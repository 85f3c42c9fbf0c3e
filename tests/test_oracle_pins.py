"""Pins of the CPU FP64 oracle against facts the paper and the mathematics fix.

Each test checks the oracle against something other than itself: values printed
in the paper (Table II weight counts, Table I ranges), closed forms, textbook
special cases, invariants, and brute force on tiny inputs.
"""
import os

import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spl

import workload as W
from oracle import decomp as dc
from oracle import dss, krylov as kr, schwarz as sw

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden(name):
    rows = []
    for line in open(os.path.join(GOLDEN, name)):
        line = line.strip()
        if line and not line.startswith("#"):
            rows.append([float(x) for x in line.split()])
    return np.array(rows)


@pytest.fixture(scope="module")
def small():
    p = W.make_problem(5, 1800, 4, 0.2)
    dec = dc.decompose(p.n, p.mesh.tri, p.mesh.dirichlet, p.part, p.n_parts, 2)
    return p, dec


# ------------------------------------------------------------------ weights
def test_table2_weight_counts():
    """Table II: the oracle's layout reproduces every printed weight count."""
    for kbar, d, n in _golden("table2_weights.txt"):
        assert dss.n_weights(int(kbar), int(d)) == int(n)
        th = np.zeros(int(n), np.float32)
        blocks = dss.unpack(th, int(kbar), int(d))
        assert len(blocks) == int(kbar)
    with pytest.raises(ValueError):
        dss.unpack(np.zeros(37531), 30, 10)


# ------------------------------------------------------------------ decomposition
def test_overlap_matches_breadth_first_distance(small):
    p, _ = small
    n = p.n
    adj = [set() for _ in range(n)]
    for a, b, c in p.mesh.tri:
        for u, v in ((a, b), (b, c), (c, a)):
            adj[u].add(v); adj[v].add(u)
    for delta in (0, 1, 2, 4):
        ptr, nodes = dc.expand_overlap(n, p.mesh.tri, p.part, p.n_parts, delta)
        for i in range(p.n_parts):
            dist = np.full(n, 10 ** 9)
            front = list(np.flatnonzero(p.part == i))
            dist[front] = 0
            while front:
                nxt = []
                for u in front:
                    for v in adj[u]:
                        if dist[v] > dist[u] + 1:
                            dist[v] = dist[u] + 1
                            nxt.append(v)
                front = nxt
            expect = np.flatnonzero(dist <= delta)
            assert np.array_equal(nodes[ptr[i]:ptr[i + 1]], expect)


def test_partition_of_unity_and_coarse_basis(small):
    p, dec = small
    s = np.zeros(p.n)
    np.add.at(s, dec.sub_nodes, dec.weights)
    free = p.mesh.dirichlet == 0
    assert np.abs(s[free] - 1.0).max() <= 1e-15
    assert not s[~free].any()
    Z = dc.nicolaides_basis(dec)
    assert np.abs(Z @ np.ones(dec.K) - free).max() <= 1e-15
    A0 = (Z.T @ (p.A.to_scipy() @ Z)).toarray()
    assert np.abs(A0 - A0.T).max() <= 1e-12 * np.abs(A0).max()
    assert np.linalg.eigvalsh(A0).min() > 0


def test_local_graph_direction_rule(small):
    """Edges inside a sub-mesh are bidirectional except at Dirichlet nodes, which only send."""
    p, dec = small
    for i in range(dec.K):
        nodes = dec.nodes(i)
        g = dc.local_graph(nodes, p.mesh.tri, p.mesh.xy, p.mesh.dirichlet)
        inset = set(nodes.tolist())
        pos = {v: k for k, v in enumerate(nodes.tolist())}
        expect = set()
        for a, b, c in p.mesh.tri:
            for u, v in ((a, b), (b, c), (c, a)):
                if u in inset and v in inset:
                    if not p.mesh.dirichlet[u]:
                        expect.add((pos[u], pos[v]))
                    if not p.mesh.dirichlet[v]:
                        expect.add((pos[v], pos[u]))
        got = list(zip(g.recv.tolist(), g.send.tolist()))
        assert len(got) == len(set(got)) == len(expect)
        assert set(got) == expect
        assert got == sorted(got)
        assert not g.dirichlet[g.recv].any()


# ------------------------------------------------------------------ DSS forward
def _laplacian_dense(g):
    k = g.k
    L = np.zeros((k, k))
    for j, l in zip(g.recv, g.send):
        L[j, j] += 1.0
        L[j, l] -= 1.0
    return L


def test_dss_constructed_richardson_equals_plain_loop(small):
    """Weights realising v <- v + w (c - L v): the DSS must equal kbar Richardson steps."""
    p, dec = small
    g = dc.local_graph(dec.nodes(1), p.mesh.tri, p.mesh.xy, p.mesh.dirichlet)
    rng = np.random.default_rng(0)
    c = rng.standard_normal(g.k)
    omega = np.linspace(0.05, 0.2, 30)
    th = W.smoother_theta(30, 10, 1e-3, omega, 1.5).astype(np.float64)
    out = dss.forward(dss.unpack(th, 30, 10), g, c, 1e-3, 10)
    L = _laplacian_dense(g)
    v = np.zeros(g.k)
    for k in range(30):
        w = float(np.float32(omega[k] / 1e-3)) * 1e-3
        v = v + w * (c - L @ v)
    assert np.abs(out - 1.5 * v).max() <= 1e-13 * np.abs(v).max()
    # Dirichlet nodes receive nothing: they only integrate their own c
    dn = g.dirichlet == 1
    if dn.any():
        w_sum = sum(float(np.float32(o / 1e-3)) * 1e-3 for o in omega)
        assert np.allclose(out[dn], 1.5 * w_sum * c[dn], rtol=1e-13, atol=0)


def _geometry_theta(kbar, d, alpha):
    """phi_out[1] = d_x, phi_in[2] = (d_lj)_x, phi_out[3] = |d|; Psi adds them to h[1..3]/alpha*alpha."""
    z = lambda *s: np.zeros(s)
    blocks = []
    for k in range(kbar):
        W1 = z(d, 2 * d + 3); W2 = z(d, d)
        W1[0, 2 * d], W1[1, 2 * d] = 1.0, -1.0          # relu(dx), relu(-dx)
        W1[2, 2 * d + 2] = 1.0                          # relu(|d|)
        W2[1, 0], W2[1, 1], W2[3, 2] = 1.0, -1.0, 1.0
        V1 = z(d, 2 * d + 3); V2 = z(d, d)
        V1[0, 2 * d], V1[1, 2 * d] = 1.0, -1.0          # relu(dx of d_lj)
        V2[2, 0], V2[2, 1] = 1.0, -1.0
        P1 = z(d, 3 * d + 1); P2 = z(d, d)
        # hidden pairs carry phi_out[1], phi_in[2], phi_out[3] (>= 0)
        P1[0, d + 1 + 1], P1[1, d + 1 + 1] = 1.0, -1.0
        P1[2, d + 1 + d + 2], P1[3, d + 1 + d + 2] = 1.0, -1.0
        P1[4, d + 1 + 3] = 1.0
        P2[1, 0], P2[1, 1] = 1 / alpha, -1 / alpha
        P2[2, 2], P2[2, 3] = 1 / alpha, -1 / alpha
        P2[3, 4] = 1 / alpha
        D1 = z(d, d); D2 = z(1, d)
        D1[0, 1], D1[1, 1], D1[2, 2], D1[3, 2], D1[4, 3] = 1, -1, 1, -1, 1
        D2[0, :5] = [1.0, -1.0, 10.0, -10.0, 100.0]
        blocks.append(dict(phi_out=(W1, z(d), W2, z(d)), phi_in=(V1, z(d), V2, z(d)),
                           psi=(P1, z(d), P2, z(d)), dec=(D1, z(d), D2, z(1))))
    return W.pack_theta(blocks, d).astype(np.float64)


def test_dss_edge_features_sign_and_norm(small):
    """Pins d_jl = x_l - x_j for Phi_out, d_lj = -d_jl for Phi_in, and |d| (eqs. (14)-(15))."""
    p, dec = small
    g = dc.local_graph(dec.nodes(2), p.mesh.tri, p.mesh.xy, p.mesh.dirichlet)
    kbar, d, alpha = 3, 10, 1e-3
    th = _geometry_theta(kbar, d, alpha)
    out = dss.forward(dss.unpack(th, kbar, d), g, np.zeros(g.k), alpha, d)
    sx = np.zeros(g.k); sn = np.zeros(g.k)
    for j, l in zip(g.recv, g.send):
        dx = g.xy[l] - g.xy[j]
        sx[j] += dx[0]
        sn[j] += np.hypot(dx[0], dx[1])
    a = float(np.float32(1 / alpha)) * alpha
    expect = kbar * a * (sx + 10.0 * (-sx) + 100.0 * sn)
    assert np.abs(out - expect).max() <= 1e-12 * max(1.0, np.abs(expect).max())


def _brute_mlp(x, W1, b1, W2, b2):
    hid = [max(0.0, sum(W1[u][i] * x[i] for i in range(len(x))) + b1[u]) for u in range(len(b1))]
    return [sum(W2[o][u] * hid[u] for u in range(len(hid))) + b2[o] for o in range(len(b2))]


def test_dss_brute_force_tiny_mesh():
    """Two triangles, four nodes, random weights: per-node Python loops vs the oracle."""
    xy = np.array([[0.0, 0.0], [1.0, 0.1], [0.2, 0.9], [1.1, 1.2]])
    tri = np.array([[0, 1, 2], [1, 3, 2]], np.int32)
    dirichlet = np.array([1, 0, 0, 0], np.uint8)
    g = dc.local_graph(np.arange(4), tri, xy, dirichlet)
    kbar, d, alpha = 3, 4, 0.3
    rng = np.random.default_rng(7)
    th = rng.uniform(-1, 1, dss.n_weights(kbar, d))
    blocks = dss.unpack(th, kbar, d)
    c = np.array([0.0, 0.6, -0.8, 0.2])
    nbrs = {0: [], 1: [0, 2, 3], 2: [0, 1, 3], 3: [1, 2]}
    H = [[0.0] * d for _ in range(4)]
    for blk in blocks:
        newH = []
        for j in range(4):
            po = [0.0] * d; pi = [0.0] * d
            for l in nbrs[j]:
                dj = [xy[l][0] - xy[j][0], xy[l][1] - xy[j][1]]
                nr = (dj[0] ** 2 + dj[1] ** 2) ** 0.5
                mo = _brute_mlp(H[j] + H[l] + dj + [nr], *[m.tolist() for m in
                                (blk.phi_out.W1, blk.phi_out.b1, blk.phi_out.W2, blk.phi_out.b2)])
                mi = _brute_mlp(H[j] + H[l] + [-dj[0], -dj[1]] + [nr], *[m.tolist() for m in
                                (blk.phi_in.W1, blk.phi_in.b1, blk.phi_in.W2, blk.phi_in.b2)])
                po = [a + b for a, b in zip(po, mo)]
                pi = [a + b for a, b in zip(pi, mi)]
            ps = _brute_mlp(H[j] + [c[j]] + po + pi, *[m.tolist() for m in
                            (blk.psi.W1, blk.psi.b1, blk.psi.W2, blk.psi.b2)])
            newH.append([h + alpha * q for h, q in zip(H[j], ps)])
        H = newH
        last = blk
    expect = [_brute_mlp(H[j], *[m.tolist() for m in (last.dec.W1, last.dec.b1, last.dec.W2, last.dec.b2)])[0]
              for j in range(4)]
    out = dss.forward(blocks, g, c, alpha, d)
    assert np.abs(out - np.array(expect)).max() <= 1e-13


def test_dss_permutation_and_translation_invariance(small):
    p, dec = small
    nodes = dec.nodes(0)
    g = dc.local_graph(nodes, p.mesh.tri, p.mesh.xy, p.mesh.dirichlet)
    blocks = dss.unpack(W.xavier_theta(3), 30, 10)
    rng = np.random.default_rng(1)
    c = rng.standard_normal(g.k)
    c /= np.linalg.norm(c)
    out = dss.forward(blocks, g, c, 1e-3, 10)
    perm = rng.permutation(g.k)
    inv = np.argsort(perm)
    recv, send = inv[g.recv], inv[g.send]
    o = np.lexsort((send, recv))
    gp = dc.LocalGraph(recv[o], send[o], g.xy[perm], g.dirichlet[perm])
    outp = dss.forward(blocks, gp, c[perm], 1e-3, 10)
    assert np.abs(outp - out[perm]).max() <= 1e-13 * np.abs(out).max()
    gt = dc.LocalGraph(g.recv, g.send, g.xy + np.array([3.25, -7.5]), g.dirichlet)
    outt = dss.forward(blocks, gt, c, 1e-3, 10)
    assert np.abs(outt - out).max() <= 1e-12 * np.abs(out).max()


# ------------------------------------------------------------------ two-level apply
def _identity_dss_theta(alpha):
    """kbar = 1 block whose output is exactly c (Psi = c/alpha, decoder = identity)."""
    d = 10
    z = lambda *s: np.zeros(s)
    P1 = z(d, 3 * d + 1); P2 = z(d, d)
    P1[0, d], P1[1, d] = 1.0, -1.0
    P2[0, 0], P2[0, 1] = 1.0 / alpha, -1.0 / alpha
    D1 = z(d, d); D2 = z(1, d)
    D1[0, 0], D1[1, 0] = 1.0, -1.0
    D2[0, 0], D2[0, 1] = 1.0, -1.0
    blk = dict(phi_out=(z(d, 2 * d + 3), z(d), z(d, d), z(d)), phi_in=(z(d, 2 * d + 3), z(d), z(d, d), z(d)),
               psi=(P1, z(d), P2, z(d)), dec=(D1, z(d), D2, z(1)))
    return W.pack_theta([blk], d)


def test_apply_glue_with_identity_local_solver(small):
    """With DSS(c) = c: z = r_c + sum_i R_i^T w_i |R_i r| c_i = r_c + sum_i R_i^T w_i R_i r (gluing step)."""
    p, dec = small
    A = p.A.to_scipy()
    alpha = 0.5  # 1/alpha exact in float32 so DSS(c) = c up to one rounding
    th = _identity_dss_theta(alpha)
    rng = np.random.default_rng(3)
    r = rng.standard_normal(p.n)
    r[p.mesh.dirichlet == 1] = 0.0
    # independent coarse correction: Z built element by element
    Z = np.zeros((p.n, dec.K))
    for i in range(dec.K):
        for node, w in zip(dec.nodes(i), dec.w(i)):
            Z[node, i] = w
    A0 = Z.T @ A.toarray() @ Z
    rc = Z @ np.linalg.solve(A0, Z.T @ r)
    mult = np.bincount(dec.sub_nodes, minlength=p.n)
    for prolong, local in (("pou", r), ("unweighted", mult * r)):
        M = sw.DDMGNN(A, p.mesh.xy, p.mesh.tri, p.mesh.dirichlet, dec, th, kbar=1, d=10, alpha=alpha,
                      prolong=prolong)
        z = M(r)
        expect = rc + local
        expect[p.mesh.dirichlet == 1] = 0
        assert np.abs(z - expect).max() <= 1e-11 * np.abs(expect).max()


def test_apply_positive_homogeneity_bitexact(small):
    """c is unchanged by r -> 2^k r, so Apply(2^k r) = 2^k Apply(r) exactly."""
    p, dec = small
    A = p.A.to_scipy()
    M = sw.DDMGNN(A, p.mesh.xy, p.mesh.tri, p.mesh.dirichlet, dec, W.xavier_theta(42))
    r = p.b - A @ p.u0
    z = M(r)
    for k in (-3, 5):
        assert np.array_equal(M(r * 2.0 ** k), z * 2.0 ** k)


def test_apply_zero_norm_subdomain_contributes_nothing(small):
    p, dec = small
    A = p.A.to_scipy()
    M = sw.DDMGNN(A, p.mesh.xy, p.mesh.tri, p.mesh.dirichlet, dec, W.xavier_theta(42), coarse=False)
    r = np.zeros(p.n)
    assert not M(r).any()
    only = dec.nodes(0)[~np.isin(dec.nodes(0), np.concatenate([dec.nodes(i) for i in range(1, dec.K)]))]
    r[only[:5]] = 1.0
    r[p.mesh.dirichlet == 1] = 0
    z = M(r)
    s, rt = M.local(0, r)
    expect = np.zeros(p.n)
    expect[dec.nodes(0)] = dec.w(0) * s * rt
    expect[p.mesh.dirichlet == 1] = 0
    assert np.array_equal(z, expect)


def test_coarse_galerkin_identity(small):
    p, dec = small
    A = p.A.to_scipy()
    C = sw.Coarse(A, dec)
    r = np.random.default_rng(2).standard_normal(p.n)
    rc = C(r)
    assert np.abs(C.Z.T @ (A @ rc) - C.Z.T @ r).max() <= 1e-10 * np.abs(C.Z.T @ r).max()


def test_ddmlu_unweighted_symmetric_positive_definite():
    p = W.make_problem(8, 700, 3)
    dec = dc.decompose(p.n, p.mesh.tri, p.mesh.dirichlet, p.part, p.n_parts, 2)
    A = p.A.to_scipy()
    M = sw.DDMLU(A, p.mesh.dirichlet, dec, prolong="unweighted")
    free = np.flatnonzero(p.mesh.dirichlet == 0)
    E = np.zeros((p.n, free.size))
    E[free, np.arange(free.size)] = 1.0
    Md = np.stack([M(E[:, k]) for k in range(free.size)], 1)[free]
    assert np.abs(Md - Md.T).max() <= 1e-12 * np.abs(Md).max()
    assert np.linalg.eigvalsh(0.5 * (Md + Md.T)).min() > 0


def test_ddmlu_both_glues_match_elementwise_construction():
    """eq. (7) written out with explicit matrices: R_i as a 0/1 matrix, A_i = R_i A R_i^T,
    the local solve by a general dense solve, D_i as a diagonal, the Nicolaides Z
    element by element; z = sum_i R_i^T W_i A_i^{-1} R_i r + Z A_0^{-1} Z^T r with
    W_i = D_i (partition of unity) or I (the paper's glue), zero at Dirichlet nodes."""
    p = W.make_problem(12, 500, 3)
    dec = dc.decompose(p.n, p.mesh.tri, p.mesh.dirichlet, p.part, p.n_parts, 2)
    A = p.A.to_scipy().toarray()
    rng = np.random.default_rng(5)
    r = rng.standard_normal(p.n)
    r[p.mesh.dirichlet == 1] = 0.0
    Z = np.zeros((p.n, dec.K))
    for i in range(dec.K):
        for node, w in zip(dec.nodes(i), dec.w(i)):
            Z[node, i] = w
    rc = Z @ np.linalg.solve(Z.T @ A @ Z, Z.T @ r)
    for prolong in ("pou", "unweighted"):
        expect = rc.copy()
        for i in range(dec.K):
            nodes = dec.nodes(i)
            R = np.zeros((nodes.size, p.n))
            R[np.arange(nodes.size), nodes] = 1.0
            Wi = np.diag(dec.w(i)) if prolong == "pou" else np.eye(nodes.size)
            expect += R.T @ (Wi @ np.linalg.solve(R @ A @ R.T, R @ r))
        expect[p.mesh.dirichlet == 1] = 0.0
        z = sw.DDMLU(p.A.to_scipy(), p.mesh.dirichlet, dec, prolong=prolong)(r)
        assert np.abs(z - expect).max() <= 1e-11 * np.abs(expect).max(), prolong
    # the two glues differ wherever sub-meshes overlap (the pin sees the weights)
    zp = sw.DDMLU(p.A.to_scipy(), p.mesh.dirichlet, dec, prolong="pou")(r)
    zu = sw.DDMLU(p.A.to_scipy(), p.mesh.dirichlet, dec, prolong="unweighted")(r)
    assert np.abs(zp - zu).max() > 1e-3 * np.abs(zu).max()


def test_ddmlu_single_subdomain_is_exact_inverse():
    p = W.make_problem(8, 900, 1)
    dec = dc.decompose(p.n, p.mesh.tri, p.mesh.dirichlet, p.part, 1, 0)
    A = p.A.to_scipy()
    M = sw.DDMLU(A, p.mesh.dirichlet, dec, coarse=False)
    res = kr.pcg(A, p.b, p.u0, M, 1e-10)
    assert res.iterations == 1


# ------------------------------------------------------------------ Krylov
def test_identity_preconditioner_fcg_pcg_cg_agree(small):
    p, _ = small
    A = p.A.to_scipy()
    a = kr.cg(A, p.b, p.u0, 1e-8)
    b = kr.pcg(A, p.b, p.u0, lambda r: r.copy(), 1e-8)
    c = kr.fcg(A, p.b, p.u0, lambda r: r.copy(), 1e-8)
    assert a.iterations == b.iterations == c.iterations
    assert np.abs(a.u - c.u).max() <= 1e-10 * np.abs(a.u).max()
    h = min(len(b.history), len(c.history), 40)
    assert np.allclose(b.history[:h], c.history[:h], rtol=1e-8)


def test_fcg1_equals_pcg_for_fixed_spd_preconditioner(small):
    p, dec = small
    A = p.A.to_scipy()
    M = sw.DDMLU(A, p.mesh.dirichlet, dec, prolong="unweighted")
    a = kr.pcg(A, p.b, p.u0, M, 1e-10, max_it=20)
    b = kr.fcg(A, p.b, p.u0, M, 1e-10, max_it=20, m_max=1)
    h = min(len(a.history), len(b.history))
    assert h >= 10
    assert np.allclose(a.history[:h], b.history[:h], rtol=1e-9)


def test_cg_finite_termination_tiny_dense():
    rng = np.random.default_rng(5)
    for n in (5, 12, 20):
        Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
        A = Q @ np.diag(rng.uniform(1, 10, n)) @ Q.T
        b = rng.standard_normal(n)
        res = kr.fcg(A, b, np.zeros(n), lambda r: r.copy(), 1e-10, max_it=n + 1)
        assert res.converged and res.iterations <= n
        assert np.abs(A @ res.u - b).max() <= 1e-8 * np.abs(b).max()


# ------------------------------------------------------------------ flexible GMRES
def test_fgmres_matches_least_squares_definition():
    """k GMRES steps (M = I) give min |b - A(u0 + K c)| over the Krylov matrix
    K = [r0, A r0, ..., A^(k-1) r0], solved here by a dense least-squares routine."""
    rng = np.random.default_rng(11)
    n = 40
    A = np.eye(n) * 4 + rng.standard_normal((n, n)) * 0.3   # nonsymmetric, well conditioned
    b = rng.standard_normal(n)
    u0 = np.zeros(n)
    res = kr.fgmres(A, b, u0, lambda r: r.copy(), 1e-14, max_it=8, restart=50)
    r0 = b - A @ u0
    for k in range(1, 9):
        K = np.stack([np.linalg.matrix_power(A, i) @ r0 for i in range(k)], 1)
        c = np.linalg.lstsq(A @ K, r0, rcond=None)[0]
        ls = np.linalg.norm(r0 - A @ K @ c) / np.linalg.norm(r0)
        assert abs(res.history[k] - ls) <= 1e-9 * max(ls, 1e-12) + 1e-13, (k, res.history[k], ls)


def test_fgmres_exact_preconditioner_one_iteration(small):
    p, _ = small
    A = p.A.to_scipy().tocsc()
    lu = spl.splu(A)
    res = kr.fgmres(A, p.b, p.u0, lambda r: lu.solve(r), 1e-10)
    assert res.converged and res.iterations == 1 and res.true_rel_residual <= 1e-10


def test_fgmres_residual_not_above_cg_and_pcg(small):
    """Same Krylov space, GMRES minimises the residual norm: |r_k| <= CG's |r_k| (M = I)
    and <= PCG's with a fixed SPD M (right preconditioning, x0 + M K_k(AM, r0))."""
    p, dec = small
    A = p.A.to_scipy()
    g = kr.fgmres(A, p.b, p.u0, lambda r: r.copy(), 1e-8, max_it=60, restart=200)
    c = kr.cg(A, p.b, p.u0, 1e-8, max_it=60)
    for k in range(1, min(len(g.history), len(c.history))):
        assert g.history[k] <= c.history[k] * (1 + 1e-7), k
    M = sw.DDMLU(A, p.mesh.dirichlet, dec, prolong="unweighted")
    g = kr.fgmres(A, p.b, p.u0, M, 1e-10, max_it=40, restart=200)
    c = kr.pcg(A, p.b, p.u0, M, 1e-10, max_it=40)
    for k in range(1, min(len(g.history), len(c.history))):
        assert g.history[k] <= c.history[k] * (1 + 1e-7), k


def test_fgmres_finite_termination_and_restarts():
    rng = np.random.default_rng(5)
    for n in (6, 12, 20):
        A = np.eye(n) * 3 + rng.standard_normal((n, n))
        b = rng.standard_normal(n)
        res = kr.fgmres(A, b, np.zeros(n), lambda r: r.copy(), 1e-10, max_it=n + 1, restart=n + 5)
        assert res.converged and res.iterations <= n
        assert np.abs(A @ res.u - b).max() <= 1e-8 * np.abs(b).max()
    # restarted: residual non-increasing across cycles, estimate = true residual at the end
    A = np.eye(30) * 3 + rng.standard_normal((30, 30)) * 0.5
    b = rng.standard_normal(30)
    res = kr.fgmres(A, b, np.zeros(30), lambda r: r.copy(), 1e-9, max_it=300, restart=4)
    assert res.converged
    assert all(res.history[i + 1] <= res.history[i] * (1 + 1e-9) for i in range(len(res.history) - 1))
    assert abs(res.true_rel_residual - res.history[-1]) <= 1e-6 * res.history[-1] + 1e-14


def test_fgmres_nonlinear_preconditioner_converges(small):
    """The flexible variant with the (nonlinear) DDM-GNN preconditioner reaches the
    direct solution."""
    p, dec = small
    A = p.A.to_scipy()
    M = sw.DDMGNN(A, p.mesh.xy, p.mesh.tri, p.mesh.dirichlet, dec, W.smoother_theta(omega=0.15, out_scale=1.7))
    res = kr.fgmres(A, p.b, p.u0, M, 1e-10, max_it=300, restart=30)
    u_direct = spl.spsolve(A.tocsc(), p.b)
    assert res.converged and res.true_rel_residual <= 1e-9
    assert np.linalg.norm(res.u - u_direct) / np.linalg.norm(u_direct) <= 1e-8


def test_solution_matches_direct_solve(small):
    p, dec = small
    A = p.A.to_scipy()
    u_direct = spl.spsolve(A.tocsc(), p.b)
    M = sw.DDMGNN(A, p.mesh.xy, p.mesh.tri, p.mesh.dirichlet, dec, W.smoother_theta(omega=0.15, out_scale=1.7))
    res = kr.fcg(A, p.b, p.u0, M, 1e-10, max_it=500)
    assert res.converged and res.true_rel_residual <= 2e-10
    assert np.linalg.norm(res.u - u_direct) / np.linalg.norm(u_direct) <= 1e-8


@pytest.mark.slow
def test_table1_ddmlu_and_cg_ballpark():
    """Sanity only (different generator): iteration counts near Table I's DDM-LU and CG columns."""
    rows = _golden("table1_iterations.txt")
    N, Ns, K, ov, lu_mean, lu_std, cg_mean, cg_std = rows[0]
    counts_lu, counts_cg = [], []
    for seed in range(3):
        p = W.make_problem(100 + seed, int(N), int(K))
        dec = dc.decompose(p.n, p.mesh.tri, p.mesh.dirichlet, p.part, p.n_parts, int(ov))
        A = p.A.to_scipy()
        counts_lu.append(kr.pcg(A, p.b, p.u0, sw.DDMLU(A, p.mesh.dirichlet, dec), 1e-6).iterations)
        counts_cg.append(kr.cg(A, p.b, p.u0, 1e-6).iterations)
    assert 0.5 * lu_mean <= np.mean(counts_lu) <= 2.0 * lu_mean, counts_lu
    assert 0.5 * cg_mean <= np.mean(counts_cg) <= 2.0 * cg_mean, counts_cg
