"""C ABI on the host: exports, validation, and setup structures against the oracle (no GPU)."""
import copy
import os
import re

import numpy as np
import pytest

import paper_2402_08296_amd as dg
import workload as W
from oracle import decomp as dc
from tests._cases import small_problem

HEADER = os.path.join(os.path.dirname(os.path.dirname(__file__)), "include", "ddmgnn.h")


def test_library_exports_every_declared_symbol():
    L = dg.lib()
    names = set(re.findall(r"\b(ddmgnn_[a-z_0-9]+)\s*\(", open(HEADER).read()))
    assert len(names) > 20
    for name in sorted(names):
        assert hasattr(L, name), name
    assert b"gfx950" in L.ddmgnn_version()
    assert L.ddmgnn_max_subdomain_nodes() == 16384


def test_overlap_bitexact_vs_oracle():
    for seed, n, parts, delta in [(1, 2500, 5, 2), (2, 4000, 9, 1), (3, 3000, 4, 4)]:
        p = W.make_problem(seed, n, parts, 0.3)
        ptr, nodes = dg.expand_overlap(p.n, p.mesh.tri, p.part, parts, delta)
        optr, onodes = dc.expand_overlap(p.n, p.mesh.tri, p.part, parts, delta)
        assert np.array_equal(ptr, optr) and np.array_equal(nodes, onodes)
        w = dg.pou_weights(p.n, p.mesh.dirichlet, ptr, nodes)
        ow = dc.pou_weights(p.n, p.mesh.dirichlet, optr, onodes)
        assert w.tobytes() == ow.tobytes()


def test_local_graphs_bitexact_vs_oracle():
    p, hp = small_problem()
    for i in range(hp.K):
        rowptr, col = dg.setup_local_graph(hp, i)
        nodes = hp.sub_nodes[hp.sub_ptr[i]:hp.sub_ptr[i + 1]]
        g = dc.local_graph(nodes, p.mesh.tri, p.mesh.xy, p.mesh.dirichlet)
        recv = np.repeat(np.arange(nodes.size), np.diff(rowptr))
        assert np.array_equal(recv, g.recv) and np.array_equal(col, g.send)


def test_coarse_operator_vs_oracle():
    p, hp = small_problem()
    a0, a0inv = dg.setup_coarse(hp)
    dec = dc.Decomposition(p.n, hp.sub_ptr, hp.sub_nodes, hp.weights)
    Z = dc.nicolaides_basis(dec)
    ref = (Z.T @ (p.A.to_scipy() @ Z)).toarray()
    assert np.abs(a0 - ref).max() <= 1e-13 * np.abs(ref).max()
    assert np.abs(a0inv @ ref - np.eye(hp.K)).max() <= 1e-10


def test_local_inverse_vs_definition():
    """(R_i A R_i^T)^{-1} of the exact local solver: the restriction picks rows and
    columns of A (eq. (7)), and the product with that matrix is the identity."""
    p, hp = small_problem()
    A = p.A.to_scipy().tocsr()
    for i in range(hp.K):
        idx = hp.sub_nodes[hp.sub_ptr[i]:hp.sub_ptr[i + 1]]
        Ai = A[idx][:, idx].toarray()
        inv = dg.setup_local_inverse(hp, i)
        assert inv.shape == Ai.shape
        assert np.array_equal(inv, inv.T)
        assert np.abs(inv @ Ai - np.eye(idx.size)).max() <= 1e-10
        ref = np.linalg.inv(Ai)
        assert np.abs(inv - ref).max() <= 1e-10 * np.abs(ref).max()
    with pytest.raises(dg.DDMGNNError):
        dg.setup_local_inverse(hp, hp.K)


def _offdiag(h):
    rows = np.repeat(np.arange(h.n), np.diff(h.rowptr))
    return int(np.flatnonzero(rows != h.col)[0])


def _desc_copy(hp):
    return copy.deepcopy(hp)


@pytest.mark.parametrize("mutate,msg", [
    (lambda h: h.val.__setitem__(_offdiag(h), h.val[_offdiag(h)] + 1.0), "symmetric"),
    (lambda h: h.col.__setitem__(3, h.n + 7), "out of range"),
    (lambda h: h.weights.__setitem__(0, h.weights[0] + 0.5) if not h.dirichlet[h.sub_nodes[0]] else
     h.weights.__setitem__(np.flatnonzero(h.dirichlet[h.sub_nodes] == 0)[0],
                           h.weights[np.flatnonzero(h.dirichlet[h.sub_nodes] == 0)[0]] + 0.5), "partition of unity"),
    (lambda h: h.b.__setitem__(10, np.nan), "non-finite"),
    (lambda h: h.sub_nodes.__setitem__(slice(0, 2), h.sub_nodes[0:2][::-1].copy()), "ascending"),
    (lambda h: h.dirichlet.__setitem__(0, 2), "0 or 1"),
])
def test_validate_rejects(mutate, msg):
    _, hp = small_problem()
    dg.validate(hp)
    bad = _desc_copy(hp)
    mutate(bad)
    with pytest.raises(dg.DDMGNNError) as ei:
        dg.validate(bad)
    assert ei.value.code == -1 and msg in str(ei.value)


def test_validate_rejects_oversized_subdomain_and_uncovered_node():
    p = W.make_problem(2, 17000, 1)
    hp = dg.host_problem(p.mesh.xy, p.mesh.tri, p.mesh.dirichlet, p.A.rowptr, p.A.col, p.A.val, p.b, p.u0,
                         p.part, 1, 0)
    with pytest.raises(dg.DDMGNNError, match="maximum"):
        dg.validate(hp)
    p = W.make_problem(2, 1500, 3)
    hp = dg.host_problem(p.mesh.xy, p.mesh.tri, p.mesh.dirichlet, p.A.rowptr, p.A.col, p.A.val, p.b, p.u0,
                         p.part, 3, 1)
    drop = hp.sub_nodes[hp.sub_ptr[0]:hp.sub_ptr[1]]
    keep = np.ones(hp.sub_nodes.size, bool)
    keep[:hp.sub_ptr[1]] = False
    hp2 = dg.HostProblem(hp.xy, hp.tri, hp.dirichlet, hp.rowptr, hp.col, hp.val, hp.b, hp.u0,
                         np.concatenate([[0], hp.sub_ptr[2:] - hp.sub_ptr[1]]), hp.sub_nodes[keep], hp.weights[keep])
    assert drop.size > 0
    with pytest.raises(dg.DDMGNNError):
        dg.validate(hp2)


def test_setup_detects_singular_coarse():
    """Two identical sub-meshes make R_0 A R_0^T singular: setup reports E_NOT_SPD."""
    p, hp = small_problem()
    sp = np.concatenate([hp.sub_ptr, [hp.sub_ptr[-1] + hp.sub_ptr[1]]])
    sn = np.concatenate([hp.sub_nodes, hp.sub_nodes[:hp.sub_ptr[1]]])
    w = np.concatenate([hp.weights, hp.weights[:hp.sub_ptr[1]]])
    # keep a partition of unity: halve the weights of the duplicated sub-mesh
    w[:hp.sub_ptr[1]] *= 0.5
    w[hp.sub_ptr[-1]:] *= 0.5
    hp2 = dg.HostProblem(hp.xy, hp.tri, hp.dirichlet, hp.rowptr, hp.col, hp.val, hp.b, hp.u0, sp, sn, w)
    with pytest.raises(dg.DDMGNNError) as ei:
        dg.setup_coarse(hp2)
    assert ei.value.code == -4


def test_tune_cache_roundtrip(tmp_path):
    """The autotuner cache: one autotune per (arch, config class), later problems of the
    class get the cached schedule (no GPU: a stand-in problem records the calls)."""
    from paper_2402_08296_amd import tune

    class FakeProb:
        def __init__(self):
            self.calls, self.set = 0, None

        def autotune(self, opts, iterations):
            self.calls += 1
            return dg.Tuning(64 * 1024, 512), 0.5

        def set_tuning(self, small_lds=0, vec_blocks=0):
            self.set = (small_lds, vec_blocks)

    _, hp = small_problem()
    opts = dg.default_opts(precision="bf16")
    path = str(tmp_path / "cache.json")
    a = FakeProb()
    r1 = tune.tuned(a, hp, opts, "gfx950", path)
    assert a.calls == 1 and not r1["cached"] and r1["tuning"] == {"small_lds": 65536, "vec_blocks": 512}
    b = FakeProb()
    r2 = tune.tuned(b, hp, opts, "gfx950", path)
    assert b.calls == 0 and r2["cached"] and b.set == (65536, 512) and r2["key"] == r1["key"]
    c = FakeProb()
    tune.tuned(c, hp, dg.default_opts(precision="fp32"), "gfx950", path)  # another class
    assert c.calls == 1
    assert tune.config_class(hp.n, hp.sub_ptr, opts) == tune.config_class(hp.n, list(hp.sub_ptr), opts)


def test_library_xavier_matches_generator():
    """ddmgnn_model_init_xavier and the seeded input generator build the same weights, bit for bit."""
    for seed, kbar, d in [(42, 30, 10), (7, 5, 5), (3, 10, 20)]:
        a = dg.init_xavier(seed, kbar, d)
        b = W.xavier_theta(seed, kbar, d)
        assert a.dtype == b.dtype and a.tobytes() == b.tobytes()
    with pytest.raises(dg.DDMGNNError):
        desc = dg.ModelDesc(30, 10, 1e-3)
        import ctypes
        th = np.empty(10, dtype=np.float32)
        dg._check(dg.lib().ddmgnn_model_init_xavier(ctypes.byref(desc), 1, th.ctypes.data_as(ctypes.c_void_p), 10))


def test_validate_rejects_oversized_and_empty():
    """A sub-mesh above the register-resident kernels' size (2048 nodes) is accepted, one above
    the library's limit (16384 nodes, 16-bit local ids) and an empty problem are refused on
    the host."""
    p = W.make_problem(33, 3000, 1)
    hp = host_problem_for(p)
    assert hp.sub_ptr[1] > 2048
    dg.validate(hp)
    p = W.make_problem(34, 16600, 1)
    hp = host_problem_for(p)
    assert hp.sub_ptr[1] > 16384
    with pytest.raises(dg.DDMGNNError, match="larger than"):
        dg.validate(hp)
    d = hp.desc()
    d.n_nodes = 0
    import ctypes
    assert dg.lib().ddmgnn_validate_problem(ctypes.byref(d)) != 0


def host_problem_for(p):
    from tests._cases import host_problem
    return host_problem(p, delta=0)
