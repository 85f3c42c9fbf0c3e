"""Overlapping decomposition, partition of unity, coarse basis, local graphs.

Test infrastructure only (see the package docstring).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp


def mesh_adjacency(n: int, tri: np.ndarray) -> sp.csr_matrix:
    """Boolean node adjacency of the mesh graph (pairs of nodes sharing an edge)."""
    t = np.asarray(tri, np.int64)
    rows = np.concatenate([t[:, 0], t[:, 1], t[:, 2], t[:, 1], t[:, 2], t[:, 0]])
    cols = np.concatenate([t[:, 1], t[:, 2], t[:, 0], t[:, 0], t[:, 1], t[:, 2]])
    G = sp.csr_matrix((np.ones(rows.size, np.int8), (rows, cols)), shape=(n, n))
    G.data[:] = 1
    return G


def expand_overlap(n: int, tri: np.ndarray, part: np.ndarray, n_parts: int, delta: int):
    """Sub-meshes Omega_{h,i}: part i grown by `delta` layers of mesh adjacency.

    Sec. II.A (overlapping decomposition into K sub-meshes with k_i nodes) and
    Sec. IV.A (overlap of 2). Returns (sub_ptr[K+1], sub_nodes[sum k_i]) with
    each sub-mesh's global node ids in ascending order; the local index of a
    node is its rank in that list, which defines the boolean restriction R_i.
    """
    G = mesh_adjacency(n, tri)
    ptr = [0]
    nodes = []
    for i in range(n_parts):
        member = part == i
        for _ in range(delta):
            member = member | (G @ member.astype(np.int8) > 0)
        ids = np.flatnonzero(member).astype(np.int32)
        nodes.append(ids)
        ptr.append(ptr[-1] + ids.size)
    return np.array(ptr, np.int64), np.concatenate(nodes)


def pou_weights(n: int, dirichlet: np.ndarray, sub_ptr: np.ndarray, sub_nodes: np.ndarray) -> np.ndarray:
    """Partition-of-unity weights D_i(n) = 1/multiplicity(n), 0 at Dirichlet nodes.

    Then sum_i R_i^T D_i R_i 1 = 1 at every free node.
    """
    mult = np.bincount(sub_nodes, minlength=n).astype(np.float64)
    w = 1.0 / mult[sub_nodes]
    w[dirichlet[sub_nodes] == 1] = 0.0
    return w


@dataclass
class Decomposition:
    n: int
    sub_ptr: np.ndarray
    sub_nodes: np.ndarray
    weights: np.ndarray   # PoU weights D_i, aligned with sub_nodes

    @property
    def K(self) -> int:
        return self.sub_ptr.size - 1

    def nodes(self, i: int) -> np.ndarray:
        return self.sub_nodes[self.sub_ptr[i]:self.sub_ptr[i + 1]]

    def w(self, i: int) -> np.ndarray:
        return self.weights[self.sub_ptr[i]:self.sub_ptr[i + 1]]


def decompose(n, tri, dirichlet, part, n_parts, delta=2) -> Decomposition:
    ptr, nodes = expand_overlap(n, tri, part, n_parts, delta)
    return Decomposition(n, ptr, nodes, pou_weights(n, dirichlet, ptr, nodes))


def nicolaides_basis(dec: Decomposition) -> sp.csr_matrix:
    """Z (N x K): column i is R_i^T D_i R_i 1, so R_0 = Z^T (Sec. II.A, eq. (7)).

    The Nicolaides coarse space has one vector per sub-domain; with the
    partition-of-unity weights the columns sum to one at free nodes.
    """
    rows = dec.sub_nodes.astype(np.int64)
    cols = np.repeat(np.arange(dec.K), np.diff(dec.sub_ptr))
    return sp.csr_matrix((dec.weights, (rows, cols)), shape=(dec.n, dec.K))


@dataclass
class LocalGraph:
    """Directed DSS graph of one sub-mesh (Sec. III.B).

    recv/send are local indices of each directed edge send -> recv. Edges are
    sorted by (recv, send). Every mesh edge {j, l} inside the sub-mesh gives
    l -> j when j is not a Dirichlet node and j -> l when l is not: the graph is
    undirected except at (global) Dirichlet nodes, whose edges only point
    inward. xy holds the node coordinates.
    """
    recv: np.ndarray
    send: np.ndarray
    xy: np.ndarray
    dirichlet: np.ndarray

    @property
    def k(self) -> int:
        return self.xy.shape[0]


def local_graph(nodes: np.ndarray, tri: np.ndarray, xy: np.ndarray, dirichlet: np.ndarray) -> LocalGraph:
    k = nodes.size
    loc = -np.ones(xy.shape[0], np.int64)
    loc[nodes] = np.arange(k)
    t = loc[np.asarray(tri, np.int64)]
    inside = (t >= 0).all(axis=1)
    t = t[inside]
    a = np.concatenate([t[:, 0], t[:, 1], t[:, 2]])
    b = np.concatenate([t[:, 1], t[:, 2], t[:, 0]])
    und = np.unique(np.stack([np.minimum(a, b), np.maximum(a, b)], 1), axis=0)
    dl = dirichlet[nodes]
    recv, send = [], []
    for j, l in und:
        if not dl[j]:
            recv.append(j); send.append(l)
        if not dl[l]:
            recv.append(l); send.append(j)
    recv = np.array(recv, np.int64)
    send = np.array(send, np.int64)
    order = np.lexsort((send, recv))
    return LocalGraph(recv[order], send[order], xy[nodes].astype(np.float64), dl.copy())
