"""Two-level Schwarz preconditioners: DDM-GNN, DDM-LU, one-level ASM.

Test infrastructure only (see the package docstring).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from . import decomp as dc
from . import dss


class Coarse:
    """Nicolaides coarse problem r_c = R_0^T (R_0 A R_0^T)^{-1} R_0 r (Sec. III.A step 1).

    The paper factors the coarse matrix by LU; it is symmetric positive
    definite, so a Cholesky factor gives the same solve up to rounding.
    """

    def __init__(self, A: sp.csr_matrix, dec: dc.Decomposition):
        self.Z = dc.nicolaides_basis(dec)
        self.A0 = (self.Z.T @ (A @ self.Z)).toarray()
        self.factor = sla.cho_factor(self.A0, lower=True)

    def __call__(self, r: np.ndarray) -> np.ndarray:
        y = sla.cho_solve(self.factor, self.Z.T @ r)
        return self.Z @ y


class DDMGNN:
    """The DDM-GNN apply z = M(r) (Sec. III.A, steps 1-3).

    For each sub-mesh i: s_i = |R_i r|, c_i = R_i r / s_i, r~_i = DSS(G_i, c_i);
    z = r_c + sum_i R_i^T (w_i * s_i * r~_i) with w_i = 1 (the paper's glue) or
    the partition-of-unity weights D_i. A sub-mesh with s_i = 0 contributes 0
    (the limit of s * DSS(c) as s -> 0). z is zero at Dirichlet nodes.
    """

    def __init__(self, A, mesh_xy, tri, dirichlet, dec: dc.Decomposition, theta, kbar=30, d=10,
                 alpha=1e-3, prolong="pou", coarse=True):
        self.dec = dec
        self.dirichlet = np.asarray(dirichlet)
        self.blocks = dss.unpack(theta, kbar, d)
        self.alpha, self.d = alpha, d
        self.graphs = [dc.local_graph(dec.nodes(i), tri, mesh_xy, self.dirichlet) for i in range(dec.K)]
        self.prolong = prolong
        self.coarse = Coarse(A, dec) if coarse else None

    def local(self, i: int, r: np.ndarray):
        """(s_i, r~_i) of sub-mesh i; r~_i is None when s_i == 0."""
        ri = r[self.dec.nodes(i)]
        s = float(np.sqrt(np.dot(ri, ri)))
        if s == 0.0:
            return s, None
        return s, dss.forward(self.blocks, self.graphs[i], ri / s, self.alpha, self.d)

    def __call__(self, r: np.ndarray) -> np.ndarray:
        z = np.zeros_like(r)
        for i in range(self.dec.K):
            s, rt = self.local(i, r)
            if rt is None:
                continue
            w = self.dec.w(i) if self.prolong == "pou" else 1.0
            z[self.dec.nodes(i)] += w * s * rt
        if self.coarse is not None:
            z += self.coarse(r)
        z[self.dirichlet == 1] = 0.0
        return z


class DDMLU:
    """Two-level additive Schwarz with exact local solves, eq. (7) (the paper's DDM-LU).

    Local matrices R_i A R_i^T are factored densely by Cholesky. With
    prolong="unweighted" this is M^{-1}_{ASM,2} of eq. (7); with "pou" the local
    solutions are weighted by D_i before extension.
    """

    def __init__(self, A: sp.csr_matrix, dirichlet, dec: dc.Decomposition, prolong="unweighted",
                 coarse=True):
        self.dec = dec
        self.dirichlet = np.asarray(dirichlet)
        A = sp.csr_matrix(A)
        self.factors = []
        for i in range(dec.K):
            idx = dec.nodes(i)
            Ai = A[idx][:, idx].toarray()
            self.factors.append(sla.cho_factor(Ai, lower=True))
        self.prolong = prolong
        self.coarse = Coarse(A, dec) if coarse else None

    def __call__(self, r: np.ndarray) -> np.ndarray:
        z = np.zeros_like(r)
        for i in range(self.dec.K):
            idx = self.dec.nodes(i)
            v = sla.cho_solve(self.factors[i], r[idx])
            w = self.dec.w(i) if self.prolong == "pou" else 1.0
            z[idx] += w * v
        if self.coarse is not None:
            z += self.coarse(r)
        z[self.dirichlet == 1] = 0.0
        return z
