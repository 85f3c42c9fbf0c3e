"""Krylov solvers in float64: PCG (Algorithm 1), flexible CG, flexible GMRES, plain CG.

Test infrastructure only (see the package docstring).

Convergence is measured as the relative residual |r_i| / |r_0| with u_0 the
lifted Dirichlet data (Sec. IV.C uses a relative residual tolerance of 1e-6).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass
class Result:
    u: np.ndarray
    iterations: int
    converged: bool
    history: list = field(default_factory=list)   # |r_i| / |r_0| for i = 0..iterations
    true_rel_residual: float = float("nan")


def _finish(A, b, u, r0n, it, conv, hist):
    res = Result(u, it, conv, hist)
    res.true_rel_residual = float(np.linalg.norm(b - A @ u) / r0n) if r0n > 0 else 0.0
    return res


def pcg(A, b, u0, M, rtol=1e-6, max_it=10_000) -> Result:
    """Preconditioned CG exactly as Algorithm 1 (Fletcher-Reeves beta = rho_{i+1}/rho_i).

    The preconditioner M is a callable r -> z (the red steps of Algorithm 1).
    """
    u = u0.copy()
    r = b - A @ u
    r0n = np.linalg.norm(r)
    hist = [1.0]
    if r0n == 0.0:
        return _finish(A, b, u, r0n, 0, True, hist)
    z = M(r)
    p = z.copy()
    rho = r @ z
    for i in range(max_it):
        q = A @ p
        alpha = rho / (p @ q)
        u = u + alpha * p
        r = r - alpha * q
        rel = np.linalg.norm(r) / r0n
        hist.append(rel)
        if rel < rtol:
            return _finish(A, b, u, r0n, i + 1, True, hist)
        z = M(r)
        rho_new = r @ z
        beta = rho_new / rho
        rho = rho_new
        p = z + beta * p
    return _finish(A, b, u, r0n, max_it, False, hist)


def fcg(A, b, u0, M, rtol=1e-6, max_it=10_000, m_max=1) -> Result:
    """Flexible CG with truncated A-orthogonalisation against the last m_max directions.

    For i = 0, 1, ...: stop when |r_i| <= rtol |r_0|; z_i = M(r_i);
    p_i = z_i - sum_k (<z_i, q_k> / <p_k, q_k>) p_k over the last m_max (p_k, q_k);
    q_i = A p_i; alpha_i = <p_i, r_i> / <p_i, q_i>; u += alpha_i p_i; r -= alpha_i q_i.
    Each step minimises the A-norm of the error along p_i, so it remains a valid
    descent method when M is nonlinear or varies between iterations.
    """
    u = u0.copy()
    r = b - A @ u
    r0n = np.linalg.norm(r)
    hist = [1.0]
    if r0n == 0.0:
        return _finish(A, b, u, r0n, 0, True, hist)
    P, Q, PQ = [], [], []
    it = 0
    while True:
        rel = np.linalg.norm(r) / r0n
        if it > 0:
            hist.append(rel)
        if rel <= rtol:
            return _finish(A, b, u, r0n, it, True, hist)
        if it >= max_it:
            return _finish(A, b, u, r0n, it, False, hist)
        z = M(r)
        p = z.copy()
        for pk, qk, pqk in zip(P, Q, PQ):
            p -= (z @ qk) / pqk * pk
        q = A @ p
        pq = p @ q
        alpha = (p @ r) / pq
        u = u + alpha * p
        r = r - alpha * q
        P.append(p); Q.append(q); PQ.append(pq)
        if len(P) > m_max:
            P.pop(0); Q.pop(0); PQ.pop(0)
        it += 1


def fgmres(A, b, u0, M, rtol=1e-6, max_it=10_000, restart=30) -> Result:
    """Restarted flexible GMRES (Saad's right-preconditioned variant for a preconditioner
    that may change between iterations; the paper's flexible alternative to FCG).

    A cycle starts from r = b - A u, beta = |r|, v_0 = r / beta. Step j: z_j = M(v_j),
    w = A z_j, Arnoldi against v_0..v_j by modified Gram-Schmidt (h_ij = <w, v_i>,
    w -= h_ij v_i), h_{j+1,j} = |w|, v_{j+1} = w / h_{j+1,j}. Givens rotations keep the
    Hessenberg matrix triangular; |g_{j+1}| is the residual norm of the least-squares
    iterate u + Z y, which the history records as |g_{j+1}| / |r_0|. The cycle ends when
    that is <= rtol, after `restart` steps, or when |w| = 0; then y solves the triangular
    system and u += Z y. Iterations count preconditioner applications.
    """
    u = u0.copy()
    r = b - A @ u
    r0n = np.linalg.norm(r)
    hist = [1.0]
    if r0n == 0.0:
        return _finish(A, b, u, r0n, 0, True, hist)
    it = 0
    while True:
        beta = np.linalg.norm(r)
        V = [r / beta]
        Z = []
        H = np.zeros((restart + 1, restart))
        cs = np.zeros(restart)
        sn = np.zeros(restart)
        g = np.zeros(restart + 1)
        g[0] = beta
        k = 0
        done = False
        for j in range(restart):
            z = M(V[j])
            Z.append(z)
            w = A @ z
            for i in range(j + 1):
                H[i, j] = w @ V[i]
                w = w - H[i, j] * V[i]
            hn = np.linalg.norm(w)
            H[j + 1, j] = hn
            for i in range(j):
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            d = np.hypot(H[j, j], H[j + 1, j])
            cs[j], sn[j] = H[j, j] / d, H[j + 1, j] / d
            H[j, j], H[j + 1, j] = d, 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            it += 1
            k = j + 1
            rel = abs(g[j + 1]) / r0n
            hist.append(rel)
            done = rel <= rtol or hn == 0.0
            if done or it >= max_it:
                break
            V.append(w / hn)
        y = np.zeros(k)
        for i in range(k - 1, -1, -1):
            y[i] = (g[i] - H[i, i + 1:k] @ y[i + 1:k]) / H[i, i]
        for i in range(k):
            u = u + y[i] * Z[i]
        r = b - A @ u
        if done:
            return _finish(A, b, u, r0n, it, True, hist)
        if it >= max_it:
            return _finish(A, b, u, r0n, it, False, hist)


def cg(A, b, u0, rtol=1e-6, max_it=100_000) -> Result:
    """Unpreconditioned CG (Algorithm 1 with M = I, restricted to free nodes by the lift)."""
    return pcg(A, b, u0, lambda r: r.copy(), rtol, max_it)
