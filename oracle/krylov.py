"""Krylov solvers in float64: PCG (Algorithm 1), flexible CG, plain CG.

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


def cg(A, b, u0, rtol=1e-6, max_it=100_000) -> Result:
    """Unpreconditioned CG (Algorithm 1 with M = I, restricted to free nodes by the lift)."""
    return pcg(A, b, u0, lambda r: r.copy(), rtol, max_it)
