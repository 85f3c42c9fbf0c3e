"""Training objective of DSS_theta and its gradient, in float64 (test infrastructure only).

Sec. II.B defines L_res(u, G), the mean over the N nodes of G of the squared
residual (A u - b)_j. Sec. III.B trains DSS_theta on the sum over blocks
k = 1..kbar of L_res of the decoded state D^k(H^k) of each block (the
intermediate decoders exist for this loss only). Sec. IV.B: local problems of
the two-level Schwarz preconditioner, Adam, gradient clipping at 1e-2.

A local problem is one sub-mesh i with the local matrix A_i = R_i A R_i^T and
the right-hand side c (the normalised restriction of a residual, Sec. III.A).
The functions here take the sum of squared residuals over all nodes and blocks
times a caller-chosen ``scale`` (1 / sum of the batch's node counts gives the
mean over a batch taken as one graph). The gradient comes from PyTorch autograd
in float64 on the CPU, through the per-edge MLPs as the paper writes them (the
messages of every edge are evaluated one by one: no factorisation).

Pins (tests): central finite differences of the loss; theta = 0 gives
kbar * scale * |c|^2; weights realising Richardson steps give the loss of the
Richardson iterates computed by a plain loop; Adam against its closed form after
one step.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import torch

from .decomp import LocalGraph
from .dss import n_weights


def local_matrix(A: sp.csr_matrix, nodes: np.ndarray) -> sp.csr_matrix:
    """A_i = R_i A R_i^T: the rows and columns of the sub-mesh's nodes (Sec. II.A)."""
    return sp.csr_matrix(A[nodes][:, nodes])


def local_rhs(A: sp.csr_matrix, b: np.ndarray, u: np.ndarray, nodes: np.ndarray) -> np.ndarray:
    """Right-hand side of a local problem at the iterate u: c_i = R_i r / |R_i r| with
    r = b - A u (the normalised restriction of Sec. III.A); zero when R_i r = 0."""
    r = (b - A @ u)[nodes]
    s = float(np.sqrt(r @ r))
    return r / s if s > 0 else np.zeros_like(r)


def _mlp(x, W1, b1, W2, b2):
    return torch.relu(x @ W1.T + b1) @ W2.T + b2


def _blocks(theta: torch.Tensor, kbar: int, d: int):
    """Views of theta in the weight layout of the forward pass (dss.unpack)."""
    pos = 0

    def take(*shape):
        nonlocal pos
        size = int(np.prod(shape))
        out = theta[pos:pos + size].reshape(shape)
        pos += size
        return out

    blocks = []
    for _ in range(kbar):
        blk = []
        for fan_in, fan_out in [(2 * d + 3, d), (2 * d + 3, d), (3 * d + 1, d), (d, 1)]:
            blk.append((take(d, fan_in), take(d), take(fan_out, d), take(fan_out)))
        blocks.append(blk)
    return blocks


def loss_torch(theta: torch.Tensor, graph: LocalGraph, Ai: sp.csr_matrix, c: np.ndarray, alpha: float,
               kbar: int, d: int, scale: float) -> torch.Tensor:
    """scale * sum_{k=1..kbar} sum_j ((A_i D^k(H^k))_j - c_j)^2 for one local problem."""
    k = graph.k
    j = torch.as_tensor(graph.recv, dtype=torch.long)
    l = torch.as_tensor(graph.send, dtype=torch.long)
    xy = torch.as_tensor(graph.xy, dtype=torch.float64)
    d_jl = xy[l] - xy[j]
    norm = torch.sqrt((d_jl ** 2).sum(dim=1, keepdim=True))
    ct = torch.as_tensor(c, dtype=torch.float64)
    Ad = torch.as_tensor(Ai.toarray(), dtype=torch.float64)
    H = torch.zeros(k, d, dtype=torch.float64)
    total = torch.zeros((), dtype=torch.float64)
    for (po, pi, ps, de) in _blocks(theta, kbar, d):
        # messages of every edge, summed per receiver (Sec. III.B)
        m_out = _mlp(torch.cat([H[j], H[l], d_jl, norm], dim=1), *po)
        m_in = _mlp(torch.cat([H[j], H[l], -d_jl, norm], dim=1), *pi)
        phi_out = torch.zeros(k, d, dtype=torch.float64).index_add(0, j, m_out)
        phi_in = torch.zeros(k, d, dtype=torch.float64).index_add(0, j, m_in)
        H = H + alpha * _mlp(torch.cat([H, ct[:, None], phi_out, phi_in], dim=1), *ps)
        r_hat = _mlp(H, *de)[:, 0]
        total = total + ((Ad @ r_hat - ct) ** 2).sum()
    return scale * total


def loss_and_grad(theta: np.ndarray, samples, alpha: float, kbar: int, d: int, scale: float):
    """Loss and gradient over a batch. samples: (graph, A_i, c) triples."""
    if theta.size != n_weights(kbar, d):
        raise ValueError("weight count does not match kbar*(11d^2+15d+1)")
    t = torch.tensor(np.asarray(theta, np.float64), requires_grad=True)
    total = torch.zeros((), dtype=torch.float64)
    for g, Ai, c in samples:
        total = total + loss_torch(t, g, Ai, c, alpha, kbar, d, scale)
    total.backward()
    return float(total.detach()), t.grad.numpy().copy()


def adam_step(theta, grad, m, v, t: int, lr: float, beta1=0.9, beta2=0.999, eps=1e-8, clip=0.0):
    """One Adam step with bias correction (the optimiser of Sec. IV.B), after scaling the
    gradient down to L2 norm `clip` when it is larger (clip <= 0: no clipping).
    Returns the new (theta, m, v)."""
    g = np.asarray(grad, np.float64)
    nrm = float(np.sqrt((g * g).sum()))
    if clip > 0 and nrm > clip:
        g = g * (clip / nrm)
    m = beta1 * m + (1 - beta1) * g
    v = beta2 * v + (1 - beta2) * g * g
    mh = m / (1 - beta1 ** t)
    vh = v / (1 - beta2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v
