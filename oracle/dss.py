"""DSS_theta forward pass in float64 (Sec. III.B).

Test infrastructure only (see the package docstring).

The model acts on a latent state H = (h_j), h_j in R^d, of one sub-mesh:
  * initialisation: H^0 = 0;
  * k = 1..kbar message-passing blocks (eqs. (14)-(17)): for every node j,
        phi_out_j = sum_{l in N(j)} Phi_out^k(h_j, h_l, d_jl, |d_jl|)
        phi_in_j  = sum_{l in N(j)} Phi_in^k (h_j, h_l, d_lj, |d_lj|)
        h_j      <- h_j + alpha * Psi^k(h_j, c_j, phi_out_j, phi_in_j)
    where every node reads the previous state H^{k-1};
  * decoding (eq. (18)): the output is D^{kbar}(H^{kbar}).
Every MLP has one hidden layer with ReLU (Sec. IV.B); the output layer is linear.
d_jl = x_l - x_j is the relative position of the sender seen from the receiver
and d_lj = -d_jl.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp

from .decomp import LocalGraph


@dataclass
class MLP:
    W1: np.ndarray
    b1: np.ndarray
    W2: np.ndarray
    b2: np.ndarray

    def __call__(self, x: np.ndarray) -> np.ndarray:
        hidden = np.maximum(x @ self.W1.T + self.b1, 0.0)
        return hidden @ self.W2.T + self.b2


@dataclass
class Block:
    phi_out: MLP
    phi_in: MLP
    psi: MLP
    dec: MLP


def n_weights(kbar: int, d: int) -> int:
    """Parameter count kbar * (11 d^2 + 15 d + 1) with hidden width d (Table II)."""
    per_block = 0
    for fan_in, fan_out in [(2 * d + 3, d), (2 * d + 3, d), (3 * d + 1, d), (d, 1)]:
        per_block += d * fan_in + d + fan_out * d + fan_out
    return kbar * per_block


def unpack(theta: np.ndarray, kbar: int, d: int) -> list[Block]:
    """Split the flat weight vector into kbar blocks (layout of the weight file).

    Per block: Phi_out {W1[d,2d+3], b1[d], W2[d,d], b2[d]}, Phi_in {same},
    Psi {W1[d,3d+1], b1[d], W2[d,d], b2[d]}, Dec {W1[d,d], b1[d], W2[1,d], b2[1]}.
    """
    theta = np.asarray(theta, np.float64)
    if theta.size != n_weights(kbar, d):
        raise ValueError("weight count does not match kbar*(11d^2+15d+1)")
    pos = 0

    def take(shape):
        nonlocal pos
        size = int(np.prod(shape))
        out = theta[pos:pos + size].reshape(shape)
        pos += size
        return out

    def mlp(fan_in, fan_out):
        return MLP(take((d, fan_in)), take((d,)), take((fan_out, d)), take((fan_out,)))

    blocks = []
    for _ in range(kbar):
        blocks.append(Block(mlp(2 * d + 3, d), mlp(2 * d + 3, d), mlp(3 * d + 1, d), mlp(d, 1)))
    return blocks


def forward(blocks: list[Block], graph: LocalGraph, c: np.ndarray, alpha: float, d: int) -> np.ndarray:
    """r_hat = DSS_theta(G_i) for one sub-mesh with normalised residual c."""
    k = graph.k
    j, l = graph.recv, graph.send
    d_jl = graph.xy[l] - graph.xy[j]
    norm = np.sqrt((d_jl ** 2).sum(axis=1, keepdims=True))
    # S[j, e] = 1 when edge e is received by node j: S @ messages sums over N(j).
    S = sp.csr_matrix((np.ones(j.size), (j, np.arange(j.size))), shape=(k, j.size))
    H = np.zeros((k, d))
    for blk in blocks:
        x_out = np.concatenate([H[j], H[l], d_jl, norm], axis=1)
        x_in = np.concatenate([H[j], H[l], -d_jl, norm], axis=1)
        phi_out = S @ blk.phi_out(x_out)
        phi_in = S @ blk.phi_in(x_in)
        H = H + alpha * blk.psi(np.concatenate([H, c[:, None], phi_out, phi_in], axis=1))
    return blocks[-1].dec(H)[:, 0]
