"""Rounding model of the matrix-core DSS forward: the tolerance of its parity tests.

The DSS_theta forward of Sec. III.B (eqs. (14)-(18)) in float64, with the
values rounded where the matrix-core kernel rounds them:

  * MFMA operands in bf16 (8-bit significand): the latent state h, the
    sub-mesh-centred coordinates (as a hi + lo pair), c, the weights and
    biases of the message first layers, of Psi's hidden layer (with the
    folded deg * b2 term) and of its output layer, and of the decoder;
  * the per-node projections P' and Q' stored in FP16, the |d| weights and
    edge lengths in FP16, and every step of the per-edge update
    S <- S + ReLU(P' + Q' + w |d|) in FP16 (add, fused multiply-add, add);
  * the message sums and the folded second message layers M = W1_psi W2_phi
    enter Psi's hidden layer in FP16;
  * ReLU(hidden) in bf16, and the state h, the products and the output in FP32.

Summation orders inside a product are not modelled (FP32 accumulation of at
most 16 terms), and the edge sums run over each receiver's in-edges in
ascending sender order, where the kernel uses its bank-aware slot order; the
kernel's error against the float64 oracle is therefore expected to be close to
the model's, not equal to it, and the GPU tests allow twice the model's error.
With every rounding switched off the model is the oracle's forward pass
(pinned in tests/test_bf16_model.py).
"""
from __future__ import annotations

import numpy as np


def bf16(x) -> np.ndarray:
    """Round to bfloat16 (round to nearest, ties to even), returned as float64."""
    a = np.ascontiguousarray(x, np.float64).astype(np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def f16(x) -> np.ndarray:
    """Round to IEEE binary16 (round to nearest, ties to even), returned as float64."""
    return np.asarray(x, np.float64).astype(np.float16).astype(np.float64)


def f32(x) -> np.ndarray:
    return np.asarray(x, np.float64).astype(np.float32).astype(np.float64)


def _exact(x) -> np.ndarray:
    return np.asarray(x, np.float64)


def forward(blocks, graph, c: np.ndarray, alpha: float, d: int, rounding: bool = True) -> np.ndarray:
    """DSS_theta(G_i) for one sub-mesh with the kernel's roundings (or none)."""
    rb, rh, rs = (bf16, f16, f32) if rounding else (_exact, _exact, _exact)
    k = graph.k
    j, l = graph.recv, graph.send
    centred = rs(graph.xy - graph.xy.mean(axis=0))
    hi = rb(centred)
    xy = hi + rb(centred - hi)
    d_jl = graph.xy[l] - graph.xy[j]
    nd = rh(np.sqrt((d_jl ** 2).sum(axis=1)))
    deg = np.bincount(j, minlength=k).astype(np.float64)
    # in-edges by receiver, then by sender: rank r of an edge among its receiver's
    order = np.lexsort((l, j))
    jo, lo, ndo = j[order], l[order], nd[order]
    first = np.searchsorted(jo, np.arange(k))
    rank = np.arange(jo.size) - first[jo]
    ranks = [np.flatnonzero(rank == r) for r in range(int(rank.max(initial=-1)) + 1)]
    cb = rb(rs(c))
    H = np.zeros((k, d))
    for blk in blocks:
        hb = rb(H)
        sums = []
        for m, sgn in ((blk.phi_out, 1.0), (blk.phi_in, -1.0)):
            w_r, w_s = rb(m.W1[:, :d]), rb(m.W1[:, d:2 * d])
            w_d, w_n = rb(m.W1[:, 2 * d:2 * d + 2]), rh(m.W1[:, 2 * d + 2])
            P = rh(hb @ w_r.T + rb(m.b1) - sgn * xy @ w_d.T)
            Q = rh(hb @ w_s.T + sgn * xy @ w_d.T)
            S = np.zeros((k, d))
            for idx in ranks:  # one in-edge of every receiver at a time, in order
                t = rh(P[jo[idx]] + Q[lo[idx]])
                t = rh(np.outer(ndo[idx], w_n) + t)
                S[jo[idx]] = rh(S[jo[idx]] + np.maximum(t, 0.0))
            sums.append(S)
        psi = blk.psi
        w1_out, w1_in = psi.W1[:, d + 1:2 * d + 1], psi.W1[:, 2 * d + 1:]
        m_out, m_in = rh(w1_out @ blk.phi_out.W2), rh(w1_in @ blk.phi_in.W2)
        degb = rb(w1_out @ blk.phi_out.b2 + w1_in @ blk.phi_in.b2)
        hid = (hb @ rb(psi.W1[:, :d]).T + rb(psi.b1) + np.outer(cb, rb(psi.W1[:, d])) + np.outer(deg, degb)
               + sums[0] @ m_out.T + sums[1] @ m_in.T)
        bh = rb(np.maximum(rs(hid), 0.0))
        o = rs(bh @ rb(psi.W2).T + rb(psi.b2))
        H = rs(H + rs(alpha) * o)
    dec = blocks[-1].dec
    hd = rb(np.maximum(rs(rb(H) @ rb(dec.W1).T + rb(dec.b1)), 0.0))
    return rs(hd @ rb(dec.W2).T + rs(dec.b2))[:, 0]


def tolerance(blocks, graphs, cs, alpha: float, d: int, factor: float = 2.0) -> float:
    """factor x the model's worst error relative to the largest output magnitude,
    over the given sub-meshes (each compared with the float64 forward pass)."""
    worst = 0.0
    for g, c in zip(graphs, cs):
        ref = forward(blocks, g, c, alpha, d, rounding=False)
        got = forward(blocks, g, c, alpha, d)
        worst = max(worst, float(np.abs(got - ref).max() / np.abs(ref).max()))
    return factor * worst
