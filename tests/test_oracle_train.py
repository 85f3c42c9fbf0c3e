"""Pins of the oracle's training objective (Sec. II.B residual loss summed over the blocks
as in Sec. III.B) and of its Adam step: finite differences, closed forms and a plain loop."""
import numpy as np
import pytest

import workload as W
from oracle import decomp as dc
from oracle import dss
from oracle import train as tr


@pytest.fixture(scope="module")
def tiny():
    p = W.make_problem(7, 420, 3, 0.2)
    dec = dc.decompose(p.n, p.mesh.tri, p.mesh.dirichlet, p.part, p.n_parts, 2)
    out = []
    for i in range(dec.K):
        nodes = dec.nodes(i)
        g = dc.local_graph(nodes, p.mesh.tri, p.mesh.xy, p.mesh.dirichlet)
        out.append((g, tr.local_matrix(p.A.to_scipy(), nodes)))
    return p, out


def _theta(seed, kbar, d=10, bias=0.3):
    rng = np.random.default_rng(seed)
    th = W.xavier_theta(seed, kbar, d).astype(np.float64)
    return th + bias * rng.standard_normal(th.size) * (th == 0)  # nonzero biases too


def _rhs(g, seed):
    c = np.random.default_rng(seed).standard_normal(g.k)
    c[g.dirichlet == 1] = 0.0
    return c / np.linalg.norm(c)


def test_gradient_matches_central_differences(tiny):
    _, subs = tiny
    kbar, d, alpha = 2, 10, 0.5
    th = _theta(1, kbar, d)
    samples = [(g, A, _rhs(g, 10 + i)) for i, (g, A) in enumerate(subs[:2])]
    scale = 1.0 / sum(g.k for g, _, _ in samples)
    L, grad = tr.loss_and_grad(th, samples, alpha, kbar, d, scale)
    rng = np.random.default_rng(3)
    idx = rng.choice(th.size, 40, replace=False)
    idx = np.concatenate([idx, np.argsort(-np.abs(grad))[:10]])
    h = 1e-6
    for i in idx:
        tp, tm = th.copy(), th.copy()
        tp[i] += h
        tm[i] -= h
        fd = (tr.loss_and_grad(tp, samples, alpha, kbar, d, scale)[0]
              - tr.loss_and_grad(tm, samples, alpha, kbar, d, scale)[0]) / (2 * h)
        assert abs(fd - grad[i]) <= 1e-6 * np.abs(grad).max() + 1e-7 * abs(grad[i]), (i, fd, grad[i])


def test_zero_weights_give_kbar_times_rhs_norm(tiny):
    _, subs = tiny
    g, A = subs[0]
    c = _rhs(g, 5)
    kbar = 4
    L, grad = tr.loss_and_grad(np.zeros(dss.n_weights(kbar, 10)), [(g, A, c)], 1e-3, kbar, 10, 0.25)
    assert L == pytest.approx(kbar * 0.25 * float(c @ c), rel=1e-15)
    # only the output biases of the decoders see a gradient at theta = 0: -2 scale sum_j (A^T c)_j
    per = dss.n_weights(1, 10)
    expect = -2 * 0.25 * float((A.T @ c).sum())
    for k in range(kbar):
        assert grad[k * per + per - 1] == pytest.approx(expect, rel=1e-13)
    others = np.delete(grad, [k * per + per - 1 for k in range(kbar)])
    assert np.abs(others).max() == 0.0


def test_richardson_weights_give_the_loss_of_the_plain_iterates(tiny):
    """Weights realising v <- v + w (c - L v) with every decoder returning s v: the loss is
    sum_k |A_i (s v_k) - c|^2 of the plain Richardson iterates v_k."""
    _, subs = tiny
    g, A = subs[1]
    c = _rhs(g, 8)
    kbar, alpha, s = 6, 1e-3, 1.5
    omega = np.linspace(0.05, 0.2, kbar)
    th = W.smoother_theta(kbar, 10, alpha, omega, s).astype(np.float64)
    L, _ = tr.loss_and_grad(th, [(g, A, c)], alpha, kbar, 10, 1.0)
    Lap = np.zeros((g.k, g.k))
    for j, l in zip(g.recv, g.send):
        Lap[j, j] += 1.0
        Lap[j, l] -= 1.0
    Ad = A.toarray()
    v = np.zeros(g.k)
    expect = 0.0
    for k in range(kbar):
        w = float(np.float32(omega[k] / alpha)) * alpha
        v = v + w * (c - Lap @ v)
        res = Ad @ (s * v) - c
        expect += float(res @ res)
    assert L == pytest.approx(expect, rel=1e-12)


def test_last_block_output_matches_the_forward_pass(tiny):
    """The torch loss path and the numpy forward agree on D^kbar(H^kbar): with the decoder of
    every block but the last zeroed, the loss is |A r - c|^2 + (kbar - 1) |c|^2."""
    _, subs = tiny
    g, A = subs[2]
    c = _rhs(g, 9)
    kbar, d, alpha = 3, 10, 0.3
    th = _theta(4, kbar, d)
    per = dss.n_weights(1, d)
    dec0 = per - (d * d + d + d + 1)
    for k in range(kbar - 1):
        th[k * per + dec0:(k + 1) * per] = 0.0
    r = dss.forward(dss.unpack(th, kbar, d), g, c, alpha, d)
    L, _ = tr.loss_and_grad(th, [(g, A, c)], alpha, kbar, d, 1.0)
    res = A @ r - c
    assert L == pytest.approx(float(res @ res) + (kbar - 1) * float(c @ c), rel=1e-12)


def test_adam_first_step_closed_form():
    """After one step from m = v = 0 the bias-corrected update is lr * g / (|g| + eps)."""
    rng = np.random.default_rng(0)
    th, g = rng.standard_normal(50), rng.standard_normal(50)
    new, m, v = tr.adam_step(th, g, np.zeros(50), np.zeros(50), 1, 1e-2)
    assert np.allclose(new, th - 1e-2 * g / (np.abs(g) + 1e-8), rtol=1e-13, atol=1e-15)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)
    # clipping scales the gradient to the clip norm; the first step is invariant to that scale
    new_c, m_c, _ = tr.adam_step(th, g, np.zeros(50), np.zeros(50), 1, 1e-2, clip=1e-2)
    assert np.linalg.norm(m_c / 0.1) == pytest.approx(1e-2, rel=1e-12)
    assert np.allclose(new_c, th - 1e-2 * (g * 1e-2 / np.linalg.norm(g)) / (np.abs(g) * 1e-2 / np.linalg.norm(g) + 1e-8))


def test_local_rhs_definition(tiny):
    """c_i is the unit vector along R_i (b - A u), by an explicit row loop; the exact
    solution gives zero right-hand sides."""
    p, _ = tiny
    A = p.A.to_scipy()
    rng = np.random.default_rng(2)
    u = p.u0 + rng.standard_normal(p.n) * (p.mesh.dirichlet == 0)
    nodes = np.arange(10, 90)
    r = np.array([p.b[j] - sum(p.A.val[q] * u[p.A.col[q]] for q in range(p.A.rowptr[j], p.A.rowptr[j + 1]))
                  for j in nodes])
    c = tr.local_rhs(A, p.b, u, nodes)
    assert np.linalg.norm(c) == pytest.approx(1.0, rel=1e-14)
    assert np.allclose(c * np.linalg.norm(r), r, rtol=1e-12, atol=1e-12 * np.abs(r).max())
    import scipy.sparse.linalg as spl
    ex = spl.spsolve(A.tocsc(), p.b)
    assert np.abs(tr.local_rhs(A, p.b, ex, nodes)).max() <= 1.0  # defined (unit or zero)
    assert np.all(tr.local_rhs(A, A @ ex, ex, nodes) == 0.0)
