"""Pins of the rounding model that sets the BF16 DSS tolerance (tests/_bf16_model.py).

* The rounding helpers round to nearest with ties to even at 8 (bf16) and 11
  (binary16) significant bits.
* With its roundings switched off the model is the oracle's DSS forward pass
  (Sec. III.B), for both weight sets and two widths: a dropped term, a wrong
  sign or a transposed weight in the model fails this.
* With them on, its error against the oracle is of the order the formats
  allow (well above FP32 effects, well below the outputs).
"""
import numpy as np
import pytest

import workload as W
from oracle import decomp as dc, dss
from tests import _bf16_model as bm


def test_bf16_rounding_ties_to_even():
    one = 1.0
    assert bm.bf16(one) == 1.0
    assert bm.bf16(one + 2.0 ** -8) == 1.0                       # tie, 1.0 is even
    assert bm.bf16(one + 3 * 2.0 ** -8) == one + 2.0 ** -6       # tie, rounds up to the even neighbour
    assert bm.bf16(one + 2.0 ** -8 + 2.0 ** -20) == one + 2.0 ** -7  # above the tie
    assert bm.bf16(-(one + 3 * 2.0 ** -8)) == -(one + 2.0 ** -6)
    assert bm.bf16(3.0) == 3.0 and bm.bf16(0.0) == 0.0


def test_rounding_helpers_bounds():
    x = np.random.default_rng(0).standard_normal(10_000) * np.exp(np.random.default_rng(1).uniform(-8, 8, 10_000))
    for f, bits in ((bm.bf16, 8), (bm.f16, 11)):
        y = f(x)
        assert np.all(np.abs(y - x) <= 2.0 ** -bits * np.abs(x) * (1 + 1e-12) + (0 if bits == 8 else 2.0 ** -25))
        # the result has at most `bits` significant bits
        m, _ = np.frexp(y[y != 0])
        assert np.all(m * 2.0 ** bits == np.round(m * 2.0 ** bits))
    assert np.array_equal(bm.f16(x), x.astype(np.float16).astype(np.float64))


@pytest.fixture(scope="module")
def small():
    p = W.make_problem(31, 1500, 3, 0.2)
    dec = dc.decompose(p.n, p.mesh.tri, p.mesh.dirichlet, p.part, p.n_parts, 2)
    r = np.random.default_rng(2).standard_normal(p.n)
    r[p.mesh.dirichlet == 1] = 0
    graphs, cs = [], []
    for i in range(dec.K):
        nodes = dec.sub_nodes[dec.sub_ptr[i]:dec.sub_ptr[i + 1]]
        graphs.append(dc.local_graph(nodes, p.mesh.tri, p.mesh.xy, p.mesh.dirichlet))
        cs.append(r[nodes] / np.linalg.norm(r[nodes]))
    return graphs, cs


@pytest.mark.parametrize("kind,kbar,d", [("xavier", 30, 10), ("smoother", 30, 10), ("xavier", 5, 5),
                                         ("smoother", 10, 5)])
def test_model_without_rounding_is_the_oracle(small, kind, kbar, d):
    graphs, cs = small
    theta = W.xavier_theta(3, kbar, d) if kind == "xavier" else W.smoother_theta(kbar=kbar, d=d, omega=0.15,
                                                                                  out_scale=1.7)
    blocks = dss.unpack(theta, kbar, d)
    for g, c in zip(graphs, cs):
        ref = dss.forward(blocks, g, c, 1e-3, d)
        got = bm.forward(blocks, g, c, 1e-3, d, rounding=False)
        assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()


def test_model_error_is_of_the_formats_order(small):
    graphs, cs = small
    blocks = dss.unpack(W.xavier_theta(W.THETA_SEED), 30, 10)
    tol = bm.tolerance(blocks, graphs, cs, 1e-3, 10, factor=1.0)
    assert 2.0 ** -11 < tol < 0.1
