"""Shared problem builders for the tests (generator + library host helpers)."""
import numpy as np

import paper_2402_08296_amd as dg
import workload as W


def host_problem(p, delta=2):
    return dg.host_problem(p.mesh.xy, p.mesh.tri, p.mesh.dirichlet, p.A.rowptr, p.A.col, p.A.val, p.b, p.u0,
                           p.part, p.n_parts, delta)


def small_problem(seed=5, n=1800, parts=4, jitter=0.2):
    p = W.make_problem(seed, n, parts, jitter)
    return p, oracle_problem(p)


def oracle_problem(p, delta=2):
    """Problem arrays with the oracle's own overlapping decomposition and weights
    (oracle.decomp.decompose): what the GPU tests hand to the library, so that no
    oracle input comes from the library (its overlap expansion is pinned to the
    oracle's bit for bit in test_abi_host)."""
    from oracle import decomp as dc
    dec = dc.decompose(p.n, p.mesh.tri, p.mesh.dirichlet, p.part, p.n_parts, delta)
    return dg.HostProblem(p.mesh.xy, p.mesh.tri, p.mesh.dirichlet, p.A.rowptr, p.A.col, p.A.val, p.b, p.u0,
                          dec.sub_ptr, dec.sub_nodes, dec.weights)
