#!/usr/bin/env python
"""Benchmark of the DDM-GNN preconditioned flexible-CG solver on one MI355X.

One step is one complete solve A u = b from u0 to relative residual 1e-6 of
the ~1M-node, 1500-sub-mesh problem (every FCG iteration runs SpMV, dots,
updates, convergence test, restriction, coarse solve, the 30-block DSS forward
on every sub-mesh and the gluing). Inputs are resident in HBM before the timed
region. `value` is solves per second, one solve after another.

The same JSON line carries:
  * roofline: the dominant kernel (the DSS forward), timed with HIP events on
    its stream, against the composite peak of its flop mix, with the HBM
    traffic of the committed counter summary while the kernel is unchanged;
  * batched: the same problem 8 times in one batched solve, and the batch of
    64 problems of 10k-200k nodes, batched and one after another;
  * serve: a bounded prefix of the request stream (Poisson arrivals, 5k-2M
    nodes) through the serving loop, with p50/p99 latency;
  * train / trained_weights: training steps of DSS_theta on local problems of the
    main mesh, and a short training run on generated meshes followed by a solve
    of the main problem with the trained weights;
  * cpu_baseline: the CPU oracle timed on a bounded sample of the main workload
    (and its training step on two local problems).

  python bench.py --pmc-workload    copies of known size and a few applies of the
                                    main workload, for rocprofv3 counter passes
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

FP32_VALU_TF = 157.3    # MI355X FP32 vector peak
FP64_VALU_TF = 78.6
FP16_PACKED_TF = FP32_VALU_TF  # packed FP16 VALU: two FP16 lanes per FP32 lane, the packed FP32 rate
BF16_MFMA_TF = 2500.0   # dense BF16 matrix-core peak
HBM_GBPS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "dss_mfma_kernel_c3_bf16_traffic.md")
LU_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "lu_local_kernel_c3_traffic.md")
PMC_COPY_BYTES = 1 << 30


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


LDS_TBPS = 128 * 256 * 2.4e9 / 1e12  # LDS: 128 B per clock per compute unit, 256 units, 2.4 GHz


def dss_work(kbar: int, d: int, sum_k: int, n_edges: int) -> dict:
    """Algorithmic work of one DSS forward launch in the factorised form (multiply-add =
    2 flops), from the actual node and edge counts.

    Dense 10-wide layers per node and block (matrix cores): neighbour projections
    Q' 4d^2 (both directions, coordinate terms folded in), receiver projections P'
    4d^2+2d, message second layers 4d^2+2d, Psi 8d^2+7d (2110 at d = 10); the
    final decoder 2d^2+4d+1 per node. Per directed edge and block (vector ALU), for
    each of the 2d message units: P'+Q', the |d| term (multiply-add), ReLU and the
    sum, 5 operations (100 at d = 10). LDS: per edge and block the gather of the
    sender's Q' row, 2d FP16 values."""
    per_node = 4 * d * d + (4 * d * d + 2 * d) + (4 * d * d + 2 * d) + (8 * d * d + 7 * d)
    dense = kbar * per_node * sum_k + (2 * d * d + 4 * d + 1) * sum_k
    edge = float(kbar * 2 * d * 5 * n_edges)
    lds = float(kbar * 2 * d * 2 * n_edges)
    return {"flops_mfma": float(dense), "flops_valu": edge, "lds_bytes": lds}


def dss_roofline(work: dict, t_ms: float, hbm_bytes: float, precision: str) -> dict:
    """Fraction of the binding roof: the largest of the floors work/peak over matrix
    cores, vector ALU, LDS and HBM, divided by the measured time. The MFMA kernel
    runs the dense layers on BF16/FP16 matrix cores and the edge work on packed FP16
    vector ALU (157.3 TFLOP/s, the packed FP32 rate); the VALU kernels run both on
    FP32 or FP64 vector ALU."""
    t = t_ms * 1e-3
    if precision == "bf16":
        floors = {"mfma": work["flops_mfma"] / (BF16_MFMA_TF * 1e12),
                  "valu": work["flops_valu"] / (FP16_PACKED_TF * 1e12)}
        valu_peak = FP16_PACKED_TF
    else:
        valu_peak = FP64_VALU_TF if precision == "fp64" else FP32_VALU_TF
        floors = {"valu": (work["flops_mfma"] + work["flops_valu"]) / (valu_peak * 1e12)}
    floors["lds"] = work["lds_bytes"] / (LDS_TBPS * 1e12)
    floors["hbm"] = hbm_bytes / (HBM_GBPS * 1e9)
    bound = max(floors, key=floors.get)
    out = {"binding": bound, "floors_us": {k: v * 1e6 for k, v in floors.items()},
           "frac_binding": floors[bound] / t}
    if precision == "bf16":
        out["achieved_valu_tflops"] = work["flops_valu"] / t / 1e12
        out["valu_peak_tflops"] = valu_peak
        out["mfma_frac"] = work["flops_mfma"] / t / 1e12 / BF16_MFMA_TF
    return out


def apply_bytes(n: int, K: int, sum_k: int, n_edges: int, xy_bytes: int = 8) -> float:
    """Compulsory HBM bytes of one preconditioner apply (each array touched once).

    restrict + DSS: r gather 8, sub_nodes 4, weights 8, coordinates xy_bytes,
    edge_ptr 4 per slot; edge_src 2 per edge; local output 8 per slot;
    coarse: A0^{-1} 8 K^2; gluing: node_ptr 4 + dirichlet 1 + z 8 + previous
    q 8 per node, node_slots 4 + slot_sub 4 + weights 8 + local 8 per slot.
    """
    return (sum_k * (8 + 4 + 8 + xy_bytes + 4 + 8) + 2 * n_edges + 8.0 * K * K
            + n * (4 + 1 + 8 + 8) + sum_k * (4 + 4 + 8 + 8))


def dss_hbm_bytes(sum_k: int, n_edges: int) -> float:
    """Compulsory HBM bytes of one DSS forward launch: per slot the r gather 8,
    sub_nodes 4, weights 8, tile record 16 and local output 8; per edge its 4-byte
    record."""
    return 44.0 * sum_k + 4.0 * n_edges


_DIRECT = {}


def _direct_solve_task():
    import scipy.sparse.linalg as spl
    A, b = _DIRECT["A"], _DIRECT["b"]
    return spl.spsolve(A.tocsc(), b)


class DirectSolve:
    """scipy's sparse direct solve of A u = b in one forked worker process (started
    before the GPU is touched, so it runs beside the GPU legs); result() joins it."""

    def __init__(self, p):
        import multiprocessing as mp
        _DIRECT.update(A=p.A.to_scipy(), b=p.b)
        self.pool = mp.get_context("fork").Pool(1)
        self.job = self.pool.apply_async(_direct_solve_task)
        _DIRECT.clear()

    def result(self):
        try:
            return self.job.get(timeout=1800)
        finally:
            self.pool.close()
            self.pool.join()


def lu_local_bytes(K: int, sum_k: int, sum_k2: int) -> float:
    """Compulsory HBM bytes of one exact local-solve launch (DDM-LU): the inverses
    8 sum k_i^2; per slot r gather 8, sub_nodes 4, weights 8, local output 8;
    per sub-mesh sub_ptr 4, lu_off 8, s and y0 outputs 16."""
    return 8.0 * sum_k2 + sum_k * (8 + 4 + 8 + 8) + K * (4 + 8 + 16)


def bench_lu(dg, prob, u, hp, steps: int) -> dict:
    """DDM-LU (eq. (7): exact local solves, unweighted glue, PCG) on the same problem."""
    import torch
    opts = dg.default_opts(krylov=dg.PCG, local_solver=dg.LOCAL_LU, prolong=dg.PROLONG_UNWEIGHTED,
                           precision="fp64", rtol=1e-6, max_it=5000, check_every=16)
    t = time.perf_counter()
    first = prob.solve(u, opts, check=False)  # assembles and inverts the local matrices on the device
    setup_s = time.perf_counter() - t - first.solve_ms * 1e-3
    log(f"DDM-LU first solve: iterations={first.iterations} factorisation={setup_s:.3f}s")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        st = prob.solve(u, opts, check=False)
    torch.cuda.synchronize()
    elapsed = (time.perf_counter() - t0) / steps
    sp = prob.solve(u, dg.default_opts(krylov=dg.PCG, local_solver=dg.LOCAL_LU, prolong=dg.PROLONG_UNWEIGHTED,
                                       precision="fp64", rtol=1e-6, max_it=5000, profile=1), check=False)
    n_it = max(1, sp.dss_launches)
    k = np.diff(hp.sub_ptr).astype(np.int64)
    nbytes = lu_local_bytes(hp.K, int(k.sum()), int((k * k).sum()))
    local_ms = sp.dss_ms / n_it
    achieved = nbytes / (local_ms * 1e-3) / 1e9
    from paper_2402_08296_amd import profiling
    tr = profiling.read_traffic(LU_TRAFFIC_FILE)
    traffic = None
    if tr and tr.get("source_hash") == profiling.source_hash("lu_local_kernel"):
        traffic = tr["traffic_bytes_per_dispatch"]
    return {"krylov": "PCG", "prolong": "unweighted", "iterations": st.iterations, "converged": bool(st.converged),
            "true_rel_residual": st.true_rel_residual, "time_to_solution_ms": 1e3 * elapsed,
            "solves_per_s": 1.0 / elapsed, "factorisation_s": setup_s,
            "factorisation": "R_i A R_i^T assembled and inverted on the device (blocked Gauss-Jordan, FP64)",
            "device_bytes": prob.device_bytes(),
            "breakdown_ms_per_iteration": {"local": local_ms, "coarse": sp.coarse_ms / n_it,
                                           "prolong": sp.prolong_ms / n_it, "krylov": sp.krylov_ms / n_it},
            "roofline": {"kernel": "lu_local_kernel", "bound": "hbm", "achieved": achieved, "peak": HBM_GBPS,
                         "unit": "GB/s", "frac": achieved / HBM_GBPS, "traffic": traffic, "bytes_per_launch": nbytes,
                         "avg_launch_ms": local_ms}}


def oracle_train_per_sample(p, hp, subs) -> dict:
    """The oracle's loss and gradient (float64 autograd, kbar 30) on a few local problems of
    the same mesh, seeded right-hand sides: CPU seconds per sample."""
    import torch
    import workload as W
    from oracle import decomp as dc
    from oracle import train as tro
    A = p.A.to_scipy()
    samples = []
    for i in subs:
        nodes = hp.sub_nodes[hp.sub_ptr[i]:hp.sub_ptr[i + 1]]
        g = dc.local_graph(nodes, p.mesh.tri, p.mesh.xy, p.mesh.dirichlet)
        c = np.random.default_rng(int(i)).standard_normal(g.k)
        c[g.dirichlet == 1] = 0.0
        samples.append((g, tro.local_matrix(A, nodes), c / np.linalg.norm(c)))
    th = W.xavier_theta(0, 30, 10).astype(np.float64)
    t0 = time.perf_counter()
    tro.loss_and_grad(th, samples, 1e-3, 30, 10, 1.0 / sum(g.k for g, _, _ in samples))
    el = time.perf_counter() - t0
    return {"s_per_sample": el / len(samples), "samples": len(samples),
            "nodes": int(sum(g.k for g, _, _ in samples)), "threads": torch.get_num_threads(),
            "kind": "oracle (float64 autograd on the CPU)"}


def bench_train(dg, ctx, prob, steps: int, batch: int = 100) -> dict:
    """Training throughput of DSS_theta (kbar 30, d 10, alpha 1e-3, Xavier start): `steps`
    Adam steps over batches of `batch` local problems of this mesh, each a forward and
    backward over all blocks (Sec. III.B loss) then an Adam step (Sec. IV.B)."""
    import torch
    import workload as W
    from paper_2402_08296_amd import train as T
    data = T.harvest(prob, [0])
    st = T.init_state(torch.tensor(W.xavier_theta(0, 30, 10), device="cuda"))
    rng = np.random.default_rng(0)
    ptr = prob.hp.sub_ptr
    batches = []
    for _ in range(steps + 1):
        subs = rng.choice(prob.K, size=min(batch, prob.K), replace=False)
        batches.append((subs, [int(ptr[i]) for i in subs]))
    def one(subs, offs):
        loss, gn = prob.train_grad(st.theta, subs, data.c, offs, st.grad)
        st.step += 1
        dg.adam_step(ctx, st.theta, st.grad, st.m, st.v, gn, st.step, lr=1e-2, clip=1e-2)
        return loss
    one(*batches[0])  # warm-up: builds the local matrices and edge transposes
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    losses = [one(*b) for b in batches[1:]]
    torch.cuda.synchronize()
    el = (time.perf_counter() - t0) / steps
    nodes = float(np.mean([sum(int(ptr[i + 1] - ptr[i]) for i in b[0]) for b in batches[1:]]))
    return {"kbar": 30, "d": 10, "batch": batch, "steps": steps, "ms_per_step": 1e3 * el,
            "samples_per_s": batch / el, "nodes_per_batch": nodes, "loss_first": losses[0], "loss_last": losses[-1],
            "data": "local right-hand sides of the initial residual (iterate 0) of this mesh",
            "timing": "host clock around train_grad + adam_step, both synchronous"}


def bench_trained(dg, ctx, hp, opts, epochs: int) -> dict:
    """The paper's pipeline end to end: train DSS_theta from Xavier weights on local problems of
    generated 7k-node meshes (8 meshes, sub-meshes of about 1000 nodes, DDM-LU-PCG harvest), then
    solve the main problem with the trained weights (same options as the main solve)."""
    import torch
    from paper_2402_08296_amd import train as T
    theta, info = T.train_on_generated(ctx, epochs=epochs, log=log)
    model = dg.Model(ctx, theta)
    prob = dg.Problem(ctx, hp, model)
    u = torch.empty(prob.n, dtype=torch.float64, device="cuda")
    prob.solve(u, opts, check=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st = prob.solve(u, opts, check=False)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    info.update({"solve_iterations": st.iterations, "solve_converged": bool(st.converged),
                 "solve_true_rel_residual": st.true_rel_residual, "solve_time_ms": 1e3 * el})
    prob.close()
    model.close()
    return info


def bench_variant(dg, prob, u, opts, popts) -> dict:
    """One warm-up solve (graph capture), one timed solve, one profiled solve of the main problem."""
    import torch
    prob.solve(u, opts, check=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st = prob.solve(u, opts, check=False)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    sp = prob.solve(u, popts, check=False)
    n_it = max(1, sp.dss_launches)
    return {"iterations": st.iterations, "converged": bool(st.converged), "rel_residual": st.rel_residual,
            "true_rel_residual": st.true_rel_residual, "time_to_solution_ms": 1e3 * elapsed,
            "breakdown_ms_per_iteration": {"dss": sp.dss_ms / n_it, "coarse": sp.coarse_ms / n_it,
                                           "prolong": sp.prolong_ms / n_it, "krylov": sp.krylov_ms / n_it}}


def _make(spec):
    """(seed, target_nodes, n_parts, jitter) -> (problem, host arrays); runs in a worker process."""
    import paper_2402_08296_amd as dg
    import workload as W
    seed, nn, parts, jit = spec
    p = W.make_problem(seed, nn, parts, jit)
    hp = dg.host_problem(p.mesh.xy, p.mesh.tri, p.mesh.dirichlet, p.A.rowptr, p.A.col, p.A.val, p.b, p.u0,
                         p.part, p.n_parts, 2)
    return p, hp


def generate(specs, workers: int):
    """Host problems of the given specs, built in worker processes (before the GPU is touched)."""
    if workers <= 1 or len(specs) <= 1:
        return [_make(s) for s in specs]
    import multiprocessing as mp
    pool = mp.get_context("fork").Pool(min(workers, len(specs)))
    try:
        out = pool.map(_make, specs, chunksize=1)
        pool.close()
    except BaseException:
        pool.terminate()
        raise
    finally:
        pool.join()
    return out


_ORACLE = {}


def _oracle_worker(w: int, nproc: int, bar, out):
    """Forked worker of oracle_apply_parallel: builds the local graphs of its sub-meshes
    (untimed), then runs their DSS forward passes between two barriers and returns their
    local terms s_i r~_i."""
    import threadpoolctl

    from oracle import decomp as dc, dss
    o = _ORACLE
    mine = o["order"][w::nproc]
    with threadpoolctl.threadpool_limits(1):
        graphs = [dc.local_graph(o["sub_nodes"][o["sub_ptr"][i]:o["sub_ptr"][i + 1]], o["tri"], o["xy"],
                                 o["dirichlet"]) for i in mine]
        bar.wait(timeout=900)
        res = []
        for i, g in zip(mine, graphs):
            ri = o["r"][o["sub_nodes"][o["sub_ptr"][i]:o["sub_ptr"][i + 1]]]
            s = float(np.linalg.norm(ri))
            res.append((int(i), s * dss.forward(o["blocks"], g, ri / s, 1e-3, 10) if s > 0 else np.zeros(ri.size)))
        bar.wait(timeout=900)
    out.put(res)


def oracle_apply_parallel(p, hp, theta, nproc: int) -> dict:
    """The oracle's preconditioner apply with one process per core: every sub-mesh's DSS
    forward (the sub-meshes dealt round-robin by decreasing size), timed between two
    barriers once every process has built its graphs, then the gluing and the coarse
    solve in this process, and the rest of an FCG iteration (SpMV, dots, updates).
    Forks before the GPU is touched; every process is joined."""
    import multiprocessing as mp

    import threadpoolctl

    from oracle import decomp as dc, dss, schwarz as sw
    A = p.A.to_scipy()
    r = np.ascontiguousarray(p.b - A @ p.u0)
    k = np.diff(hp.sub_ptr)
    _ORACLE.update(sub_ptr=hp.sub_ptr, sub_nodes=hp.sub_nodes, r=r, blocks=dss.unpack(theta, 30, 10),
                   tri=p.mesh.tri, xy=p.mesh.xy, dirichlet=p.mesh.dirichlet, order=np.argsort(-k, kind="stable"))
    nproc = max(1, min(nproc, hp.K))
    ctx = mp.get_context("fork")
    bar = ctx.Barrier(nproc + 1)
    out = ctx.Queue()
    procs = [ctx.Process(target=_oracle_worker, args=(w, nproc, bar, out)) for w in range(nproc)]
    for pr in procs:
        pr.start()
    try:
        bar.wait(timeout=900)
        t0 = time.perf_counter()
        bar.wait(timeout=900)
        t_local = time.perf_counter() - t0
        loc = {}
        for _ in range(nproc):
            loc.update(out.get(timeout=900))
    finally:
        for pr in procs:
            pr.join(timeout=60)
        _ORACLE.clear()
    dec = dc.Decomposition(p.n, hp.sub_ptr, hp.sub_nodes, hp.weights)
    coarse = sw.Coarse(A, dec)
    with threadpoolctl.threadpool_limits(1):
        t0 = time.perf_counter()
        z = np.zeros(p.n)
        for i in range(hp.K):
            sl = slice(hp.sub_ptr[i], hp.sub_ptr[i + 1])
            z[hp.sub_nodes[sl]] += hp.weights[sl] * loc[i]
        z += coarse(r)
        z[p.mesh.dirichlet == 1] = 0.0
        t_glue = time.perf_counter() - t0
        t0 = time.perf_counter()
        q = A @ z
        _ = (z @ q, z @ r, np.linalg.norm(r))
        u = p.u0 + 0.5 * z
        r2 = r - 0.5 * q
        t_krylov = time.perf_counter() - t0
    del u, r2
    return {"local_s": t_local, "glue_coarse_s": t_glue, "krylov_s": t_krylov,
            "apply_s": t_local + t_glue, "iteration_s": t_local + t_glue + t_krylov, "processes": nproc}


def cpu_baseline(p, hp, theta, nproc: int) -> dict:
    """The CPU oracle on the main workload: one whole iteration (the apply over all
    sub-meshes on nproc processes, one thread each, then the SpMV and vector work),
    timed before the GPU is touched; scaled to solves/s by the GPU solve's iteration
    count once that is known."""
    t = oracle_apply_parallel(p, hp, theta, nproc)
    t["sample"] = (f"one oracle FCG iteration of the whole workload: DSS forward of all {hp.K} sub-meshes "
                   f"({hp.sub_nodes.size} slots) on {t['processes']} processes (one BLAS thread each), then "
                   f"gluing, coarse solve, SpMV, dots and updates in one process")
    return t


def oracle_small_cpu(theta, workers: int) -> dict:
    """c1 and c2: the oracle's preconditioner apply timed with one thread and with one
    process per core over the sub-meshes, before the GPU is touched.
    Returns {name: (p, hp, timings)}."""
    import threadpoolctl
    import workload as W
    from oracle import decomp as dc, schwarz as sw
    out = {}
    for name in ("c1", "c2"):
        cfg = W.CONFIGS[name]
        p, hp = _make((cfg["seeds"][0], cfg["target_nodes"], cfg["n_parts"], cfg["jitter"]))
        A = p.A.to_scipy()
        r = np.ascontiguousarray(p.b - A @ p.u0)
        dec = dc.Decomposition(p.n, hp.sub_ptr, hp.sub_nodes, hp.weights)
        M = sw.DDMGNN(A, p.mesh.xy, p.mesh.tri, p.mesh.dirichlet, dec, theta)
        with threadpoolctl.threadpool_limits(1):
            t0 = time.perf_counter()
            M(r)
            one = time.perf_counter() - t0
        par = oracle_apply_parallel(p, hp, theta, workers)
        log(f"{name}: oracle apply {one:.2f} s (1 thread), {par['apply_s']:.2f} s ({par['processes']} processes)")
        out[name] = (p, hp, {"oracle_apply_s_1thread": one, "oracle_apply_s_allcore": par["apply_s"],
                             "oracle_processes": par["processes"]})
    return out


def gpu_small(dg, ctx, model, cpu: dict) -> dict:
    """GPU solve and apply of c1 (FP64) and c2 (FP32) beside the oracle timings of oracle_small_cpu."""
    import torch
    out = {}
    for name, prec in (("c1", "fp64"), ("c2", "fp32")):
        p, hp, t = cpu[name]
        prob = dg.Problem(ctx, hp, model)
        u = torch.empty(p.n, dtype=torch.float64, device="cuda")
        opts = dg.default_opts(precision=prec, rtol=1e-6, max_it=5000)
        prob.solve(u, opts, check=False)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = prob.solve(u, opts, check=False)
        torch.cuda.synchronize()
        gpu_solve = time.perf_counter() - t0
        rt = torch.from_numpy(np.ascontiguousarray(p.b - p.A.to_scipy() @ p.u0)).cuda()
        gl, gc, gg = prob.time_apply_stages(rt, torch.empty_like(rt), opts, reps=10)
        out[name] = {"nodes": p.n, "subdomains": hp.K, "precision": prec, "gpu_iterations": st.iterations,
                     "gpu_solve_ms": 1e3 * gpu_solve, "gpu_apply_ms": gl + gc + gg, **t,
                     "oracle_solve_s_1thread": t["oracle_apply_s_1thread"] * st.iterations,
                     "oracle_solve_s_allcore": t["oracle_apply_s_allcore"] * st.iterations,
                     "note": "oracle per-solve = its apply time x the GPU's iteration count (the oracle's own "
                             "FCG takes the same number up to the precision gap)"}
        log(f"{name}: GPU {1e3 * gpu_solve:.1f} ms/solve, {st.iterations} iterations")
    return out


def bench_batched(dg, ctx, model, items, opts, reps: int, sequential: bool, schedule=None) -> dict:
    """One batched solve of all items (after a warm-up), and optionally the same one after another.
    schedule: a tuning (dict) applied to every problem."""
    import torch
    probs = [dg.Problem(ctx, hp, model) for _, hp in items]
    for pr in probs:
        if schedule:
            pr.set_tuning(**schedule)
    outs = [torch.empty(pr.n, dtype=torch.float64, device="cuda") for pr in probs]
    dg.solve_batch(ctx, probs, outs, opts, check=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        sts = dg.solve_batch(ctx, probs, outs, opts, check=False)
    torch.cuda.synchronize()
    t_batch = (time.perf_counter() - t0) / reps
    res = {"problems": len(probs), "nodes": int(sum(pr.n for pr in probs)),
           "subdomains": int(sum(pr.K for pr in probs)),
           "batched_s": t_batch, "batched_solves_per_s": len(probs) / t_batch,
           "converged": int(sum(1 for s in sts if s.converged)),
           "iterations_max": int(max(s.iterations for s in sts)),
           "iterations_mean": float(np.mean([s.iterations for s in sts]))}
    # every member's solution checked on the host (scipy, FP64)
    worst = 0.0
    for (q, _), ub in zip(items, outs):
        A = q.A.to_scipy()
        ug = ub.cpu().numpy()
        worst = max(worst, float(np.linalg.norm(q.b - A @ ug) / np.linalg.norm(q.b - A @ q.u0)))
    res["max_host_rel_residual"] = worst
    if sequential:
        for pr, u in zip(probs, outs):  # warm (graph capture per problem)
            pr.solve(u, opts, check=False)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for pr, u in zip(probs, outs):
            pr.solve(u, opts, check=False)
        torch.cuda.synchronize()
        t_seq = time.perf_counter() - t0
        res.update({"sequential_s": t_seq, "sequential_solves_per_s": len(probs) / t_seq,
                    "batch_speedup": t_seq / t_batch})
    for pr in probs:
        pr.close()
    return res


def bench_serve(dg, model, stream, opts, budget: int, check_solutions: bool = True) -> dict:
    """Replays a stream of requests (arrival offsets in s) through the serving loop.

    Latency is counted from each request's scheduled arrival: the server's own figure
    (submission to completion) plus the time by which the submission call returned
    after the scheduled arrival. Every returned solution is checked on the host: its
    relative residual |b - A u| / |b - A u0| recomputed with scipy in FP64."""
    import scipy.sparse as sp
    import torch
    sctx = dg.Context(torch.cuda.Stream())
    srv = dg.Server(sctx, model, hbm_budget=budget, max_active=64, setup_threads=8)
    t0 = time.perf_counter()
    tickets, lags = [], []
    for t_arr, hp in stream:
        wait = t0 + t_arr - time.perf_counter()
        if wait > 0:
            time.sleep(wait)
        tickets.append(srv.submit(hp, opts))
        lags.append(time.perf_counter() - (t0 + t_arr))
    srv.drain()
    makespan = time.perf_counter() - t0
    lat, its, ok, status, stages, worst = [], [], 0, {}, {"setup": [], "queue": [], "upload": [], "solve": []}, 0.0
    for t, lag, (_, hp) in zip(tickets, lags, stream):
        rc, st, u = srv.poll(t, with_solution=check_solutions)
        lat.append(st.latency_ms + 1e3 * lag)
        its.append(st.iterations)
        ok += int(rc == 0)
        name = dg.STATUS.get(rc, str(rc))
        status[name] = status.get(name, 0) + 1
        stages["setup"].append(st.setup_ms)
        stages["queue"].append(st.queue_ms)
        stages["upload"].append(st.upload_ms)
        stages["solve"].append(st.solve_ms)
        if check_solutions and rc == 0:
            A = sp.csr_matrix((hp.val, hp.col, hp.rowptr), shape=(hp.n, hp.n))
            res = np.linalg.norm(hp.b - A @ u) / np.linalg.norm(hp.b - A @ hp.u0)
            worst = max(worst, float(res))
    srv.close()
    sctx.close()
    nodes = sum(hp.n for _, hp in stream)
    offered = len(stream) / max(stream[-1][0], 1e-9)
    served = len(stream) / makespan
    out = {"requests": len(stream), "completed_ok": ok, "status": status, "makespan_s": makespan,
           "solves_per_s": served, "offered_rate_per_s": offered, "nodes_total": int(nodes),
           "nodes_per_s": nodes / makespan,
           "p50_latency_ms": float(np.percentile(lat, 50)), "p99_latency_ms": float(np.percentile(lat, 99)),
           "max_latency_ms": float(np.max(lat)), "iterations_mean": float(np.mean(its)),
           "submit_lag_ms_max": 1e3 * float(np.max(lags)),
           "stage_p50_ms": {k: float(np.percentile(v, 50)) for k, v in stages.items()},
           "stage_p99_ms": {k: float(np.percentile(v, 99)) for k, v in stages.items()},
           "latency": "scheduled arrival to completion",
           "regime": "overloaded (served rate below the offered rate: the queue grows over the replay, so the "
                     "percentiles depend on the stream length)" if served < 0.95 * offered else "stable"}
    if check_solutions:
        out["max_host_rel_residual"] = worst
    return out


def pmc_workload(args):
    """Copies of known size (counter calibration) and a few DSS applies of the main workload."""
    import torch

    import paper_2402_08296_amd as dg
    import workload as W
    p, hp = _make((W.CONFIGS[args.config]["seeds"][0], W.CONFIGS[args.config]["target_nodes"],
                   W.CONFIGS[args.config]["n_parts"], W.CONFIGS[args.config]["jitter"]))
    torch.cuda.set_device(0)
    ctx = dg.Context()
    model = dg.Model(ctx, W.smoother_theta(omega=0.15, out_scale=1.7))
    prob = dg.Problem(ctx, hp, model)
    if args.tune:  # the schedule of the measured run (cached by it on this machine)
        from paper_2402_08296_amd import tune
        tinfo = tune.tuned(prob, hp, dg.default_opts(precision=args.precision, rtol=1e-6, max_it=5000,
                                                     check_every=16),
                           dg.lib().ddmgnn_version().decode().split()[-1], args.tune_cache)
        log(f"schedule {tinfo['tuning']}")
    x = torch.ones(PMC_COPY_BYTES // 8, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    r = torch.from_numpy(np.ascontiguousarray(p.b - p.A.to_scipy() @ p.u0)).cuda()
    z = torch.empty_like(r)
    opts = dg.default_opts(precision=args.precision)
    for _ in range(6):
        prob.apply(r, z, opts)
    torch.cuda.synchronize()
    u = torch.empty_like(r)
    prob.solve(u, dg.default_opts(precision=args.precision, max_it=8, graph=0), check=False)
    torch.cuda.synchronize()
    lu = dg.default_opts(local_solver=dg.LOCAL_LU, prolong=dg.PROLONG_UNWEIGHTED)
    for _ in range(4):
        prob.apply(r, z, lu)
    torch.cuda.synchronize()
    log(f"pmc workload done: 3 copies of {PMC_COPY_BYTES} B, 6 DSS applies ({args.precision}), 8 FCG iterations, "
        "4 DDM-LU applies")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="c3", choices=["c1", "c2", "c3"])
    ap.add_argument("--precision", default="bf16", choices=["bf16", "fp32", "fp64"])
    ap.add_argument("--m-max", type=int, default=4, help="directions kept by FCG (truncated flexible CG)")
    ap.add_argument("--theta", default="smoother", choices=["smoother", "xavier"])
    ap.add_argument("--cpu-baseline", type=int, default=1,
                    help="time one oracle iteration of the main workload on --workers processes (0: skip)")
    ap.add_argument("--direct", type=int, default=1,
                    help="scipy direct solve of the main problem in a worker process, for the solution's L2 error (0: skip)")
    ap.add_argument("--batch8", type=int, default=8, help="copies of the main problem in one batch (0: skip)")
    ap.add_argument("--batch", type=int, default=64, help="problems of the 10k-200k batch (0: skip)")
    ap.add_argument("--serve", type=int, default=500, help="requests of the c5 stream (500: all; 0: skip)")
    ap.add_argument("--serve-slow-rate", type=float, default=6.0, help="arrival rate of the sustained replay (1/s)")
    ap.add_argument("--serve-slow", type=int, default=150, help="requests of the sustained replay (0: skip)")
    ap.add_argument("--workers", type=int, default=min(16, os.cpu_count() or 1))
    ap.add_argument("--lu-steps", type=int, default=1, help="timed DDM-LU solves of the main problem (0: skip)")
    ap.add_argument("--train-steps", type=int, default=5, help="timed training steps of DSS_theta (0: skip)")
    ap.add_argument("--trained-epochs", type=int, default=40,
                    help="train DSS_theta for this many epochs, then solve the main problem with it (0: skip)")
    ap.add_argument("--variants", type=int, default=1, help="FGMRES and rtol 1e-9 legs on the main problem (0: skip)")
    ap.add_argument("--oracle-small", type=int, default=1, help="c1/c2 GPU and oracle timings (0: skip)")
    ap.add_argument("--tune", type=int, default=1, help="autotune the main problem's schedule (0: default schedule)")
    ap.add_argument("--tune-cache", default=None, help="autotuner cache file (default: ~/.cache/ddmgnn_tune.json)")
    ap.add_argument("--pmc-workload", action="store_true")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: this build runs on one GPU only (no multi-GPU path); use --gpus 1", file=sys.stderr)
        sys.exit(2)
    if args.pmc_workload:
        pmc_workload(args)
        return

    import workload as W

    # ---- all host inputs first, in worker processes, before the GPU is touched
    t = time.perf_counter()
    cfg = W.CONFIGS[args.config]
    p, hp = _make((cfg["seeds"][0], cfg["target_nodes"], cfg["n_parts"], cfg["jitter"]))
    log(f"problem {args.config}: N={p.n} nnz={p.A.val.size} K={hp.K} sum_k={hp.sub_nodes.size} "
        f"({time.perf_counter() - t:.1f}s)")
    batch_items = []
    if args.batch > 0:
        t = time.perf_counter()
        batch_items = generate(W.batch_specs("c4", args.batch), args.workers)
        log(f"batch c4: {len(batch_items)} problems, {sum(q.n for q, _ in batch_items)} nodes "
            f"({time.perf_counter() - t:.1f}s)")
    stream, stream_slow = [], []
    if args.serve > 0:
        t = time.perf_counter()
        specs = W.stream_specs("c5", args.serve)
        made = generate([s[1:] for s in specs], args.workers)
        stream = [(s[0], hp_) for s, (_, hp_) in zip(specs, made)]
        # the first requests again at a rate one GPU sustains
        if args.serve_slow > 0:
            slow = W.stream_specs("c5", min(args.serve_slow, args.serve), rate=args.serve_slow_rate)
            stream_slow = [(s[0], hp_) for s, (_, hp_) in zip(slow, made)]
        log(f"stream c5: {len(stream)} requests, {sum(h.n for _, h in stream)} nodes over "
            f"{specs[-1][0]:.2f}s of arrivals ({time.perf_counter() - t:.1f}s)")

    small_cpu = {}
    if args.oracle_small > 0:
        # the oracle's c1/c2 applies, timed before the GPU is touched (worker processes)
        log("c1 and c2: CPU oracle")
        theta_s = W.smoother_theta(omega=0.15, out_scale=1.7) if args.theta == "smoother" else \
            W.xavier_theta(W.THETA_SEED)
        small_cpu = oracle_small_cpu(theta_s, args.workers)
    theta = W.smoother_theta(omega=0.15, out_scale=1.7) if args.theta == "smoother" else \
        W.xavier_theta(W.THETA_SEED)
    cpu_it = None
    if args.cpu_baseline > 0:
        log(f"{args.config}: one oracle iteration on {args.workers} processes")
        cpu_it = cpu_baseline(p, hp, theta, args.workers)
        log(f"{args.config}: oracle iteration {cpu_it['iteration_s']:.2f} s")
    direct = DirectSolve(p) if args.direct > 0 else None  # scipy, in a forked worker, beside the GPU legs

    import torch

    import paper_2402_08296_amd as dg
    from paper_2402_08296_amd import profiling

    torch.cuda.set_device(0)
    ctx = dg.Context()
    model = dg.Model(ctx, theta)
    t = time.perf_counter()
    prob = dg.Problem(ctx, hp, model)
    log(f"library setup {time.perf_counter() - t:.1f}s; edges={prob.n_edges}")
    u = torch.empty(p.n, dtype=torch.float64, device="cuda")
    max_it = 5000 if args.theta == "smoother" else 200
    opts = dg.default_opts(precision=args.precision, rtol=1e-6, max_it=max_it, check_every=16, m_max=args.m_max)
    tuning = None
    if args.tune:
        from paper_2402_08296_amd import tune
        t = time.perf_counter()
        tuning = tune.tuned(prob, hp, opts, dg.lib().ddmgnn_version().decode().split()[-1], args.tune_cache)
        tuning["seconds"] = time.perf_counter() - t
        log(f"schedule {tuning['tuning']} ({'cached' if tuning['cached'] else 'autotuned'}, "
            f"{tuning['seconds']:.2f}s)")
    popts = dg.default_opts(precision=args.precision, rtol=1e-6, max_it=max_it, profile=1, check_every=16,
                            m_max=args.m_max)
    for w in range(args.warmup):
        st = prob.solve(u, opts, check=False)
        log(f"warmup {w}: iterations={st.iterations} status={st.status} true_rel={st.true_rel_residual:.2e}")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    t_prev = t0
    stats, step_s = [], []
    for k in range(args.steps):
        st = prob.solve(u, opts, check=False)
        stats.append((st.iterations, st.converged, st.true_rel_residual, st.solve_ms))
        step_s.append(time.perf_counter() - t_prev)
        t_prev = time.perf_counter()
        log(f"step {k}: iterations={st.iterations} converged={st.converged} true_rel={st.true_rel_residual:.2e} "
            f"solve_ms={st.solve_ms:.1f}")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    u_host = u.cpu().numpy()
    A_host = p.A.to_scipy()
    host_res = float(np.linalg.norm(p.b - A_host @ u_host) / np.linalg.norm(p.b - A_host @ p.u0))
    log(f"solution: scipy relative residual {host_res:.3e}")
    # One more solve with HIP events around every stage (outside the timed steps).
    sp = prob.solve(u, popts, check=False)
    # The stages of one apply as the solve's graphs run them (two forked DSS launches
    # under the split schedule), each captured 20 times over in one graph timed
    # between events.
    r0 = torch.from_numpy(np.ascontiguousarray(p.b - p.A.to_scipy() @ p.u0)).cuda()
    zt = torch.empty_like(r0)
    g_local, g_coarse, g_glue = prob.time_apply_stages(r0, zt, opts, reps=20)
    log(f"apply stages (graph replay): local {g_local * 1e3:.1f} us, coarse {g_coarse * 1e3:.1f} us, "
        f"glue {g_glue * 1e3:.1f} us")
    dss_kernel = {0: "dss_kernel<double>", 1: "dss_kernel<float>", 2: "dss_mfma_kernel<1024>"}[sp.dss_kernel]
    if sp.dss_kernel == 2 and prob.tuning().small_lds > 0:
        dss_kernel += "+dss_mfma_kernel<512>"  # sub-meshes split over the two workgroup sizes
    n_it = max(1, sp.dss_launches)
    dss_avg_ms = g_local
    work = dss_work(30, 10, prob.sum_k, prob.n_edges)
    run_prec = args.precision if sp.dss_kernel == 2 or args.precision != "bf16" else "fp32"
    rl = dss_roofline(work, dss_avg_ms, dss_hbm_bytes(prob.sum_k, prob.n_edges), run_prec)
    t_s = dss_avg_ms * 1e-3
    if rl["binding"] == "mfma":
        bound, achieved, peak, unit = "mfma", work["flops_mfma"] / t_s / 1e12, BF16_MFMA_TF, "TFLOP/s"
    elif rl["binding"] == "valu":
        f = work["flops_valu"] if run_prec == "bf16" else work["flops_valu"] + work["flops_mfma"]
        peak = FP16_PACKED_TF if run_prec == "bf16" else (FP64_VALU_TF if run_prec == "fp64" else FP32_VALU_TF)
        bound, achieved, unit = "alu", f / t_s / 1e12, "TFLOP/s"
    elif rl["binding"] == "lds":
        bound, achieved, peak, unit = "lds", work["lds_bytes"] / t_s / 1e9, LDS_TBPS * 1e3, "GB/s"
    else:
        bound, achieved, peak, unit = "hbm", dss_hbm_bytes(prob.sum_k, prob.n_edges) / t_s / 1e9, HBM_GBPS, "GB/s"
    apply_ms = g_local + g_coarse + g_glue
    abytes = apply_bytes(prob.n, prob.K, prob.sum_k, prob.n_edges, 8 if args.precision == "fp64" else 4)
    traffic = None
    tr = profiling.read_traffic(TRAFFIC_FILE)
    if tr and tr.get("kernel") == dss_kernel and tr.get("source_hash") == profiling.source_hash("dss_mfma_kernel"):
        traffic = tr["traffic_bytes_per_dispatch"]
    iters = stats[-1][0]
    out = {
        "metric": "time-to-1e-6 residual & solves/s at 1M nodes; precond-apply HBM GB/s; p99 latency",
        "value": args.steps / elapsed,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"bf16": "bf16+f16+f32+f64", "fp32": "f32+f64", "fp64": "f64"}[args.precision],
        "data": "synthetic",
        "config": {"workload": f"{args.config}: P1-FEM Poisson on a Delaunay mesh of a star polygon, "
                               f"N={p.n}, K={hp.K} sub-meshes (overlap 2), sum k_i={hp.sub_nodes.size}, "
                               f"DSS kbar=30 d=10 ({args.theta} weights), FCG({args.m_max}) to rel. residual 1e-6",
                   "nodes": p.n, "subdomains": hp.K, "dss_precision": args.precision, "weights": args.theta,
                   "schedule": "autotuned" if args.tune else "default",
                   "target_nodes": cfg["target_nodes"]},
        "iterations": iters,
        "converged": bool(stats[-1][1]),
        "true_rel_residual": stats[-1][2],
        "time_to_solution_ms": 1e3 * elapsed / args.steps,
        "time_to_solution_median_ms": 1e3 * float(np.median(step_s)),
        "apply_ms": apply_ms,
        "apply_hbm_GBps": abytes / (apply_ms * 1e-3) / 1e9,
        "breakdown_ms_per_iteration": {"dss": sp.dss_ms / n_it, "coarse": sp.coarse_ms / n_it,
                                       "prolong": sp.prolong_ms / n_it, "krylov": sp.krylov_ms / n_it,
                                       "timing": "eager solve with events between stages"},
        "apply_stages_graph_ms": {"local": g_local, "coarse": g_coarse, "glue": g_glue,
                                  "timing": "each stage captured 20 times over in one HIP graph, mean per stage"},
        "roofline": {"kernel": dss_kernel, "bound": bound, "achieved": achieved, "peak": peak, "unit": unit,
                     "frac": achieved / peak, "traffic": traffic, **rl, **work,
                     "avg_launch_ms": dss_avg_ms,
                     "avg_launch_timing": "DSS stage of one apply (both forked launches) in a replayed HIP graph",
                     "algorithmic_hbm_bytes_per_launch": dss_hbm_bytes(prob.sum_k, prob.n_edges),
                     "algorithmic_bytes_per_apply": abytes},
        "solution_check": {"host_rel_residual": host_res,
                           "method": "u copied to the host after the timed solves; |b - A u| / |b - A u0| by scipy "
                                     "in FP64"},
        "p99_latency_ms": None,
        "tuning": tuning,
    }
    if args.variants > 0:
        other = 1 if args.m_max != 1 else 4
        log(f"FGMRES(30), FCG({other}) and rtol 1e-9 on the same problem")
        mk = lambda **kw: (dg.default_opts(precision=args.precision, max_it=max_it, check_every=16, **kw),
                           dg.default_opts(precision=args.precision, max_it=max_it, check_every=16, profile=1, **kw))
        out["fgmres30_c3"] = bench_variant(dg, prob, u, *mk(krylov=dg.FGMRES, restart=30, rtol=1e-6))
        out[f"fcg{other}_c3"] = bench_variant(dg, prob, u, *mk(m_max=other, rtol=1e-6))
        out["fcg_rtol1e-9_c3"] = bench_variant(dg, prob, u, *mk(m_max=args.m_max, rtol=1e-9))
        out["fgmres30_rtol1e-9_c3"] = bench_variant(dg, prob, u, *mk(krylov=dg.FGMRES, restart=30, rtol=1e-9))
        log("plain FP64 form: FP64 DSS, eager launches (no graph), convergence read every iteration")
        plain = dg.default_opts(precision="fp64", rtol=1e-6, max_it=max_it, check_every=1, graph=0)
        out["fp64_plain_c3"] = bench_variant(dg, prob, u, plain,
                                             dg.default_opts(precision="fp64", rtol=1e-6, max_it=max_it,
                                                             check_every=1, graph=0, profile=1))
        out["fp64_plain_c3"]["krylov"] = "FCG(1)"
        out["fp64_plain_c3"]["main_speedup"] = out["fp64_plain_c3"]["time_to_solution_ms"] / out["time_to_solution_ms"]
    if args.train_steps > 0:
        log("training steps of DSS_theta on the same mesh")
        out["train"] = bench_train(dg, ctx, prob, args.train_steps)
    if args.trained_epochs > 0:
        log(f"trained DSS_theta ({args.trained_epochs} epochs on generated meshes) on the main problem")
        out["trained_weights"] = bench_trained(dg, ctx, hp, opts, args.trained_epochs)
    if args.lu_steps > 0:
        log("DDM-LU on the same problem")
        out["ddm_lu"] = bench_lu(dg, prob, u, hp, args.lu_steps)
        out["ddm_lu"]["gnn_vs_lu_time"] = out["ddm_lu"]["time_to_solution_ms"] / out["time_to_solution_ms"]
        del prob  # frees the inverses before the batched legs
        torch.cuda.synchronize()
    if args.batch8 > 1:
        log(f"{args.config} x{args.batch8} in one batch")
        out["batched_same_x8"] = bench_batched(dg, ctx, model, [(p, hp)] * args.batch8, opts, 1, False,
                                               tuning["tuning"] if tuning else None)
        out["batched_same_x8"]["schedule"] = "autotuned (main problem's)" if tuning else "default"
        out["batched_same_x8"]["vs_sequential_value"] = out["batched_same_x8"]["batched_solves_per_s"] / out["value"]
    if batch_items:
        log("batch c4")
        out["batch_c4"] = bench_batched(dg, ctx, model, batch_items, opts, 2, True)
    if stream:
        log("stream c5")
        sopts = dg.default_opts(precision=args.precision, rtol=1e-6, max_it=max_it, check_every=8, graph=0,
                                m_max=args.m_max)
        out["serve_c5"] = bench_serve(dg, model, stream, sopts, 64 << 30)
        out["serve_c5"]["rate_per_s"] = W.STREAM_CONFIGS["c5"]["rate"]
        log(f"c5: {out['serve_c5']['solves_per_s']:.2f} solves/s served of {out['serve_c5']['offered_rate_per_s']:.2f} "
            f"offered; p50 {out['serve_c5']['p50_latency_ms']:.0f} ms p99 {out['serve_c5']['p99_latency_ms']:.0f} ms")
        if stream_slow:
            out["serve_c5_sustained"] = bench_serve(dg, model, stream_slow, sopts, 64 << 30)
            out["serve_c5_sustained"]["rate_per_s"] = args.serve_slow_rate
        if len(stream) == W.STREAM_CONFIGS["c5"]["count"]:  # p99 of the configured stream only
            out["p99_latency_ms"] = out["serve_c5"]["p99_latency_ms"]
    if cpu_it is not None:
        per_solve = iters * cpu_it["iteration_s"]
        out["cpu_baseline"] = {"value": 1.0 / per_solve, "unit": "solves/s", "cores": cpu_it["processes"],
                               "kind": "oracle",
                               "sample": cpu_it["sample"] + f"; {cpu_it['iteration_s']:.2f} s per iteration x the "
                                         f"GPU solve's {iters} iterations = {per_solve:.0f} s per solve",
                               "iteration_s": cpu_it["iteration_s"], "local_s": cpu_it["local_s"],
                               "glue_coarse_s": cpu_it["glue_coarse_s"], "krylov_s": cpu_it["krylov_s"],
                               "threads_per_process": 1}
        if "train" in out:  # the oracle's training step beside the GPU's
            orc = oracle_train_per_sample(p, hp, [0, 1])
            out["cpu_baseline"]["train_step"] = orc
            out["train"]["oracle_s_per_sample"] = orc["s_per_sample"]
            out["train"]["gpu_speedup_per_sample"] = orc["s_per_sample"] * out["train"]["samples_per_s"]
    if small_cpu:
        log("c1 and c2 on the GPU")
        out["oracle_c1_c2"] = gpu_small(dg, ctx, model, small_cpu)
    if direct is not None:
        log("waiting for the direct solve")
        ud = direct.result()
        out["solution_check"]["l2_vs_direct"] = float(np.linalg.norm(u_host - ud) / np.linalg.norm(ud))
        out["solution_check"]["direct"] = "scipy.sparse.linalg.spsolve (SuperLU) in FP64 in a worker process"
        log(f"solution: relative L2 distance to the direct solve {out['solution_check']['l2_vs_direct']:.3e}")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
