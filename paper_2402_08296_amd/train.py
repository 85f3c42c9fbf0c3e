"""Training driver for DSS_theta (Sec. IV.A data, Sec. IV.B set-up).

The data are local problems of the two-level Schwarz preconditioner met during a
PCG solve with exact local solves (DDM-LU): at each harvested iterate u_t, every
sub-mesh i gives the sample (i, c_i = R_i r_t / |R_i r_t|). Training runs the
library's forward/backward kernel over batches of samples and the library's Adam
step with gradient clipping, and lowers the learning rate by a factor when the
epoch loss stops improving (a plateau schedule). Every arithmetic step runs in
the library's kernels; this module only orders the calls.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import (FP64, LOCAL_LU, PCG, PROLONG_UNWEIGHTED, Context, Problem, adam_step, default_opts)


@dataclass
class Harvest:
    """Right-hand sides of all K sub-meshes at T iterates: c[t * sum_k + slot]."""
    c: object          # device float32 tensor, T * sum_k
    iterates: list     # the PCG iteration of each block of sum_k values
    sum_k: int
    K: int

    def samples(self):
        """(iterate index, sub-mesh) of every sample."""
        return [(t, i) for t in range(len(self.iterates)) for i in range(self.K)]


def harvest(prob: Problem, iterates) -> Harvest:
    """Local right-hand sides at the given DDM-LU-PCG iterations (0 = the initial guess).
    Iterate t comes from a solve capped at t iterations (the iteration is deterministic)."""
    import torch
    dev = prob.ctx.stream.device
    sum_k = prob.sum_k
    c = torch.empty(len(iterates) * sum_k, dtype=torch.float32, device=dev)
    u = torch.empty(prob.n, dtype=torch.float64, device=dev)
    for t, it in enumerate(iterates):
        if it == 0:
            u.copy_(torch.as_tensor(prob.hp.u0, device=dev))
        else:
            o = default_opts(krylov=PCG, local_solver=LOCAL_LU, prolong=PROLONG_UNWEIGHTED, precision=FP64,
                             rtol=1e-300, max_it=it)
            prob.solve(u, o, check=False)
        prob.train_rhs(u, c[t * sum_k:(t + 1) * sum_k])
    return Harvest(c, list(iterates), sum_k, prob.K)


@dataclass
class TrainState:
    theta: object
    m: object
    v: object
    grad: object
    step: int = 0
    lr: float = 1e-2
    best: float = float("inf")
    stale: int = 0
    history: list = field(default_factory=list)


def init_state(theta0, lr: float = 1e-2) -> TrainState:
    import torch
    th = theta0.detach().clone().float().contiguous()
    return TrainState(th, torch.zeros_like(th), torch.zeros_like(th), torch.empty_like(th), lr=lr)


def train_epoch(ctx: Context, pairs, st: TrainState, batch: int = 100, kbar: int = 30, alpha: float = 1e-3,
                clip: float = 1e-2, seed: int = 0, patience: int = 10, factor: float = 0.1) -> float:
    """One pass over the samples of every (problem, harvest) pair in a seeded order (a batch
    holds samples of one problem); returns the mean batch loss."""
    batches = []
    rng = np.random.default_rng(seed)
    for q, (prob, data) in enumerate(pairs):
        samples = data.samples()
        order = rng.permutation(len(samples))
        for b0 in range(0, len(order), batch):
            batches.append((q, [samples[i] for i in order[b0:b0 + batch]]))
    losses = []
    for bi in rng.permutation(len(batches)):
        q, sel = batches[bi]
        prob, data = pairs[q]
        ptr = prob.hp.sub_ptr
        subs = [i for _, i in sel]
        offs = [t * data.sum_k + int(ptr[i]) for t, i in sel]
        loss, gn = prob.train_grad(st.theta, subs, data.c, offs, st.grad, kbar=kbar, alpha=alpha)
        st.step += 1
        adam_step(ctx, st.theta, st.grad, st.m, st.v, gn, st.step, lr=st.lr, clip=clip)
        losses.append(loss)
    mean = float(np.mean(losses))
    plateau(st, mean, patience, factor)
    return mean


def plateau(st: TrainState, loss: float, patience: int = 10, factor: float = 0.1) -> None:
    """Record an epoch loss; after more than `patience` epochs without a new best, scale the
    learning rate by `factor` and start counting again."""
    st.history.append(loss)
    if loss < st.best:
        st.best, st.stale = loss, 0
    else:
        st.stale += 1
        if st.stale > patience:
            st.lr *= factor
            st.stale = 0


def train_on_generated(ctx: Context, problems: int = 8, nodes: int = 7000, parts: int = 7, epochs: int = 100,
                       batch: int = 100, lr: float = 1e-2, clip: float = 1e-2, kbar: int = 30,
                       alpha: float = 1e-3, seed: int = 0, log=None):
    """Harvest the local problems of DDM-LU-PCG solves on `problems` generated meshes (seeds
    100, 101, ...) and train from Xavier weights. Returns (theta numpy, info dict)."""
    import time
    import torch
    import workload as W
    from . import Model
    th0 = W.xavier_theta(seed, kbar, 10)
    model = Model(ctx, th0, kbar=kbar, alpha=alpha)
    pairs, t0 = [], time.perf_counter()
    for s in range(100, 100 + problems):
        p, hp = generated(s, nodes, parts)
        prob = Problem(ctx, hp, model)
        u = torch.empty(prob.n, dtype=torch.float64, device="cuda")
        st = prob.solve(u, default_opts(krylov=PCG, local_solver=LOCAL_LU, prolong=PROLONG_UNWEIGHTED,
                                        precision=FP64, rtol=1e-6, max_it=500), check=False)
        pairs.append((prob, harvest(prob, list(range(st.iterations)))))
    t_harvest = time.perf_counter() - t0
    state = init_state(torch.tensor(th0, device="cuda"), lr=lr)
    t0 = time.perf_counter()
    losses = []
    for e in range(epochs):
        losses.append(train_epoch(ctx, pairs, state, batch, kbar, alpha, clip, seed=e))
        if log and (e % 10 == 0 or e == epochs - 1):
            log(f"epoch {e}: loss {losses[-1]:.5g} lr {state.lr:.1e}")
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    info = {"problems": problems, "nodes": nodes, "parts": parts, "samples": sum(len(d.samples()) for _, d in pairs),
            "epochs": epochs, "steps": state.step, "harvest_s": t_harvest, "train_s": t_train,
            "loss_first": losses[0], "loss_last": losses[-1], "lr_final": state.lr}
    return state.theta.cpu().numpy(), info


def generated(seed: int, nodes: int, parts: int):
    """A generated problem (seeded mesh, P1 system, partition) and its host arrays."""
    import workload as W
    from . import host_problem
    p = W.make_problem(seed, nodes, parts, 0.0)
    return p, host_problem(p.mesh.xy, p.mesh.tri, p.mesh.dirichlet, p.A.rowptr, p.A.col, p.A.val, p.b, p.u0,
                           p.part, p.n_parts, 2)


def main():
    """Train DSS_theta on local problems of generated meshes (the Sec. IV.A recipe at the
    generator's shapes) and compare FCG iterations on a held-out problem."""
    import argparse
    import json
    import torch
    import workload as W
    from . import FCG, FP32, Model
    ap = argparse.ArgumentParser()
    ap.add_argument("--problems", type=int, default=8)
    ap.add_argument("--nodes", type=int, default=7000)
    ap.add_argument("--parts", type=int, default=7)
    ap.add_argument("--epochs", type=int, default=100)
    ap.add_argument("--batch", type=int, default=100)
    ap.add_argument("--lr", type=float, default=1e-2)
    ap.add_argument("--clip", type=float, default=1e-2)
    ap.add_argument("--kbar", type=int, default=30)
    ap.add_argument("--alpha", type=float, default=1e-3)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--out", default=None, help="write the trained weights here (.npy)")
    a = ap.parse_args()
    ctx = Context()
    theta, info = train_on_generated(ctx, a.problems, a.nodes, a.parts, a.epochs, a.batch, a.lr, a.clip, a.kbar,
                                     a.alpha, a.seed, log=lambda m: print(m, flush=True))
    if a.out:
        np.save(a.out, theta)
    p, hp = generated(0, a.nodes, a.parts)  # held out
    res = {}
    for name, th in (("xavier", W.xavier_theta(a.seed, a.kbar, 10)), ("trained", theta)):
        m = Model(ctx, th, kbar=a.kbar, alpha=a.alpha)
        prob = Problem(ctx, hp, m)
        u = torch.empty(prob.n, dtype=torch.float64, device="cuda")
        st = prob.solve(u, default_opts(krylov=FCG, precision=FP32, rtol=1e-6, max_it=600), check=False)
        res[name] = {"iterations": st.iterations, "converged": bool(st.converged),
                     "rel_residual": st.rel_residual}
    info["held_out_fcg"] = res
    print(json.dumps(info))


if __name__ == "__main__":
    main()
