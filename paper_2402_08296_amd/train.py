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
    """Right-hand sides of all sub-meshes at T iterates: c[t * sum_k + slot]."""
    c: object          # device float32 tensor, T * sum_k
    iterates: list     # the PCG iteration of each block
    sum_k: int

    def samples(self):
        return [(t, i) for t in range(len(self.iterates)) for i in range(self._K)]

    _K: int = 0


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
    h = Harvest(c, list(iterates), sum_k)
    h._K = prob.K
    return h


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


def train_epoch(ctx: Context, prob: Problem, data: Harvest, st: TrainState, batch: int = 100, kbar: int = 30,
                alpha: float = 1e-3, clip: float = 1e-2, seed: int = 0, patience: int = 10,
                factor: float = 0.1) -> float:
    """One pass over the samples in a seeded order; returns the mean batch loss."""
    samples = data.samples()
    order = np.random.default_rng(seed).permutation(len(samples))
    ptr = prob.hp.sub_ptr
    losses = []
    for b0 in range(0, len(order), batch):
        sel = [samples[q] for q in order[b0:b0 + batch]]
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
