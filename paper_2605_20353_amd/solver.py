"""GCP-Adam solver: epochs of synchronous sampled-gradient Adam iterations
(Alg. gcp-sgd-iter on one device) with the paper's safeguard -- the objective
is estimated on a fixed sample set after every epoch; an epoch that does not
lower it is undone (model and Adam state restored) and the rate is multiplied
by `decay`; after `max_fails` such epochs the solver stops (Sec. 5, the
experiments' epoch loop with 100 iterations per epoch and the rate / decay
parameters of the hyperparameter tables).

Every numerical step runs in the HIP kernels through the C ABI; this module
only sequences the calls and copies device buffers for the restore.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import torch

from . import _lib as G

OBJECTIVE_CLIENT = 1 << 62     # Philox key word of the fixed objective sample set


@dataclass
class SolverConfig:
    R: int
    loss: str = "poisson"
    sampling: str = "stratified"       # or "semi_stratified" / "uniform" (dense tensors)
    p: int = 1 << 16                   # per-iteration samples (uniform: all samples)
    q: int = 1 << 16
    obj_p: int = 1 << 18               # fixed objective set
    obj_q: int = 1 << 18
    iters_per_epoch: int = 100
    max_epochs: int = 50
    lr: float = 1e-3
    decay: float = 0.1
    max_fails: int = 3
    beta1: float = 0.9
    beta2: float = 0.999
    eps: float = 1e-8
    lower: float = float("-inf")
    seed: int = 20353
    tile: G.Tile | None = None
    fused: bool = True                 # False: the non-fused gradient (write the sampled tensor, then MTTKRP)


@dataclass
class SolverResult:
    A: torch.Tensor
    objective: list = field(default_factory=list)   # after each accepted epoch (index 0: initial)
    rates: list = field(default_factory=list)       # rate used in each epoch
    accepted: list = field(default_factory=list)
    fails: int = 0
    iterations: int = 0


def gcp_adam(tensor, A0: torch.Tensor, cfg: SolverConfig) -> SolverResult:
    """Run GCP-Adam on `tensor` from the model A0 ([sum_k I_k, R], copied)."""
    A = A0.detach().reshape(-1).contiguous().clone()
    B = torch.zeros_like(A)
    C = torch.zeros_like(A)
    Gr = torch.zeros_like(A)
    obj_sp = G.SampleParams(cfg.sampling, cfg.obj_p, cfg.obj_q if cfg.sampling != "uniform" else 0,
                            seed=cfg.seed, step=0, client=OBJECTIVE_CLIENT)

    def objective() -> float:
        _, L = G.gcp_loss_grad(tensor, obj_sp, A, cfg.R, cfg.loss, loss_only=True)
        return float(L.item())

    nonfused_bufs = None
    if not cfg.fused:
        n = cfg.p + (cfg.q if cfg.sampling != "uniform" else 0)
        nonfused_bufs = (torch.empty(n, tensor.d, dtype=torch.int64, device=A.device),
                         torch.empty(n, dtype=A.dtype, device=A.device))

    def gradient(sp):
        if cfg.fused:
            G.gcp_loss_grad(tensor, sp, A, cfg.R, cfg.loss, G=Gr, accumulate=True, want_loss=False, tile=cfg.tile)
        else:
            # Sec. 3.1.2 without fusion: the sampled tensor (coordinates and
            # derivative values) goes to memory, then the MTTKRP reads it and
            # gathers the factor rows a second time
            coords, y = nonfused_bufs
            G.gcp_sample_y(tensor, sp, A, cfg.R, cfg.loss, coords=coords, y=y)
            G.gcp_mttkrp(tensor, coords, y, A, cfg.R, G=Gr, accumulate=True, tile=cfg.tile)

    res = SolverResult(A=A)
    f_prev = objective()
    res.objective.append(f_prev)
    rate = cfg.lr
    t = 0                      # Adam update count
    it = 0                     # iterations taken, accepted or not (drives the RNG step)
    for _ in range(cfg.max_epochs):
        saved = (A.clone(), B.clone(), C.clone(), t)
        for _ in range(cfg.iters_per_epoch):
            sp = G.SampleParams(cfg.sampling, cfg.p, cfg.q if cfg.sampling != "uniform" else 0,
                                seed=cfg.seed, step=it)
            gradient(sp)
            t += 1
            it += 1
            G.gcp_adam_step(A, Gr, B, C, t, lr=rate, beta1=cfg.beta1, beta2=cfg.beta2, eps=cfg.eps,
                            lower=cfg.lower, zero_grad=True)
        tensor.status()
        f = objective()
        res.rates.append(rate)
        if f < f_prev:
            f_prev = f
            res.objective.append(f)
            res.accepted.append(True)
        else:
            A.copy_(saved[0])
            B.copy_(saved[1])
            C.copy_(saved[2])
            t = saved[3]
            rate *= cfg.decay
            res.fails += 1
            res.accepted.append(False)
            if res.fails >= cfg.max_fails:
                break
    res.iterations = it
    return res
