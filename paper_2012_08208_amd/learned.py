"""Training driver of the learned preconditioner (host orchestration only).

Pairs (r, e = K^{-1} r) come from multigrid PCG solves along seeded SIMP
histories: the library advances the design with its own SIMP iteration and
harvests the iterates of a PCG solve at the current design
(``topo_precond_harvest``).  Training steps, the loss, the backward pass and
Adam all run in the library's kernels (``topo_precond_train_step``).  This
module only chooses which pair to feed next, keeps the pairs in device
memory, and records losses.
"""

from __future__ import annotations

import dataclasses
from typing import List, Sequence

import numpy as np

from .binding import TOPO_FP64, TOPO_PC_GMG, Topo, num_params


@dataclasses.dataclass
class PairSet:
    rhos: list          # density tensors, one per design
    R: object           # [n_pairs, n_dofs] float64 (device)
    E: object           # [n_pairs, n_dofs] float64 (device)
    design: np.ndarray  # design index of each pair
    iters: List[int]    # PCG iterations of each harvest solve


def harvest_history(t: Topo, n_designs: int, simp_steps: int, harvest_iters: Sequence[int],
                    rho0=None, presmooth: bool = True) -> PairSet:
    """Runs ``simp_steps`` SIMP iterations between harvests on context ``t``
    (GMG preconditioner, one load case) and harvests pairs at the listed PCG
    iterations of a solve at each design (pre-smoothed as the learned cycle
    sees them, unless ``presmooth`` is false)."""
    torch = t.torch
    dev = t.device
    rho = (torch.full((t.n_cells,), t.prob.volfrac, dtype=torch.float64, device=dev)
           if rho0 is None else rho0.clone())
    u = torch.zeros(t.vec_numel(), dtype=torch.float64, device=dev)
    its = list(int(k) for k in harvest_iters)
    rhos, Rs, Es, des, solves = [], [], [], [], []
    for d in range(n_designs):
        if simp_steps > 0:
            t.iterate(rho, u, simp_steps)
        R = torch.empty(len(its) * t.n_dofs, dtype=torch.float64, device=dev)
        E = torch.empty_like(R)
        n, fin = t.precond_harvest(rho, its, R, E, presmooth)
        keep = [i for i in range(n) if its[i] < fin]
        R = R.view(len(its), t.n_dofs)[keep]
        E = E.view(len(its), t.n_dofs)[keep]
        rhos.append(rho.clone())
        Rs.append(R)
        Es.append(E)
        des += [d] * len(keep)
        solves.append(fin)
    return PairSet(rhos, torch.cat(Rs), torch.cat(Es), np.asarray(des, dtype=np.int64), solves)


def choose_gamma(ps: PairSet) -> float:
    """Output gain: the median ratio rms(e) / rms(r) over the pairs, so the
    network's target e / rms(r) is O(1) after division by gamma."""
    torch = __import__("torch")
    re = torch.sqrt(torch.mean(ps.E * ps.E, dim=1)) / torch.sqrt(torch.mean(ps.R * ps.R, dim=1))
    return float(torch.median(re).item())


def init_weights(seed: int, device) -> object:
    """He-style normal initialisation (variance 2 / fan_in) of the hidden
    layers and a zero output layer, FP32."""
    import torch
    spec = [(8, 16, 1), (16, 16, 1), (16, 32, 1), (32, 32, 1), (32, 64, 1), (64, 64, 1),
            (64, 64, 1), (64, 64, 1), (128, 64, 1), (96, 32, 1), (48, 16, 1), (16, 3, 0)]
    g = torch.Generator().manual_seed(int(seed))
    parts = []
    for cin, cout, act in spec:
        std = float(np.sqrt((2.0 if act else 1.0) / (27 * cin)))
        parts.append(torch.randn(cout * 27 * cin, generator=g, dtype=torch.float32) * std)
    parts[-1].zero_()   # the output layer starts at zero: no correction, loss 1
    w = torch.cat(parts)
    assert w.numel() == num_params()
    return w.to(device)


def train(t: Topo, ps: PairSet, steps: int, lr: float, seed: int = 0, lr_final: float | None = None):
    """``steps`` Adam steps on pairs drawn uniformly (seeded); cosine decay
    from ``lr`` to ``lr_final`` when given.  Returns the device tensor of
    per-step losses."""
    torch = t.torch
    rng = np.random.default_rng(seed)
    losses = torch.zeros(steps, dtype=torch.float64, device=t.device)
    n = ps.R.shape[0]
    for s in range(steps):
        i = int(rng.integers(n))
        a = lr
        if lr_final is not None and steps > 1:
            a = lr_final + 0.5 * (lr - lr_final) * (1 + np.cos(np.pi * s / (steps - 1)))
        t.precond_train_step(ps.rhos[int(ps.design[i])], ps.R[i], ps.E[i], a, losses[s:s + 1])
    return losses


def learned_context(p, weights, gamma: float, fcg_maxit: int = 500, smooth: int = 1, rtol=None,
                    maxit: int = 20000, device="cuda") -> Topo:
    """A TOPO_PC_LEARNED context for problem ``p`` with the given weights."""
    from .binding import TOPO_PC_LEARNED
    t = Topo.from_problem(p, precision=TOPO_FP64, precond=TOPO_PC_LEARNED, rtol=rtol, maxit=maxit,
                          device=device)
    t.precond_attach()
    t.precond_set_weights(weights)
    t.precond_config(gamma, fcg_maxit, smooth)
    return t


def gmg_context(p, rtol=None, maxit: int = 20000, device="cuda") -> Topo:
    """A multigrid-PCG context (FP64) with a network workspace attached, for
    harvesting and training."""
    t = Topo.from_problem(p, precision=TOPO_FP64, precond=TOPO_PC_GMG, rtol=rtol, maxit=maxit,
                          device=device)
    t.precond_attach()
    return t
