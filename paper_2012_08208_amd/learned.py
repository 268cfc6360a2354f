"""Training driver of the learned preconditioner (host orchestration only).

Pairs (r, e = K^{-1} r) come from multigrid PCG solves along seeded SIMP
histories: the library advances the design with its own SIMP iteration and
harvests the iterates of a PCG solve at the current design
(``topo_precond_harvest``).  Training steps, the loss, the backward pass and
Adam all run in the library's kernels (``topo_precond_train_step``).  This
module only chooses which pair to feed next, keeps the pairs in device
memory (a fixed pair set, or a replay buffer that pairs stream through),
and records losses.
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


class Replay:
    """Ring buffer of (r, e) pairs in device memory, with a ring of the
    designs they were harvested at.  New pairs overwrite the oldest; a pair
    whose design slot has since been reused is never drawn."""

    def __init__(self, t: Topo, capacity: int, design_capacity: int):
        torch = t.torch
        self.torch = torch
        self.R = torch.empty((capacity, t.n_dofs), dtype=torch.float64, device=t.device)
        self.E = torch.empty_like(self.R)
        self.rhos = torch.empty((design_capacity, t.n_cells), dtype=torch.float64, device=t.device)
        self.pair_design = np.full(capacity, -1, dtype=np.int64)   # design serial of each slot
        self.slot_serial = np.full(design_capacity, -1, dtype=np.int64)
        self.head = 0
        self.dhead = 0
        self.pairs_seen = 0
        self.designs_seen = 0

    @property
    def capacity(self) -> int:
        return self.R.shape[0]

    def add_design(self, rho) -> int:
        """Stores a design; returns its serial number."""
        slot = self.dhead
        self.rhos[slot].copy_(rho)
        serial = self.designs_seen
        self.slot_serial[slot] = serial
        self.dhead = (self.dhead + 1) % self.rhos.shape[0]
        self.designs_seen += 1
        return serial

    def add_pairs(self, serial: int, R, E) -> None:
        for i in range(R.shape[0]):
            self.R[self.head].copy_(R[i])
            self.E[self.head].copy_(E[i])
            self.pair_design[self.head] = serial
            self.head = (self.head + 1) % self.capacity
            self.pairs_seen += 1

    def valid(self) -> np.ndarray:
        """Slots whose design is still held."""
        ds = self.pair_design
        ok = ds >= 0
        slots = ds % self.rhos.shape[0]
        ok &= self.slot_serial[np.where(ok, slots, 0)] == ds
        return np.nonzero(ok)[0]

    def design_of(self, i: int):
        return self.rhos[int(self.pair_design[i] % self.rhos.shape[0])]


def stream_train(t: Topo, histories, n_pairs: int, harvest_iters: Sequence[int], capacity: int,
                 steps_per_pair: float, lr: float, lr_final: float, seed: int,
                 simp_steps: int = 1, designs_per_history: int = 40, log=None) -> dict:
    """Streams about ``n_pairs`` harvested pairs through a replay buffer of
    ``capacity`` pairs while training the network of context ``t``.

    ``histories(h)`` returns the problem of the h-th seeded SIMP history (the
    same grid and supports as ``t``'s problem).  Each history starts from the
    uniform design; every ``simp_steps`` SIMP iterations its design is
    stored and a multigrid PCG solve there is harvested at ``harvest_iters``
    (pre-smoothed pairs).  After each harvest, ``steps_per_pair`` training
    steps per new pair draw pairs uniformly from the buffer; the learning
    rate follows a cosine from ``lr`` to ``lr_final`` over the planned
    steps.  Returns the device tensor of losses and counts and times."""
    import time
    torch = t.torch
    rng = np.random.default_rng(seed)
    its = [int(k) for k in harvest_iters]
    per_design = len(its)
    design_capacity = capacity // max(1, per_design) + 8
    buf = Replay(t, capacity, design_capacity)
    planned = max(1, int(round(n_pairs * steps_per_pair)))
    losses = torch.zeros(planned, dtype=torch.float64, device=t.device)
    step = 0
    credit = 0.0
    h = 0
    t_harvest = t_train = 0.0
    solve_iters = []
    R = torch.empty(per_design * t.n_dofs, dtype=torch.float64, device=t.device)
    E = torch.empty_like(R)
    while buf.pairs_seen < n_pairs:
        th = gmg_context(histories(h), rtol=t.prob.rtol, device=t.device)
        rho = torch.full((t.n_cells,), th.prob.volfrac, dtype=torch.float64, device=t.device)
        u = torch.zeros(th.vec_numel(), dtype=torch.float64, device=t.device)
        for d in range(designs_per_history):
            if buf.pairs_seen >= n_pairs:
                break
            a = time.perf_counter()
            th.iterate(rho, u, simp_steps)
            n, fin = th.precond_harvest(rho, its, R, E, True)
            keep = [i for i in range(n) if its[i] < fin]
            serial = buf.add_design(rho)
            buf.add_pairs(serial, R.view(per_design, t.n_dofs)[keep],
                          E.view(per_design, t.n_dofs)[keep])
            solve_iters.append(fin)
            torch.cuda.synchronize()
            b = time.perf_counter()
            t_harvest += b - a
            credit += steps_per_pair * len(keep)
            valid = buf.valid()
            while credit >= 1.0 and step < planned:
                i = int(valid[int(rng.integers(len(valid)))])
                c = 0.5 * (1.0 + np.cos(np.pi * step / max(1, planned - 1)))
                t.precond_train_step(buf.design_of(i), buf.R[i], buf.E[i],
                                     lr_final + (lr - lr_final) * c, losses[step:step + 1])
                step += 1
                credit -= 1.0
            torch.cuda.synchronize()
            t_train += time.perf_counter() - b
            if log is not None and d == 0:
                log(f"history {h}: {buf.pairs_seen} pairs, {step} steps, "
                    f"harvest {t_harvest:.1f} s, train {t_train:.1f} s")
        th.close()
        h += 1
    return {"losses": losses[:step], "pairs": buf.pairs_seen, "designs": buf.designs_seen,
            "histories": h, "steps": step, "capacity": capacity, "harvest_s": t_harvest,
            "train_s": t_train, "solve_iters_mean": float(np.mean(solve_iters)) if solve_iters else 0.0}


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
    harvesting and training.  Its hierarchy goes down to 128 DOFs: the pairs
    are errors of a multigrid PCG iterate, and with a large coarsest level
    solved exactly (the 3D default) the errors that PCG leaves are mostly
    rough, while the network serves as the coarse correction between two
    smoothings, whose job is the smooth part; on 24 x 12 x 12 a network
    trained on those pairs did not beat the cycle without it (342 against
    329 FCG iterations; 210 against 336 with this hierarchy)."""
    t = Topo.from_problem(p, precision=TOPO_FP64, precond=TOPO_PC_GMG, rtol=rtol, maxit=maxit,
                          device=device, gmg_dense=128)
    t.precond_attach()
    return t
