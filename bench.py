#!/usr/bin/env python3
"""Benchmark: SIMP iterations per second on one MI355X.

Workload (default): the 3D cantilever of 192 x 96 x 96 unit cubes, each cut
into 6 Kuhn tetrahedra (10,616,832 cells, 5,447,811 DOFs), face x = 0
clamped, four unit line-load cases solved as four batched right-hand sides
(compliance summed), volfrac 0.3, p = 3, rmin 2.5 cells, CG relative
residual 1e-8 per load case.  One step is one full SIMP iteration (solve,
sensitivity, filter, OC update) on device-resident data; the design evolves
from step to step as in a real run, starting from rho = volfrac, so the
default 2 warmup + 48 timed steps are iterations 3..50 of a 50-iteration
run.  Default solve: multigrid-preconditioned CG with the FP32 V-cycle
inside FP64 flexible CG.

Printed: one JSON line with the throughput, the live roofline of the
operator-apply kernel (algorithmic bytes per launch / mean launch time from
HIP events on the library stream), and the CPU oracle timed on a bounded
sample of the same workload.
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "SIMP iters/s + matvec HBM GB/s, 3D 5.4M DOF; mixed/learned vs FP64 PCG"
HBM_PEAK_GBS = 8000.0


def workload(name: str):
    import synth
    if name == "cantilever3d":
        return synth.cantilever3d(192, 96, 96, nrhs=4, volfrac=0.3, rmin=2.5, rtol=1e-8)
    if name == "cantilever3d-small":
        return synth.cantilever3d(48, 24, 24, nrhs=4, volfrac=0.3, rmin=2.5, rtol=1e-8)
    if name == "cantilever2d":
        return synth.cantilever2d(60, 30, rtol=1e-10)
    raise SystemExit(f"unknown workload {name}")


def apply_bytes(p, precision: str) -> int:
    """Algorithmic bytes of one operator apply over all load cases: read x,
    write y (nrhs x N_d values each), read one modulus per cell, read the
    one-byte node mask."""
    sv = 8 if precision == "fp64" else 4
    se = 8 if precision == "fp64" else 4
    return p.nrhs * p.n_dofs * sv * 2 + p.n_cells * se + p.n_nodes


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in ("apply.hip", "element.h"):
        with open(os.path.join(ROOT, "paper_2012_08208_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def load_traffic(wl: str, precision: str):
    path = os.path.join(ROOT, "profiles", "apply_traffic.json")
    if not os.path.exists(path):
        return None
    try:
        d = json.load(open(path))
    except Exception:
        return None
    key = f"{wl}:{precision}"
    rec = d.get(key)
    if not rec or rec.get("kernel_hash") != kernel_source_hash():
        return None
    return rec.get("bytes_per_launch")


def cpu_baseline(p_full, sample_nel=(32, 16, 16)):
    """The oracle as it stands, one SIMP iteration on a sub-box of the same
    workload (same BCs, loads, rmin, volfrac, 4 load cases), rate scaled to
    the full mesh by the cell-count ratio (linear scaling favours the CPU:
    sparse LU grows faster than linearly)."""
    import synth
    from oracle import simp
    p = synth.cantilever3d(*sample_nel, nrhs=p_full.nrhs, volfrac=p_full.volfrac,
                           rmin=p_full.rmin)
    S = simp.setup(p)
    t0 = time.perf_counter()
    simp.iterate(S, 1)
    dt = time.perf_counter() - t0
    scale = p.n_cells / p_full.n_cells
    return {
        "value": scale / dt,
        "unit": "SIMP iter/s",
        "cores": 1,
        "kind": "oracle",
        "sample": (f"one oracle SIMP iteration (sparse LU solve of 4 load cases, k-d tree "
                   f"filter, bisection OC) on {sample_nel[0]}x{sample_nel[1]}x{sample_nel[2]} "
                   f"cubes ({p.n_cells} cells, {p.n_dofs} DOFs) in {dt:.2f} s; rate scaled by "
                   f"the cell ratio {scale:.3e}; SuperLU and NumPy single-threaded; host "
                   f"{platform.processor() or platform.machine()}, {os.cpu_count()} cores visible"),
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=48)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="cantilever3d")
    ap.add_argument("--precision", default="mixed", choices=["fp64", "mixed", "mixed-ir"])
    ap.add_argument("--precond", default="gmg", choices=["jacobi", "gmg"])
    ap.add_argument("--maxit", type=int, default=40000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (got --gpus {args.gpus}); "
              "the multi-GPU decomposition is a design note, not an implemented path",
              file=sys.stderr)
        return 2

    import numpy as np
    import torch
    from paper_2012_08208_amd import (LOG_LEN, TOPO_FP64, TOPO_MIXED_FP32, TOPO_MIXED_IR,
                                      TOPO_PC_GMG, TOPO_PC_JACOBI, Topo)

    p = workload(args.workload)
    dev = torch.device("cuda:0")
    prec = {"fp64": TOPO_FP64, "mixed": TOPO_MIXED_FP32, "mixed-ir": TOPO_MIXED_IR}[args.precision]
    pc = TOPO_PC_JACOBI if args.precond == "jacobi" else TOPO_PC_GMG
    t = Topo.from_problem(p, precision=prec, precond=pc, maxit=args.maxit, device=dev)
    rho = torch.full((p.n_cells,), p.volfrac, dtype=torch.float64, device=dev)
    u = torch.zeros(p.nrhs * p.n_dofs, dtype=torch.float64, device=dev)
    log = torch.zeros(max(1, args.steps) * LOG_LEN, dtype=torch.float64, device=dev)
    print(f"[bench] {args.workload} nel={p.nel} nrhs={p.nrhs} cells={p.n_cells} dofs={p.n_dofs} "
          f"precision={args.precision} precond={args.precond}", file=sys.stderr, flush=True)
    for w in range(args.warmup):
        t.iterate(rho, u, 1, 0.0, None)
        torch.cuda.synchronize()
        print(f"[bench] warmup step {w + 1}/{args.warmup} done", file=sys.stderr, flush=True)
    t.timing_enable(True)
    t.timing_read()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(args.steps):
        t.iterate(rho, u, 1, 0.0, log[s * LOG_LEN:(s + 1) * LOG_LEN])
        print(f"[bench] timed step {s + 1}/{args.steps} queued", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    n_apply, apply_ms = t.timing_read()
    status = t.sync()
    lg = log.cpu().numpy().reshape(-1, LOG_LEN)
    dt = t1 - t0
    ms_step = 1e3 * dt / args.steps
    bytes_apply = apply_bytes(p, args.precision)
    avg_apply_s = (apply_ms / n_apply) * 1e-3 if n_apply else float("nan")
    achieved = bytes_apply / avg_apply_s / 1e9 if n_apply else None
    traffic = load_traffic(args.workload, args.precision)
    rec = {
        "metric": METRIC,
        "value": args.steps / dt,
        "unit": "SIMP iter/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {
            "workload": (f"{args.workload}: {'x'.join(map(str, p.nel))} cells "
                         f"({p.n_cells} simplices, {p.n_dofs} DOFs), {p.nrhs} load cases, "
                         f"volfrac {p.volfrac}, p {p.penal}, rmin {p.rmin}, CG rtol {p.rtol}"),
            "precision": args.precision,
            "precond": args.precond,
            "status": int(status),
            "cg_iters_per_step": lg[:, 5].tolist(),
            "compliance": lg[:, 0].tolist(),
            "apply_launches": n_apply,
            "apply_ms_mean": (apply_ms / n_apply) if n_apply else None,
            "apply_share_of_step": (apply_ms / (dt * 1e3)) if n_apply else None,
        },
        "roofline": {
            "kernel": "apply3d" if p.dim == 3 else "apply2d",
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": (achieved / HBM_PEAK_GBS) if achieved else None,
            "traffic": traffic,
            "algorithmic_bytes_per_launch": bytes_apply,
        },
    }
    if not args.no_cpu_baseline and p.dim == 3:
        print("[bench] timing the CPU oracle on a bounded sample", file=sys.stderr, flush=True)
        rec["cpu_baseline"] = cpu_baseline(p)
    else:
        rec["cpu_baseline"] = None
    t.close()
    print(json.dumps(rec))
    return 0


if __name__ == "__main__":
    sys.exit(main())
