"""Writes mbb2d_1200x400.json: oracle values for the full-size 2D MBB
half-beam (1200 x 400 squares, 960,000 P1 triangles, 963,202 DOFs) at a
seeded density field, for tests/test_gpu_fullsize_mbb2d.py.

Calls only the oracle (FP64 sparse assembly and SuperLU solve, k-d tree
filter rows, bisection OC), about two minutes on one core:

    python tests/golden/make_mbb2d_fullsize.py

Stored: the compliance f^T u (Sec. 3.2), u at sampled nodes, the exact
sensitivity and the filtered sensitivity at sampled cells (Sec. 3.2,
Sec. 3.2.2 eq. filter), the OC multiplier, volume and design at sampled
cells (Sec. 3.2 eq. update).
"""

import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import synth  # noqa: E402
from oracle import fem, filt, mesh as M, oc  # noqa: E402

RHO_SEED, RHO_LO, RHO_HI = 5, 0.05, 0.75


def main():
    p = synth.mbb2d()                                   # 1200 x 400, the configured size
    m = M.build(2, p.nel, p.split)
    rho = synth.rho_random(RHO_SEED, m.n_cells, RHO_LO, RHO_HI)
    E = fem.simp_modulus(rho, p.E0, p.Emin, p.penal)
    K = fem.assemble(m, E, p.nu)
    f = p.loads.reshape(1, -1)
    u = fem.solve(K, f, p.fixed.ravel())
    c = fem.compliance(f, u)
    rng = np.random.default_rng(6)
    nodes = np.unique(np.concatenate([rng.integers(0, m.n_nodes, 40), [0, m.n_nodes - 1, 1200, 400 * 1201]]))
    cells = np.unique(np.concatenate([rng.integers(0, m.n_cells, 40), [0, 1, m.n_cells - 1, 2 * 1199]]))
    w = fem.element_energy(m, u, p.nu)
    dc = fem.sensitivity(rho, w, p.E0, p.Emin, p.penal)
    cent = M.centroids(m)
    dcf_rows, _ = filt.apply_rows(cent, p.rmin, rho, dc, cells)
    # the full filtered field for the OC step (every row by the same rule)
    W = filt.weights_sparse(cent, p.rmin)
    dcf = filt.apply(W, filt.row_sums(W), rho, dc)
    rho_new, lam, vol, change, _ = oc.update(rho, dcf, p.volfrac, p.move, p.eta, p.rho_min)
    out = {
        "problem": "mbb2d 1200x400, volfrac 0.4, rmin 3.0, uniform split",
        "rho": {"seed": RHO_SEED, "lo": RHO_LO, "hi": RHO_HI},
        "compliance": c,
        "nodes": nodes.tolist(),
        "u": u.reshape(2, -1)[:, nodes].tolist(),
        "cells": cells.tolist(),
        "dc": dc[cells].tolist(),
        "dcf": dcf_rows.tolist(),
        "oc": {"lambda": lam, "volume": vol, "change": change, "rho_new": rho_new[cells].tolist()},
    }
    with open(os.path.join(HERE, "mbb2d_1200x400.json"), "w") as fh:
        json.dump(out, fh, indent=1)
    print("compliance", c, "lambda", lam)


if __name__ == "__main__":
    main()
