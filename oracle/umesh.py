"""The SIMP iteration on an arbitrary P1 simplex mesh (test oracle, FP64).

Test infrastructure: only ``tests/``, the entry module's ``smoke()`` and the
CPU-baseline leg of the benchmark may import it.

Section 6.1 runs the loop of the Appendix code unchanged on an imported
tetrahedral mesh: the finite-element steps (Sec. 3.1, eq. fe_form; Sec. 2,
eq. simp) are written over whatever cells the mesh has, and the filter
takes its weights from the distances between the actual cell midpoints
(Sec. 3.2.2, eq. filter; Sec. 4.5, eq. filter_mat; the weight matrix built
in chunks, Sec. 6.2).  On such a mesh the cells differ in volume, and two
choices of the listing then matter; this oracle follows the listing:

* the sensitivity it filters is a value per unit volume, the derivative of
  the energy density -p rho^(p-1) psi_e: here s_e = (dc/drho_e) / |T_e|,
  which is -p rho^(p-1) (E0 - Emin) 2 psi_e (the constant 2 (E0 - Emin)
  scales every cell alike and cancels in the OC multiplier);
* the OC volume constraint counts cells, sum_e rho_e = volfrac * N_c
  (Sec. 3.2.1 and the listing's bisection test).

Every step is the plain definition: the assembled sparse stiffness, a
direct solve per load case, element energies from the strains, the
midpoint weights from a k-d tree (pinned elsewhere to the brute-force
pairwise distances), and the bisection OC update.
"""

from __future__ import annotations

import dataclasses
from typing import List

import numpy as np

from . import fem, filt, mesh as mesh_mod, oc


@dataclasses.dataclass
class USetup:
    mesh: mesh_mod.Mesh
    K0: np.ndarray
    vol: np.ndarray
    fixed_flat: np.ndarray
    f: np.ndarray      # [nrhs, N_d], node-major within a component: f[r, c*N + n]
    W: object
    R: np.ndarray
    prob: object


def setup(p) -> USetup:
    """p: an object with dim, coords [N, dim], cells [N_c, dim+1], fixed
    [dim][N], loads [nrhs][dim][N] and the SIMP parameters."""
    m = mesh_mod.Mesh(p.dim, None, np.asarray(p.coords, dtype=np.float64),
                      np.asarray(p.cells, dtype=np.int64))
    K0 = fem.element_K0(m, p.nu)
    vol, _ = mesh_mod.geometry(m)
    fixed_flat = np.asarray(p.fixed).reshape(-1)
    f = np.asarray(p.loads, dtype=np.float64).reshape(p.loads.shape[0], -1)
    W = filt.weights_sparse(mesh_mod.centroids(m), p.rmin)
    return USetup(m, K0, vol, fixed_flat, f, W, filt.row_sums(W), p)


def solve_state(S: USetup, rho):
    """u, compliance, element energies w_e = sum_r u_e^T K0_e u_e, the exact
    derivative dc/drho_e and the per-volume sensitivity s_e = dc_e / |T_e|."""
    p = S.prob
    E = fem.simp_modulus(rho, p.E0, p.Emin, p.penal)
    K = fem.assemble(S.mesh, E, p.nu, False, S.K0)
    u = fem.solve(K, S.f, S.fixed_flat)
    c = fem.compliance(S.f, u)
    w = fem.element_energy(S.mesh, u, p.nu)
    dc = fem.sensitivity(rho, w, p.E0, p.Emin, p.penal)
    return u, c, w, dc, dc / S.vol, E


def iterate(S: USetup, n_iter: int, rho0=None) -> tuple:
    """The loop (solve, sensitivity per unit volume, midpoint filter, OC by
    cell count); returns (rho, log), one dict per iteration."""
    p = S.prob
    rho = np.full(S.mesh.n_cells, p.volfrac) if rho0 is None else np.array(rho0, dtype=np.float64)
    log: List[dict] = []
    for it in range(n_iter):
        u, c, w, dc, s, E = solve_state(S, rho)
        c_paper = float(np.sum(E * w / (2.0 * S.vol)))
        sf = filt.apply(S.W, S.R, rho, s)
        rho_new, lam, vol, change, passes = oc.update(rho, sf, p.volfrac, p.move, p.eta, p.rho_min)
        log.append(dict(it=it + 1, c=c, c_paper=c_paper, vol=vol / rho.size, change=change,
                        lam=lam, passes=passes))
        rho = rho_new
    return rho, log
