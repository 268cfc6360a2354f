"""The SIMP iteration loop (test oracle, FP64).

Section 4.3-4.5 and the Appendix code: starting from rho = volfrac in every
cell, each iteration (1) solves K(rho) u = f, (2) evaluates the compliance
and its sensitivity, (3) filters the sensitivity, (4) updates rho by the
optimality criteria with bisection, and (5) records the change
max |rho_new - rho|.  Multiple load cases (Section 5.3) are solved one by
one; compliances and sensitivities are summed over the cases.  Step (3)
uses the distance-weighted filter, or the Helmholtz PDE filter
(oracle/helm.py) when the problem's ``filter`` is 1.  With ``filter`` 2
(density filter) the physics of steps (1)-(2) sees x~ = W x / R, step (3)
is the chain rule back to the design x, and the OC volume is that of x~.

The logged objective is the compliance c = sum_r f_r^T u_r; ``c_paper`` is
sum_e E_e w_e / (2|T_e|), the sum of rho^p psi_e that the listing prints
(equal to c / (2|T|) on these equal-volume meshes).
"""

from __future__ import annotations

import dataclasses
from typing import List

import numpy as np

from . import fem, filt, helm, mesh as mesh_mod, oc


@dataclasses.dataclass
class Setup:
    mesh: mesh_mod.Mesh
    K0: np.ndarray
    fixed_flat: np.ndarray
    f: np.ndarray          # [nrhs, N_d]
    W: object
    R: np.ndarray
    prob: object
    helm_mats: object = None


def _helmholtz(prob) -> bool:
    return getattr(prob, "filter", 0) == 1


def setup(prob, dense_filter: bool = False) -> Setup:
    m = mesh_mod.build(prob.dim, prob.nel, prob.split)
    K0 = fem.element_K0(m, prob.nu, prob.paper_mode)
    fixed_flat = np.asarray(prob.fixed).reshape(-1)
    f = np.asarray(prob.loads, dtype=np.float64).reshape(prob.loads.shape[0], -1)
    cent = mesh_mod.centroids(m)
    W = filt.weights_dense(cent, prob.rmin) if dense_filter else filt.weights_sparse(cent, prob.rmin)
    R = filt.row_sums(W) if not dense_filter else W.sum(axis=1)
    hm = helm.matrices(m) if _helmholtz(prob) else None
    return Setup(m, K0, fixed_flat, f, W, R, prob, hm)


def filter_sensitivity(S: Setup, rho, s):
    """Step (3): the configured sensitivity filter."""
    if _helmholtz(S.prob):
        return helm.sensitivity_filter(S.mesh, S.prob.rmin, rho, s, S.helm_mats)
    return filt.apply(S.W, S.R, rho, s)


def modulus(S: Setup, rho):
    p = S.prob
    return fem.simp_modulus(rho, p.E0, p.Emin, p.penal, p.paper_mode)


def solve_state(S: Setup, rho):
    """u, compliance, element energies and sensitivity at design rho."""
    p = S.prob
    E = modulus(S, rho)
    K = fem.assemble(S.mesh, E, p.nu, p.paper_mode, S.K0)
    u = fem.solve(K, S.f, S.fixed_flat)
    c = fem.compliance(S.f, u)
    w = fem.element_energy(S.mesh, u, p.nu, p.paper_mode)
    s = fem.sensitivity(rho, w, p.E0, p.Emin, p.penal, p.paper_mode)
    if p.paper_mode:
        s = s * fem.paper_sensitivity_scale(S.mesh)
    return u, c, w, s, E


def iterate(S: Setup, n_iter: int, rho0=None, change_tol: float = 0.0) -> tuple:
    """Run the loop; returns (rho, log) where log has one dict per iteration."""
    p = S.prob
    rho = np.full(S.mesh.n_cells, p.volfrac) if rho0 is None else np.array(rho0, dtype=np.float64)
    log: List[dict] = []
    vol_cell, _ = mesh_mod.geometry(S.mesh)
    dens = getattr(p, "filter", 0) == 2
    dv = filt.density_grad(S.W, S.R, np.ones(S.mesh.n_cells)) if dens else None
    phys = (lambda x: filt.density(S.W, S.R, x)) if dens else None
    for it in range(n_iter):
        u, c, w, s, E = solve_state(S, phys(rho) if dens else rho)
        c_paper = float(np.sum(E * w / (2.0 * vol_cell)))
        sf = filt.density_grad(S.W, S.R, s) if dens else filter_sensitivity(S, rho, s)
        rho_new, lam, vol, change, passes = oc.update(rho, sf, p.volfrac, p.move, p.eta,
                                                      p.rho_min,
                                                      passive=getattr(p, "passive", None),
                                                      dv=dv, phys=phys)
        log.append(dict(it=it + 1, c=c, c_paper=c_paper, vol=vol / rho.size, change=change,
                        lam=lam, passes=passes))
        rho = rho_new
        if change_tol > 0.0 and change < change_tol:
            break
    return rho, log
