"""Finite-element steps of the SIMP iteration (test oracle, FP64).

* Material law: isotropic linear elasticity with stress
  sigma = lambda tr(eps) I + 2 mu eps and strain-energy density
  psi = lambda/2 tr(eps)^2 + mu tr(eps^2) (Section 2, eq. str_energy;
  Section 4.2, eq. stress and eq. energy).  Here it is written in Voigt
  form with engineering shear strains.  Two-dimensional problems use plane
  stress with (E, nu); the "paper mode" uses the listing's Lame constants
  mu = 0.4, lambda = 0.6 directly.
* SIMP interpolation (Section 2, eq. simp_fn and eq. simp): the stiffness
  of cell e is E_e D_unit with E_e = Emin + rho_e^p (E0 - Emin); the paper
  itself uses E_e = rho_e^p (paper mode, Emin = 0).
* Discrete form (Section 3.1, eq. fe_form): P1 Galerkin, so the strain is
  constant per cell and K_e = |T_e| B_e^T D B_e exactly.
* Dirichlet conditions (Section 4.3.2) are imposed by eliminating the
  fixed DOFs; the reduced system is solved with a sparse LU factorisation,
  the paper's default solver (Section 4.3.4).
* Compliance c = sum_r f_r^T u_r and its exact derivative
  dc/drho_e = -p rho_e^(p-1) (E0 - Emin) sum_r u_{r,e}^T K0_e u_{r,e}
  (Section 3.2: sensitivity of f; the paper's per-cell value is this
  derivative divided by 2|T_e|, i.e. -p rho^(p-1) psi_e).

Global DOF numbering is structure-of-arrays: dof(c, n) = c * N_n + n.
"""

from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .mesh import Mesh, geometry

PAPER_MU = 0.4
PAPER_LAMBDA = 0.6


def material_D(dim: int, nu: float, paper_mode: bool = False) -> np.ndarray:
    """Unit-modulus constitutive matrix in Voigt form (engineering shear).

    2D order (xx, yy, xy); 3D order (xx, yy, zz, yz, xz, xy)."""
    if dim == 2:
        if paper_mode:
            lam, mu = PAPER_LAMBDA, PAPER_MU
            return np.array([[lam + 2 * mu, lam, 0.0], [lam, lam + 2 * mu, 0.0], [0.0, 0.0, mu]])
        c = 1.0 / (1.0 - nu * nu)
        return c * np.array([[1.0, nu, 0.0], [nu, 1.0, 0.0], [0.0, 0.0, 0.5 * (1.0 - nu)]])
    if paper_mode:
        lam, mu = PAPER_LAMBDA, PAPER_MU
    else:
        lam = nu / ((1.0 + nu) * (1.0 - 2.0 * nu))
        mu = 1.0 / (2.0 * (1.0 + nu))
    D = np.zeros((6, 6))
    D[:3, :3] = lam
    D[0, 0] = D[1, 1] = D[2, 2] = lam + 2 * mu
    D[3, 3] = D[4, 4] = D[5, 5] = mu
    return D


def B_matrices(grads: np.ndarray) -> np.ndarray:
    """Strain-displacement matrices [n, nstrain, (d+1)*d]; element DOF order
    is node-major: local dof = a*d + c."""
    n, nv, d = grads.shape
    if d == 2:
        B = np.zeros((n, 3, nv * 2), dtype=grads.dtype)
        for a in range(nv):
            gx, gy = grads[:, a, 0], grads[:, a, 1]
            B[:, 0, 2 * a] = gx
            B[:, 1, 2 * a + 1] = gy
            B[:, 2, 2 * a] = gy
            B[:, 2, 2 * a + 1] = gx
        return B
    B = np.zeros((n, 6, nv * 3), dtype=grads.dtype)
    for a in range(nv):
        gx, gy, gz = grads[:, a, 0], grads[:, a, 1], grads[:, a, 2]
        B[:, 0, 3 * a] = gx
        B[:, 1, 3 * a + 1] = gy
        B[:, 2, 3 * a + 2] = gz
        B[:, 3, 3 * a + 1] = gz
        B[:, 3, 3 * a + 2] = gy
        B[:, 4, 3 * a] = gz
        B[:, 4, 3 * a + 2] = gx
        B[:, 5, 3 * a] = gy
        B[:, 5, 3 * a + 1] = gx
    return B


def element_K0(mesh: Mesh, nu: float, paper_mode: bool = False, cells=None) -> np.ndarray:
    """Unit-modulus element matrices |T| B^T D B, shape [n, m, m]."""
    vol, g = geometry(mesh, cells)
    B = B_matrices(g)
    D = material_D(mesh.dim, nu, paper_mode)
    return vol[:, None, None] * np.einsum("eki,kl,elj->eij", B, D, B)


def element_dofs(mesh: Mesh, cells=None) -> np.ndarray:
    """Global SoA DOF ids of each cell, node-major: [n, (d+1)*d]."""
    cells = mesh.cells if cells is None else cells
    d = mesh.dim
    N = mesh.n_nodes
    out = np.empty((cells.shape[0], cells.shape[1] * d), dtype=np.int64)
    for a in range(cells.shape[1]):
        for c in range(d):
            out[:, a * d + c] = c * N + cells[:, a]
    return out


def simp_modulus(rho, E0=1.0, Emin=1e-9, penal=3.0, paper_mode=False):
    """E_e = Emin + rho^p (E0 - Emin); paper mode E_e = rho^p."""
    if paper_mode:
        return rho ** penal
    return Emin + rho ** penal * (E0 - Emin)


def bf16_modulus(E):
    """The BF16 copy of the moduli that the BF16 mixed-precision mode keeps
    for its FP32 multigrid cycle: each FP64 value rounded once to the
    nearest number with 8 significant bits, ties to even, returned as FP64.
    Written with frexp: E = m 2^e with m in [0.5, 1), so the kept
    significand is round(m * 256) (NumPy rounds halves to even).  Values
    must lie in BF16's normal range, [2^-126, 2^128)."""
    E = np.asarray(E, dtype=np.float64)
    a = np.abs(E)
    assert np.all((a == 0) | ((a >= 2.0 ** -126) & (a < 2.0 ** 128)))
    m, e = np.frexp(E)
    return np.ldexp(np.round(m * 256.0), e - 8)


def assemble(mesh: Mesh, E, nu, paper_mode=False, K0=None):
    """Global stiffness sum_e E_e K0_e as CSR (duplicates summed)."""
    if K0 is None:
        K0 = element_K0(mesh, nu, paper_mode)
    dofs = element_dofs(mesh)
    m = dofs.shape[1]
    rows = np.repeat(dofs, m, axis=1).ravel()
    cols = np.tile(dofs, (1, m)).ravel()
    vals = (np.asarray(E)[:, None, None] * K0).ravel()
    nd = mesh.dim * mesh.n_nodes
    return sp.coo_matrix((vals, (rows, cols)), shape=(nd, nd)).tocsr()


def apply_operator(K, x, fixed_flat):
    """y = Z K Z x with Z zeroing fixed DOFs (the constrained operator)."""
    free = fixed_flat == 0
    y = K @ (x * free)
    return y * free


def jacobi_diag(K, fixed_flat):
    """diag(K) on free DOFs, 1 on fixed DOFs."""
    d = K.diagonal().copy()
    d[fixed_flat != 0] = 1.0
    return d


def solve(K, f, fixed_flat):
    """Direct solve of the reduced SPD system for each load case.

    f: [nrhs, N_d] (flat SoA per case). Returns u [nrhs, N_d] with zeros on
    fixed DOFs."""
    free = np.flatnonzero(fixed_flat == 0)
    Kff = K[free][:, free].tocsc()
    lu = spla.splu(Kff)
    f = np.atleast_2d(f)
    u = np.zeros(f.shape, dtype=np.result_type(K.dtype, f.dtype))
    for r in range(f.shape[0]):
        u[r, free] = lu.solve(f[r, free].astype(u.dtype))
    return u


def element_energy(mesh: Mesh, u, nu: float, paper_mode: bool = False, cells=None):
    """w_e = sum_r u_{r,e}^T K0_e u_{r,e} (unit modulus).

    Evaluated from the strain, w_e = |T_e| eps_e^T D eps_e with
    eps_e = B_e u_e: the energy density is a function of the strain
    (Section 2, eq. str_energy), and forming the strain first avoids the
    cancellation of the quadratic form u^T K0 u when u_e is close to a
    rigid motion."""
    dofs = element_dofs(mesh, cells)
    vol, g = geometry(mesh, cells)
    B = B_matrices(g)
    D = material_D(mesh.dim, nu, paper_mode)
    u = np.atleast_2d(u)
    w = np.zeros(dofs.shape[0], dtype=u.dtype)
    for r in range(u.shape[0]):
        eps = np.einsum("eki,ei->ek", B, u[r][dofs])
        w = w + vol * np.einsum("ek,kl,el->e", eps, D, eps)
    return w


def compliance(f, u):
    """c = sum_r f_r^T u_r."""
    return float(np.sum(np.atleast_2d(f) * np.atleast_2d(u)))


def sensitivity(rho, w, E0=1.0, Emin=1e-9, penal=3.0, paper_mode=False):
    """dc/drho_e = -p rho^(p-1) (E0 - Emin) w_e (exact derivative)."""
    if paper_mode:
        return -penal * rho ** (penal - 1.0) * w
    return -penal * rho ** (penal - 1.0) * (E0 - Emin) * w


def paper_sensitivity_scale(mesh: Mesh) -> np.ndarray:
    """1/(2|T_e|): converts the exact derivative to the listing's per-cell
    value -p rho^(p-1) psi_e."""
    vol, _ = geometry(mesh)
    return 1.0 / (2.0 * vol)


def matvec_ebe(mesh: Mesh, E, x, nu, paper_mode=False, chunk=1 << 18):
    """Element-by-element y = sum_e E_e P_e^T K0_e P_e x without assembling
    (for meshes too large for a CSR matrix).  x: [nrhs, N_d]."""
    x = np.atleast_2d(x)
    y = np.zeros_like(x)
    for s in range(0, mesh.n_cells, chunk):
        cells = mesh.cells[s:s + chunk]
        K0 = element_K0(mesh, nu, paper_mode, cells)
        dofs = element_dofs(mesh, cells)
        Ec = np.asarray(E)[s:s + chunk]
        for r in range(x.shape[0]):
            ye = Ec[:, None] * np.einsum("eij,ej->ei", K0, x[r][dofs])
            np.add.at(y[r], dofs.ravel(), ye.ravel())
    return y
