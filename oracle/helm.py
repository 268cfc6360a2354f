"""Helmholtz-type PDE sensitivity filter (test oracle, FP64).

Section 6.3 replaces the distance-weighted filter by the PDE filter of
Lazarov and Sigmund (2011) for parallel runs; the paper gives no formula,
so the one below is the reading taken (the cited paper is not reproduced
here):

* continuous problem: -r^2 lap(psi~) + psi~ = psi in the domain, zero normal
  derivative on its boundary, with psi piecewise constant on the cells;
* length scale r = rmin / (2 sqrt(3)): a one-dimensional hat of radius rmin
  and the one-dimensional Green's function exp(-|x|/r) / (2r) then have the
  same second moment (rmin^2 / 6 = 2 r^2);
* P1 Galerkin discretisation on the same simplex mesh as the elasticity
  problem: (r^2 K + M) x = T psi, with K_ab = sum_e |T_e| grad N_a . grad N_b,
  M_ab = sum_e int_e N_a N_b and T_ne = int_e N_n = |T_e| / (d+1) when node
  n is a vertex of cell e;
* the filtered cell value is the cell mean of the P1 field, i.e. the mean of
  x over the cell's d+1 vertices;
* as a *sensitivity* filter (the role of eq. filter, Section 3.2.2):
  s~_e = F(rho s)_e / rho_e.

Test infrastructure only: imported by tests/, the smoke check and the CPU
baseline of bench.py, never by the library.
"""

from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .mesh import Mesh, geometry


def radius(rmin: float) -> float:
    """PDE-filter length scale for a cone radius rmin (reading above)."""
    return rmin / (2.0 * np.sqrt(3.0))


def mass_element(vol: np.ndarray, d: int) -> np.ndarray:
    """Consistent P1 mass of each cell: int_e lambda_a lambda_b dx =
    |T| (1 + delta_ab) / ((d+1)(d+2)) (integral of barycentric monomials)."""
    n = d + 1
    base = (np.ones((n, n)) + np.eye(n)) / ((d + 1) * (d + 2))
    return vol[:, None, None] * base[None]


def matrices(mesh: Mesh):
    """Assembled Laplacian stiffness K, consistent mass M (N_n x N_n, CSR)
    and the cell-to-node load matrix T (N_n x N_c)."""
    vol, g = geometry(mesh)
    d = mesh.dim
    Ke = vol[:, None, None] * np.einsum("eai,ebi->eab", g, g)
    Me = mass_element(vol, d)
    cells = mesh.cells
    n = d + 1
    rows = np.repeat(cells, n, axis=1).ravel()
    cols = np.tile(cells, (1, n)).ravel()
    N = mesh.coords.shape[0]
    K = sp.csr_matrix((Ke.ravel(), (rows, cols)), shape=(N, N))
    M = sp.csr_matrix((Me.ravel(), (rows, cols)), shape=(N, N))
    tr = cells.ravel()
    tc = np.repeat(np.arange(cells.shape[0]), n)
    tv = np.repeat(vol / n, n)
    T = sp.csr_matrix((tv, (tr, tc)), shape=(N, cells.shape[0]))
    return K, M, T


def smooth(mesh: Mesh, r: float, psi: np.ndarray, mats=None) -> np.ndarray:
    """The PDE filter F applied to a cellwise field psi: the cell means of
    the P1 solution of (r^2 K + M) x = T psi."""
    K, M, T = matrices(mesh) if mats is None else mats
    A = (r * r * K + M).tocsc()
    x = spla.spsolve(A, T @ np.asarray(psi, dtype=np.float64))
    return x[mesh.cells].mean(axis=1)


def sensitivity_filter(mesh: Mesh, rmin: float, rho, s, mats=None) -> np.ndarray:
    """s~ = F(rho s) / rho with r = radius(rmin)."""
    rho = np.asarray(rho, dtype=np.float64)
    return smooth(mesh, radius(rmin), rho * np.asarray(s, dtype=np.float64), mats) / rho
