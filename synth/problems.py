"""Problem definitions: grid sizes, parameters, Dirichlet masks and nodal loads.

The workloads follow the paper's cantilever family (two-dimensional
cantilever with a tip load, Section 4; three-dimensional cantilever,
Section 5.1; two load cases summed, Section 5.3) at the sizes of the
benchmark configurations, plus closed-form bar problems used as pins.

Loads are nodal vectors built with consistent P1 lumping:

* a point load at a non-nodal position along an edge is split linearly
  between the two nodes of the unit segment that holds it;
* a line load of intensity q along a row of unit segments puts q on each
  interior node and q/2 on the two end nodes;
* a uniform face traction q on a face of the three-dimensional grid is
  lumped over the boundary triangles of the Kuhn split, whose diagonal in
  each unit square of a face x = const runs from (y, z) to (y+1, z+1):
  every boundary triangle (area 1/2) gives q/6 to each of its vertices.
"""

from __future__ import annotations

import dataclasses
from typing import List, Sequence

import numpy as np

SPLIT_ALT_ROWS = 0
SPLIT_UNIFORM = 1


def n_nodes(nel: Sequence[int]) -> int:
    out = 1
    for n in nel:
        out *= int(n) + 1
    return out


def n_cells(nel: Sequence[int]) -> int:
    out = 1
    for n in nel:
        out *= int(n)
    return out * (2 if len(nel) == 2 else 6)


def node_id(nel: Sequence[int], i, j, k=0):
    nx, ny = int(nel[0]), int(nel[1])
    return (np.asarray(k) * (ny + 1) + np.asarray(j)) * (nx + 1) + np.asarray(i)


@dataclasses.dataclass
class Problem:
    """One SIMP problem on a structured simplex grid.

    ``fixed`` is uint8 ``[dim][N_n]``; ``loads`` is float64
    ``[nrhs][dim][N_n]``.  Parameters follow the paper's notation: penal p,
    volume fraction k (``volfrac``), filter radius rmin, OC move limit m and
    damping eta, density lower bound ``rho_min``.
    """

    name: str
    dim: int
    nel: tuple
    split: int
    fixed: np.ndarray
    loads: np.ndarray
    E0: float = 1.0
    Emin: float = 1e-9
    nu: float = 0.3
    penal: float = 3.0
    volfrac: float = 0.5
    rmin: float = 1.5
    move: float = 0.2
    eta: float = 0.5
    rho_min: float = 1e-3
    paper_mode: bool = False
    rtol: float = 1e-10
    n_iter: int = 50
    passive: object = None   # None, or uint8 [N_c]: 0 free, 1 void, 2 solid
    filter: int = 0          # 0: distance-weighted filter, 1: Helmholtz PDE filter

    @property
    def nrhs(self) -> int:
        return int(self.loads.shape[0])

    @property
    def n_nodes(self) -> int:
        return n_nodes(self.nel)

    @property
    def n_cells(self) -> int:
        return n_cells(self.nel)

    @property
    def n_dofs(self) -> int:
        return self.dim * self.n_nodes

    def with_loads(self, loads: np.ndarray) -> "Problem":
        return dataclasses.replace(self, loads=np.ascontiguousarray(loads, dtype=np.float64))


def _edge_point_load(nel, fixed_axis_val, along_axis, pos, comp, value, dim):
    """Lump a point load at fractional position ``pos`` along a grid line."""
    f = np.zeros((dim, n_nodes(nel)))
    lo = int(np.floor(pos))
    hi_lim = nel[along_axis]
    lo = min(max(lo, 0), hi_lim)
    frac = pos - lo
    if lo == hi_lim:
        frac = 0.0
    idx = [0, 0, 0]
    for ax, v in fixed_axis_val.items():
        idx[ax] = v
    idx[along_axis] = lo
    f[comp, node_id(nel, *idx[:max(dim, 2)])] += value * (1.0 - frac)
    if frac > 0.0:
        idx[along_axis] = lo + 1
        f[comp, node_id(nel, *idx[:max(dim, 2)])] += value * frac
    return f


def cantilever2d(nelx=60, nely=30, volfrac=0.5, rmin=1.5, load_pos=None,
                 split=SPLIT_ALT_ROWS, n_iter=50, rtol=1e-10, **kw) -> Problem:
    """Left edge clamped, unit downward point load on the right edge.

    ``load_pos`` is the load height as a fraction of ``nely`` (default 0.5,
    the right-edge midpoint)."""
    nel = (int(nelx), int(nely))
    N = n_nodes(nel)
    fixed = np.zeros((2, N), np.uint8)
    j = np.arange(nely + 1)
    fixed[:, node_id(nel, 0, j)] = 1
    pos = 0.5 * nely if load_pos is None else float(load_pos) * nely
    f = _edge_point_load(nel, {0: nelx}, 1, pos, 1, -1.0, 2)
    return Problem("cantilever2d", 2, nel, split, fixed, f[None].copy(),
                   volfrac=volfrac, rmin=rmin, n_iter=n_iter, rtol=rtol, **kw)


def cantilever2d_hole(nelx=180, nely=60, volfrac=0.5, rmin=3.0, **kw) -> Problem:
    """The cantilever of ``cantilever2d`` with a circular hole of passive void
    cells (Section 5.4's example: centre (nelx/3, nely/2), radius nely/4, at
    180 x 60, volfrac 0.5, rmin 3).  A cell is passive when all four corners
    of its unit square lie in the closed disc, so both triangles of a square
    share the mark."""
    p = cantilever2d(nelx, nely, volfrac=volfrac, rmin=rmin, **kw)
    x0, y0, r = nelx / 3.0, nely / 2.0, nely / 4.0
    i = np.arange(nelx)[None, :]
    j = np.arange(nely)[:, None]
    inside = np.ones((nely, nelx), bool)
    for di in (0, 1):
        for dj in (0, 1):
            inside &= (i + di - x0) ** 2 + (j + dj - y0) ** 2 <= r * r
    p.passive = np.repeat(inside.reshape(-1).astype(np.uint8), 2)   # cells 2s, 2s + 1
    p.name = "cantilever2d_hole"
    return p


def propped_cantilever2d(nelx=180, nely=60, volfrac=0.5, rmin=3.0, **kw) -> Problem:
    """The cantilever of ``cantilever2d`` with a prop: u_y = 0 at the single
    node (nelx, 0) (Section 5.2's pointwise support)."""
    p = cantilever2d(nelx, nely, volfrac=volfrac, rmin=rmin, **kw)
    p.fixed[1, node_id(p.nel, nelx, 0)] = 1
    p.name = "propped_cantilever2d"
    return p


def mbb2d(nelx=1200, nely=400, volfrac=0.4, rmin=3.0, split=SPLIT_UNIFORM,
          n_iter=100, rtol=1e-8, **kw) -> Problem:
    """MBB half-beam: symmetry rollers (u_x = 0) on the left edge, a roller
    (u_y = 0) at the bottom-right corner, unit downward load at the top-left."""
    nel = (int(nelx), int(nely))
    N = n_nodes(nel)
    fixed = np.zeros((2, N), np.uint8)
    fixed[0, node_id(nel, 0, np.arange(nely + 1))] = 1
    fixed[1, node_id(nel, nelx, 0)] = 1
    f = np.zeros((1, 2, N))
    f[0, 1, node_id(nel, 0, nely)] = -1.0
    return Problem("mbb2d", 2, nel, split, fixed, f, volfrac=volfrac, rmin=rmin,
                   n_iter=n_iter, rtol=rtol, **kw)


def _line_load_z(nel, i, j, comp, q):
    """Line load of intensity q along the z-directed grid line (i, j, *)."""
    nz = nel[2]
    f = np.zeros((3, n_nodes(nel)))
    k = np.arange(nz + 1)
    w = np.full(nz + 1, q)
    w[0] *= 0.5
    w[-1] *= 0.5
    f[comp, node_id(nel, i, j, k)] = w
    return f


def cantilever3d(nelx=192, nely=96, nelz=96, nrhs=4, volfrac=0.3, rmin=2.5,
                 n_iter=50, rtol=1e-8, **kw) -> Problem:
    """Face x = 0 clamped; up to four unit line-load cases on the x = L face:

    1. (0, -1, 0) along the bottom edge {x = L, y = 0};
    2. (0, +1, 0) along the top edge {x = L, y = H};
    3. (0, 0, +1) along the bottom edge (z-shear);
    4. (0, 0, -1) along the top edge (z-shear).
    """
    nel = (int(nelx), int(nely), int(nelz))
    N = n_nodes(nel)
    fixed = np.zeros((3, N), np.uint8)
    jj, kk = np.meshgrid(np.arange(nely + 1), np.arange(nelz + 1), indexing="ij")
    fixed[:, node_id(nel, 0, jj.ravel(), kk.ravel())] = 1
    cases = [
        _line_load_z(nel, nelx, 0, 1, -1.0),
        _line_load_z(nel, nelx, nely, 1, +1.0),
        _line_load_z(nel, nelx, 0, 2, +1.0),
        _line_load_z(nel, nelx, nely, 2, -1.0),
    ]
    if not 1 <= nrhs <= 4:
        raise ValueError("nrhs must be 1..4")
    f = np.stack(cases[:nrhs])
    return Problem("cantilever3d", 3, nel, SPLIT_UNIFORM, fixed, f, volfrac=volfrac,
                   rmin=rmin, n_iter=n_iter, rtol=rtol, **kw)


def learned3d(nelx=128, nely=64, nelz=64, **kw) -> Problem:
    """Cantilever of the learned-preconditioner workload: load case 1 only."""
    kw.setdefault("volfrac", 0.3)
    kw.setdefault("rmin", 2.5)
    p = cantilever3d(nelx, nely, nelz, nrhs=1, **kw)
    p.name = "learned3d"
    return p


def bar2d(nelx=8, nely=4, q=1.0, split=SPLIT_ALT_ROWS, **kw) -> Problem:
    """Plane-stress bar: u_x = 0 on x = 0, u_y = 0 on y = 0, uniform traction
    q in +x on the edge x = L (lumped as a line load)."""
    nel = (int(nelx), int(nely))
    N = n_nodes(nel)
    fixed = np.zeros((2, N), np.uint8)
    fixed[0, node_id(nel, 0, np.arange(nely + 1))] = 1
    fixed[1, node_id(nel, np.arange(nelx + 1), 0)] = 1
    f = np.zeros((1, 2, N))
    w = np.full(nely + 1, q)
    w[0] *= 0.5
    w[-1] *= 0.5
    f[0, 0, node_id(nel, nelx, np.arange(nely + 1))] = w
    return Problem("bar2d", 2, nel, split, fixed, f, **kw)


def bar3d(nelx=6, nely=3, nelz=2, q=1.0, **kw) -> Problem:
    """3D bar: u_x = 0 on x = 0, u_y = 0 on y = 0, u_z = 0 on z = 0, uniform
    traction q in +x on the face x = L (lumped over the face triangles)."""
    nel = (int(nelx), int(nely), int(nelz))
    N = n_nodes(nel)
    fixed = np.zeros((3, N), np.uint8)
    I, J, K = np.meshgrid(np.arange(nelx + 1), np.arange(nely + 1), np.arange(nelz + 1),
                          indexing="ij")
    I, J, K = I.ravel(), J.ravel(), K.ravel()
    fixed[0, node_id(nel, I[I == 0], J[I == 0], K[I == 0])] = 1
    fixed[1, node_id(nel, I[J == 0], J[J == 0], K[J == 0])] = 1
    fixed[2, node_id(nel, I[K == 0], J[K == 0], K[K == 0])] = 1
    f = np.zeros((1, 3, N))
    for j in range(nely):
        for k in range(nelz):
            # two triangles of the unit face square, diagonal (j,k)-(j+1,k+1)
            for tri in (((j, k), (j + 1, k), (j + 1, k + 1)), ((j, k), (j, k + 1), (j + 1, k + 1))):
                for (a, b) in tri:
                    f[0, 0, node_id(nel, nelx, a, b)] += q / 6.0
    return Problem("bar3d", 3, nel, SPLIT_UNIFORM, fixed, f, **kw)


def batch2d(seed: int = 20120820, count: int = 64, nx_lo: int = 80, nx_hi: int = 640,
            **kw) -> List[Problem]:
    """Uneven batch of 2D cantilevers: nx ~ U{nx_lo..nx_hi}, ny = nx // 2, tip
    load height ~ U[0,1] * ny on the right edge, volfrac ~ U[0.3, 0.5],
    rmin ~ U[1.5, 3]; runs until max |d rho| < 0.01 (cap 2000)."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        nx = int(rng.integers(nx_lo, nx_hi + 1))
        ny = nx // 2
        pos = float(rng.uniform(0.0, 1.0))
        vf = float(rng.uniform(0.3, 0.5))
        rm = float(rng.uniform(1.5, 3.0))
        p = cantilever2d(nx, ny, volfrac=vf, rmin=rm, load_pos=pos, split=SPLIT_UNIFORM,
                         n_iter=2000, rtol=1e-8, **kw)
        p.name = "batch2d"
        out.append(p)
    return out


def describe(p: Problem) -> dict:
    return {"name": p.name, "dim": p.dim, "nel": list(p.nel), "nrhs": p.nrhs,
            "n_cells": p.n_cells, "n_dofs": p.n_dofs, "volfrac": p.volfrac,
            "rmin": p.rmin, "penal": p.penal, "split": p.split}
