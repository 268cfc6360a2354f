"""Seeded unstructured simplex meshes that stand in for imported meshes.

The paper runs its loop unchanged on an imported tetrahedral mesh (the
bridge of Sec. 6.1, meshed by an external generator); that mesh is not
available here.  These meshes have what such a mesh has and a grid does
not: nodes at irregular positions (so every cell has its own shape,
volume and midpoint), an irregular boundary around holes, and node and
cell numberings with no order.  They are built from a structured split
(two triangles per square, six Kuhn tetrahedra per cube), then

* every node strictly inside the box moves by an independent seeded
  U[-jitter, jitter] per coordinate (box faces stay planar, so supports and
  loads stay where the structured problem has them);
* ``holes`` spherical voids (centres and radii seeded, kept clear of the
  supported and loaded faces) remove every cell whose vertices all lie
  inside one;
* nodes no cell uses are dropped, then nodes and cells are shuffled by a
  seeded permutation (``permute``).

The problem is the cantilever family: face x = 0 clamped, unit line loads
along edges of the face x = L, lumped onto the edge nodes (q per interior
node, q/2 at the two ends).  Nothing here computes a stiffness, a strain,
a filter weight or an update: these arrays are the method's input.

Layout: ``coords[n, c]`` (float64), ``cells[e, a]`` (int64 node ids, the
vertex order of the structured split), ``fixed[c][n]`` (uint8),
``loads[r][c][n]`` (float64).
"""

from __future__ import annotations

import dataclasses
import itertools

import numpy as np


@dataclasses.dataclass
class UProblem:
    name: str
    dim: int
    coords: np.ndarray
    cells: np.ndarray
    fixed: np.ndarray
    loads: np.ndarray
    E0: float = 1.0
    Emin: float = 1e-9
    nu: float = 0.3
    penal: float = 3.0
    volfrac: float = 0.3
    rmin: float = 2.0
    move: float = 0.2
    eta: float = 0.5
    rho_min: float = 1e-3
    rtol: float = 1e-10
    paper_mode: bool = False

    @property
    def nrhs(self) -> int:
        return int(self.loads.shape[0])

    @property
    def n_nodes(self) -> int:
        return int(self.coords.shape[0])

    @property
    def n_cells(self) -> int:
        return int(self.cells.shape[0])

    @property
    def n_dofs(self) -> int:
        return self.dim * self.n_nodes


def _grid(nel):
    """Nodes (x-fastest) and cells of the structured split, in the cell
    order and vertex order of the structured library convention (2D: the
    uniform diagonal split; 3D: six Kuhn tetrahedra per cube)."""
    dim = len(nel)
    axes = [np.arange(n + 1, dtype=np.float64) for n in nel]
    g = np.meshgrid(*reversed(axes), indexing="ij")
    coords = np.stack([a.ravel() for a in reversed(g)], axis=1)
    nx, ny = nel[0], nel[1]
    if dim == 2:
        j, i = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
        n00 = (j * (nx + 1) + i).ravel()
        n10, n01 = n00 + 1, n00 + nx + 1
        n11 = n01 + 1
        cells = np.stack([np.stack([n00, n10, n11], 1), np.stack([n00, n11, n01], 1)], 1)
        return coords, cells.reshape(-1, 3)
    nz = nel[2]
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    base = np.stack([i.ravel(), j.ravel(), k.ravel()], 1)
    cells = np.empty((base.shape[0], 6, 4), dtype=np.int64)
    for t, perm in enumerate(itertools.permutations(range(3))):
        p = base.copy()
        cells[:, t, 0] = (p[:, 2] * (ny + 1) + p[:, 1]) * (nx + 1) + p[:, 0]
        for v, ax in enumerate(perm):
            p[:, ax] += 1
            cells[:, t, v + 1] = (p[:, 2] * (ny + 1) + p[:, 1]) * (nx + 1) + p[:, 0]
    return coords, cells.reshape(-1, 4)


def _edge_load(coords, at, comp, q):
    """Line load q along the edge {x_a = at[a] for every a in at}: q on
    interior edge nodes, q/2 on the two end nodes (unit node spacing)."""
    on = np.ones(coords.shape[0], dtype=bool)
    for a, v in at.items():
        on &= coords[:, a] == v
    idx = np.flatnonzero(on)
    free_axis = [a for a in range(coords.shape[1]) if a not in at][0]
    t = coords[idx, free_axis]
    w = np.full(idx.size, q)
    w[t == t.min()] *= 0.5
    w[t == t.max()] *= 0.5
    f = np.zeros((coords.shape[1], coords.shape[0]))
    f[comp, idx] = w
    return f


def jittered_cantilever(nel, nrhs: int = 1, seed: int = 2012, jitter: float = 0.15,
                        holes: int = 0, rlo: float = 0.12, rhi: float = 0.2,
                        permute: bool = True, **params) -> UProblem:
    """Cantilever on a jittered, holed, shuffled simplex mesh over ``nel``
    unit cells (2D or 3D), face x = 0 clamped.  3D load cases (as the
    structured cantilever): (0,-1,0) along {x=L, y=0}, (0,+1,0) along
    {x=L, y=H}, (0,0,+1) along {x=L, y=0}, (0,0,-1) along {x=L, y=H}.
    2D load cases: unit point loads (0,-1) at (L, 0) and (0,+1) at (L, H)."""
    nel = tuple(int(v) for v in nel)
    dim = len(nel)
    rng = np.random.default_rng(seed)
    coords, cells = _grid(nel)
    ext = np.array(nel, dtype=np.float64)
    inner = np.all((coords > 0) & (coords < ext), axis=1)
    coords = coords.copy()
    coords[inner] += rng.uniform(-jitter, jitter, (int(inner.sum()), dim))
    if holes:
        keep = np.ones(cells.shape[0], dtype=bool)
        for _ in range(holes):
            c = rng.uniform(0.25, 0.75, dim) * ext
            r = rng.uniform(rlo, rhi) * float(ext.min())
            inside = np.sum((coords - c) ** 2, axis=1) <= r * r
            keep &= ~np.all(inside[cells], axis=1)
        cells = cells[keep]
    used = np.zeros(coords.shape[0], dtype=bool)
    used[cells.ravel()] = True
    new_id = np.cumsum(used) - 1
    coords = coords[used]
    cells = new_id[cells]
    if permute:
        pn = rng.permutation(coords.shape[0])          # new position of old node i
        inv = np.empty_like(pn)
        inv[pn] = np.arange(pn.size)
        coords = coords[inv]
        cells = pn[cells]
        cells = cells[rng.permutation(cells.shape[0])]
    N = coords.shape[0]
    fixed = np.zeros((dim, N), np.uint8)
    fixed[:, coords[:, 0] == 0.0] = 1
    L, H = ext[0], ext[1]
    if dim == 3:
        cases = [_edge_load(coords, {0: L, 1: 0.0}, 1, -1.0),
                 _edge_load(coords, {0: L, 1: H}, 1, +1.0),
                 _edge_load(coords, {0: L, 1: 0.0}, 2, +1.0),
                 _edge_load(coords, {0: L, 1: H}, 2, -1.0)]
    else:
        cases = []
        for y, s in ((0.0, -1.0), (H, +1.0)):
            f = np.zeros((2, N))
            f[1, np.flatnonzero((coords[:, 0] == L) & (coords[:, 1] == y))] = s
            cases.append(f)
    if not 1 <= nrhs <= len(cases):
        raise ValueError(f"nrhs must be 1..{len(cases)}")
    loads = np.ascontiguousarray(np.stack(cases[:nrhs]))
    return UProblem("jittered_cantilever", dim, np.ascontiguousarray(coords),
                    np.ascontiguousarray(cells, dtype=np.int64), fixed, loads, **params)


def from_structured(p) -> UProblem:
    """A structured-grid problem (synth.problems.Problem with the uniform
    2D split or in 3D) given as unstructured data: the same nodes, cells,
    supports and loads, in the structured numbering."""
    coords, cells = _grid(tuple(int(v) for v in p.nel))
    keys = ("E0", "Emin", "nu", "penal", "volfrac", "rmin", "move", "eta", "rho_min", "rtol")
    return UProblem(p.name + "_as_unstructured", p.dim, coords, cells,
                    np.ascontiguousarray(p.fixed), np.ascontiguousarray(p.loads),
                    **{k: getattr(p, k) for k in keys})
