"""Structured P1 simplex meshes with explicit coordinates (test oracle).

Section 3.1 discretises the body with three-noded triangles (2D) or
four-noded tetrahedra (3D) and one density value per cell; Section 4.3.1
builds the 2D mesh from ``nelx x nely`` unit rectangles, each cut into two
triangles, and Section 5.1 uses a box mesh for 3D.  The paper leaves the cut
rule to the mesh generator, so this module fixes it:

* 2D, diagonal "A" joins (0,0)-(1,1) of a unit square: t=0 is
  (0,0),(1,0),(1,1) and t=1 is (0,0),(1,1),(0,1); diagonal "B" joins
  (1,0)-(0,1): t=0 is (0,0),(1,0),(0,1) and t=1 is (1,0),(1,1),(0,1).
  Split "alternating rows" uses A on even rows and B on odd rows; split
  "uniform" uses A everywhere.
* 3D, each unit cube is cut into the six Kuhn simplices: for the
  permutation pi of the axes (lexicographic order t = 0..5) the vertices
  are the cube corner v0, v1 = v0 + e_pi1, v2 = v1 + e_pi2 and the far
  corner v0 + (1,1,1).

Node numbering is x-fastest; cells are numbered 2*(square)+t or 6*(cube)+t.
Everything geometric (cell volumes, barycentric gradients, centroids) is
computed from the vertex coordinates, not from tables.
"""

from __future__ import annotations

import dataclasses
import itertools

import numpy as np

SPLIT_ALT_ROWS = 0
SPLIT_UNIFORM = 1

PERMS3 = list(itertools.permutations(range(3)))  # lexicographic order


@dataclasses.dataclass
class Mesh:
    dim: int
    nel: tuple
    coords: np.ndarray  # [N_n, dim]
    cells: np.ndarray   # [N_c, dim+1] node ids

    @property
    def n_nodes(self):
        return self.coords.shape[0]

    @property
    def n_cells(self):
        return self.cells.shape[0]


def _square_cells(i, j, nx, split):
    n00 = j * (nx + 1) + i
    n10 = n00 + 1
    n01 = n00 + (nx + 1)
    n11 = n01 + 1
    use_a = (split == SPLIT_UNIFORM) or (j % 2 == 0)
    if use_a:
        return [(n00, n10, n11), (n00, n11, n01)]
    return [(n00, n10, n01), (n10, n11, n01)]


def grid2d(nx, ny, split=SPLIT_ALT_ROWS) -> Mesh:
    ii, jj = np.meshgrid(np.arange(nx + 1), np.arange(ny + 1), indexing="xy")
    coords = np.stack([ii.ravel(), jj.ravel()], axis=1).astype(np.float64)
    cells = []
    for j in range(ny):
        for i in range(nx):
            cells.extend(_square_cells(i, j, nx, split))
    return Mesh(2, (nx, ny), coords, np.asarray(cells, dtype=np.int64).reshape(-1, 3))


def cube_cells(i, j, k, nx, ny):
    """The six Kuhn tetrahedra of unit cube (i, j, k), as node-id tuples."""
    def nid(a, b, c):
        return (c * (ny + 1) + b) * (nx + 1) + a
    out = []
    for perm in PERMS3:
        p = [i, j, k]
        verts = [nid(*p)]
        for ax in perm:
            p[ax] += 1
            verts.append(nid(*p))
        out.append(tuple(verts))
    return out


def grid3d(nx, ny, nz) -> Mesh:
    kk, jj, ii = np.meshgrid(np.arange(nz + 1), np.arange(ny + 1), np.arange(nx + 1),
                             indexing="ij")
    coords = np.stack([ii.ravel(), jj.ravel(), kk.ravel()], axis=1).astype(np.float64)
    # vectorised version of cube_cells over all cubes (same rule)
    ck, cj, ci = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    base = np.stack([ci.ravel(), cj.ravel(), ck.ravel()], axis=1)
    cells = np.empty((base.shape[0], 6, 4), dtype=np.int64)

    def nid(p):
        return (p[:, 2] * (ny + 1) + p[:, 1]) * (nx + 1) + p[:, 0]
    for t, perm in enumerate(PERMS3):
        p = base.copy()
        cells[:, t, 0] = nid(p)
        for v, ax in enumerate(perm):
            p[:, ax] += 1
            cells[:, t, v + 1] = nid(p)
    return Mesh(3, (nx, ny, nz), coords, cells.reshape(-1, 4))


def build(dim, nel, split=SPLIT_ALT_ROWS) -> Mesh:
    if dim == 2:
        return grid2d(int(nel[0]), int(nel[1]), split)
    return grid3d(int(nel[0]), int(nel[1]), int(nel[2]))


def centroids(mesh: Mesh) -> np.ndarray:
    """Vertex average of every cell (the cell midpoint used by the filter)."""
    return mesh.coords[mesh.cells].mean(axis=1)


def geometry(mesh: Mesh, cells=None):
    """Signed-volume-checked cell measures and barycentric gradients.

    Returns (vol [n], grads [n, dim+1, dim]) where grads[e, a] is the
    gradient of the P1 basis function of local vertex a, obtained by
    inverting the Jacobian of the affine map from the reference simplex.
    """
    cells = mesh.cells if cells is None else cells
    X = mesh.coords[cells]                      # [n, d+1, d]
    J = (X[:, 1:, :] - X[:, :1, :])             # rows: x_a - x_0, a = 1..d
    det = np.linalg.det(J)
    d = mesh.dim
    fact = 2.0 if d == 2 else 6.0
    vol = np.abs(det) / fact
    # grad N_a for a>=1 are the columns of J^{-1}; grad N_0 = -sum
    Jinv = np.linalg.inv(J)                      # [n, d, d]
    g = np.empty((cells.shape[0], d + 1, d))
    g[:, 1:, :] = np.transpose(Jinv, (0, 2, 1))
    g[:, 0, :] = -g[:, 1:, :].sum(axis=1)
    return vol, g
