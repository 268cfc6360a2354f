"""Seeded cell-midpoint clouds that stand in for unstructured meshes.

The paper's filter works on any mesh through the midpoints of its cells
(Sec. 3.2.2, Sec. 6.1); its unstructured examples (the bridge and the
ground structures) are imported meshes that are not available here.  These
clouds have the spacing, count and irregularity of such meshes: one point
per simplex at the positions the simplices of a structured split would
have, each moved by an independent seeded uniform jitter, with cells
inside seeded holes removed (the "complex ground structure" of Sec. 6.1).
No filter arithmetic happens here: the points are the filter's input.

Layout: ``mid[c, a]`` is coordinate c of point a (float64, SoA, C order).
"""

from __future__ import annotations

import itertools

import numpy as np

# in-cube offsets of the six 3D points (one per axis permutation: the
# coordinate along the permutation's first axis is 3/4, second 1/2, third
# 1/4) and of the two 2D points (one per triangle of a square)
_OFF3 = np.array([[0.0] * 3 for _ in range(6)])
for _t, _p in enumerate(itertools.permutations(range(3))):
    for _r, _ax in enumerate(_p):
        _OFF3[_t, _ax] = (3 - _r) / 4.0
_OFF2 = np.array([[2.0 / 3.0, 1.0 / 3.0], [1.0 / 3.0, 2.0 / 3.0]])


def _holes(rng, mid, extent, count, rlo, rhi):
    keep = np.ones(mid.shape[1], dtype=bool)
    dim = mid.shape[0]
    for _ in range(count):
        c = rng.uniform(0.0, 1.0, dim) * extent
        r = rng.uniform(rlo, rhi) * float(min(extent))
        d2 = np.zeros(mid.shape[1])
        for a in range(dim):
            d2 += (mid[a] - c[a]) ** 2
        keep &= d2 >= r * r
    return np.ascontiguousarray(mid[:, keep])


def cloud(nel, seed: int, jitter: float = 0.2, holes: int = 0, rlo: float = 0.08,
          rhi: float = 0.16, origin=None) -> np.ndarray:
    """Midpoint cloud over ``nel`` unit cells (2 points per square in 2D,
    6 per cube in 3D), x-fastest cell order, each point moved by
    U[-jitter, jitter] per coordinate, then ``holes`` spherical voids of
    radius U[rlo, rhi] times the shortest side removed.  ``origin`` shifts
    every point (checks hashing of negative and large coordinates)."""
    nel = tuple(int(v) for v in nel)
    dim = len(nel)
    rng = np.random.default_rng(seed)
    off = _OFF2 if dim == 2 else _OFF3
    grids = np.meshgrid(*[np.arange(n, dtype=np.float64) for n in reversed(nel)], indexing="ij")
    base = np.stack([g.ravel() for g in reversed(grids)])            # [dim, cells], x fastest
    mid = (base[:, :, None] + off.T[:, None, :]).reshape(dim, -1)    # point = cell * k + t
    mid = mid + rng.uniform(-jitter, jitter, mid.shape)
    if holes:
        mid = _holes(rng, mid, np.array(nel, dtype=np.float64), holes, rlo, rhi)
    if origin is not None:
        mid = mid + np.asarray(origin, dtype=np.float64)[:, None]
    return np.ascontiguousarray(mid)
