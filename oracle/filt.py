"""Distance-weighted sensitivity filter (test oracle, FP64).

Section 3.2.2 (eq. filter, eq. filter_cond) and Section 4.5 (eq. filter_mat):
with cell midpoints x_a, weights W_ab = max(0, rmin - |x_a - x_b|_2) and
row sums R_a = sum_b W_ab, the filtered sensitivity is

    s~_a = (sum_b W_ab rho_b s_b) / (rho_a R_a).

The weight is zero at and beyond rmin, so "dist <= rmin" and clipping at
zero select the same pairs.  Distances are formed from direct coordinate
differences.  Cells near the domain boundary simply have fewer neighbours
(no padding), exactly as a weight matrix over the existing cells does.
"""

from __future__ import annotations

import numpy as np
import scipy.sparse as sp
from scipy.spatial import cKDTree


def weights_dense(cent: np.ndarray, rmin: float) -> np.ndarray:
    """Brute force N x N weight matrix (small meshes only)."""
    diff = cent[:, None, :] - cent[None, :, :]
    dist = np.sqrt(np.sum(diff * diff, axis=-1))
    return np.maximum(0.0, rmin - dist)


def weights_sparse(cent: np.ndarray, rmin: float, chunk: int = 1 << 16) -> sp.csr_matrix:
    """The same matrix from a k-d tree neighbour search, built in chunks of
    rows so that memory stays proportional to the number of nonzeros."""
    tree = cKDTree(cent)
    n = cent.shape[0]
    rows, cols, vals = [], [], []
    for s in range(0, n, chunk):
        idx = np.arange(s, min(n, s + chunk))
        nb = tree.query_ball_point(cent[idx], r=rmin)
        cnt = np.fromiter((len(v) for v in nb), dtype=np.int64, count=len(nb))
        r = np.repeat(idx, cnt)
        c = np.fromiter((j for v in nb for j in v), dtype=np.int64, count=int(cnt.sum()))
        d = cent[r] - cent[c]
        w = np.maximum(0.0, rmin - np.sqrt(np.sum(d * d, axis=1)))
        keep = w > 0.0
        rows.append(r[keep])
        cols.append(c[keep])
        vals.append(w[keep])
    W = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(n, n))
    return W


def row_sums(W) -> np.ndarray:
    return np.asarray(W.sum(axis=1)).ravel()


def apply(W, R, rho, s):
    """s~ = W (rho * s) / (rho * R)."""
    return (W @ (rho * s)) / (rho * R)


def apply_rows(cent: np.ndarray, rmin: float, rho, s, rows: np.ndarray, tree=None):
    """Filtered values for selected cells only (sampled checks at full size)."""
    tree = cKDTree(cent) if tree is None else tree
    out = np.empty(len(rows))
    Rout = np.empty(len(rows))
    for q, a in enumerate(rows):
        nb = np.asarray(tree.query_ball_point(cent[a], r=rmin), dtype=np.int64)
        d = cent[nb] - cent[a]
        w = np.maximum(0.0, rmin - np.sqrt(np.sum(d * d, axis=1)))
        Rout[q] = w.sum()
        out[q] = np.dot(w, rho[nb] * s[nb]) / (rho[a] * Rout[q])
    return out, Rout


# ---------------------------------------------------------------------------
# Density-filter mode (not in the paper, whose filter acts on sensitivities):
# the physics sees the filtered design x~ = W x / R.  By the chain rule the
# design gradient of a function f(x~) is W^T (df/dx~ / R), and W is
# symmetric; the volume sum x~ has gradient W^T (1 / R).


def density(W, R, x):
    """x~ = W x / R."""
    return (W @ np.asarray(x, dtype=np.float64)) / R


def density_grad(W, R, g):
    """Design gradient W^T (g / R) of a function with gradient g in x~."""
    return W.T @ (np.asarray(g, dtype=np.float64) / R)
