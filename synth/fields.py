"""Seeded density fields and vectors (no method arithmetic)."""

from __future__ import annotations

import numpy as np


def rho_uniform(n_cells: int, volfrac: float) -> np.ndarray:
    """Iteration-0 density: every cell at the volume fraction."""
    return np.full(int(n_cells), float(volfrac))


def rho_random(seed: int, n_cells: int, lo: float = 1e-3, hi: float = 1.0) -> np.ndarray:
    """i.i.d. U[lo, hi] densities: a numerical stress case for the solvers."""
    rng = np.random.default_rng(seed)
    return rng.uniform(lo, hi, int(n_cells))


def rho_smooth(seed: int, n_cells: int, lo: float = 1e-3, sharp: float = 8.0,
               fill: float = 0.5) -> np.ndarray:
    """A 0/1-contrast field shaped like a mid-run SIMP design: a smoothed
    random walk over the cell index, pushed through a steep logistic so that
    roughly ``fill`` of the cells are near 1 and the rest near ``lo``."""
    rng = np.random.default_rng(seed)
    w = np.cumsum(rng.standard_normal(int(n_cells)))
    k = max(1, int(n_cells) // 64)
    kern = np.ones(k) / k
    w = np.convolve(w, kern, mode="same")
    w = (w - np.quantile(w, 1.0 - fill)) / (np.std(w) + 1e-30)
    s = 1.0 / (1.0 + np.exp(-sharp * w))
    return lo + (1.0 - lo) * s


def vec_random(seed: int, shape, fixed: np.ndarray | None = None) -> np.ndarray:
    """N(0, 1) nodal vector ``[nrhs][dim][N_n]``, zero on fixed DOFs."""
    rng = np.random.default_rng(seed)
    x = rng.standard_normal(shape)
    if fixed is not None:
        x = x * (fixed[None] == 0) if x.ndim == 3 else x * (fixed == 0)
    return np.ascontiguousarray(x)
