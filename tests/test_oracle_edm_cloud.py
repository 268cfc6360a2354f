"""The oracle's distance filter on irregular midpoint clouds (unstructured
stand-ins), pinned to the Euclidean distance matrix of Sec. 4.5 computed by
scipy's pairwise-distance routine and to closed forms of eq. filter."""

import numpy as np
import pytest
from scipy.spatial.distance import cdist

from oracle import filt
from synth import clouds

CASES = [
    ((20, 10), 11, 1.5, 2, None),
    ((9, 6, 5), 12, 2.5, 2, None),
    ((8, 5, 4), 13, 1.2, 1, (-1.0e6, 3.0e5, -7.5)),
]


@pytest.mark.parametrize("nel,seed,rmin,holes,origin", CASES)
def test_sparse_weights_match_the_distance_matrix(nel, seed, rmin, holes, origin):
    mid = clouds.cloud(nel, seed, holes=holes, origin=origin)
    pts = mid.T
    W = filt.weights_sparse(pts, rmin).toarray()
    D = cdist(pts, pts)                                 # eq. EDM, library routine
    ref = np.where(D < rmin, rmin - D, 0.0)             # eq. filter_cond
    assert np.max(np.abs(W - ref)) <= 1e-12 * max(1.0, rmin)
    assert np.allclose(np.diag(W), rmin, rtol=0, atol=0)
    assert np.array_equal(W, W.T)


def test_filter_returns_s_when_rho_s_is_constant():
    """eq. filter: with rho_b s_b = c for every b, the weighted mean is c and
    s~_a = c / rho_a = s_a whatever the weights are."""
    mid = clouds.cloud((10, 6, 4), 5, holes=1)
    pts = mid.T
    W = filt.weights_sparse(pts, 2.0)
    R = filt.row_sums(W)
    rng = np.random.default_rng(3)
    rho = rng.uniform(0.05, 1.0, pts.shape[0])
    s = -2.5 / rho
    assert np.max(np.abs(filt.apply(W, R, rho, s) / s - 1.0)) <= 1e-13


def test_isolated_points_keep_their_sensitivity():
    """Below the nearest-neighbour distance W = rmin I, so s~ = s."""
    mid = clouds.cloud((6, 4), 2, jitter=0.0)
    pts = mid.T
    D = cdist(pts, pts) + np.eye(pts.shape[0]) * 1e9
    rmin = 0.5 * D.min()
    W = filt.weights_sparse(pts, rmin)
    assert W.nnz == pts.shape[0]
    rng = np.random.default_rng(4)
    rho, s = rng.uniform(0.1, 1, pts.shape[0]), rng.normal(size=pts.shape[0])
    assert np.allclose(filt.apply(W, filt.row_sums(W), rho, s), s, rtol=1e-15, atol=0)


def test_cloud_generator_is_seeded_and_shaped():
    a = clouds.cloud((7, 3, 2), 9, holes=1)
    b = clouds.cloud((7, 3, 2), 9, holes=1)
    assert np.array_equal(a, b)
    assert clouds.cloud((7, 3, 2), 9).shape == (3, 7 * 3 * 2 * 6)
    assert clouds.cloud((7, 3), 9).shape == (2, 7 * 3 * 2)
    assert a.shape[1] < 7 * 3 * 2 * 6 and a.flags.c_contiguous
