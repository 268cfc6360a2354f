"""Pins for the oracle's Helmholtz PDE filter (oracle/helm.py).

* the assembled Laplacian equals the textbook finite-difference stencils at
  interior nodes: 5-point on right-triangle meshes (either split), 7-point
  on the Kuhn split (the P1 stiffness of these meshes couples only grid
  neighbours along the axes, with weight -1, diagonal 2d);
* the element mass equals an independent degree-2-exact quadrature, and
  the mass rows sum to each node's share of the domain (1 inside);
* the filter keeps constants, conserves the integral, is self-adjoint and
  a contraction in the cell-volume inner product;
* for a very large radius it returns the domain mean, and its radius rule
  r = rmin / (2 sqrt 3) is applied by the sensitivity form.
"""

import numpy as np
import pytest

from oracle import filt, helm, mesh as M


def _interior_nodes(m):
    nel = m.nel
    X = m.coords
    inside = np.ones(X.shape[0], bool)
    for a in range(m.dim):
        inside &= (X[:, a] > 0.5) & (X[:, a] < nel[a] - 0.5)
    return np.flatnonzero(inside)


@pytest.mark.parametrize("dim,split", [(2, M.SPLIT_ALT_ROWS), (2, M.SPLIT_UNIFORM), (3, 0)])
def test_laplacian_is_fd_stencil_inside(dim, split):
    nel = (7, 6) if dim == 2 else (5, 4, 4)
    m = M.build(dim, nel, split)
    K, Mm, T = helm.matrices(m)
    K = K.tocsr()
    N = m.coords.shape[0]
    strides = [1, nel[0] + 1] + ([(nel[0] + 1) * (nel[1] + 1)] if dim == 3 else [])
    for n in _interior_nodes(m):
        row = K.getrow(n).toarray().ravel()
        want = np.zeros(N)
        want[n] = 2.0 * dim
        for s in strides:
            want[n + s] = -1.0
            want[n - s] = -1.0
        np.testing.assert_allclose(row, want, atol=1e-13)
    # the operator annihilates constants everywhere (Neumann problem)
    np.testing.assert_allclose(K @ np.ones(N), 0.0, atol=1e-13)


def _quad_mass(m):
    """Element mass from published degree-2-exact rules: the 3 edge
    midpoints with weight 1/3 (triangle), the 4-point rule with
    a = 0.5854101966249685, b = 0.1381966011250105, weight 1/4 (tetrahedron)."""
    vol, _ = M.geometry(m)
    d = m.dim
    if d == 2:
        pts = np.array([[0.5, 0.5, 0.0], [0.0, 0.5, 0.5], [0.5, 0.0, 0.5]])
        w = np.full(3, 1.0 / 3.0)
    else:
        a, b = 0.5854101966249685, 0.1381966011250105
        pts = np.full((4, 4), b) + np.eye(4) * (a - b)
        w = np.full(4, 0.25)
    # barycentric coordinates are the basis values at the points
    loc = np.einsum("q,qa,qb->ab", w, pts, pts)
    return vol[:, None, None] * loc[None]


@pytest.mark.parametrize("dim", [2, 3])
def test_mass_matches_quadrature_and_row_sums(dim):
    nel = (5, 4) if dim == 2 else (3, 3, 2)
    m = M.build(dim, nel)
    vol, _ = M.geometry(m)
    np.testing.assert_allclose(helm.mass_element(vol, dim), _quad_mass(m), rtol=1e-14)
    _, Mm, T = helm.matrices(m)
    N = m.coords.shape[0]
    rs = np.asarray(Mm.sum(axis=1)).ravel()
    # node share of the measure: the domain split among nodes by the T map
    np.testing.assert_allclose(rs, np.asarray(T.sum(axis=1)).ravel(), rtol=1e-13)
    np.testing.assert_allclose(rs[_interior_nodes(m)], 1.0, rtol=1e-13)
    np.testing.assert_allclose(rs.sum(), np.prod(nel), rtol=1e-13)
    assert N == rs.size


@pytest.mark.parametrize("dim", [2, 3])
def test_filter_constants_conservation_symmetry_contraction(dim):
    nel = (9, 6) if dim == 2 else (5, 4, 3)
    m = M.build(dim, nel)
    vol, _ = M.geometry(m)
    mats = helm.matrices(m)
    r = helm.radius(2.5)
    rng = np.random.default_rng(31 + dim)
    n = m.cells.shape[0]
    np.testing.assert_allclose(helm.smooth(m, r, np.full(n, 3.7), mats), 3.7, rtol=1e-13)
    psi = rng.standard_normal(n)
    phi = rng.standard_normal(n)
    Fpsi = helm.smooth(m, r, psi, mats)
    Fphi = helm.smooth(m, r, phi, mats)
    np.testing.assert_allclose(np.sum(vol * Fpsi), np.sum(vol * psi), rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(np.sum(vol * phi * Fpsi), np.sum(vol * Fphi * psi), rtol=1e-11)
    assert np.sum(vol * psi * Fpsi) >= 0.0
    assert np.sum(vol * Fpsi ** 2) <= np.sum(vol * psi ** 2)
    # a larger radius smooths more
    F2 = helm.smooth(m, 4 * r, psi, mats)
    assert np.sum(vol * F2 ** 2) < np.sum(vol * Fpsi ** 2)
    # a huge radius leaves the mean
    Finf = helm.smooth(m, 1e4, psi, mats)
    mean = np.sum(vol * psi) / np.sum(vol)
    np.testing.assert_allclose(Finf, mean, atol=1e-6 * np.max(np.abs(psi)))


def test_sensitivity_form_and_radius_rule():
    m = M.build(2, (8, 5))
    n = m.cells.shape[0]
    rng = np.random.default_rng(5)
    rho = rng.uniform(0.05, 1.0, n)
    s = -rng.lognormal(0.0, 1.0, n)
    got = helm.sensitivity_filter(m, 3.0, rho, s)
    want = helm.smooth(m, 3.0 / (2.0 * np.sqrt(3.0)), rho * s) / rho
    np.testing.assert_allclose(got, want, rtol=1e-13)
    # rho = 1 and a constant sensitivity are kept
    np.testing.assert_allclose(helm.sensitivity_filter(m, 3.0, np.ones(n), np.full(n, -2.0)),
                               -2.0, rtol=1e-13)
    # negative sensitivities stay negative on average (conservation of rho s)
    vol, _ = M.geometry(m)
    np.testing.assert_allclose(np.sum(vol * rho * got), np.sum(vol * rho * s), rtol=1e-12)


def test_cosine_mode_response():
    """Continuous Neumann problem: psi = cos(kappa x) with kappa = 2 pi / L
    is an eigenfunction, F psi = psi / (1 + r^2 kappa^2).  On a 64-cell strip
    the P1 filter reproduces that factor to O(h^2) (here < 1%); this pins
    the r^2 scaling of the Laplacian term and the sign of the operator."""
    L = 64
    m = M.build(2, (L, 3))
    cx = M.centroids(m)[:, 0]
    kappa = 2.0 * np.pi / L
    psi = np.cos(kappa * cx)
    for r in (2.0, 5.0):
        F = helm.smooth(m, r, psi)
        want = 1.0 / (1.0 + (r * kappa) ** 2)
        sel = np.abs(psi) > 0.5
        ratio = F[sel] / psi[sel]
        np.testing.assert_allclose(ratio, want, rtol=1e-2)


def test_loop_with_helmholtz_filter_symmetry_and_volume():
    """The 60 x 30 cantilever loop with the PDE filter: the design stays
    mirror-symmetric (mesh, loads and filter are), the volume is held, and
    the compliance falls."""
    import dataclasses
    import synth
    from oracle import simp
    p = dataclasses.replace(synth.cantilever2d(60, 30), filter=1)
    S = simp.setup(p)
    c = M.centroids(S.mesh)
    key = {tuple(np.round(x * 3).astype(int)): i for i, x in enumerate(c)}
    mir = c.copy()
    mir[:, 1] = 30 - mir[:, 1]
    perm = np.array([key[tuple(np.round(x * 3).astype(int))] for x in mir])
    rho, log = simp.iterate(S, 12)
    np.testing.assert_allclose(rho, rho[perm], atol=1e-8)
    for rec in log:
        assert abs(rec["vol"] - 0.5) <= 1e-12
    assert log[-1]["c"] < 0.6 * log[0]["c"]


def test_radius_rule_matches_the_distance_filter_second_moment():
    """The reading r = rmin / (2 sqrt 3) equates the second moment of the
    PDE filter's kernel with that of the distance filter's hat weights in
    one dimension (2 r^2 = rmin^2 / 6).  On a one-row strip, the x second
    moment of the oracle's P1 Helmholtz response to a one-square impulse
    and that of the distance filter's weights around the same square agree
    to discretisation error: 0.6% at rmin 12, shrinking about fourfold per
    doubling of rmin (second order).  A radius off by any constant factor
    (r = rmin / 2, rmin / sqrt 3, rmin / (4 sqrt 3)) fails by 30% or more."""
    gaps = []
    for rmin, L in ((12, 240), (24, 400), (48, 800)):
        m = M.build(2, (L, 1), M.SPLIT_UNIFORM)
        cen = M.centroids(m)
        vol, _ = M.geometry(m)
        i0 = L // 2
        psi = ((np.arange(m.n_cells) // 2) == i0).astype(float)
        x0 = i0 + 0.5
        F = helm.smooth(m, helm.radius(rmin), psi)
        m_helm = np.sum(vol * F * (cen[:, 0] - x0) ** 2) / np.sum(vol * F)
        W = filt.weights_sparse(cen, rmin)
        w = np.asarray(W.T @ psi).ravel()
        m_dist = np.sum(w * (cen[:, 0] - x0) ** 2) / np.sum(w)
        # both near the 1D hat's rmin^2 / 6
        assert abs(m_dist - rmin ** 2 / 6) <= 0.01 * rmin ** 2 / 6
        gaps.append(abs(m_helm - m_dist) / m_dist)
        for wrong in (rmin / 2.0, rmin / np.sqrt(3.0), rmin / (4.0 * np.sqrt(3.0))):
            Fw = helm.smooth(m, wrong, psi)
            mw = np.sum(vol * Fw * (cen[:, 0] - x0) ** 2) / np.sum(vol * Fw)
            assert abs(mw - m_dist) / m_dist > 0.3
    assert gaps[0] < 0.01
    assert gaps[1] < 0.35 * gaps[0] and gaps[2] < 0.35 * gaps[1]
