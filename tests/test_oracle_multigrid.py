"""Pins of the Galerkin coarse operator that the geometric multigrid
preconditioner stores (the coarse moduli of each level), written with the
oracle's assembly on explicit meshes only:

* prolongation P is the coarse P1 function evaluated at the fine nodes
  (barycentric coordinates in the containing coarse Kuhn simplex);
* the Galerkin operator P^T K_f P equals the coarse P1 operator on cells of
  twice the size whose moduli are the means of their children's moduli
  (the nested Kuhn split, Sec. 3.1; fine cells outside an odd-sized grid
  count as void);
* on unit cells that operator needs moduli of 2x the children's mean in 3D
  and 1x in 2D: a P1 element matrix scales as h^(dim-2) (Sec. 3.1, eq.
  fe_form: cell measure times squared gradients).

The multigrid kernels run every level on unit cells, so these fix the
factor their 3D coarse moduli carry.
"""

import itertools

import numpy as np
import pytest

from oracle import fem, mesh as M

NU = 0.3


def _scaled(m, h):
    return M.Mesh(m.dim, m.nel, m.coords * h, m.cells)


def _prolongation(fine, coarse_nel, dim):
    """P[fine dof, coarse dof]: the coarse P1 function at each fine node."""
    if dim == 3:
        ncx, ncy, ncz = coarse_nel
        nid = lambda i, j, k: (k * (ncy + 1) + j) * (ncx + 1) + i   # noqa: E731
        ext = np.array([ncx, ncy, ncz])
    else:
        ncx, ncy = coarse_nel
        nid = lambda i, j: j * (ncx + 1) + i                         # noqa: E731
        ext = np.array([ncx, ncy])
    n_c = int(np.prod(ext + 1))
    P1 = np.zeros((fine.n_nodes, n_c))
    for f, x in enumerate(fine.coords):
        y = x / 2.0
        base = np.minimum(np.floor(y).astype(int), ext - 1)
        t = y - base
        # Kuhn simplex {t_p0 >= t_p1 (>= t_p2)}: walk the sorted axes
        order = np.argsort(-t, kind="stable")
        p = base.copy()
        ts = np.concatenate(([1.0], t[order], [0.0]))
        for v in range(dim + 1):
            w = ts[v] - ts[v + 1]
            if w != 0.0:
                P1[f, nid(*p)] += w
            if v < dim:
                p[order[v]] += 1
    # vector P1: the same weights for every component (SoA dofs)
    return np.kron(np.eye(dim), P1)


def _coarse_moduli(fine, coarse, E_f):
    """Mean of the children's moduli per coarse cell (void children: 0);
    coarse is given in fine-grid coordinates."""
    dim = fine.dim
    cen_c = M.centroids(coarse)
    cen_f = M.centroids(fine)
    E_c = np.zeros(coarse.n_cells)
    nkids = 8 if dim == 3 else 4
    # locate each fine cell in a coarse cell by barycentric containment
    X = coarse.coords[coarse.cells]
    J = X[:, 1:, :] - X[:, :1, :]
    Jinv = np.linalg.inv(J)
    for e, y in enumerate(cen_f):
        near = np.argsort(np.sum((cen_c - y) ** 2, axis=1))[:12]
        for c in near:
            lam = (y - X[c, 0]) @ Jinv[c]
            if np.all(lam >= -1e-12) and lam.sum() <= 1 + 1e-12:
                E_c[c] += E_f[e] / nkids
                break
        else:
            raise AssertionError("fine cell not inside any coarse cell")
    return E_c


CASES = [(3, (4, 2, 2)), (3, (3, 3, 1)), (2, (6, 4)), (2, (5, 3))]


@pytest.mark.parametrize("dim,nel_f", CASES)
def test_galerkin_operator_is_the_coarse_p1_operator_on_doubled_cells(dim, nel_f):
    rng = np.random.default_rng(3 + sum(nel_f))
    split = M.SPLIT_UNIFORM
    fine = M.build(dim, nel_f, split)
    nel_c = tuple((n + 1) // 2 for n in nel_f)
    coarse = M.build(dim, nel_c, split)
    E_f = rng.uniform(0.05, 1.0, fine.n_cells)
    E_c = _coarse_moduli(fine, _scaled(coarse, 2.0), E_f)
    assert np.isclose(E_c.sum(), E_f.sum() / (8 if dim == 3 else 4))
    P = _prolongation(fine, nel_c, dim)
    # P reproduces the coarse linear functions exactly at the fine nodes
    a = rng.normal(size=dim)
    lin_c = (2.0 * coarse.coords) @ a
    np.testing.assert_allclose(P[:fine.n_nodes, :coarse.n_nodes] @ lin_c, fine.coords @ a,
                               atol=1e-13)
    K_f = fem.assemble(fine, E_f, NU).toarray()
    G = P.T @ K_f @ P
    K_2h = fem.assemble(_scaled(coarse, 2.0), E_c, NU).toarray()
    scale = np.max(np.abs(G))
    assert np.max(np.abs(G - K_2h)) <= 1e-13 * scale
    factor = 2.0 if dim == 3 else 1.0
    K_unit = fem.assemble(coarse, factor * E_c, NU).toarray()
    assert np.max(np.abs(G - K_unit)) <= 1e-13 * scale
    # and with the plain mean on unit cells the 3D operator is half of it
    if dim == 3:
        K_mean = fem.assemble(coarse, E_c, NU).toarray()
        np.testing.assert_allclose(2.0 * K_mean, G, atol=1e-13 * scale)


def test_p1_element_matrix_scales_as_h_to_dim_minus_2():
    for dim, nel in ((2, (1, 1)), (3, (1, 1, 1))):
        m = M.build(dim, nel, M.SPLIT_UNIFORM)
        for h in (0.5, 2.0, 3.0):
            K1 = fem.element_K0(m, NU)
            Kh = fem.element_K0(_scaled(m, h), NU)
            np.testing.assert_allclose(Kh, h ** (dim - 2) * K1, rtol=1e-13, atol=1e-15)


def test_kuhn_children_fill_each_coarse_simplex():
    """Every coarse Kuhn simplex holds exactly 8 fine ones (2D: 4) of total
    measure equal to its own."""
    for dim, nel in ((3, (2, 2, 2)), (2, (2, 2))):
        fine = M.build(dim, nel, M.SPLIT_UNIFORM)
        coarse = _scaled(M.build(dim, tuple(n // 2 for n in nel), M.SPLIT_UNIFORM), 2.0)
        counts = _coarse_moduli(fine, coarse, np.ones(fine.n_cells)) * (8 if dim == 3 else 4)
        np.testing.assert_allclose(counts, 8 if dim == 3 else 4)
        vol_f, _ = M.geometry(fine)
        vol_c, _ = M.geometry(coarse)
        np.testing.assert_allclose(vol_c, vol_f.sum() / coarse.n_cells)
    assert list(itertools.permutations(range(3))) == M.PERMS3
