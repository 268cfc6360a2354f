"""Pins of the unstructured-mesh oracle (oracle/umesh.py) to what the paper
and the mathematics fix, on jittered, holed, shuffled simplex meshes
(synth/umesh.py):

* patch test: an affine displacement gives every cell the strain sym(A)
  exactly and zero force at every interior node (P1 reproduces linear
  fields on any mesh, Sec. 3.1);
* each element matrix has the rigid motions (3 in 2D, 6 in 3D) as its
  exact kernel, on cells of arbitrary shape;
* the sensitivity is the derivative of the compliance: complex-step
  derivative on a tiny jittered mesh (Sec. 3.2);
* on a grid (no jitter, no holes, no shuffling) the per-volume sensitivity
  and the cell-count volume reduce to the structured oracle's exact
  derivative and volume, so the two loops give the same trajectory
  (equal cell volumes: the filter is linear and the OC step is invariant
  to scaling the sensitivity);
* the midpoint weights equal the brute-force pairwise distances;
* the OC volume is met by cell count to 1e-12 N_c every iteration.
"""

import numpy as np
import pytest

import synth
from oracle import fem, filt, mesh as M, simp, umesh


def _mesh(p):
    return M.Mesh(p.dim, None, p.coords, p.cells)


@pytest.mark.parametrize("dim", [2, 3])
def test_patch_test_on_jittered_holed_mesh(dim):
    nel = (10, 6) if dim == 2 else (7, 4, 4)
    p = synth.jittered_cantilever(nel, seed=5, holes=1, jitter=0.2)
    m = _mesh(p)
    rng = np.random.default_rng(6)
    A = rng.normal(size=(dim, dim))
    b = rng.normal(size=dim)
    u = (p.coords @ A.T + b).T.reshape(-1)             # [dim][N]
    vol, g = M.geometry(m)
    eps = np.einsum("eaj,eai->eij", g, u.reshape(dim, -1).T[p.cells])
    np.testing.assert_allclose(eps, np.broadcast_to(A, eps.shape), atol=1e-12)
    K = fem.assemble(m, np.full(m.n_cells, 0.7), p.nu)   # one material throughout
    r = (K @ u).reshape(dim, -1)
    ext = np.array(nel, dtype=float)
    inner = np.all((p.coords > 1e-9) & (p.coords < ext - 1e-9), axis=1)
    # nodes on a hole's rim are boundary nodes too: keep the nodes whose
    # every incident cell is present (full star) by comparing with the
    # unholed mesh's incidence counts
    full = synth.jittered_cantilever(nel, seed=5, holes=0, jitter=0.2)
    cnt = np.bincount(p.cells.ravel(), minlength=p.n_nodes)
    cnt_full = np.bincount(full.cells.ravel(), minlength=full.n_nodes)
    interior_count = cnt_full[np.all((full.coords > 0) & (full.coords < ext), axis=1)].max()
    star = cnt == interior_count
    sel = inner & star
    assert sel.sum() > 10
    assert np.max(np.abs(r[:, sel])) <= 1e-11 * np.max(np.abs(K @ u) + 1.0)


@pytest.mark.parametrize("dim", [2, 3])
def test_element_kernels_are_the_rigid_motions(dim):
    nel = (6, 4) if dim == 2 else (4, 3, 3)
    p = synth.jittered_cantilever(nel, seed=8, jitter=0.2)
    m = _mesh(p)
    K0 = fem.element_K0(m, p.nu)
    nz = 3 if dim == 2 else 6
    for e in range(0, m.n_cells, max(1, m.n_cells // 17)):
        w = np.linalg.eigvalsh(K0[e])
        assert np.all(w[:nz] <= 1e-12 * w[-1]) and w[nz] > 1e-6 * w[-1]


def test_sensitivity_is_the_complex_step_derivative_on_a_jittered_mesh():
    p = synth.jittered_cantilever((4, 3, 2), nrhs=2, seed=9, jitter=0.2)
    S = umesh.setup(p)
    rho = synth.rho_random(10, S.mesh.n_cells, 0.2, 1.0)
    u, c, w, dc, s, E = umesh.solve_state(S, rho)
    h = 1e-30
    for e in (0, 7, S.mesh.n_cells // 2, S.mesh.n_cells - 1):
        rc = rho.astype(complex)
        rc[e] += 1j * h
        Ec = fem.simp_modulus(rc, p.E0, p.Emin, p.penal)
        K = fem.assemble(S.mesh, Ec, p.nu, False, S.K0)
        uc = fem.solve(K, S.f, S.fixed_flat)
        cs = np.sum(S.f * uc).imag / h
        assert abs(cs - dc[e]) <= 1e-10 * abs(dc[e])
    np.testing.assert_allclose(s, dc / S.vol, rtol=0)
    assert np.all(dc <= 0)


def test_grid_as_unstructured_data_gives_the_structured_trajectory():
    p3 = synth.cantilever3d(10, 5, 5, nrhs=2, volfrac=0.3, rmin=1.5)
    pu = synth.from_structured(p3)
    ref_rho, ref_log = simp.iterate(simp.setup(p3), 12)
    rho, log = umesh.iterate(umesh.setup(pu), 12)
    c_ref = np.array([r["c"] for r in ref_log])
    c = np.array([r["c"] for r in log])
    np.testing.assert_allclose(c, c_ref, rtol=1e-12)
    assert np.max(np.abs(rho - ref_rho)) <= 1e-10


def test_midpoint_weights_equal_brute_force_and_volume_counts_cells():
    p = synth.jittered_cantilever((8, 5, 4), nrhs=1, seed=11, holes=1, jitter=0.2, rmin=1.7,
                                  volfrac=0.35)
    S = umesh.setup(p)
    Wd = filt.weights_dense(M.centroids(S.mesh), p.rmin)
    np.testing.assert_allclose(S.W.toarray(), Wd, atol=1e-14)
    rho, log = umesh.iterate(S, 6)
    N = S.mesh.n_cells
    for r in log:
        assert abs(r["vol"] * N - p.volfrac * N) <= 1e-12 * N
    assert abs(rho.sum() - p.volfrac * N) <= 1e-12 * N
