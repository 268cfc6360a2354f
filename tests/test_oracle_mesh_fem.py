"""Pins for the oracle's mesh and finite-element steps.

Each check compares the oracle with something the mathematics fixes:
simplex tilings, rigid-body null spaces, the energy density of the paper's
material law (eq. str_energy) under constant strain, the patch test, the
closed-form bar solution, reciprocity and the compliance identities.
"""

import collections
import itertools

import numpy as np
import pytest

import synth
from oracle import fem, mesh as M


def _facets(cells):
    d1 = cells.shape[1]
    out = collections.Counter()
    for c in cells:
        for f in itertools.combinations(sorted(c), d1 - 1):
            out[f] += 1
    return out


@pytest.mark.parametrize("split", [M.SPLIT_ALT_ROWS, M.SPLIT_UNIFORM])
def test_2d_mesh_is_conforming_tiling(split):
    nx, ny = 5, 4
    m = M.grid2d(nx, ny, split)
    assert m.n_nodes == (nx + 1) * (ny + 1) and m.n_cells == 2 * nx * ny
    vol, _ = M.geometry(m)
    np.testing.assert_allclose(vol, 0.5, rtol=0, atol=1e-15)
    cnt = _facets(m.cells)
    assert set(cnt.values()) <= {1, 2}
    # boundary edges are exactly the perimeter's unit segments
    assert sum(v == 1 for v in cnt.values()) == 2 * (nx + ny)


def test_3d_mesh_is_conforming_tiling():
    nx, ny, nz = 3, 2, 2
    m = M.grid3d(nx, ny, nz)
    assert m.n_cells == 6 * nx * ny * nz
    vol, _ = M.geometry(m)
    np.testing.assert_allclose(vol, 1.0 / 6.0, rtol=0, atol=1e-15)
    cnt = _facets(m.cells)
    assert set(cnt.values()) <= {1, 2}
    assert sum(v == 1 for v in cnt.values()) == 2 * 2 * (nx * ny + ny * nz + nx * nz)


def test_kuhn_centroids_closed_form():
    # the Kuhn simplex of permutation pi is {1 >= q_pi1 >= q_pi2 >= q_pi3 >= 0};
    # its centroid has coordinates 3/4, 1/2, 1/4 along pi1, pi2, pi3
    m = M.grid3d(1, 1, 1)
    c = M.centroids(m)
    for t, perm in enumerate(itertools.permutations(range(3))):
        want = np.zeros(3)
        want[perm[0]], want[perm[1]], want[perm[2]] = 0.75, 0.5, 0.25
        np.testing.assert_allclose(c[t], want, atol=1e-15)


def test_alt_rows_mirror_symmetric():
    nx, ny = 6, 4
    m = M.grid2d(nx, ny, M.SPLIT_ALT_ROWS)
    c = M.centroids(m)
    mir = c.copy()
    mir[:, 1] = ny - mir[:, 1]
    a = np.round(c * 3).astype(int)
    b = np.round(mir * 3).astype(int)
    assert set(map(tuple, a)) == set(map(tuple, b))


def _rigid_modes(coords):
    d = coords.shape[1]
    modes = []
    for c in range(d):
        v = np.zeros_like(coords)
        v[:, c] = 1.0
        modes.append(v.ravel())
    axes = [(0, 1)] if d == 2 else [(0, 1), (1, 2), (0, 2)]
    for a, b in axes:
        v = np.zeros_like(coords)
        v[:, a] = -coords[:, b]
        v[:, b] = coords[:, a]
        modes.append(v.ravel())
    return np.array(modes)


@pytest.mark.parametrize("dim", [2, 3])
def test_element_matrix_null_space(dim):
    m = M.grid2d(1, 2, M.SPLIT_ALT_ROWS) if dim == 2 else M.grid3d(1, 1, 1)
    K0 = fem.element_K0(m, 0.3)
    nz = 3 if dim == 2 else 6
    for e in range(m.n_cells):
        k = K0[e]
        np.testing.assert_allclose(k, k.T, atol=1e-14)
        ev = np.linalg.eigvalsh(k)
        assert np.all(ev > -1e-13)
        assert np.sum(np.abs(ev) < 1e-12) == nz
        R = _rigid_modes(m.coords[m.cells[e]])   # node-major element DOFs
        np.testing.assert_allclose(k @ R.T, 0.0, atol=1e-13)


def _psi(eps, lam, mu):
    # Section 2, eq. str_energy: psi = lam/2 tr(eps)^2 + mu tr(eps^2)
    return 0.5 * lam * np.trace(eps) ** 2 + mu * np.trace(eps @ eps)


@pytest.mark.parametrize("dim,paper", [(2, False), (2, True), (3, False), (3, True)])
def test_constant_strain_energy_matches_paper_energy_density(dim, paper):
    nu = 0.3
    m = M.grid2d(1, 2, M.SPLIT_ALT_ROWS) if dim == 2 else M.grid3d(1, 1, 1)
    K0 = fem.element_K0(m, nu, paper)
    if paper:
        lam, mu = 0.6, 0.4
    elif dim == 2:   # plane stress at E = 1: effective lambda* = nu / (1 - nu^2)
        lam, mu = nu / (1 - nu * nu), 1.0 / (2 * (1 + nu))
    else:
        lam, mu = nu / ((1 + nu) * (1 - 2 * nu)), 1.0 / (2 * (1 + nu))
    rng = np.random.default_rng(0)
    vol, _ = M.geometry(m)
    for _ in range(5):
        A = rng.standard_normal((dim, dim))
        eps = 0.5 * (A + A.T)
        for e in range(m.n_cells):
            X = m.coords[m.cells[e]]
            ue = (X @ A.T).ravel()      # u(x) = A x at the vertices, node-major
            energy = ue @ K0[e] @ ue
            np.testing.assert_allclose(energy, 2 * vol[e] * _psi(eps, lam, mu), rtol=1e-13)


@pytest.mark.parametrize("dim", [2, 3])
def test_patch_test_interior_equilibrium(dim):
    m = M.grid2d(4, 4, M.SPLIT_ALT_ROWS) if dim == 2 else M.grid3d(3, 3, 3)
    K = fem.assemble(m, np.ones(m.n_cells), 0.3)
    rng = np.random.default_rng(1)
    A = rng.standard_normal((dim, dim))
    b = rng.standard_normal(dim)
    u = (m.coords @ A.T + b).T.ravel()   # SoA
    y = (K @ u).reshape(dim, -1)
    X = m.coords
    nel = m.nel
    interior = np.all([(X[:, a] > 0) & (X[:, a] < nel[a]) for a in range(dim)], axis=0)
    np.testing.assert_allclose(y[:, interior], 0.0, atol=1e-12)


def test_bar_closed_form_2d():
    # plane stress, E = 1: u_x = q x / E, u_y = -nu q y / E; c = q^2 L H / E
    for split in (M.SPLIT_ALT_ROWS, M.SPLIT_UNIFORM):
        p = synth.bar2d(8, 4, q=0.7, split=split)
        m = M.build(2, p.nel, p.split)
        E = fem.simp_modulus(np.ones(m.n_cells), p.E0, p.Emin, p.penal)
        K = fem.assemble(m, E, p.nu)
        f = p.loads.reshape(1, -1)
        u = fem.solve(K, f, p.fixed.ravel()).reshape(2, -1)
        np.testing.assert_allclose(u[0], 0.7 * m.coords[:, 0], atol=1e-12)
        np.testing.assert_allclose(u[1], -0.3 * 0.7 * m.coords[:, 1], atol=1e-12)
        c = fem.compliance(f, u.ravel())
        np.testing.assert_allclose(c, 0.7 ** 2 * 8 * 4, rtol=1e-12)


def test_bar_closed_form_3d():
    p = synth.bar3d(4, 3, 2, q=1.3)
    m = M.build(3, p.nel)
    K = fem.assemble(m, np.ones(m.n_cells), p.nu)
    f = p.loads.reshape(1, -1)
    np.testing.assert_allclose(f.sum(), 1.3 * 3 * 2, rtol=1e-14)   # resultant
    u = fem.solve(K, f, p.fixed.ravel()).reshape(3, -1)
    np.testing.assert_allclose(u[0], 1.3 * m.coords[:, 0], atol=1e-12)
    np.testing.assert_allclose(u[1], -0.3 * 1.3 * m.coords[:, 1], atol=1e-12)
    np.testing.assert_allclose(u[2], -0.3 * 1.3 * m.coords[:, 2], atol=1e-12)
    np.testing.assert_allclose(fem.compliance(f, u.ravel()), 1.3 ** 2 * 4 * 3 * 2, rtol=1e-12)


def test_loads_resultants():
    p = synth.cantilever2d(60, 30)
    assert p.loads.sum() == -1.0 and p.loads[0, 1, synth.node_id(p.nel, 60, 15)] == -1.0
    p = synth.cantilever2d(20, 9, load_pos=0.5)
    np.testing.assert_allclose(p.loads.sum(), -1.0)
    p = synth.cantilever3d(6, 3, 3, nrhs=4)
    np.testing.assert_allclose(p.loads.sum(axis=(1, 2)), [-3.0, 3.0, 3.0, -3.0])


@pytest.mark.parametrize("dim", [2, 3])
def test_reciprocity_and_compliance_identities(dim):
    if dim == 2:
        p = synth.cantilever2d(12, 6)
    else:
        p = synth.cantilever3d(6, 3, 3, nrhs=2)
    m = M.build(dim, p.nel, p.split)
    rho = synth.rho_random(3, m.n_cells)
    E = fem.simp_modulus(rho, p.E0, p.Emin, p.penal)
    K0 = fem.element_K0(m, p.nu)
    K = fem.assemble(m, E, p.nu, K0=K0)
    fixed = p.fixed.ravel()
    rng = np.random.default_rng(5)
    F = rng.standard_normal((2, K.shape[0])) * (fixed == 0)
    U = fem.solve(K, F, fixed)
    np.testing.assert_allclose(F[0] @ U[1], F[1] @ U[0], rtol=1e-11)
    # residual of the direct solve on free DOFs
    r = fem.apply_operator(K, U[0], fixed) - F[0]
    assert np.linalg.norm(r) <= 1e-12 * np.linalg.norm(F[0])
    # c = f^T u = u^T K u = sum_e E_e u_e^T K0_e u_e
    c = F[0] @ U[0]
    np.testing.assert_allclose(U[0] @ (K @ U[0]), c, rtol=1e-11)
    w = fem.element_energy(m, U[0], p.nu)
    np.testing.assert_allclose(np.sum(E * w), c, rtol=1e-11)


def test_matvec_ebe_matches_assembled():
    p = synth.cantilever3d(4, 2, 3, nrhs=2)
    m = M.build(3, p.nel)
    rho = synth.rho_random(7, m.n_cells)
    E = fem.simp_modulus(rho)
    K = fem.assemble(m, E, p.nu)
    x = synth.vec_random(8, (2, 3, m.n_nodes)).reshape(2, -1)
    y = fem.matvec_ebe(m, E, x, p.nu, chunk=37)
    np.testing.assert_allclose(y, (K @ x.T).T, rtol=1e-13, atol=1e-13)


def test_bf16_modulus_rounding():
    """The BF16 copy of the moduli: against torch's FP32 -> BF16 conversion
    (nearest, ties to even) on FP32-exact values, which one rounding of the
    FP64 value must reproduce; and hand cases where rounding through FP32
    first would differ (double rounding), plus ties both ways."""
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(11)
    x = np.concatenate([rng.uniform(1e-9, 1.0, 4000), 10.0 ** rng.uniform(-30, 3, 4000)])
    x32 = x.astype(np.float32).astype(np.float64)
    ref = torch.from_numpy(x32.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(fem.bf16_modulus(x32), ref)
    one = 1.0
    cases = [
        (one + 2.0 ** -8, one),                            # tie, kept bit even: down
        (one + 3 * 2.0 ** -8, one + 2.0 ** -6),            # tie, kept bit odd: up
        (one + 2.0 ** -8 + 2.0 ** -40, one + 2.0 ** -7),   # above the tie only in FP64
        (one + 2.0 ** -8 - 2.0 ** -40, one),               # below the tie
        (0.75 * (1 + 2.0 ** -9), 0.75),                    # well below the tie
        (2.0 ** -30, 2.0 ** -30),                          # a power of two is exact
    ]
    for v, want in cases:
        assert fem.bf16_modulus(np.array([v]))[0] == want, v
    # the FP32 route gets the third case wrong, so one rounding is required
    v = np.float32(one + 2.0 ** -8 + 2.0 ** -40)
    assert torch.tensor([float(v)], dtype=torch.float32).to(torch.bfloat16).item() == 1.0
    # relative error at most half a BF16 ulp (2^-8 of the value)
    y = fem.bf16_modulus(x)
    assert np.all(np.abs(y - x) <= 2.0 ** -8 * np.abs(x))


def _affine_gradients(coords, cells, u_nodes):
    """Per-cell displacement gradient of the P1 field, fitted directly from
    the vertex coordinates: solve [x_v - x_0] G^T = [u_v - u_0]."""
    d = coords.shape[1]
    X = coords[cells]                       # [e, d+1, d]
    U = u_nodes[cells]                      # [e, d+1, d]
    dX = X[:, 1:, :] - X[:, :1, :]
    dU = U[:, 1:, :] - U[:, :1, :]
    Gt = np.linalg.solve(dX, dU)            # [e, d, d]: row j = d u / d x_j
    return np.transpose(Gt, (0, 2, 1))      # G[e, a, j] = d u_a / d x_j


@pytest.mark.parametrize("dim", [2, 3])
def test_paper_mode_sensitivity_is_minus_p_rho_pm1_energy_density(dim):
    """The listing's per-cell sensitivity (Sec. 3.2) is -p rho^(p-1) psi_e with
    psi the strain-energy density of eq. str_energy at the listing's Lame
    constants lambda = 0.6, mu = 0.4.  Here psi is formed independently of
    the oracle's element matrices: the strain comes from an affine fit of
    the nodal displacements on each cell's vertex coordinates, and
    psi = lambda/2 tr(eps)^2 + mu eps:eps.  The oracle's paper-mode
    sensitivity times paper_sensitivity_scale must equal it; a dropped
    factor 2|T|, the exact-derivative scale or the plane-stress law in
    place of the listing's fails by 2% (3D, whose nu = 0.3 Lame constants
    are close to the listing's) to 28% (2D) or more."""
    m = M.build(dim, (5, 4) if dim == 2 else (3, 3, 2))
    rng = np.random.default_rng(90 + dim)
    u = rng.standard_normal((dim, m.n_nodes))
    rho = rng.uniform(0.05, 1.0, m.n_cells)
    p = 3.0
    G = _affine_gradients(m.coords, m.cells, u.T)
    eps = 0.5 * (G + np.transpose(G, (0, 2, 1)))
    tr = np.trace(eps, axis1=1, axis2=2)
    psi = 0.5 * 0.6 * tr ** 2 + 0.4 * np.einsum("eij,eij->e", eps, eps)
    want = -p * rho ** (p - 1.0) * psi
    w = fem.element_energy(m, u.reshape(1, -1), 0.3, paper_mode=True)
    got = fem.sensitivity(rho, w, 1.0, 1e-9, p, paper_mode=True) * fem.paper_sensitivity_scale(m)
    np.testing.assert_allclose(got, want, rtol=1e-12)
    # the non-paper law differs: plane stress (2D) / nu = 0.3 Lame (3D)
    w_ns = fem.element_energy(m, u.reshape(1, -1), 0.3, paper_mode=False)
    got_ns = fem.sensitivity(rho, w_ns, 1.0, 1e-9, p) * fem.paper_sensitivity_scale(m)
    assert np.max(np.abs(got_ns - want) / np.abs(want)) > 0.02
    # without the scale the value is the exact derivative, 2|T| times it
    vol, _ = M.geometry(m)
    np.testing.assert_allclose(fem.sensitivity(rho, w, 1.0, 1e-9, p, paper_mode=True),
                               2.0 * vol * want, rtol=1e-12)
