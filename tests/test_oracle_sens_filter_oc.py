"""Pins for the oracle's sensitivity, filter, OC update and loop.

* sensitivities against complex-step and central finite differences of the
  compliance (Section 3.2: sensitivity of f);
* the filter (Section 3.2.2, eq. filter / eq. filter_cond; Section 4.5,
  eq. filter_mat) against brute force, constant fields, conservation,
  the identity limit and an exact-rational lattice enumeration of the
  interior neighbourhoods;
* the OC update (Section 3.2, eq. update; Section 3.2.1) against an
  independent exact breakpoint solver and its invariants;
* the loop: mirror symmetry of the 60 x 30 cantilever and the volume held
  at every iteration.
"""

import fractions
import itertools

import numpy as np
import pytest

import synth
from oracle import fem, filt, mesh as M, oc, simp


def _compliance_of(m, K0, rho, f, fixed, p):
    E = fem.simp_modulus(rho, p.E0, p.Emin, p.penal)
    K = fem.assemble(m, E, p.nu, K0=K0)
    u = fem.solve(K, f, fixed)
    return np.sum(f * u), u


@pytest.mark.parametrize("dim", [2, 3])
def test_sensitivity_complex_step(dim):
    if dim == 2:
        p = synth.cantilever2d(4, 2)
    else:
        p = synth.cantilever3d(2, 1, 1, nrhs=2)
    m = M.build(dim, p.nel, p.split)
    K0 = fem.element_K0(m, p.nu)
    fixed = p.fixed.ravel()
    f = p.loads.reshape(p.nrhs, -1)
    rho = synth.rho_random(11, m.n_cells, 0.2, 1.0)
    c, u = _compliance_of(m, K0, rho, f, fixed, p)
    w = fem.element_energy(m, u, p.nu)
    s = fem.sensitivity(rho, w, p.E0, p.Emin, p.penal)
    h = 1e-30
    for e in range(0, m.n_cells, max(1, m.n_cells // 8)):
        rc = rho.astype(complex)
        rc[e] += 1j * h
        cc, _ = _compliance_of(m, K0, rc, f.astype(complex), fixed, p)
        np.testing.assert_allclose(s[e], cc.imag / h, rtol=1e-10)
        dh = 1e-6
        rp, rm = rho.copy(), rho.copy()
        rp[e] += dh
        rm[e] -= dh
        fd = (_compliance_of(m, K0, rp, f, fixed, p)[0] - _compliance_of(m, K0, rm, f, fixed, p)[0]) / (2 * dh)
        np.testing.assert_allclose(s[e], fd, rtol=1e-5)
    assert np.all(s <= 0)
    # sum_e rho_e s_e = -p (c - Emin sum_e w_e)
    np.testing.assert_allclose(np.sum(rho * s), -p.penal * (c - p.Emin * w.sum()), rtol=1e-12)


def _lattice_neighbourhood(dim, split, rmin):
    """Exact-rational enumeration of the interior cell neighbourhoods: for
    each cell class of a central square/cube, the count of cells whose
    centroid lies strictly within rmin and the sum of rmin - dist."""
    F = fractions.Fraction
    r2 = F(rmin).limit_denominator(1000) ** 2
    if dim == 2:
        def cls(i, j):
            a = (split == M.SPLIT_UNIFORM) or (j % 2 == 0)
            return [(F(2, 3), F(1, 3)), (F(1, 3), F(2, 3))] if a else [(F(1, 3), F(1, 3)), (F(2, 3), F(2, 3))]
        out = []
        for t in range(2):
            ca = cls(0, 0)[t]
            n, s = 0, 0.0
            reach = int(np.ceil(rmin)) + 1
            for i, j in itertools.product(range(-reach, reach + 1), repeat=2):
                for cb in cls(i, j):
                    d2 = (i + cb[0] - ca[0]) ** 2 + (j + cb[1] - ca[1]) ** 2
                    if d2 < r2:
                        n += 1
                        s += rmin - float(d2) ** 0.5
            out.append((n, s))
        return out
    cents = []
    for perm in itertools.permutations(range(3)):
        c = [F(0)] * 3
        c[perm[0]], c[perm[1]], c[perm[2]] = F(3, 4), F(1, 2), F(1, 4)
        cents.append(c)
    out = []
    for ca in cents:
        n, s = 0, 0.0
        reach = int(np.ceil(rmin)) + 1
        for off in itertools.product(range(-reach, reach + 1), repeat=3):
            for cb in cents:
                d2 = sum((off[a] + cb[a] - ca[a]) ** 2 for a in range(3))
                if d2 < r2:
                    n += 1
                    s += rmin - float(d2) ** 0.5
        out.append((n, s))
    return out


@pytest.mark.parametrize("dim,split,rmin,count,rsum", [
    (2, M.SPLIT_UNIFORM, 1.5, 17, 7.208059),
    (2, M.SPLIT_ALT_ROWS, 1.5, 14, 7.493284),
    (3, M.SPLIT_UNIFORM, 1.5, 87, None),
    (3, M.SPLIT_UNIFORM, 2.5, 405, 245.602905),
])
def test_filter_interior_rows_match_lattice(dim, split, rmin, count, rsum):
    lat = _lattice_neighbourhood(dim, split, rmin)
    if dim == 2:
        m = M.grid2d(12, 12, split)
        e0 = 2 * (6 * 12 + 6)          # square (6, 6): an even row
    else:
        m = M.grid3d(10, 10, 10)
        e0 = 6 * ((5 * 10 + 5) * 10 + 5)
    cent = M.centroids(m)
    W = filt.weights_sparse(cent, rmin)
    R = filt.row_sums(W)
    for t, (n, s) in enumerate(lat):
        row = W.getrow(e0 + t)
        assert row.nnz == n == count
        np.testing.assert_allclose(R[e0 + t], s, rtol=1e-13)
        if rsum is not None:
            np.testing.assert_allclose(R[e0 + t], rsum, atol=5e-7)


@pytest.mark.parametrize("dim", [2, 3])
def test_filter_brute_force_and_invariants(dim):
    m = M.grid2d(9, 5, M.SPLIT_ALT_ROWS) if dim == 2 else M.grid3d(4, 3, 3)
    cent = M.centroids(m)
    rmin = 1.7 if dim == 2 else 1.6
    Wd = filt.weights_dense(cent, rmin)
    Ws = filt.weights_sparse(cent, rmin, chunk=17)
    np.testing.assert_allclose(Ws.toarray(), Wd, atol=1e-15)
    np.testing.assert_allclose(Wd, Wd.T, atol=0)
    R = Wd.sum(1)
    rng = np.random.default_rng(2)
    rho = rng.uniform(0.001, 1, m.n_cells)
    s = -rng.uniform(0, 5, m.n_cells)
    sf = filt.apply(Wd, R, rho, s)
    # explicit per-cell sum
    a = 7
    want = sum(max(0.0, rmin - np.linalg.norm(cent[a] - cent[b])) * rho[b] * s[b]
               for b in range(m.n_cells)) / (rho[a] * R[a])
    np.testing.assert_allclose(sf[a], want, rtol=1e-13)
    # conservation: sum_a rho_a R_a s~_a = sum_b rho_b R_b s_b
    np.testing.assert_allclose(np.sum(rho * R * sf), np.sum(rho * R * s), rtol=1e-12)
    # constant fields are reproduced
    np.testing.assert_allclose(filt.apply(Wd, R, np.full_like(rho, 0.4), np.full_like(s, -2.5)),
                               -2.5, rtol=1e-14)
    # linear in s
    s2 = -rng.uniform(0, 5, m.n_cells)
    np.testing.assert_allclose(filt.apply(Wd, R, rho, 2 * s - 3 * s2),
                               2 * sf - 3 * filt.apply(Wd, R, rho, s2), rtol=1e-12, atol=1e-12)
    # identity limit: rmin below the smallest centroid distance
    r_id = 0.45 if dim == 2 else 0.34
    Wi = filt.weights_dense(cent, r_id)
    np.testing.assert_allclose(Wi, r_id * np.eye(m.n_cells), atol=1e-15)
    np.testing.assert_allclose(filt.apply(Wi, Wi.sum(1), rho, s), s, rtol=1e-14)


def test_filter_apply_rows_matches_matrix():
    m = M.grid3d(5, 4, 3)
    cent = M.centroids(m)
    W = filt.weights_sparse(cent, 2.5)
    R = filt.row_sums(W)
    rng = np.random.default_rng(4)
    rho = rng.uniform(0.001, 1, m.n_cells)
    s = -rng.uniform(0, 1, m.n_cells)
    rows = np.array([0, 17, 100, m.n_cells - 1])
    vals, Rr = filt.apply_rows(cent, 2.5, rho, s, rows)
    np.testing.assert_allclose(vals, filt.apply(W, R, rho, s)[rows], rtol=1e-13)
    np.testing.assert_allclose(Rr, R[rows], rtol=1e-14)


def test_oc_matches_exact_root_and_invariants():
    rng = np.random.default_rng(9)
    n = 400
    rho = rng.uniform(0.001, 1.0, n)
    sf = -rng.lognormal(0.0, 2.0, n)
    vf = 0.4
    rn, lam, vol, change, passes = oc.update(rho, sf, vf)
    assert abs(rn.sum() - vf * n) <= 1e-12 * n
    lo = np.maximum(1e-3, rho - 0.2)
    hi = np.minimum(1.0, rho + 0.2)
    assert np.all(rn >= lo) and np.all(rn <= hi)
    free = (rn > lo) & (rn < hi)
    assert free.sum() > 10
    np.testing.assert_allclose(rn[free], rho[free] * np.sqrt(-sf[free] / lam), rtol=1e-12)
    re, lam_e = oc.exact_root(rho, sf, vf)
    np.testing.assert_allclose(rn, re, rtol=0, atol=1e-12)
    np.testing.assert_allclose(lam, lam_e, rtol=1e-10)
    # invariance to positive scaling of the sensitivity (lambda scales too)
    rn2, lam2, *_ = oc.update(rho, 37.0 * sf, vf)
    np.testing.assert_allclose(rn2, rn, atol=1e-12)
    np.testing.assert_allclose(lam2, 37.0 * lam, rtol=1e-10)
    assert change == np.max(np.abs(rn - rho))


def test_oc_uniform_fixed_point_and_bracket_growth():
    n = 1000
    rho = np.full(n, 0.3)
    rn, lam, *_ = oc.update(rho, np.full(n, -4.0), 0.3)
    np.testing.assert_allclose(rn, 0.3, atol=1e-13)
    np.testing.assert_allclose(lam, 4.0, rtol=1e-12)
    # lambda* far beyond the initial bracket [0, 1e5]
    rn, lam, *_ = oc.update(rho, np.full(n, -4.0e7), 0.3)
    np.testing.assert_allclose(rn, 0.3, atol=1e-13)
    np.testing.assert_allclose(lam, 4.0e7, rtol=1e-12)


def _mirror_perm(m):
    c = M.centroids(m)
    key = {tuple(np.round(x * 3).astype(int)): i for i, x in enumerate(c)}
    ny = m.nel[1]
    mir = c.copy()
    mir[:, 1] = ny - mir[:, 1]
    return np.array([key[tuple(np.round(x * 3).astype(int))] for x in mir])


def test_loop_cantilever_mirror_symmetry_and_volume():
    p = synth.cantilever2d(60, 30)
    S = simp.setup(p)
    perm = _mirror_perm(S.mesh)
    rho, log = simp.iterate(S, 50)
    np.testing.assert_allclose(rho, rho[perm], atol=1e-8)
    for rec in log:
        assert abs(rec["vol"] - 0.5) <= 1e-12
    cs = [r["c"] for r in log]
    assert cs[-1] < 0.25 * cs[0]
    # iteration 1 is the homogeneous problem: c scales as 1/E(rho)
    E_half = fem.simp_modulus(0.5)
    S1 = simp.setup(p)
    _, c_unit, *_ = simp.solve_state(S1, np.ones(S1.mesh.n_cells))
    np.testing.assert_allclose(cs[0], c_unit / E_half, rtol=1e-9)


def test_oc_passive_cells():
    """Passive cells (Section 5.4): void cells at rho_min and solid cells at
    1 after the update; the volume constraint counts them; free cells obey
    the OC formula at the returned multiplier; and the bisection (which
    overwrites passive cells after the clamp) agrees with the exact
    breakpoint root written with pinned bounds and zero coefficients."""
    rng = np.random.default_rng(19)
    n = 500
    rho = rng.uniform(0.001, 1.0, n)
    sf = -rng.lognormal(0.0, 2.0, n)
    passive = np.zeros(n, np.uint8)
    passive[rng.choice(n, 60, replace=False)] = oc.VOID
    passive[rng.choice(np.flatnonzero(passive == 0), 25, replace=False)] = oc.SOLID
    vf = 0.4
    rn, lam, vol, change, _ = oc.update(rho, sf, vf, passive=passive)
    assert np.all(rn[passive == oc.VOID] == 1e-3)
    assert np.all(rn[passive == oc.SOLID] == 1.0)
    assert abs(rn.sum() - vf * n) <= 1e-12 * n
    lo = np.maximum(1e-3, rho - 0.2)
    hi = np.minimum(1.0, rho + 0.2)
    free = (passive == 0) & (rn > lo) & (rn < hi)
    assert free.sum() > 10
    np.testing.assert_allclose(rn[free], rho[free] * np.sqrt(-sf[free] / lam), rtol=1e-12)
    re, lam_e = oc.exact_root(rho, sf, vf, passive=passive)
    np.testing.assert_allclose(rn, re, rtol=0, atol=1e-12)
    np.testing.assert_allclose(lam, lam_e, rtol=1e-10)
    # an all-free mask is the plain update
    r0, l0, *_ = oc.update(rho, sf, vf, passive=np.zeros(n, np.uint8))
    r1, l1, *_ = oc.update(rho, sf, vf)
    assert np.array_equal(r0, r1) and l0 == l1
    # the multiplier moves: the free cells carry the volume the passive ones do not
    _, lam_free, *_ = oc.update(rho, sf, vf)
    assert lam != lam_free


def test_loop_hole_keeps_passive_void():
    """The hole example at 60 x 30 (same rule, disc at (20, 15), radius 7.5):
    every passive cell is at rho_min after each iteration, the volume is
    held, and the design stays mirror-symmetric (the disc is symmetric about
    y = 15 and the alternating-rows mesh is too)."""
    p = synth.cantilever2d_hole(60, 30, rmin=1.5)
    assert p.passive.sum() > 0
    S = simp.setup(p)
    perm = _mirror_perm(S.mesh)
    assert np.array_equal(p.passive, p.passive[perm])
    rho, log = simp.iterate(S, 12)
    assert np.all(rho[p.passive == oc.VOID] == p.rho_min)
    for rec in log:
        assert abs(rec["vol"] - p.volfrac) <= 1e-12
    np.testing.assert_allclose(rho, rho[perm], atol=1e-8)
