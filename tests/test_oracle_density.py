"""Pins for the oracle's density-filter mode (oracle/filt.py density and
density_grad, oracle/oc.py with dv and phys, oracle/simp.py filter 2).

* the filter keeps constants and its adjoint is the chain-rule map
  (<F x, y> = <x, F^T y>);
* the design gradient of the compliance through the filter matches central
  finite differences of c(F(x));
* the volume gradient dv is exact (the filter is linear);
* OC holds the filtered volume to rounding, and the weighted sum
  sum dv x_new equals it;
* the 60 x 30 loop keeps mirror symmetry and the filtered volume.
"""

import dataclasses

import numpy as np

import synth
from oracle import fem, filt, mesh as M, oc, simp


def _wr(m, rmin):
    W = filt.weights_sparse(M.centroids(m), rmin)
    return W, filt.row_sums(W)


def test_density_filter_constants_and_adjoint():
    m = M.build(2, (11, 7))
    W, R = _wr(m, 2.5)
    n = m.cells.shape[0]
    np.testing.assert_allclose(filt.density(W, R, np.full(n, 0.37)), 0.37, rtol=1e-14)
    rng = np.random.default_rng(3)
    x, y = rng.standard_normal(n), rng.standard_normal(n)
    np.testing.assert_allclose(np.dot(filt.density(W, R, x), y), np.dot(x, filt.density_grad(W, R, y)),
                               rtol=1e-12)
    # against the dense brute-force weights
    Wd = filt.weights_dense(M.centroids(m), 2.5)
    np.testing.assert_allclose(filt.density(W, R, x), Wd @ x / Wd.sum(axis=1), rtol=1e-12)


def test_chain_rule_matches_finite_differences():
    p = synth.cantilever2d(8, 4, rmin=1.5)
    m = M.build(2, p.nel, p.split)
    W, R = _wr(m, p.rmin)
    K0 = fem.element_K0(m, p.nu)
    f = p.loads.reshape(1, -1)
    fixed = p.fixed.ravel()
    rng = np.random.default_rng(8)
    x = rng.uniform(0.2, 0.9, m.cells.shape[0])

    def comp(xd):
        xp = filt.density(W, R, xd)
        K = fem.assemble(m, fem.simp_modulus(xp, p.E0, p.Emin, p.penal), p.nu, K0=K0)
        u = fem.solve(K, f, fixed)
        return float(np.sum(f * u)), u, xp

    _, u, xp = comp(x)
    w = fem.element_energy(m, u, p.nu)
    g = filt.density_grad(W, R, fem.sensitivity(xp, w, p.E0, p.Emin, p.penal))
    h = 1e-6
    for j in (0, 5, 17, 40, 63):
        e = np.zeros_like(x)
        e[j] = h
        fd = (comp(x + e)[0] - comp(x - e)[0]) / (2 * h)
        np.testing.assert_allclose(g[j], fd, rtol=1e-5)
    dv = filt.density_grad(W, R, np.ones_like(x))
    for j in (0, 9, 33):
        e = np.zeros_like(x)
        e[j] = 1.0
        np.testing.assert_allclose(filt.density(W, R, e).sum(), dv[j], rtol=1e-13)


def test_oc_filtered_volume_and_weighted_sum():
    m = M.build(2, (20, 10))
    W, R = _wr(m, 3.0)
    n = m.cells.shape[0]
    rng = np.random.default_rng(12)
    rho = rng.uniform(0.05, 0.9, n)
    g = -rng.lognormal(0.0, 1.5, n)
    dv = filt.density_grad(W, R, np.ones(n))
    phys = lambda z: filt.density(W, R, z)  # noqa: E731
    rn, lam, vol, change, _ = oc.update(rho, g, 0.45, dv=dv, phys=phys)
    assert abs(phys(rn).sum() - 0.45 * n) <= 1e-12 * n
    assert abs(np.dot(dv, rn) - phys(rn).sum()) <= 1e-12 * n
    np.testing.assert_allclose(vol, phys(rn).sum(), rtol=1e-15)
    lo = np.maximum(1e-3, rho - 0.2)
    hi = np.minimum(1.0, rho + 0.2)
    free = (rn > lo) & (rn < hi)
    assert free.sum() > 10
    np.testing.assert_allclose(rn[free], rho[free] * np.sqrt(-g[free] / (dv[free] * lam)), rtol=1e-12)


def test_loop_density_filter_symmetry_and_volume():
    p = dataclasses.replace(synth.cantilever2d(60, 30), filter=2)
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
