"""GPU parity of the SIMP loop on arbitrary simplex meshes (topo_umesh_*,
Sec. 6.1) against the unstructured-mesh oracle (oracle/umesh.py), through the
C ABI:

* the structured grid given as unstructured data reproduces the structured
  apply (the same operator, Sec. 3.1 eq. fe_form), 2D and 3D;
* on jittered, holed, shuffled meshes: the apply against the oracle's
  assembled operator, the solve against its direct solve, the compliance and
  sensitivity (Sec. 3.2), the cell volumes and midpoints;
* whole loops with the midpoint filter built by the chunked distance matrix
  (Sec. 3.2.2, Sec. 4.5, Sec. 6.2) and the OC update by cell count
  (Sec. 3.2.1), against the oracle loop; and the no-wait mode gives the same
  bits as the polling one.
Bars: FP64 operator 1e-13 of max |y|; solve to rtol 1e-12; compliance 1e-9
relative every iteration; per-cell sensitivity 1e-9 in the cell-wise metric;
volume 1e-12 N_c; the design after the loop to L-inf 1e-4.
"""

import numpy as np
import pytest

import synth
from oracle import fem, mesh as M, umesh as OU

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _t(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device=DEV)


def _um(up, **kw):
    from paper_2012_08208_amd import UMesh
    return UMesh(up, device=DEV, **kw)


@pytest.mark.parametrize("case", ["3d", "2d"])
def test_grid_as_unstructured_data_matches_the_structured_apply(case):
    from paper_2012_08208_amd import Topo
    if case == "3d":
        p = synth.cantilever3d(13, 7, 6, nrhs=2, rmin=1.5)
    else:
        p = synth.cantilever2d(21, 9, split=synth.problems.SPLIT_UNIFORM)
    up = synth.from_structured(p)
    print(f"[umesh grid] {case} nel={p.nel} nrhs={p.nrhs}", flush=True)
    rho = synth.rho_random(41, p.n_cells, 0.05, 1.0)
    x = synth.vec_random(42, (p.nrhs, p.dim, p.n_nodes))
    t = Topo.from_problem(p, device=DEV)
    y_s = torch.zeros(p.nrhs * p.n_dofs, dtype=torch.float64, device=DEV)
    t.apply(_t(rho), _t(x.ravel()), y_s)
    assert t.sync() == 0
    t.close()
    u = _um(up)
    y_u = torch.zeros_like(y_s)
    u.apply(_t(rho), _t(x.ravel()), y_u)
    assert u.sync() == 0
    u.close()
    scale = float(y_s.abs().max())
    err = float((y_u - y_s).abs().max()) / scale
    print(f"  unstructured vs structured apply: {err:.2e}", flush=True)
    assert err <= 1e-13


def _jittered(dim, nrhs, holes, seed):
    nel = (12, 6, 5) if dim == 3 else (30, 14)
    return synth.jittered_cantilever(nel, nrhs=nrhs, seed=seed, holes=holes, jitter=0.2,
                                     rlo=0.3, rhi=0.4, volfrac=0.35,
                                     rmin=1.8 if dim == 3 else 2.2)


@pytest.mark.parametrize("dim", [3, 2])
def test_jittered_mesh_apply_solve_sensitivity(dim):
    up = _jittered(dim, 2, 2, 50 + dim)
    print(f"[umesh jittered] dim {dim}: {up.n_nodes} nodes, {up.n_cells} cells", flush=True)
    S = OU.setup(up)
    m = S.mesh
    rho = synth.rho_random(52, m.n_cells, 0.05, 1.0)
    x = synth.vec_random(53, (up.nrhs, dim, m.n_nodes))
    E = fem.simp_modulus(rho, up.E0, up.Emin, up.penal)
    K = fem.assemble(m, E, up.nu, False, S.K0)
    y_ref = np.stack([fem.apply_operator(K, x[r].ravel(), S.fixed_flat) for r in range(up.nrhs)])
    u = _um(up, rtol=1e-12)
    y = torch.zeros(up.nrhs * dim * m.n_nodes, dtype=torch.float64, device=DEV)
    u.apply(_t(rho), _t(x.ravel()), y)
    y2 = torch.zeros_like(y)
    u.apply(_t(rho), _t(x.ravel()), y2)
    vol = torch.zeros(m.n_cells, dtype=torch.float64, device=DEV)
    mid = torch.zeros(dim * m.n_cells, dtype=torch.float64, device=DEV)
    u.volumes(vol)
    u.midpoints(mid)
    assert u.sync() == 0
    assert torch.equal(y, y2)   # no atomics: the same bits every run
    err = np.max(np.abs(y.cpu().numpy().reshape(up.nrhs, -1) - y_ref)) / np.max(np.abs(y_ref))
    print(f"  apply vs oracle: {err:.2e}", flush=True)
    assert err <= 1e-13
    np.testing.assert_allclose(vol.cpu().numpy(), S.vol, rtol=1e-13)
    np.testing.assert_allclose(mid.cpu().numpy().reshape(dim, -1).T, M.centroids(m), rtol=0,
                               atol=1e-13)
    # solve, compliance and sensitivity against the oracle's direct solve
    u_ref, c_ref, w_ref, dc_ref, s_ref, _ = OU.solve_state(S, rho)
    uu = torch.zeros(up.nrhs * dim * m.n_nodes, dtype=torch.float64, device=DEV)
    info = torch.zeros(6, dtype=torch.float64, device=DEV)
    u.solve(_t(rho), uu, info)
    dc = torch.zeros(m.n_cells, dtype=torch.float64, device=DEV)
    c = torch.zeros(1, dtype=torch.float64, device=DEV)
    u.sensitivity(_t(rho), uu, dc, c)
    assert u.sync() == 0
    info = info.cpu().numpy()
    print(f"  CG iterations {info[0]:.0f}, residuals {info[2:2 + up.nrhs]}", flush=True)
    assert info[1] == 1.0 and np.all(info[2:2 + up.nrhs] <= 1e-12)
    uu = uu.cpu().numpy().reshape(up.nrhs, -1)
    for r in range(up.nrhs):
        assert np.linalg.norm(uu[r] - u_ref[r]) <= 1e-8 * np.linalg.norm(u_ref[r])
    assert abs(c.item() - c_ref) <= 1e-10 * abs(c_ref)
    dcg = dc.cpu().numpy()
    denom = np.maximum(np.abs(dc_ref), 1e-6 * np.max(np.abs(dc_ref)))
    assert np.max(np.abs(dcg - dc_ref) / denom) <= 1e-9
    u.close()


@pytest.mark.parametrize("dim,holes,n_iter", [(3, 2, 20), (2, 1, 30)])
def test_unstructured_loop_matches_the_oracle(dim, holes, n_iter):
    from paper_2012_08208_amd import EdmFilter, LOG_LEN, TOPO_SYNC_NONE
    up = _jittered(dim, 2, holes, 60 + dim)
    print(f"[umesh loop] dim {dim}: {up.n_nodes} nodes, {up.n_cells} cells, x{n_iter}", flush=True)
    S = OU.setup(up)
    rho_ref, log_ref = OU.iterate(S, n_iter)
    out = {}
    for mode in ("poll", "nowait"):
        um = _um(up, rtol=1e-12, maxit=3000, sync_mode=TOPO_SYNC_NONE if mode == "nowait" else 0)
        mid = torch.zeros(dim * up.n_cells, dtype=torch.float64, device=DEV)
        um.midpoints(mid)
        edm = EdmFilter(mid.reshape(dim, up.n_cells), up.rmin)
        rho = torch.full((up.n_cells,), up.volfrac, dtype=torch.float64, device=DEV)
        u = torch.zeros(up.nrhs * dim * up.n_nodes, dtype=torch.float64, device=DEV)
        log = torch.zeros(n_iter * LOG_LEN, dtype=torch.float64, device=DEV)
        um.iterate(rho, u, n_iter, edm, log)
        st = um.sync()
        um.close()
        assert st == 0, st
        out[mode] = (rho.cpu().numpy(), log.cpu().numpy().reshape(n_iter, LOG_LEN))
    rho_g, lg = out["poll"]
    assert np.array_equal(rho_g, out["nowait"][0]) and np.array_equal(lg, out["nowait"][1])
    c_ref = np.array([r["c"] for r in log_ref])
    err_c = np.max(np.abs(lg[:, 0] - c_ref) / np.abs(c_ref))
    err_rho = np.max(np.abs(rho_g - rho_ref))
    err_v = np.max(np.abs(lg[:, 2] - up.volfrac))
    print(f"  compliance rel {err_c:.2e}  rho L-inf {err_rho:.2e}  volume {err_v:.2e}", flush=True)
    assert err_c <= 1e-9
    assert err_v <= 1e-12
    assert err_rho <= 1e-4
    np.testing.assert_allclose(lg[:, 3], [r["change"] for r in log_ref], atol=1e-6)
    np.testing.assert_allclose(lg[:, 1], [r["c_paper"] for r in log_ref], rtol=1e-9)
