"""GPU parity: every step of the HIP path against the FP64 CPU oracle, called
through the C ABI, on seeded inputs spanning several tiles with ragged
tails.  Tolerances: FP64 kernels that only reorder sums are held to ~1e-12
relative; solves at rtol 1e-12 to 1e-9 relative in u; compliance and
sensitivity to 1e-9; the 50-iteration design to L-inf 1e-4 (and in practice
far tighter)."""

import numpy as np
import pytest

import synth
from oracle import fem, filt, mesh as M, oc, simp

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _topo(p, **kw):
    from paper_2012_08208_amd import Topo
    return Topo.from_problem(p, device=DEV, **kw)


def _t(a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64), device=DEV)


def _problems():
    return [
        ("2d_alt_r1", synth.cantilever2d(37, 23, rmin=1.5)),
        ("2d_uni_r1", synth.cantilever2d(31, 16, rmin=3.0, split=synth.problems.SPLIT_UNIFORM)),
        ("2d_mbb", synth.mbb2d(44, 20, rmin=3.0)),
        ("3d_r1", synth.cantilever3d(20, 17, 11, nrhs=1, rmin=1.5)),
        ("3d_r4", synth.cantilever3d(16, 9, 18, nrhs=4, rmin=2.5)),
        ("3d_r3_tiny", synth.cantilever3d(3, 2, 2, nrhs=3, rmin=1.5)),
    ]


@pytest.mark.parametrize("name,p", _problems())
def test_apply_and_diagonal(name, p):
    print(f"[apply] {name} nel={p.nel} nrhs={p.nrhs}", flush=True)
    m = M.build(p.dim, p.nel, p.split)
    rho = synth.rho_random(1, m.n_cells)
    E = fem.simp_modulus(rho, p.E0, p.Emin, p.penal)
    K = fem.assemble(m, E, p.nu)
    fixed = p.fixed.ravel()
    x = synth.vec_random(2, (p.nrhs, p.dim, m.n_nodes))
    y_ref = np.stack([fem.apply_operator(K, x[r].ravel(), fixed) for r in range(p.nrhs)])
    t = _topo(p)
    y = torch.zeros(p.nrhs * p.n_dofs, dtype=torch.float64, device=DEV)
    t.apply(_t(rho), _t(x), y)
    d = torch.zeros(p.n_dofs, dtype=torch.float64, device=DEV)
    t.diagonal(_t(rho), d)
    assert t.sync() == 0
    y = y.cpu().numpy().reshape(p.nrhs, -1)
    scale = np.max(np.abs(y_ref))
    np.testing.assert_allclose(y, y_ref, rtol=0, atol=1e-13 * scale)
    np.testing.assert_allclose(d.cpu().numpy(), fem.jacobi_diag(K, fixed), rtol=1e-13)


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
@pytest.mark.parametrize("name,p", _problems())
def test_apply_f32_and_bf16_moduli(name, p, prec):
    """The V-cycle's fine-level apply in FP32 arithmetic: with FP32 moduli
    against the oracle's FP64 operator, and with BF16 moduli against the
    oracle's operator assembled from its own BF16 rounding of the moduli.
    Bar: 2e-6 of the largest |y| (FP32 rounding of up to about 40 terms per
    row); BF16 moduli move y by about 2^-9 relative, so the BF16 case must
    match the BF16 operator and not the FP64 one."""
    from paper_2012_08208_amd import TOPO_MIXED_BF16, TOPO_MIXED_FP32
    print(f"[apply-{prec}] {name} nel={p.nel} nrhs={p.nrhs}", flush=True)
    m = M.build(p.dim, p.nel, p.split)
    rho = synth.rho_random(21, m.n_cells, 0.05, 1.0)
    E = fem.simp_modulus(rho, p.E0, p.Emin, p.penal)
    fixed = p.fixed.ravel()
    x = synth.vec_random(22, (p.nrhs, p.dim, m.n_nodes)).astype(np.float32).astype(np.float64)
    K = fem.assemble(m, E, p.nu)
    y64 = np.stack([fem.apply_operator(K, x[r].ravel(), fixed) for r in range(p.nrhs)])
    if prec == "bf16":
        Kb = fem.assemble(m, fem.bf16_modulus(E), p.nu)
        y_ref = np.stack([fem.apply_operator(Kb, x[r].ravel(), fixed) for r in range(p.nrhs)])
    else:
        y_ref = y64
    t = _topo(p, precision=TOPO_MIXED_BF16 if prec == "bf16" else TOPO_MIXED_FP32)
    y = torch.zeros(p.nrhs * p.n_dofs, dtype=torch.float32, device=DEV)
    t.apply_f32(_t(rho), torch.as_tensor(x.astype(np.float32).ravel(), device=DEV), y)
    assert t.sync() == 0
    t.close()
    y = y.double().cpu().numpy().reshape(p.nrhs, -1)
    scale = np.max(np.abs(y_ref))
    err = np.max(np.abs(y - y_ref)) / scale
    print(f"  max |y - y_ref| / max |y_ref| = {err:.2e}", flush=True)
    assert err <= 2e-6
    if prec == "bf16":
        assert np.max(np.abs(y64 - y_ref)) / scale > 10 * err


@pytest.mark.parametrize("pc", ["jacobi", "gmg", "mixed-gmg", "bf16-gmg", "ir-gmg", "ir-jacobi",
                                "ru-gmg"])
@pytest.mark.parametrize("name,p", _problems())
def test_solve_matches_direct(name, p, pc):
    from paper_2012_08208_amd import (TOPO_FP64, TOPO_MIXED_BF16, TOPO_MIXED_FP32, TOPO_MIXED_IR,
                                      TOPO_MIXED_RU, TOPO_PC_GMG, TOPO_PC_JACOBI)
    print(f"[solve] {name} {pc}", flush=True)
    m = M.build(p.dim, p.nel, p.split)
    rho = synth.rho_random(3, m.n_cells, 0.05, 1.0)
    E = fem.simp_modulus(rho, p.E0, p.Emin, p.penal)
    K = fem.assemble(m, E, p.nu)
    f = p.loads.reshape(p.nrhs, -1)
    u_ref = fem.solve(K, f, p.fixed.ravel())
    t = _topo(p, rtol=1e-12, precond=TOPO_PC_GMG if pc.endswith("gmg") else TOPO_PC_JACOBI,
              precision={"mixed": TOPO_MIXED_FP32, "ir": TOPO_MIXED_IR, "bf16": TOPO_MIXED_BF16,
                         "ru": TOPO_MIXED_RU}.get(pc.split("-")[0], TOPO_FP64))
    u = torch.zeros(p.nrhs * p.n_dofs, dtype=torch.float64, device=DEV)
    info = torch.zeros(6, dtype=torch.float64, device=DEV)
    t.solve(_t(rho), u, info)
    assert t.sync() == 0
    info = info.cpu().numpy()
    assert info[1] == 1.0 and np.all(info[2:2 + p.nrhs] <= 1e-12)
    u = u.cpu().numpy().reshape(p.nrhs, -1)
    for r in range(p.nrhs):
        err = np.linalg.norm(u[r] - u_ref[r]) / np.linalg.norm(u_ref[r])
        assert err <= 1e-8, (r, err)


@pytest.mark.parametrize("name,p", _problems())
def test_sensitivity_and_compliance(name, p):
    print(f"[sens] {name}", flush=True)
    m = M.build(p.dim, p.nel, p.split)
    rho = synth.rho_random(4, m.n_cells, 0.05, 1.0)
    K0 = fem.element_K0(m, p.nu)
    E = fem.simp_modulus(rho, p.E0, p.Emin, p.penal)
    K = fem.assemble(m, E, p.nu, K0=K0)
    f = p.loads.reshape(p.nrhs, -1)
    u = fem.solve(K, f, p.fixed.ravel())
    w = fem.element_energy(m, u, p.nu)
    s_ref = fem.sensitivity(rho, w, p.E0, p.Emin, p.penal)
    c_ref = fem.compliance(f, u)
    t = _topo(p)
    dc = torch.zeros(m.n_cells, dtype=torch.float64, device=DEV)
    c = torch.zeros(1, dtype=torch.float64, device=DEV)
    t.sensitivity(_t(rho), _t(u), dc, c)
    assert t.sync() == 0
    np.testing.assert_allclose(c.item(), c_ref, rtol=1e-12)
    dc = dc.cpu().numpy()
    denom = np.maximum(np.abs(s_ref), 1e-6 * np.max(np.abs(s_ref)))
    assert np.max(np.abs(dc - s_ref) / denom) <= 1e-11


@pytest.mark.parametrize("name,p", _problems())
def test_filter_and_rowsums(name, p):
    print(f"[filter] {name} rmin={p.rmin}", flush=True)
    m = M.build(p.dim, p.nel, p.split)
    cent = M.centroids(m)
    W = filt.weights_sparse(cent, p.rmin)
    R = filt.row_sums(W)
    rng = np.random.default_rng(5)
    rho = rng.uniform(0.001, 1.0, m.n_cells)
    dc = -rng.lognormal(0, 1, m.n_cells)
    ref = filt.apply(W, R, rho, dc)
    t = _topo(p)
    out = torch.zeros(m.n_cells, dtype=torch.float64, device=DEV)
    Rg = torch.zeros(m.n_cells, dtype=torch.float64, device=DEV)
    t.filter(_t(rho), _t(dc), out)
    t.filter_rowsums(Rg)
    assert t.sync() == 0
    np.testing.assert_allclose(Rg.cpu().numpy(), R, rtol=1e-13)
    np.testing.assert_allclose(out.cpu().numpy(), ref, rtol=1e-12)


@pytest.mark.parametrize("nx,ny,vf,seed", [(60, 30, 0.5, 0), (101, 50, 0.3, 1), (13, 7, 0.45, 2)])
def test_oc_update(nx, ny, vf, seed):
    print(f"[oc] {nx}x{ny}", flush=True)
    p = synth.cantilever2d(nx, ny, volfrac=vf)
    rng = np.random.default_rng(seed)
    ncell = p.n_cells
    # densities spread around the volume fraction so that the target lies
    # inside [sum lo, sum hi]
    rho = np.clip(rng.uniform(0.0, 2 * vf, ncell), 0.001, 1.0)
    dcf = -rng.lognormal(0, 2, ncell)
    ref, lam, vol, change, _ = oc.update(rho, dcf, vf)
    t = _topo(p)
    rn = torch.zeros(ncell, dtype=torch.float64, device=DEV)
    sc = torch.zeros(3, dtype=torch.float64, device=DEV)
    t.oc_update(_t(rho), _t(dcf), rn, sc)
    assert t.sync() == 0
    rn = rn.cpu().numpy()
    sc = sc.cpu().numpy()
    np.testing.assert_allclose(rn, ref, rtol=0, atol=1e-12)
    assert abs(rn.sum() - vf * ncell) <= 1e-12 * ncell
    np.testing.assert_allclose(sc[0], lam, rtol=1e-9)
    np.testing.assert_allclose(sc[2], change, rtol=0, atol=1e-12)


@pytest.mark.parametrize("dim", [2, 3])
def test_oc_update_passive(dim):
    """Passive cells (Section 5.4) in the OC update against the oracle:
    void cells at rho_min, solid cells at 1, the volume counted with them."""
    from paper_2012_08208_amd import TopoError
    p = synth.cantilever2d(53, 21, volfrac=0.4) if dim == 2 else \
        synth.cantilever3d(13, 7, 5, nrhs=1, volfrac=0.4)
    print(f"[oc-passive] {dim}D nel={p.nel}", flush=True)
    rng = np.random.default_rng(40 + dim)
    n = p.n_cells
    rho = np.clip(rng.uniform(0.0, 0.8, n), 0.001, 1.0)
    dcf = -rng.lognormal(0, 2, n)
    passive = np.zeros(n, np.uint8)
    passive[rng.choice(n, n // 10, replace=False)] = oc.VOID
    passive[rng.choice(np.flatnonzero(passive == 0), n // 20, replace=False)] = oc.SOLID
    ref, lam, vol, change, _ = oc.update(rho, dcf, 0.4, passive=passive)
    t = _topo(p)
    with pytest.raises(TopoError):
        t.set_passive(np.full(n, 3, np.uint8))
    t.set_passive(passive)
    rn = torch.zeros(n, dtype=torch.float64, device=DEV)
    sc = torch.zeros(3, dtype=torch.float64, device=DEV)
    t.oc_update(_t(rho), _t(dcf), rn, sc)
    assert t.sync() == 0
    got = rn.cpu().numpy()
    scv = sc.cpu().numpy()
    assert np.all(got[passive == oc.VOID] == p.rho_min) and np.all(got[passive == oc.SOLID] == 1.0)
    np.testing.assert_allclose(got, ref, rtol=0, atol=1e-12)
    np.testing.assert_allclose(scv[0], lam, rtol=1e-9)
    np.testing.assert_allclose(scv[2], change, rtol=0, atol=1e-12)
    # removing the set gives the plain update again
    t.set_passive(None)
    t.oc_update(_t(rho), _t(dcf), rn, sc)
    assert t.sync() == 0
    ref0, *_ = oc.update(rho, dcf, 0.4)
    np.testing.assert_allclose(rn.cpu().numpy(), ref0, rtol=0, atol=1e-12)
    t.close()


@pytest.mark.parametrize("nel", [(32, 16, 16), (41, 13, 9)])
def test_gmg_needs_far_fewer_iterations_than_jacobi(nel):
    from paper_2012_08208_amd import TOPO_PC_GMG, TOPO_PC_JACOBI
    p = synth.cantilever3d(*nel, nrhs=2, rtol=1e-8)
    rho = synth.rho_smooth(7, p.n_cells)
    iters = {}
    sols = {}
    for pc, code in (("jacobi", TOPO_PC_JACOBI), ("gmg", TOPO_PC_GMG)):
        print(f"[gmg-vs-jacobi] {nel} {pc}", flush=True)
        t = _topo(p, precond=code, maxit=20000)
        u = torch.zeros(p.nrhs * p.n_dofs, dtype=torch.float64, device=DEV)
        info = torch.zeros(6, dtype=torch.float64, device=DEV)
        t.solve(_t(rho), u, info)
        assert t.sync() == 0
        info = info.cpu().numpy()
        assert info[1] == 1.0
        iters[pc] = info[0]
        sols[pc] = u.cpu().numpy()
    print(f"[gmg-vs-jacobi] iterations {iters}", flush=True)
    assert iters["gmg"] * 5 < iters["jacobi"]
    rel = np.linalg.norm(sols["gmg"] - sols["jacobi"]) / np.linalg.norm(sols["jacobi"])
    assert rel < 1e-5


def test_oc_infeasible_target_is_flagged():
    # every cell can drop by at most the move limit: with all rho = 0.9 and
    # volfrac 0.3 the target lies below sum(lo) = 0.7 N
    p = synth.cantilever2d(20, 10, volfrac=0.3)
    rho = np.full(p.n_cells, 0.9)
    dcf = -np.linspace(1.0, 2.0, p.n_cells)
    t = _topo(p)
    rn = torch.zeros(p.n_cells, dtype=torch.float64, device=DEV)
    t.oc_update(_t(rho), _t(dcf), rn, None)
    assert t.sync() == -6
    np.testing.assert_allclose(rn.cpu().numpy(), 0.7, atol=1e-15)


def test_iterate_cantilever_60x30_50_iterations():
    from paper_2012_08208_amd import LOG_LEN
    p = synth.cantilever2d(60, 30)
    print("[iterate] cantilever2d 60x30 x50", flush=True)
    S = simp.setup(p)
    rho_ref, log_ref = simp.iterate(S, 50)
    t = _topo(p, rtol=1e-12)
    _run_iterate_check(t, p, rho_ref, log_ref)


def test_iterate_cantilever_60x30_50_iterations_gmg():
    from paper_2012_08208_amd import TOPO_PC_GMG
    p = synth.cantilever2d(60, 30)
    print("[iterate] cantilever2d 60x30 x50 gmg", flush=True)
    S = simp.setup(p)
    rho_ref, log_ref = simp.iterate(S, 50)
    t = _topo(p, rtol=1e-12, precond=TOPO_PC_GMG)
    _run_iterate_check(t, p, rho_ref, log_ref)


def test_iterate_cantilever_60x30_50_iterations_mixed():
    # the mixed-precision bar: compliance within rel 1e-7 of the oracle
    from paper_2012_08208_amd import TOPO_MIXED_FP32, TOPO_PC_GMG
    p = synth.cantilever2d(60, 30)
    print("[iterate] cantilever2d 60x30 x50 mixed", flush=True)
    S = simp.setup(p)
    rho_ref, log_ref = simp.iterate(S, 50)
    t = _topo(p, rtol=1e-10, precond=TOPO_PC_GMG, precision=TOPO_MIXED_FP32)
    _run_iterate_check(t, p, rho_ref, log_ref, c_rtol=1e-7)


def test_iterate_cantilever_60x30_50_iterations_mixed_bf16():
    # BF16 moduli in the V-cycle only precondition; the FP64 outer CG meets
    # the same tolerance, so the mixed bar applies
    from paper_2012_08208_amd import TOPO_MIXED_BF16, TOPO_PC_GMG
    p = synth.cantilever2d(60, 30)
    print("[iterate] cantilever2d 60x30 x50 mixed-bf16", flush=True)
    S = simp.setup(p)
    rho_ref, log_ref = simp.iterate(S, 50)
    t = _topo(p, rtol=1e-10, precond=TOPO_PC_GMG, precision=TOPO_MIXED_BF16)
    _run_iterate_check(t, p, rho_ref, log_ref, c_rtol=1e-7)


def test_iterate_cantilever_60x30_50_iterations_mixed_ir():
    from paper_2012_08208_amd import TOPO_MIXED_IR, TOPO_PC_GMG
    p = synth.cantilever2d(60, 30)
    print("[iterate] cantilever2d 60x30 x50 mixed-ir", flush=True)
    S = simp.setup(p)
    rho_ref, log_ref = simp.iterate(S, 50)
    t = _topo(p, rtol=1e-10, precond=TOPO_PC_GMG, precision=TOPO_MIXED_IR)
    _run_iterate_check(t, p, rho_ref, log_ref, c_rtol=1e-7)


def test_iterate_cantilever_60x30_50_iterations_mixed_ru():
    from paper_2012_08208_amd import TOPO_MIXED_RU, TOPO_PC_GMG
    p = synth.cantilever2d(60, 30)
    print("[iterate] cantilever2d 60x30 x50 mixed-ru", flush=True)
    S = simp.setup(p)
    rho_ref, log_ref = simp.iterate(S, 50)
    t = _topo(p, rtol=1e-10, precond=TOPO_PC_GMG, precision=TOPO_MIXED_RU)
    _run_iterate_check(t, p, rho_ref, log_ref, c_rtol=1e-7)


@pytest.mark.parametrize("case", ["hole", "propped"])
def test_iterate_extensions_60x30_50_iterations(case):
    """The paper's extensions on the 60 x 30 cantilever, 50 iterations
    against the oracle: a hole of passive void cells (Section 5.4) and a
    pointwise prop u_y = 0 at the bottom-right node (Section 5.2)."""
    from paper_2012_08208_amd import TOPO_PC_GMG
    p = synth.cantilever2d_hole(60, 30, rmin=1.5) if case == "hole" else \
        synth.propped_cantilever2d(60, 30, rmin=1.5)
    print(f"[iterate] {p.name} 60x30 x50", flush=True)
    S = simp.setup(p)
    rho_ref, log_ref = simp.iterate(S, 50)
    t = _topo(p, rtol=1e-12, precond=TOPO_PC_GMG)
    rho = _run_iterate_check(t, p, rho_ref, log_ref)
    if case == "hole":
        assert np.all(rho[p.passive == oc.VOID] == p.rho_min)


def _run_iterate_check(t, p, rho_ref, log_ref, c_rtol=1e-9):
    from paper_2012_08208_amd import LOG_LEN
    rho = torch.full((p.n_cells,), p.volfrac, dtype=torch.float64, device=DEV)
    u = torch.zeros(p.n_dofs, dtype=torch.float64, device=DEV)
    log = torch.zeros(50 * LOG_LEN, dtype=torch.float64, device=DEV)
    n = t.iterate(rho, u, 50, 0.0, log)
    assert n == 50
    assert t.sync() == 0
    lg = log.cpu().numpy().reshape(50, LOG_LEN)
    c_ref = np.array([r["c"] for r in log_ref])
    np.testing.assert_allclose(lg[:, 0], c_ref, rtol=c_rtol)
    np.testing.assert_allclose(lg[:, 2], 0.5, atol=1e-12)
    np.testing.assert_allclose(lg[:, 3], [r["change"] for r in log_ref], atol=1e-6)
    err = np.max(np.abs(rho.cpu().numpy() - rho_ref))
    print(f"[iterate] max |rho - rho_oracle| = {err:.3e}", flush=True)
    assert err <= 1e-4
    return rho.cpu().numpy()


@pytest.mark.parametrize("prec", ["fp64", "mixed", "bf16"])
def test_fused_post_smoothing_equals_separate_kernels(prec, monkeypatch):
    """The 3D degree-2 post-smoothing fused into two apply epilogues does the
    arithmetic of the separate Chebyshev kernels, operation for operation:
    the same CG iteration count and the same solution (1e-13 relative, the
    bar allows a different fused-multiply-add contraction choice)."""
    from paper_2012_08208_amd import TOPO_FP64, TOPO_MIXED_BF16, TOPO_MIXED_FP32, TOPO_PC_GMG
    code = {"fp64": TOPO_FP64, "mixed": TOPO_MIXED_FP32, "bf16": TOPO_MIXED_BF16}[prec]
    p = synth.cantilever3d(41, 23, 17, nrhs=3, rmin=1.5, rtol=1e-10)
    rho = synth.rho_random(31, p.n_cells, 0.05, 1.0)
    print(f"[fused post] {prec} nel={p.nel}", flush=True)
    out = {}
    for fused in ("1", "0"):
        monkeypatch.setenv("TOPO_CHEB_POST_FUSED", fused)
        t = _topo(p, rtol=1e-10, precond=TOPO_PC_GMG, precision=code)
        u = torch.zeros(p.nrhs * p.n_dofs, dtype=torch.float64, device=DEV)
        info = torch.zeros(6, dtype=torch.float64, device=DEV)
        t.solve(_t(rho), u, info)
        assert t.sync() == 0
        out[fused] = (u.cpu().numpy(), info.cpu().numpy())
        t.close()
    (u1, i1), (u0, i0) = out["1"], out["0"]
    print(f"  iterations {i1[0]:.0f} / {i0[0]:.0f}", flush=True)
    assert i1[0] == i0[0] and i1[1] == 1.0
    assert np.max(np.abs(u1 - u0)) <= 1e-13 * np.max(np.abs(u0))
