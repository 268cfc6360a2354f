"""The 3D operator apply with several load cases per block (the moduli, mask
and D^-1 of a tile read once for all of them) against one load case per
block, through the C ABI.

Each load case goes through the same operations in the same order whatever
the block handles, so y = Z K Z x (Sec. 3.1, eq. fe_form) must be the same
bits for every split, in FP64 and FP32 with FP32 or BF16 moduli, on a grid
whose tiles and z-chunks end in ragged tails.  Inside multigrid-
preconditioned solves (where the fused Chebyshev smoothing kernels take the
same split) only the block order of the CG dot products changes, so the
solutions agree to the solve's rounding and the iteration counts match.
"""

import numpy as np
import pytest

import synth
from oracle import fem, mesh as M

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda:0"
SPLITS = [("1", "1"), ("2", "1"), ("2", "2"), ("4", "1"), ("4", "2"), ("4", "4")]


def _t(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device=DEV)


def _apply_all(p, rho, x, monkeypatch, prec):
    from paper_2012_08208_amd import TOPO_FP64, TOPO_MIXED_BF16, TOPO_MIXED_FP32, Topo
    code = {"fp64": TOPO_FP64, "fp32": TOPO_MIXED_FP32, "bf16": TOPO_MIXED_BF16}[prec]
    out = {}
    for nrb, g in SPLITS:
        monkeypatch.setenv("TOPO_APPLY_NRB", nrb)
        monkeypatch.setenv("TOPO_APPLY_G", g)
        t = Topo.from_problem(p, precision=code, device=DEV)
        if prec == "fp64":
            y = torch.zeros(p.nrhs * p.n_dofs, dtype=torch.float64, device=DEV)
            t.apply(_t(rho), _t(x.ravel()), y)
        else:
            y = torch.zeros(p.nrhs * p.n_dofs, dtype=torch.float32, device=DEV)
            t.apply_f32(_t(rho), _t(x.ravel(), torch.float32), y)
        assert t.sync() == 0
        t.close()
        out[(nrb, g)] = y.cpu().numpy()
    return out


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16"])
def test_apply_bit_equal_for_every_load_case_split(prec, monkeypatch):
    p = synth.cantilever3d(33, 19, 21, nrhs=4, rmin=1.5)
    print(f"[apply split] {prec} nel={p.nel} nrhs={p.nrhs}", flush=True)
    m = M.build(p.dim, p.nel, p.split)
    rho = synth.rho_random(61, m.n_cells, 0.05, 1.0)
    x = synth.vec_random(62, (p.nrhs, p.dim, m.n_nodes))
    if prec != "fp64":
        x = x.astype(np.float32).astype(np.float64)
    out = _apply_all(p, rho, x, monkeypatch, prec)
    base = out[("1", "1")]
    for key, y in out.items():
        assert np.array_equal(y, base), key
    E = fem.simp_modulus(rho, p.E0, p.Emin, p.penal)
    if prec == "bf16":
        E = fem.bf16_modulus(E)
    K = fem.assemble(m, E, p.nu)
    y_ref = np.stack([fem.apply_operator(K, x[r].ravel(), p.fixed.ravel()) for r in range(p.nrhs)])
    err = np.max(np.abs(base.reshape(p.nrhs, -1) - y_ref)) / np.max(np.abs(y_ref))
    print(f"  bit-equal over {len(out)} splits; max rel err vs oracle {err:.2e}", flush=True)
    assert err <= (1e-13 if prec == "fp64" else 2e-6)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_gmg_solve_for_every_load_case_split(prec, monkeypatch):
    from paper_2012_08208_amd import TOPO_FP64, TOPO_MIXED_FP32, TOPO_PC_GMG, Topo
    p = synth.cantilever3d(41, 23, 17, nrhs=4, rmin=1.5, rtol=1e-10)
    rho = synth.rho_random(63, p.n_cells, 0.05, 1.0)
    print(f"[solve split] {prec} nel={p.nel}", flush=True)
    res = {}
    for nrb, g in SPLITS:
        monkeypatch.setenv("TOPO_APPLY_NRB", nrb)
        monkeypatch.setenv("TOPO_APPLY_G", g)
        t = Topo.from_problem(p, rtol=1e-10, precond=TOPO_PC_GMG,
                              precision=TOPO_FP64 if prec == "fp64" else TOPO_MIXED_FP32,
                              device=DEV)
        u = torch.zeros(p.nrhs * p.n_dofs, dtype=torch.float64, device=DEV)
        info = torch.zeros(6, dtype=torch.float64, device=DEV)
        t.solve(_t(rho), u, info)
        assert t.sync() == 0
        t.close()
        res[(nrb, g)] = (u.cpu().numpy(), info.cpu().numpy())
    u0, i0 = res[("1", "1")]
    for key, (u, info) in res.items():
        print(f"  split {key}: {info[0]:.0f} iterations", flush=True)
        assert info[1] == 1.0 and np.all(info[2:6] <= 1e-10)
        assert abs(info[0] - i0[0]) <= 1, key
        assert np.max(np.abs(u - u0)) <= 1e-8 * np.max(np.abs(u0)), key
