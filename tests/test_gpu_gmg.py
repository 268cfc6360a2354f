"""Multigrid preconditioner behaviour on the GPU, through the C ABI.

* With the Galerkin coarse operators (3D coarse moduli twice the mean of
  their 8 children on the unit-cell kernels) the V-cycle preconditioned CG
  needs about the same number of iterations on 24x12x12 and 48x24x24 (one
  more level): the count does not grow with the depth.
* The W-cycle on the top levels (TOPO_GMG_WLEVELS; by default the 3D levels
  whose coarse level has at least 512 nodes) is a symmetric positive
  definite preconditioner for every depth it is given: CG converges, in no
  more iterations than with the V-cycle, to the same solution.
* The hierarchy stops at the first level of at most 2048 DOFs
  (TOPO_GMG_DENSE or topo_problem.gmg_dense; 128 gives the hierarchy that
  goes down to 128 DOFs) and solves it with its exact inverse, built by
  block Gauss-Jordan elimination: on a grid that small the preconditioner
  is the inverse of K itself.
"""

import os

import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _solve(p, precision, rho_val=0.3, maxit=2000, gmg_dense=0):
    from paper_2012_08208_amd import Topo, TOPO_PC_GMG, SOLVE_INFO_LEN
    t = Topo.from_problem(p, precision=precision, precond=TOPO_PC_GMG, maxit=maxit, device=DEV,
                          gmg_dense=gmg_dense)
    if np.isscalar(rho_val):
        rho = torch.full((p.n_cells,), rho_val, dtype=torch.float64, device=DEV)
    else:
        rho = torch.as_tensor(rho_val, dtype=torch.float64, device=DEV)
    u = torch.zeros(p.nrhs * p.n_dofs, dtype=torch.float64, device=DEV)
    info = torch.zeros(SOLVE_INFO_LEN, dtype=torch.float64, device=DEV)
    t.solve(rho, u, info)
    st = t.sync()
    t.close()
    return st, info.cpu().numpy(), u.cpu().numpy()


@pytest.mark.parametrize("prec", ["fp64", "mixed-ru"])
def test_vcycle_iterations_do_not_grow_with_depth(prec, monkeypatch):
    from paper_2012_08208_amd import TOPO_FP64, TOPO_MIXED_RU
    monkeypatch.setenv("TOPO_GMG_WLEVELS", "0")
    monkeypatch.setenv("TOPO_GMG_DENSE", "128")   # 3 and 4 levels down to 3 x 2 x 2
    code = TOPO_FP64 if prec == "fp64" else TOPO_MIXED_RU
    its = []
    for nel in ((24, 12, 12), (48, 24, 24)):
        p = synth.cantilever3d(*nel, nrhs=2, volfrac=0.3, rmin=1.5, rtol=1e-8)
        print(f"[gmg depth] {prec} {nel}", flush=True)
        st, info, _ = _solve(p, code)
        assert st == 0 and info[1] == 1.0, (st, info)
        its.append(int(info[0]))
    print(f"  CG iterations {its}", flush=True)
    assert max(its) <= 25
    assert abs(its[1] - its[0]) <= 3


@pytest.mark.parametrize("wlevels", ["1", "2", "9", "auto"])
def test_wcycle_converges_to_the_vcycle_solution(wlevels, monkeypatch):
    from paper_2012_08208_amd import TOPO_FP64, TOPO_MIXED_RU
    p = synth.cantilever3d(48, 24, 24, nrhs=2, volfrac=0.3, rmin=1.5, rtol=1e-10)
    monkeypatch.setenv("TOPO_GMG_WLEVELS", "0")
    st, info_v, u_v = _solve(p, TOPO_FP64)
    assert st == 0
    for code in (TOPO_FP64, TOPO_MIXED_RU):
        if wlevels == "auto":
            monkeypatch.delenv("TOPO_GMG_WLEVELS", raising=False)   # default: by level size
        else:
            monkeypatch.setenv("TOPO_GMG_WLEVELS", wlevels)
        print(f"[gmg W] wlevels {wlevels} precision {code}", flush=True)
        st, info, u = _solve(p, code)
        print(f"  CG iterations V {info_v[0]:.0f}  W {info[0]:.0f}", flush=True)
        assert st == 0 and info[1] == 1.0, (st, info)
        assert info[0] <= info_v[0]
        for r in range(p.nrhs):
            a, b = u[r * p.n_dofs:(r + 1) * p.n_dofs], u_v[r * p.n_dofs:(r + 1) * p.n_dofs]
            assert np.linalg.norm(a - b) <= 1e-7 * np.linalg.norm(b)
    monkeypatch.delenv("TOPO_GMG_WLEVELS", raising=False)
    assert "TOPO_GMG_WLEVELS" not in os.environ


@pytest.mark.parametrize("nel", [(24, 12, 12), (40, 20, 20), (33, 17, 9), (96, 48), (75, 29)])
def test_one_block_coarse_tail_matches_the_per_level_kernels(nel, monkeypatch):
    """The FP32 cycle's small coarse levels in one work-group per load case
    (default; 3D and 2D) against the per-level kernels (TOPO_GMG_TAIL=0): the same
    preconditioner up to the order of the operator's node sums and FP32
    rounding.  After two CG iterations (plus the true-residual restart
    passes of two iterations each) the iterates agree to FP32 rounding,
    far below what a different cycle would give; whole solves reach the
    same solution in about the same iterations; two runs give the same
    bits."""
    from paper_2012_08208_amd import TOPO_MIXED_RU, TOPO_MIXED_FP32
    # the tail serves hierarchies that go down to 128 DOFs
    monkeypatch.setenv("TOPO_GMG_DENSE", "128")
    if len(nel) == 3:
        p = synth.cantilever3d(*nel, nrhs=3, volfrac=0.3, rmin=1.5, rtol=1e-9)
    else:
        # the alternating split on the fine level, diagonal A on the coarse ones
        p = synth.cantilever2d(*nel, volfrac=0.4, rmin=1.5, rtol=1e-9)
    for code in (TOPO_MIXED_FP32, TOPO_MIXED_RU):
        short, full = {}, {}
        for tail in ("0", "1", "1"):
            monkeypatch.setenv("TOPO_GMG_TAIL", tail)
            print(f"[gmg tail] {nel} precision {code} tail {tail}", flush=True)
            _, _, u2 = _solve(p, code, rho_val=0.4, maxit=2)
            st, info, u = _solve(p, code, rho_val=0.4)
            assert st == 0 and info[1] == 1.0, (st, info)
            if tail in full:
                assert np.array_equal(u, full[tail][1]) and np.array_equal(u2, short[tail])
            short[tail], full[tail] = u2, (info, u)
        (i0, u0), (i1, u1) = full["0"], full["1"]
        d2 = np.linalg.norm(short["1"] - short["0"]) / np.linalg.norm(short["0"])
        print(f"  after 2 iterations: rel diff {d2:.2e}; CG iterations per-level {i0[0]:.0f}"
              f"  one-block {i1[0]:.0f}", flush=True)
        assert d2 <= 1e-5
        assert abs(i1[0] - i0[0]) <= 3
        for r in range(p.nrhs):
            a, b = u1[r * p.n_dofs:(r + 1) * p.n_dofs], u0[r * p.n_dofs:(r + 1) * p.n_dofs]
            assert np.linalg.norm(a - b) <= 1e-6 * np.linalg.norm(b)
    monkeypatch.delenv("TOPO_GMG_TAIL", raising=False)


@pytest.mark.parametrize("env", [{"TOPO_CHEB_DEGREE": "3", "TOPO_CHEB_POST": "1"},
                                 {"TOPO_CHEB_KIND": "4"},
                                 {"TOPO_GMG_WLEVELS": "9"}])
def test_one_block_tail_follows_the_smoother_and_cycle_switches(env, monkeypatch):
    """The tail runs the same smoothing degrees, Chebyshev kind and W revisits
    as the per-level kernels: after two CG iterations the iterates agree to
    FP32 rounding (a different polynomial or cycle would differ at 1e-2)."""
    from paper_2012_08208_amd import TOPO_MIXED_FP32
    p = synth.cantilever3d(24, 12, 12, nrhs=2, volfrac=0.3, rmin=1.5, rtol=1e-9)
    monkeypatch.setenv("TOPO_GMG_DENSE", "128")
    for k, v in env.items():
        monkeypatch.setenv(k, v)
    out = {}
    for tail in ("0", "1"):
        monkeypatch.setenv("TOPO_GMG_TAIL", tail)
        _, _, u2 = _solve(p, TOPO_MIXED_FP32, rho_val=0.4, maxit=2)
        st, info, _ = _solve(p, TOPO_MIXED_FP32, rho_val=0.4)
        assert st == 0 and info[1] == 1.0, (st, info)
        out[tail] = (u2, info[0])
    d2 = np.linalg.norm(out["1"][0] - out["0"][0]) / np.linalg.norm(out["0"][0])
    print(f"[tail switches] {env}: rel diff {d2:.2e}, CG iterations {out['0'][1]:.0f} / "
          f"{out['1'][1]:.0f}", flush=True)
    assert d2 <= 1e-5
    assert abs(out["1"][1] - out["0"][1]) <= 2


_DIRECT_CASES = ([(nel, prec) for nel in [(10, 6, 5), (7, 7, 7), (30, 15), (31, 16)]
                  for prec in ("fp64", "mixed-ru")]
                 + [((4, 3, 3), "fp64"), ((11, 5), "fp64")])


@pytest.mark.parametrize("nel,prec", _DIRECT_CASES)
def test_direct_level_above_128_dofs_is_the_exact_inverse(nel, prec):
    """A grid of 128 < DOFs <= 2048 is its own coarsest level (3D: 1386 DOFs,
    padded to 1408 = 22 blocks of 64, 1536 = 24 blocks, no padding, and
    240 padded to 256 = 4 blocks; 2D: 992 DOFs padded to 1024, 1088 = 17
    blocks, and 144 padded to 192 = 3 blocks, the fewest), so the
    preconditioner is K^-1 from the block sweep.  The two smallest grids
    run in FP64 only: with the SIMP contrast on so few cells the FP32 copy
    of the inverse is too far from K^-1 for the few-iteration bound (10
    reliable-update iterations on 4 x 3 x 3).  FP64 CG stops after
    one iteration (two at most), the reliable-update CG with the FP32 copy of the inverse
    after a few, both at the direct solution (SIMP contrast 1e-9, fixed DOFs
    as identity rows)."""
    from oracle import fem, mesh as M
    from paper_2012_08208_amd import TOPO_FP64, TOPO_MIXED_RU
    if len(nel) == 3:
        p = synth.cantilever3d(*nel, nrhs=2, volfrac=0.3, rmin=1.5, rtol=1e-10)
    else:
        p = synth.cantilever2d(*nel, volfrac=0.4, rmin=1.5, rtol=1e-10)
    m = M.build(p.dim, p.nel, p.split)
    rho = synth.rho_random(5, m.n_cells, 1e-3, 1.0)
    K = fem.assemble(m, fem.simp_modulus(rho, p.E0, p.Emin, p.penal), p.nu)
    f = p.loads.reshape(p.nrhs, -1)
    u_ref = fem.solve(K, f, p.fixed.ravel())
    code = TOPO_FP64 if prec == "fp64" else TOPO_MIXED_RU
    print(f"[dense direct] {nel} {prec}", flush=True)
    st, info, u = _solve(p, code, rho_val=rho)
    print(f"  CG iterations {info[0]:.0f}", flush=True)
    assert st == 0 and info[1] == 1.0, (st, info)
    assert info[0] <= (2 if prec == "fp64" else 6)
    u = u.reshape(p.nrhs, -1)
    for r in range(p.nrhs):
        err = np.linalg.norm(u[r] - u_ref[r]) / np.linalg.norm(u_ref[r])
        assert err <= 1e-8, (r, err)


@pytest.mark.parametrize("nel", [(48, 24, 24), (33, 17, 9), (192, 64), (149, 57)])
def test_direct_2048_dof_level_against_the_128_dof_hierarchy(nel, monkeypatch):
    """The hierarchy that stops at 12 x 6 x 6 (1911 DOFs; 9 x 5 x 3, 720 DOFs,
    on the odd grid; 2D: 48 x 16, 1666 DOFs, and 38 x 15, 1248 DOFs) and solves
    it exactly, against the one that goes on down to 128 DOFs (with the
    one-block tail in the FP32 2D cycle): the same solution, in no more CG
    iterations (an exact coarse solve is at least as good as a cycle over
    the levels below it).  The size comes from topo_problem.gmg_dense, or
    from TOPO_GMG_DENSE when that field is 0 (automatic)."""
    from paper_2012_08208_amd import TOPO_FP64, TOPO_MIXED_RU
    if len(nel) == 3:
        p = synth.cantilever3d(*nel, nrhs=2, volfrac=0.3, rmin=1.5, rtol=1e-10)
    else:
        p = synth.mbb2d(*nel, volfrac=0.4, rmin=1.5, rtol=1e-10)
    for code in (TOPO_FP64, TOPO_MIXED_RU):
        out = {}
        for dense in ("128", "2048"):
            field = 128 if (dense == "128" and code == TOPO_FP64) else 0
            monkeypatch.setenv("TOPO_GMG_DENSE", "2048" if field else dense)
            print(f"[dense level] {nel} precision {code} dense {dense} (field {field})", flush=True)
            st, info, u = _solve(p, code, gmg_dense=field)
            assert st == 0 and info[1] == 1.0, (st, info)
            out[dense] = (info[0], u)
        print(f"  CG iterations 128: {out['128'][0]:.0f}  2048: {out['2048'][0]:.0f}", flush=True)
        assert out["2048"][0] <= out["128"][0] + 1
        for r in range(p.nrhs):
            sl = slice(r * p.n_dofs, (r + 1) * p.n_dofs)
            a, b = out["2048"][1][sl], out["128"][1][sl]
            assert np.linalg.norm(a - b) <= 1e-7 * np.linalg.norm(b)
    monkeypatch.delenv("TOPO_GMG_DENSE", raising=False)
