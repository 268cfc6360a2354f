"""Host-only checks of the C ABI: the library loads, exports every entry point
that include/topo.h declares, and sizes workspaces without touching a GPU."""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "topo.h")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(topo_[a-z_]+)\s*\(", txt)))


def _lib():
    from paper_2012_08208_amd import binding
    if not os.path.exists(binding.LIB_PATH):
        pytest.skip("libtopo.so not built (run __graft_entry__.build())")
    return binding


def test_header_declares_the_seven_path_calls():
    names = _declared()
    for n in ["topo_create", "topo_set_loads", "topo_solve", "topo_sensitivity", "topo_filter",
              "topo_oc_update", "topo_iterate"]:
        assert n in names


def test_library_exports_every_declared_symbol():
    b = _lib()
    lib = ctypes.CDLL(b.LIB_PATH)
    for n in _declared():
        assert hasattr(lib, n), n
    assert set(_declared()) <= set(b.EXPORTED)


def test_workspace_size_and_validation():
    b = _lib()
    lib = b.load_library()
    p = b.make_problem(3, (192, 96, 96), nrhs=4, volfrac=0.3, rmin=2.5)
    n = ctypes.c_size_t(0)
    assert lib.topo_workspace_size(ctypes.byref(p), ctypes.byref(n)) == 0
    nd = 3 * 193 * 97 * 97
    assert n.value > 4 * nd * 8 * 4          # loads + three CG vectors
    assert n.value < 8 * 1024 ** 3          # modest on a 288 GB device
    bad = b.make_problem(4, (2, 2, 2))
    assert lib.topo_workspace_size(ctypes.byref(bad), ctypes.byref(n)) == -1
    bad = b.make_problem(2, (8, 4), nrhs=5)
    assert lib.topo_workspace_size(ctypes.byref(bad), ctypes.byref(n)) == -1
    bad = b.make_problem(2, (8, 4), volfrac=0.0)
    assert lib.topo_workspace_size(ctypes.byref(bad), ctypes.byref(n)) == -1
    assert lib.topo_status_string(-7) == b"workspace too small"


def test_directly_solved_coarsest_level_size():
    """topo_problem.gmg_dense: 0 (automatic) or 128..2048 DOFs.  The 3D
    default stops the 192 x 96 x 96 hierarchy at 12 x 6 x 6 (1911 DOFs) and
    holds its padded 1920 x 1920 inverse (FP64 and, mixed, FP32); 128 goes
    on down to 3 x 2 x 2 with a 108 x 108 inverse."""
    b = _lib()
    lib = b.load_library()
    n = ctypes.c_size_t(0)
    sizes = {}
    for dense in (0, 128, 2048):
        p = b.make_problem(3, (192, 96, 96), nrhs=4, volfrac=0.3, rmin=2.5,
                           precision=b.TOPO_MIXED_RU, precond=b.TOPO_PC_GMG, gmg_dense=dense)
        assert lib.topo_workspace_size(ctypes.byref(p), ctypes.byref(n)) == 0
        sizes[dense] = n.value
    assert sizes[0] == sizes[2048]
    # the 1920 x 1920 FP64 + FP32 inverse against the levels below 12 x 6 x 6
    assert sizes[2048] - sizes[128] > 1920 * 1920 * 12 - 8 * 1024 ** 2
    # 2D: the MBB beam stops at 38 x 13 (1092 DOFs, padded to 1152) instead
    # of going on to 5 x 2
    s2 = {}
    for dense in (0, 128):
        p = b.make_problem(2, (1200, 400), nrhs=1, volfrac=0.4, rmin=3.0,
                           precision=b.TOPO_MIXED_FP32, precond=b.TOPO_PC_GMG, gmg_dense=dense)
        assert lib.topo_workspace_size(ctypes.byref(p), ctypes.byref(n)) == 0
        s2[dense] = n.value
    assert s2[0] - s2[128] > 1152 * 1152 * 12 - 4 * 1024 ** 2
    for dense in (-1, 1, 127, 2049, 4096):
        bad = b.make_problem(3, (16, 8, 8), precond=b.TOPO_PC_GMG, gmg_dense=dense)
        assert lib.topo_workspace_size(ctypes.byref(bad), ctypes.byref(n)) == -1, dense


def test_network_parameter_count_and_workspace():
    from oracle import net
    b = _lib()
    lib = b.load_library()
    assert b.num_params() == net.n_params()
    p = b.make_problem(3, (128, 64, 64), nrhs=1, precond=b.TOPO_PC_LEARNED)
    n = ctypes.c_size_t(0)
    assert lib.topo_workspace_size(ctypes.byref(p), ctypes.byref(n)) == 0
    assert lib.topo_precond_workspace_size(ctypes.byref(p), ctypes.byref(n)) == 0
    v0 = 129 * 65 * 65
    assert n.value > v0 * 2 * (8 + 16 + 48 + 16)   # level-0 activations
    assert n.value < 4 * 1024 ** 3
    # the learned preconditioner is 3D and FP64 only
    bad = b.make_problem(2, (8, 4), precond=b.TOPO_PC_LEARNED)
    assert lib.topo_workspace_size(ctypes.byref(bad), ctypes.byref(n)) == -1
    bad = b.make_problem(3, (8, 4, 4), precond=b.TOPO_PC_LEARNED, precision=b.TOPO_MIXED_FP32)
    assert lib.topo_workspace_size(ctypes.byref(bad), ctypes.byref(n)) == -1
    assert b"learned" in lib.topo_status_string(2)


def test_batch_workspace_and_validation():
    import synth
    b = _lib()
    lib = b.load_library()
    probs = synth.batch2d(count=4, nx_lo=12, nx_hi=30)
    arr = (b.CProblem * 4)()
    for i, p in enumerate(probs):
        arr[i] = b.make_problem(2, p.nel, 1, p.split, volfrac=p.volfrac, rmin=p.rmin,
                                precond=b.TOPO_PC_GMG)
    n = ctypes.c_size_t(0)
    assert lib.topo_batch_workspace_size(arr, 4, ctypes.byref(n)) == 0
    cells = sum(p.n_cells for p in probs)
    assert n.value > cells * 8 * 8
    # 3D, several load cases, Jacobi or mixed precision are rejected
    bad = (b.CProblem * 1)(b.make_problem(3, (4, 2, 2), precond=b.TOPO_PC_GMG))
    assert lib.topo_batch_workspace_size(bad, 1, ctypes.byref(n)) == -1
    bad = (b.CProblem * 1)(b.make_problem(2, (8, 4), nrhs=2, precond=b.TOPO_PC_GMG))
    assert lib.topo_batch_workspace_size(bad, 1, ctypes.byref(n)) == -1
    bad = (b.CProblem * 1)(b.make_problem(2, (8, 4), precond=b.TOPO_PC_JACOBI))
    assert lib.topo_batch_workspace_size(bad, 1, ctypes.byref(n)) == -1
    assert lib.topo_batch_workspace_size(arr, 0, ctypes.byref(n)) == -1


def test_filter_selector_and_new_modes_validate():
    """The filter selector sits at the end of topo_problem (the ctypes mirror
    must match the header's field order); the Helmholtz filter adds five
    nodal FP64 vectors to the workspace; unknown filters and precisions are
    rejected; the batch keeps the distance filter only."""
    b = _lib()
    lib = b.load_library()
    txt = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    body = re.search(r"typedef struct topo_problem \{(.*?)\} topo_problem;", txt, re.S).group(1)
    names = re.findall(r"\b([A-Za-z_][A-Za-z_0-9]*)(?:\[\d\])?\s*[,;]", body)
    assert names == [f[0] for f in b.CProblem._fields_]
    n0, n1 = ctypes.c_size_t(0), ctypes.c_size_t(0)
    p = b.make_problem(3, (24, 12, 12), nrhs=1)
    assert lib.topo_workspace_size(ctypes.byref(p), ctypes.byref(n0)) == 0
    p = b.make_problem(3, (24, 12, 12), nrhs=1, filter=b.TOPO_FILTER_HELMHOLTZ)
    assert lib.topo_workspace_size(ctypes.byref(p), ctypes.byref(n1)) == 0
    assert n1.value >= n0.value + 5 * 25 * 13 * 13 * 8
    bad = b.make_problem(2, (8, 4), filter=3)
    assert lib.topo_workspace_size(ctypes.byref(bad), ctypes.byref(n0)) == -1
    p = b.make_problem(3, (24, 12, 12), nrhs=1, filter=b.TOPO_FILTER_DENSITY)
    n2 = ctypes.c_size_t(0)
    assert lib.topo_workspace_size(ctypes.byref(p), ctypes.byref(n2)) == 0
    p = b.make_problem(3, (24, 12, 12), nrhs=1)
    assert lib.topo_workspace_size(ctypes.byref(p), ctypes.byref(n0)) == 0
    assert n2.value >= n0.value + 2 * 24 * 12 * 12 * 6 * 8   # filtered design and dv
    bad = b.make_problem(2, (8, 4), precision=5)
    assert lib.topo_workspace_size(ctypes.byref(bad), ctypes.byref(n0)) == -1
    ok = b.make_problem(2, (8, 4), precision=b.TOPO_MIXED_BF16, precond=b.TOPO_PC_GMG)
    assert lib.topo_workspace_size(ctypes.byref(ok), ctypes.byref(n0)) == 0
    bad = (b.CProblem * 1)(b.make_problem(2, (8, 4), precond=b.TOPO_PC_GMG,
                                          filter=b.TOPO_FILTER_HELMHOLTZ))
    assert lib.topo_batch_workspace_size(bad, 1, ctypes.byref(n0)) == -1


def test_edm_entry_points_reject_bad_arguments_on_the_host():
    """Argument checks of topo_edm_* return before any device work."""
    b = _lib()
    lib = b.load_library()
    fake = ctypes.c_void_p(256)           # never dereferenced: each call fails first
    assert lib.topo_edm_count(fake, 4, 10, 1.0, fake, fake, 1 << 20, None) == -1
    assert lib.topo_edm_count(fake, 3, 10, 0.0, fake, fake, 1 << 20, None) == -1
    assert lib.topo_edm_count(fake, 3, 10, float("nan"), fake, fake, 1 << 20, None) == -1
    assert lib.topo_edm_count(None, 3, 10, 1.0, fake, fake, 1 << 20, None) == -1
    assert lib.topo_edm_count(fake, 3, -1, 1.0, fake, fake, 1 << 20, None) == -2
    assert lib.topo_edm_count(fake, 3, 1 << 31, 1.0, fake, fake, 1 << 20, None) == -2
    assert lib.topo_edm_fill(fake, 2, 10, 1.0, fake, None, fake, fake, fake, 1 << 20, None) == -1
    assert lib.topo_edm_filter(-1, 0, fake, fake, fake, fake, fake, fake, fake, None) == -2
    assert lib.topo_edm_filter(10, -5, fake, fake, fake, fake, fake, fake, fake, None) == -2
    assert lib.topo_edm_filter(10, 5, fake, None, fake, fake, fake, fake, fake, None) == -1
    assert lib.topo_edm_filter(0, 0, None, None, None, None, None, None, None, None) == 0
    assert lib.topo_edm_workspace_size(-3, ctypes.byref(ctypes.c_size_t())) == -2


@pytest.mark.parametrize("dim,split,rmin", [
    (2, 0, 1.5), (2, 1, 1.5), (2, 0, 3.0), (3, 1, 1.5), (3, 1, 2.5), (3, 1, 4.4), (3, 1, 5.0),
])
def test_filter_tap_lists_are_whole_neighbourhoods(dim, split, rmin):
    """The tap lists the filter kernels walk hold every cell of an interior
    neighbourhood (Sec. 3.2.2, eq. filter): their lengths equal the
    exact-rational lattice counts, including radii whose 3D neighbourhoods
    (2137 cells at 4.4, 3119 at 5) exceed any fixed table size."""
    from test_oracle_sens_filter_oc import _lattice_neighbourhood
    b = _lib()
    lib = b.load_library()
    nt = (ctypes.c_int32 * 8)()
    ncls = ctypes.c_int32(0)
    assert lib.topo_filter_taps(dim, split, rmin, nt, ctypes.byref(ncls)) == 0
    lat = _lattice_neighbourhood(dim, split, rmin)
    want = [n for n, _ in lat]
    if dim == 2 and split == 0:
        # alternating rows: odd-row classes mirror the even-row ones
        assert ncls.value == 4 and sorted(nt[2:4]) == sorted(want)
    else:
        assert ncls.value == len(want)
    assert list(nt[:len(want)]) == want
    if dim == 3 and rmin == 5.0:
        assert want == [3119] * 6
    # the workspace grows with the neighbourhood instead of truncating it
    small = b.make_problem(3, (14, 9, 6), rmin=2.5)
    big = b.make_problem(3, (14, 9, 6), rmin=5.0)
    ns, nb = ctypes.c_size_t(0), ctypes.c_size_t(0)
    assert lib.topo_workspace_size(ctypes.byref(small), ctypes.byref(ns)) == 0
    assert lib.topo_workspace_size(ctypes.byref(big), ctypes.byref(nb)) == 0
    assert nb.value >= ns.value + 8 * (3119 - 405) * 24
    assert lib.topo_filter_taps(4, 0, 1.5, nt, ctypes.byref(ncls)) == -1
    assert lib.topo_filter_taps(3, 0, 0.0, nt, ctypes.byref(ncls)) == -1


def test_noalloc_oc_update_rejects_bad_arguments_on_the_host():
    """topo_oc_update_noalloc checks its arguments before any HIP call, so a
    bad call returns an error code here, with no GPU: sizes outside
    [1, TOPO_OC_NOALLOC_MAX_CELLS] give TOPO_E_SHAPE, null or aliased
    pointers and out-of-range parameters TOPO_E_INVALID."""
    b = _lib()
    lib = b.load_library()
    f = lib.topo_oc_update_noalloc
    r, d, o, s = 4096, 8192, 12288, 16384      # never dereferenced
    ok = dict(volfrac=0.5, move=0.2, eta=0.5, rho_min=1e-3)

    def call(n, rho=r, dcf=d, new=o, out=s, **kw):
        a = dict(ok, **kw)
        return f(n, rho, dcf, new, a["volfrac"], a["move"], a["eta"], a["rho_min"], out, None)

    assert call(b.OC_NOALLOC_MAX_CELLS + 1) == -2
    assert call(0) == -2
    assert call(-5) == -2
    assert call(10, rho=None) == -1
    assert call(10, out=None) == -1
    assert call(10, new=r) == -1
    assert call(10, new=d) == -1
    assert call(10, volfrac=0.0) == -1
    assert call(10, volfrac=1.5) == -1
    assert call(10, move=0.0) == -1
    assert call(10, eta=0.0) == -1
    assert call(10, rho_min=0.0) == -1


def test_no_wait_mode_validates_on_the_host():
    """TOPO_SYNC_NONE (no host wait inside the path calls) is accepted with
    the FP64 and mixed FP32/BF16 multigrid or Jacobi solves and every
    filter; it is refused (TOPO_E_INVALID) with the host-driven refinement
    loop of TOPO_MIXED_IR and with the learned preconditioner, and an unknown
    mode is refused."""
    b = _lib()
    lib = b.load_library()
    n = ctypes.c_size_t(0)
    for prec in (b.TOPO_FP64, b.TOPO_MIXED_FP32, b.TOPO_MIXED_BF16):
        for pc in (b.TOPO_PC_JACOBI, b.TOPO_PC_GMG):
            for flt in (b.TOPO_FILTER_DISTANCE, b.TOPO_FILTER_HELMHOLTZ, b.TOPO_FILTER_DENSITY):
                p = b.make_problem(3, (8, 4, 4), nrhs=2, precision=prec, precond=pc, filter=flt,
                                   sync_mode=b.TOPO_SYNC_NONE)
                assert lib.topo_workspace_size(ctypes.byref(p), ctypes.byref(n)) == 0
    p = b.make_problem(3, (8, 4, 4), precision=b.TOPO_MIXED_IR, precond=b.TOPO_PC_GMG,
                       sync_mode=b.TOPO_SYNC_NONE)
    assert lib.topo_workspace_size(ctypes.byref(p), ctypes.byref(n)) == -1
    p = b.make_problem(3, (8, 4, 4), precond=b.TOPO_PC_LEARNED, sync_mode=b.TOPO_SYNC_NONE)
    assert lib.topo_workspace_size(ctypes.byref(p), ctypes.byref(n)) == -1
    p = b.make_problem(3, (8, 4, 4), sync_mode=2)
    assert lib.topo_workspace_size(ctypes.byref(p), ctypes.byref(n)) == -1


def test_umesh_entry_points_validate_on_the_host():
    """topo_umesh_workspace_size and topo_umesh_create check sizes, the
    problem and the node ids before any HIP call: errors come back with no
    GPU."""
    import numpy as np
    b = _lib()
    lib = b.load_library()
    n = ctypes.c_size_t(0)
    assert lib.topo_umesh_workspace_size(3, 10, 12, 2, ctypes.byref(n)) == 0 and n.value > 0
    assert lib.topo_umesh_workspace_size(4, 10, 12, 1, ctypes.byref(n)) == -1
    assert lib.topo_umesh_workspace_size(3, 10, 12, 5, ctypes.byref(n)) == -1
    assert lib.topo_umesh_workspace_size(3, 0, 12, 1, ctypes.byref(n)) == -2
    assert lib.topo_umesh_workspace_size(3, 10, 2 ** 30, 1, ctypes.byref(n)) == -2
    coords = np.zeros((3, 4))
    cells = np.array([[0, 1, 2, 3]], dtype=np.int32)
    fixed = np.zeros((3, 4), np.uint8)
    h = ctypes.c_void_p()
    ws = ctypes.c_void_p(1 << 20)      # never touched: validation fails first
    good = b.make_problem(3, (1, 1, 1), 1)
    for bad in (b.make_problem(3, (1, 1, 1), 1, precond=b.TOPO_PC_GMG),
                b.make_problem(3, (1, 1, 1), 1, precision=b.TOPO_MIXED_FP32),
                b.make_problem(3, (1, 1, 1), 1, paper_mode=True)):
        assert lib.topo_umesh_create(ctypes.byref(bad), 4, 1, coords.ctypes.data,
                                     cells.ctypes.data, fixed.ctypes.data, ws, 1 << 30, None,
                                     ctypes.byref(h)) == -1
    bad_cells = np.array([[0, 1, 2, 7]], dtype=np.int32)
    assert lib.topo_umesh_create(ctypes.byref(good), 4, 1, coords.ctypes.data,
                                 bad_cells.ctypes.data, fixed.ctypes.data, ws, 1 << 30, None,
                                 ctypes.byref(h)) == -1
    assert lib.topo_umesh_create(ctypes.byref(good), 4, 1, coords.ctypes.data, cells.ctypes.data,
                                 fixed.ctypes.data, ws, 16, None, ctypes.byref(h)) == -7
