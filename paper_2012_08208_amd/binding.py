"""ctypes binding of the gfx950 SIMP library (argument marshalling only).

Every compute step runs in the HIP kernels of ``libtopo.so``; this module
only checks tensor shapes/dtypes/devices, passes raw device pointers and
the current torch stream, and owns the workspace tensor.  There is no CPU
path: if the library is missing the import of a context fails loudly.
"""

from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtopo.so")

TOPO_SPLIT_ALT_ROWS = 0
TOPO_SPLIT_UNIFORM = 1
TOPO_FP64 = 0
TOPO_MIXED_FP32 = 1
TOPO_MIXED_IR = 2
TOPO_MIXED_BF16 = 3
TOPO_MIXED_RU = 4
TOPO_PASSIVE_FREE = 0
TOPO_PASSIVE_VOID = 1
TOPO_PASSIVE_SOLID = 2
TOPO_FILTER_DISTANCE = 0
TOPO_FILTER_HELMHOLTZ = 1
TOPO_FILTER_DENSITY = 2
TOPO_PC_JACOBI = 0
TOPO_PC_GMG = 1
TOPO_PC_LEARNED = 2
TOPO_SYNC_POLL = 0
TOPO_SYNC_NONE = 1
TOPO_S_LEARNED_FALLBACK = 2
TOPO_S_OC_INEXACT = 3
SOLVE_INFO_LEN = 6
LOG_LEN = 8

EXPORTED = [
    "topo_workspace_size", "topo_create", "topo_destroy", "topo_set_loads", "topo_solve",
    "topo_sensitivity", "topo_filter", "topo_oc_update", "topo_iterate", "topo_apply",
    "topo_apply_f32", "topo_set_passive", "topo_density_filter", "topo_diagonal", "topo_filter_rowsums", "topo_timing_enable", "topo_timing_read",
    "topo_sync", "topo_status_string", "topo_filter_taps",
    "topo_precond_num_params", "topo_precond_workspace_size", "topo_precond_attach",
    "topo_precond_set_weights", "topo_precond_get_weights", "topo_precond_config",
    "topo_precond_apply", "topo_precond_backward", "topo_precond_train_step",
    "topo_precond_get_grad", "topo_precond_harvest", "topo_precond_stats", "topo_timing_read_net",
    "topo_batch_workspace_size", "topo_batch_create", "topo_batch_destroy", "topo_batch_set_loads",
    "topo_batch_iterate", "topo_batch_solution", "topo_batch_tile_shape", "topo_batch_sync",
    "topo_batch_uses_graphs",
    "topo_edm_workspace_size", "topo_edm_count", "topo_edm_fill", "topo_edm_filter",
    "topo_oc_update_noalloc",
    "topo_umesh_workspace_size", "topo_umesh_create", "topo_umesh_destroy",
    "topo_umesh_set_loads", "topo_umesh_midpoints", "topo_umesh_volumes", "topo_umesh_apply",
    "topo_umesh_solve", "topo_umesh_sensitivity", "topo_umesh_iterate", "topo_umesh_sync",
]
OC_NOALLOC_MAX_CELLS = 2147483647
BATCH_REC_LEN = 6


class TopoError(RuntimeError):
    pass


class CProblem(ctypes.Structure):
    _fields_ = [
        ("dim", ctypes.c_int32), ("nel", ctypes.c_int32 * 3), ("split2d", ctypes.c_int32),
        ("nrhs", ctypes.c_int32), ("E0", ctypes.c_double), ("Emin", ctypes.c_double),
        ("nu", ctypes.c_double), ("penal", ctypes.c_double), ("volfrac", ctypes.c_double),
        ("rmin", ctypes.c_double), ("move", ctypes.c_double), ("eta", ctypes.c_double),
        ("rho_min", ctypes.c_double), ("precision", ctypes.c_int32), ("precond", ctypes.c_int32),
        ("rtol", ctypes.c_double), ("maxit", ctypes.c_int32), ("paper_mode", ctypes.c_int32),
        ("warm_start", ctypes.c_int32), ("gmg_dense", ctypes.c_int32), ("filter", ctypes.c_int32),
        ("sync_mode", ctypes.c_int32),
    ]


_lib = None


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    """Loads libtopo.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise TopoError(f"HIP library not built: {path} is missing (run __graft_entry__.build())")
    lib = ctypes.CDLL(path)
    vp, i32, dbl = ctypes.c_void_p, ctypes.c_int, ctypes.c_double
    P = ctypes.POINTER
    lib.topo_workspace_size.argtypes = [P(CProblem), P(ctypes.c_size_t)]
    lib.topo_create.argtypes = [P(CProblem), vp, vp, ctypes.c_size_t, vp, P(vp)]
    lib.topo_destroy.argtypes = [vp]
    lib.topo_set_loads.argtypes = [vp, vp, i32]
    lib.topo_solve.argtypes = [vp, vp, vp, vp]
    lib.topo_sensitivity.argtypes = [vp, vp, vp, vp, vp]
    lib.topo_filter.argtypes = [vp, vp, vp, vp]
    lib.topo_oc_update.argtypes = [vp, vp, vp, vp, vp]
    lib.topo_iterate.argtypes = [vp, vp, vp, i32, dbl, vp, P(i32)]
    lib.topo_apply.argtypes = [vp, vp, vp, vp]
    lib.topo_apply_f32.argtypes = [vp, vp, vp, vp]
    lib.topo_diagonal.argtypes = [vp, vp, vp]
    lib.topo_filter_rowsums.argtypes = [vp, vp]
    lib.topo_set_passive.argtypes = [vp, vp]
    lib.topo_density_filter.argtypes = [vp, vp, vp]
    lib.topo_timing_enable.argtypes = [vp, i32]
    lib.topo_timing_read.argtypes = [vp, P(ctypes.c_int64), P(dbl)]
    lib.topo_timing_read_net.argtypes = [vp, P(ctypes.c_int64), P(dbl)]
    lib.topo_sync.argtypes = [vp, P(i32)]
    lib.topo_precond_num_params.argtypes = [P(ctypes.c_int64)]
    lib.topo_precond_workspace_size.argtypes = [P(CProblem), P(ctypes.c_size_t)]
    lib.topo_precond_attach.argtypes = [vp, vp, ctypes.c_size_t]
    lib.topo_precond_set_weights.argtypes = [vp, vp]
    lib.topo_precond_get_weights.argtypes = [vp, vp]
    lib.topo_precond_config.argtypes = [vp, dbl, i32, i32]
    lib.topo_precond_apply.argtypes = [vp, vp, vp, vp]
    lib.topo_precond_backward.argtypes = [vp, vp, vp]
    lib.topo_precond_train_step.argtypes = [vp, vp, vp, vp, ctypes.c_float, vp]
    lib.topo_precond_get_grad.argtypes = [vp, vp]
    lib.topo_precond_harvest.argtypes = [vp, vp, P(i32), i32, vp, vp, i32, P(i32)]
    lib.topo_precond_stats.argtypes = [vp, P(i32), P(i32)]
    lib.topo_batch_workspace_size.argtypes = [P(CProblem), i32, P(ctypes.c_size_t)]
    lib.topo_batch_create.argtypes = [P(CProblem), i32, vp, vp, ctypes.c_size_t, vp, P(vp)]
    lib.topo_batch_destroy.argtypes = [vp]
    lib.topo_batch_set_loads.argtypes = [vp, vp]
    lib.topo_batch_iterate.argtypes = [vp, vp, i32, dbl, vp, P(i32)]
    lib.topo_batch_solution.argtypes = [vp, vp]
    lib.topo_batch_tile_shape.argtypes = [vp, P(i32), P(i32), P(dbl)]
    lib.topo_batch_sync.argtypes = [vp, P(i32)]
    lib.topo_batch_uses_graphs.argtypes = [vp]
    i64, szt = ctypes.c_int64, ctypes.c_size_t
    lib.topo_edm_workspace_size.argtypes = [i64, P(szt)]
    lib.topo_edm_count.argtypes = [vp, i32, i64, dbl, vp, vp, szt, vp]
    lib.topo_edm_fill.argtypes = [vp, i32, i64, dbl, vp, vp, vp, vp, vp, szt, vp]
    lib.topo_edm_filter.argtypes = [i64, i64, vp, vp, vp, vp, vp, vp, vp, vp]
    lib.topo_filter_taps.argtypes = [i32, i32, dbl, P(ctypes.c_int32), P(ctypes.c_int32)]
    lib.topo_oc_update_noalloc.argtypes = [i64, vp, vp, vp, dbl, dbl, dbl, dbl, vp, vp]
    lib.topo_umesh_workspace_size.argtypes = [i32, i64, i64, i32, P(szt)]
    lib.topo_umesh_create.argtypes = [P(CProblem), i64, i64, vp, vp, vp, vp, szt, vp, P(vp)]
    lib.topo_umesh_destroy.argtypes = [vp]
    lib.topo_umesh_set_loads.argtypes = [vp, vp, i32]
    lib.topo_umesh_midpoints.argtypes = [vp, vp]
    lib.topo_umesh_volumes.argtypes = [vp, vp]
    lib.topo_umesh_apply.argtypes = [vp, vp, vp, vp]
    lib.topo_umesh_solve.argtypes = [vp, vp, vp, vp]
    lib.topo_umesh_sensitivity.argtypes = [vp, vp, vp, vp, vp]
    lib.topo_umesh_iterate.argtypes = [vp, vp, vp, i32, i64, vp, vp, vp, vp, vp]
    lib.topo_umesh_sync.argtypes = [vp, P(i32)]
    lib.topo_status_string.argtypes = [i32]
    lib.topo_status_string.restype = ctypes.c_char_p
    for name in EXPORTED:
        if name != "topo_status_string":
            getattr(lib, name).restype = i32
    _lib = lib
    return lib


def _check(rc: int, what: str) -> None:
    if rc != 0:
        msg = load_library().topo_status_string(rc).decode()
        raise TopoError(f"{what} failed: {rc} ({msg})")


def make_problem(dim: int, nel: Sequence[int], nrhs: int = 1, split: int = TOPO_SPLIT_ALT_ROWS,
                 E0: float = 1.0, Emin: float = 1e-9, nu: float = 0.3, penal: float = 3.0,
                 volfrac: float = 0.5, rmin: float = 1.5, move: float = 0.2, eta: float = 0.5,
                 rho_min: float = 1e-3, precision: int = TOPO_FP64, precond: int = TOPO_PC_JACOBI,
                 rtol: float = 1e-10, maxit: int = 20000, paper_mode: bool = False,
                 warm_start: bool = False, gmg_dense: int = 0,
                 filter: int = 0, sync_mode: int = TOPO_SYNC_POLL) -> CProblem:
    p = CProblem()
    p.dim = int(dim)
    nel3 = list(nel) + [0] * (3 - len(nel))
    for a in range(3):
        p.nel[a] = int(nel3[a])
    p.split2d = int(split)
    p.nrhs = int(nrhs)
    p.E0, p.Emin, p.nu, p.penal = float(E0), float(Emin), float(nu), float(penal)
    p.volfrac, p.rmin, p.move, p.eta, p.rho_min = (float(volfrac), float(rmin), float(move),
                                                   float(eta), float(rho_min))
    p.precision, p.precond = int(precision), int(precond)
    p.rtol, p.maxit = float(rtol), int(maxit)
    p.paper_mode, p.warm_start, p.gmg_dense = int(bool(paper_mode)), int(bool(warm_start)), int(gmg_dense)
    p.filter = int(filter)
    p.sync_mode = int(sync_mode)
    return p


class Topo:
    """One library context on the current CUDA(HIP) device and stream."""

    def __init__(self, cprob: CProblem, fixed_mask: np.ndarray, device="cuda"):
        import torch
        self.torch = torch
        self.lib = load_library()
        self.prob = cprob
        self.dim = cprob.dim
        nel = [cprob.nel[a] for a in range(cprob.dim)]
        self.nel = tuple(nel)
        self.n_nodes = int(np.prod([n + 1 for n in nel]))
        self.n_cells = int(np.prod(nel)) * (2 if cprob.dim == 2 else 6)
        self.nrhs = cprob.nrhs
        self.device = torch.device(device)
        mask = np.ascontiguousarray(fixed_mask, dtype=np.uint8).reshape(-1)
        if mask.size != self.dim * self.n_nodes:
            raise TopoError("fixed mask must have dim * n_nodes entries")
        self._mask = mask
        nbytes = ctypes.c_size_t(0)
        _check(self.lib.topo_workspace_size(ctypes.byref(cprob), ctypes.byref(nbytes)),
               "topo_workspace_size")
        self.ws = torch.empty(int(nbytes.value) + 256, dtype=torch.uint8, device=self.device)
        base = self.ws.data_ptr()
        off = (-base) % 256
        self._ws_ptr = base + off
        self._ws_bytes = int(nbytes.value)
        self.stream = torch.cuda.current_stream(self.device)
        ctx = ctypes.c_void_p()
        _check(self.lib.topo_create(ctypes.byref(cprob), mask.ctypes.data, ctypes.c_void_p(self._ws_ptr),
                                    self._ws_bytes, ctypes.c_void_p(self.stream.cuda_stream),
                                    ctypes.byref(ctx)), "topo_create")
        self.ctx = ctx

    @classmethod
    def from_problem(cls, p, precision=TOPO_FP64, precond=TOPO_PC_JACOBI, rtol=None, maxit=20000,
                     warm_start=False, device="cuda", filter=None, sync_mode=TOPO_SYNC_POLL,
                     gmg_dense=0):
        """Builds a context from any object with the problem attributes
        (dim, nel, split, loads, fixed, E0, Emin, nu, penal, volfrac, rmin,
        move, eta, rho_min, paper_mode, rtol)."""
        cp = make_problem(p.dim, p.nel, p.loads.shape[0], p.split, p.E0, p.Emin, p.nu, p.penal,
                          p.volfrac, p.rmin, p.move, p.eta, p.rho_min, precision, precond,
                          p.rtol if rtol is None else rtol, maxit, p.paper_mode, warm_start,
                          gmg_dense=gmg_dense,
                          filter=getattr(p, "filter", 0) if filter is None else filter,
                          sync_mode=sync_mode)
        t = cls(cp, p.fixed, device)
        import torch
        t.set_loads(torch.as_tensor(np.ascontiguousarray(p.loads), dtype=torch.float64,
                                    device=t.device))
        if getattr(p, "passive", None) is not None:
            t.set_passive(p.passive)
        return t

    # ---------------------------------------------------------------- utils
    def _ptr(self, t, numel: int, name: str, dtype=None):
        torch = self.torch
        if t is None:
            return None
        if dtype is None:
            dtype = torch.float64
        if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
            raise TopoError(f"{name} must be a CUDA tensor")
        if t.dtype != dtype or not t.is_contiguous() or t.numel() != numel:
            raise TopoError(f"{name} must be contiguous {dtype} with {numel} elements")
        return ctypes.c_void_p(t.data_ptr())

    @property
    def n_dofs(self):
        return self.dim * self.n_nodes

    def vec_numel(self):
        return self.nrhs * self.n_dofs

    def close(self):
        if getattr(self, "ctx", None):
            self.lib.topo_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---------------------------------------------------------------- API
    def set_loads(self, f):
        _check(self.lib.topo_set_loads(self.ctx, self._ptr(f, self.vec_numel(), "f"), self.nrhs),
               "topo_set_loads")

    def solve(self, rho, u, info=None):
        _check(self.lib.topo_solve(self.ctx, self._ptr(rho, self.n_cells, "rho"),
                                   self._ptr(u, self.vec_numel(), "u"),
                                   self._ptr(info, SOLVE_INFO_LEN, "info")), "topo_solve")

    def sensitivity(self, rho, u, dc, compliance=None):
        _check(self.lib.topo_sensitivity(self.ctx, self._ptr(rho, self.n_cells, "rho"),
                                         self._ptr(u, self.vec_numel(), "u"),
                                         self._ptr(dc, self.n_cells, "dc"),
                                         self._ptr(compliance, 1, "compliance")), "topo_sensitivity")

    def filter(self, rho, dc, dcf):
        _check(self.lib.topo_filter(self.ctx, self._ptr(rho, self.n_cells, "rho"),
                                    self._ptr(dc, self.n_cells, "dc"),
                                    self._ptr(dcf, self.n_cells, "dcf")), "topo_filter")

    def oc_update(self, rho, dcf, rho_new, scalars=None):
        _check(self.lib.topo_oc_update(self.ctx, self._ptr(rho, self.n_cells, "rho"),
                                       self._ptr(dcf, self.n_cells, "dcf"),
                                       self._ptr(rho_new, self.n_cells, "rho_new"),
                                       self._ptr(scalars, 3, "scalars")), "topo_oc_update")

    def iterate(self, rho, u, max_iter: int, change_tol: float = 0.0, log=None) -> int:
        n = ctypes.c_int(0)
        _check(self.lib.topo_iterate(self.ctx, self._ptr(rho, self.n_cells, "rho"),
                                     self._ptr(u, self.vec_numel(), "u"), int(max_iter),
                                     float(change_tol),
                                     self._ptr(log, int(max_iter) * LOG_LEN, "log"),
                                     ctypes.byref(n)), "topo_iterate")
        return int(n.value)

    def apply(self, rho, x, y):
        _check(self.lib.topo_apply(self.ctx, self._ptr(rho, self.n_cells, "rho"),
                                   self._ptr(x, self.vec_numel(), "x"),
                                   self._ptr(y, self.vec_numel(), "y")), "topo_apply")

    def apply_f32(self, rho, x, y):
        """FP32 apply of the mixed V-cycle's fine level (x, y float32; BF16
        moduli in a TOPO_MIXED_BF16 context, FP32 moduli otherwise)."""
        f32 = self.torch.float32
        _check(self.lib.topo_apply_f32(self.ctx, self._ptr(rho, self.n_cells, "rho"),
                                       self._ptr(x, self.vec_numel(), "x", f32),
                                       self._ptr(y, self.vec_numel(), "y", f32)), "topo_apply_f32")

    def set_passive(self, passive):
        """Installs passive cells (host uint8 [N_c] of TOPO_PASSIVE_*), or
        removes them with None."""
        if passive is None:
            _check(self.lib.topo_set_passive(self.ctx, None), "topo_set_passive")
            return
        a = np.ascontiguousarray(passive, dtype=np.uint8).reshape(-1)
        if a.size != self.n_cells:
            raise TopoError("passive must have one entry per cell")
        self._passive = a
        _check(self.lib.topo_set_passive(self.ctx, a.ctypes.data_as(ctypes.c_void_p)),
               "topo_set_passive")

    def density_filter(self, x, x_phys):
        """x~ = W x / R (distance weights)."""
        _check(self.lib.topo_density_filter(self.ctx, self._ptr(x, self.n_cells, "x"),
                                            self._ptr(x_phys, self.n_cells, "x_phys")),
               "topo_density_filter")

    def diagonal(self, rho, d):
        _check(self.lib.topo_diagonal(self.ctx, self._ptr(rho, self.n_cells, "rho"),
                                      self._ptr(d, self.n_dofs, "d")), "topo_diagonal")

    def filter_rowsums(self, R):
        _check(self.lib.topo_filter_rowsums(self.ctx, self._ptr(R, self.n_cells, "R")),
               "topo_filter_rowsums")

    def timing_enable(self, on: bool = True):
        _check(self.lib.topo_timing_enable(self.ctx, int(bool(on))), "topo_timing_enable")

    def timing_read(self):
        n = ctypes.c_int64(0)
        ms = ctypes.c_double(0.0)
        _check(self.lib.topo_timing_read(self.ctx, ctypes.byref(n), ctypes.byref(ms)),
               "topo_timing_read")
        return int(n.value), float(ms.value)

    def timing_read_net(self):
        n = ctypes.c_int64(0)
        ms = ctypes.c_double(0.0)
        _check(self.lib.topo_timing_read_net(self.ctx, ctypes.byref(n), ctypes.byref(ms)),
               "topo_timing_read_net")
        return int(n.value), float(ms.value)

    def sync(self) -> int:
        st = ctypes.c_int(0)
        _check(self.lib.topo_sync(self.ctx, ctypes.byref(st)), "topo_sync")
        return int(st.value)

    # ------------------------------------------------- learned preconditioner
    def precond_attach(self):
        """Allocates (torch) and attaches the network workspace."""
        nbytes = ctypes.c_size_t(0)
        _check(self.lib.topo_precond_workspace_size(ctypes.byref(self.prob), ctypes.byref(nbytes)),
               "topo_precond_workspace_size")
        self.net_ws = self.torch.empty(int(nbytes.value) + 256, dtype=self.torch.uint8,
                                       device=self.device)
        base = self.net_ws.data_ptr()
        ptr = base + (-base) % 256
        _check(self.lib.topo_precond_attach(self.ctx, ctypes.c_void_p(ptr), int(nbytes.value)),
               "topo_precond_attach")

    def precond_set_weights(self, w):
        _check(self.lib.topo_precond_set_weights(self.ctx, self._ptr(w, num_params(), "w",
                                                                     self.torch.float32)),
               "topo_precond_set_weights")

    def precond_get_weights(self, w):
        _check(self.lib.topo_precond_get_weights(self.ctx, self._ptr(w, num_params(), "w",
                                                                     self.torch.float32)),
               "topo_precond_get_weights")

    def precond_config(self, gamma: float = 1.0, fcg_maxit: int = 500, smooth: int = 1):
        _check(self.lib.topo_precond_config(self.ctx, float(gamma), int(fcg_maxit), int(smooth)),
               "topo_precond_config")

    def precond_apply(self, rho, r, z):
        _check(self.lib.topo_precond_apply(self.ctx, self._ptr(rho, self.n_cells, "rho"),
                                           self._ptr(r, self.n_dofs, "r"),
                                           self._ptr(z, self.n_dofs, "z")), "topo_precond_apply")

    def precond_backward(self, gz, grad):
        _check(self.lib.topo_precond_backward(self.ctx, self._ptr(gz, self.n_dofs, "gz"),
                                              self._ptr(grad, num_params(), "grad",
                                                        self.torch.float32)),
               "topo_precond_backward")

    def precond_train_step(self, rho, r, e, lr: float, loss=None):
        _check(self.lib.topo_precond_train_step(self.ctx, self._ptr(rho, self.n_cells, "rho"),
                                                self._ptr(r, self.n_dofs, "r"),
                                                self._ptr(e, self.n_dofs, "e"), float(lr),
                                                self._ptr(loss, 1, "loss")),
               "topo_precond_train_step")

    def precond_get_grad(self, grad):
        _check(self.lib.topo_precond_get_grad(self.ctx, self._ptr(grad, num_params(), "grad",
                                                                  self.torch.float32)),
               "topo_precond_get_grad")

    def precond_harvest(self, rho, iters, r_out, e_out, presmooth: bool = False):
        """Returns (pairs written, iterations of the solve)."""
        it = np.ascontiguousarray(iters, dtype=np.int32)
        n = it.size
        fin = ctypes.c_int(0)
        rc = self.lib.topo_precond_harvest(
            self.ctx, self._ptr(rho, self.n_cells, "rho"),
            it.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), int(n),
            self._ptr(r_out, n * self.n_dofs, "r_out"), self._ptr(e_out, n * self.n_dofs, "e_out"),
            int(bool(presmooth)), ctypes.byref(fin))
        if rc < 0:
            _check(rc, "topo_precond_harvest")
        return int(rc), int(fin.value)

    def precond_stats(self):
        it = ctypes.c_int(0)
        fb = ctypes.c_int(0)
        _check(self.lib.topo_precond_stats(self.ctx, ctypes.byref(it), ctypes.byref(fb)),
               "topo_precond_stats")
        return int(it.value), int(fb.value)


def num_params() -> int:
    n = ctypes.c_int64(0)
    _check(load_library().topo_precond_num_params(ctypes.byref(n)), "topo_precond_num_params")
    return int(n.value)


class Batch:
    """Many independent 2D problems advanced together (one library batch on
    its own stream).  Vectors are concatenated in instance order."""

    def __init__(self, problems, rtol=None, maxit: int = 20000, device="cuda"):
        import torch
        self.torch = torch
        self.lib = load_library()
        self.device = torch.device(device)
        n = len(problems)
        arr = (CProblem * n)()
        for i, p in enumerate(problems):
            if p.dim != 2 or p.loads.shape[0] != 1:
                raise TopoError("batched instances must be 2D with one load case")
            arr[i] = make_problem(p.dim, p.nel, 1, p.split, p.E0, p.Emin, p.nu, p.penal, p.volfrac,
                                  p.rmin, p.move, p.eta, p.rho_min, TOPO_FP64, TOPO_PC_GMG,
                                  p.rtol if rtol is None else rtol, maxit, p.paper_mode, False)
        self._arr = arr
        self.count = n
        self.n_cells = [int(p.n_cells) for p in problems]
        self.n_dofs = [int(p.n_dofs) for p in problems]
        self.cell_off = np.concatenate([[0], np.cumsum(self.n_cells)]).astype(np.int64)
        self.dof_off = np.concatenate([[0], np.cumsum(self.n_dofs)]).astype(np.int64)
        masks = np.ascontiguousarray(np.concatenate([np.asarray(p.fixed, np.uint8).ravel()
                                                     for p in problems]))
        nbytes = ctypes.c_size_t(0)
        _check(self.lib.topo_batch_workspace_size(arr, n, ctypes.byref(nbytes)),
               "topo_batch_workspace_size")
        self.ws = torch.empty(int(nbytes.value) + 256, dtype=torch.uint8, device=self.device)
        base = self.ws.data_ptr()
        ptr = base + (-base) % 256
        self.stream = torch.cuda.current_stream(self.device)
        h = ctypes.c_void_p()
        _check(self.lib.topo_batch_create(arr, n, masks.ctypes.data, ctypes.c_void_p(ptr),
                                          int(nbytes.value), ctypes.c_void_p(self.stream.cuda_stream),
                                          ctypes.byref(h)), "topo_batch_create")
        self.h = h
        f = np.concatenate([np.asarray(p.loads, np.float64).ravel() for p in problems])
        self.set_loads(torch.as_tensor(f, device=self.device))

    def _ptr(self, t, numel, name):
        torch = self.torch
        if not isinstance(t, torch.Tensor) or t.device.type != "cuda" or t.dtype != torch.float64 \
                or not t.is_contiguous() or t.numel() != numel:
            raise TopoError(f"{name} must be a contiguous float64 CUDA tensor of {numel} elements")
        return ctypes.c_void_p(t.data_ptr())

    @property
    def total_cells(self):
        return int(self.cell_off[-1])

    @property
    def total_dofs(self):
        return int(self.dof_off[-1])

    def set_loads(self, f):
        _check(self.lib.topo_batch_set_loads(self.h, self._ptr(f, self.total_dofs, "f")),
               "topo_batch_set_loads")

    def iterate(self, rho, max_iter: int, change_tol: float = 0.0, record=None) -> int:
        rounds = ctypes.c_int(0)
        rec = None if record is None else self._ptr(record, self.count * BATCH_REC_LEN, "record")
        _check(self.lib.topo_batch_iterate(self.h, self._ptr(rho, self.total_cells, "rho"),
                                           int(max_iter), float(change_tol), rec,
                                           ctypes.byref(rounds)), "topo_batch_iterate")
        return int(rounds.value)

    def solution(self, u):
        _check(self.lib.topo_batch_solution(self.h, self._ptr(u, self.total_dofs, "u")),
               "topo_batch_solution")

    def tile_shape(self):
        bx, by = ctypes.c_int(0), ctypes.c_int(0)
        us = (ctypes.c_double * 3)()
        _check(self.lib.topo_batch_tile_shape(self.h, ctypes.byref(bx), ctypes.byref(by), us),
               "topo_batch_tile_shape")
        return int(bx.value), int(by.value), [float(v) for v in us]

    def uses_graphs(self) -> bool:
        return self.lib.topo_batch_uses_graphs(self.h) == 1

    def sync(self) -> int:
        st = ctypes.c_int(0)
        _check(self.lib.topo_batch_sync(self.h, ctypes.byref(st)), "topo_batch_sync")
        return int(st.value)

    def close(self):
        if getattr(self, "h", None):
            self.lib.topo_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class EdmFilter:
    """Distance-weighted filter over arbitrary cell midpoints: the CSR
    weight matrix and its row sums are built on the device once
    (``topo_edm_count`` then ``topo_edm_fill``); ``filter`` is the
    per-iteration ``topo_edm_filter``."""

    def __init__(self, mid, rmin: float):
        import torch
        self.torch = torch
        self.lib = load_library()
        if not isinstance(mid, torch.Tensor) or mid.device.type != "cuda":
            raise TopoError("mid must be a CUDA tensor")
        if mid.dtype != torch.float64 or mid.dim() != 2 or mid.shape[0] not in (2, 3):
            raise TopoError("mid must be float64 of shape [dim, n], dim 2 or 3")
        self.mid = mid.contiguous()
        self.dim, self.n = int(mid.shape[0]), int(mid.shape[1])
        self.rmin = float(rmin)
        dev = mid.device
        self.stream = torch.cuda.current_stream(dev)
        st = ctypes.c_void_p(self.stream.cuda_stream)
        nbytes = ctypes.c_size_t(0)
        _check(self.lib.topo_edm_workspace_size(self.n, ctypes.byref(nbytes)),
               "topo_edm_workspace_size")
        self.work = torch.empty(int(nbytes.value) + 256, dtype=torch.uint8, device=dev)
        wp = self.work.data_ptr() + (-self.work.data_ptr()) % 256
        self.rowptr = torch.empty(self.n + 1, dtype=torch.int64, device=dev)
        _check(self.lib.topo_edm_count(ctypes.c_void_p(self.mid.data_ptr()), self.dim, self.n,
                                       self.rmin, ctypes.c_void_p(self.rowptr.data_ptr()),
                                       ctypes.c_void_p(wp), int(nbytes.value), st),
               "topo_edm_count")
        self.stream.synchronize()
        self.nnz = int(self.rowptr[-1].item())
        self.col = torch.empty(max(self.nnz, 1), dtype=torch.int32, device=dev)
        self.w = torch.empty(max(self.nnz, 1), dtype=torch.float64, device=dev)
        self.R = torch.empty(max(self.n, 1), dtype=torch.float64, device=dev)
        _check(self.lib.topo_edm_fill(ctypes.c_void_p(self.mid.data_ptr()), self.dim, self.n,
                                      self.rmin, ctypes.c_void_p(self.rowptr.data_ptr()),
                                      ctypes.c_void_p(self.col.data_ptr()),
                                      ctypes.c_void_p(self.w.data_ptr()),
                                      ctypes.c_void_p(self.R.data_ptr()), ctypes.c_void_p(wp),
                                      int(nbytes.value), st), "topo_edm_fill")
        self.work = None   # the hash order is needed only by the fill

    def _vec(self, t, name):
        torch = self.torch
        if (not isinstance(t, torch.Tensor) or t.device.type != "cuda" or t.dtype != torch.float64
                or not t.is_contiguous() or t.numel() != self.n):
            raise TopoError(f"{name} must be a contiguous float64 CUDA tensor of {self.n} elements")
        return ctypes.c_void_p(t.data_ptr())

    def filter(self, rho, dc, dcf):
        if dcf.data_ptr() in (rho.data_ptr(), dc.data_ptr()):
            raise TopoError("dcf must not alias rho or dc")
        _check(self.lib.topo_edm_filter(self.n, self.nnz, ctypes.c_void_p(self.rowptr.data_ptr()),
                                        ctypes.c_void_p(self.col.data_ptr()),
                                        ctypes.c_void_p(self.w.data_ptr()),
                                        ctypes.c_void_p(self.R.data_ptr()), self._vec(rho, "rho"),
                                        self._vec(dc, "dc"), self._vec(dcf, "dcf"),
                                        ctypes.c_void_p(self.stream.cuda_stream)),
               "topo_edm_filter")


class UMesh:
    """The SIMP loop on an arbitrary simplex mesh (topo_umesh_*), on the
    current torch stream.  ``up`` has dim, coords [N, dim], cells
    [N_c, dim+1], fixed [dim][N], loads [nrhs][dim][N] and the SIMP
    parameters (synth.UProblem)."""

    def __init__(self, up, rtol=None, maxit: int = 20000, warm_start: bool = False,
                 sync_mode: int = TOPO_SYNC_POLL, device="cuda"):
        import torch
        self.torch = torch
        self.lib = load_library()
        self.dim, self.nrhs = int(up.dim), int(up.loads.shape[0])
        self.n_nodes, self.n_cells = int(up.coords.shape[0]), int(up.cells.shape[0])
        self.device = torch.device(device)
        cp = make_problem(self.dim, (1,) * self.dim, self.nrhs, TOPO_SPLIT_UNIFORM, up.E0, up.Emin,
                          up.nu, up.penal, up.volfrac, 1.0, up.move, up.eta, up.rho_min, TOPO_FP64,
                          TOPO_PC_JACOBI, up.rtol if rtol is None else rtol, maxit, False,
                          warm_start, sync_mode=sync_mode)
        self.prob = cp
        coords = np.ascontiguousarray(np.asarray(up.coords, dtype=np.float64).T)
        cells = np.ascontiguousarray(np.asarray(up.cells), dtype=np.int32)
        fixed = np.ascontiguousarray(np.asarray(up.fixed), dtype=np.uint8)
        if coords.shape != (self.dim, self.n_nodes) or cells.shape != (self.n_cells, self.dim + 1) \
                or fixed.shape != (self.dim, self.n_nodes):
            raise TopoError("coords [N, dim], cells [N_c, dim+1] and fixed [dim][N] expected")
        nbytes = ctypes.c_size_t(0)
        _check(self.lib.topo_umesh_workspace_size(self.dim, self.n_nodes, self.n_cells, self.nrhs,
                                                  ctypes.byref(nbytes)), "topo_umesh_workspace_size")
        self.ws = torch.empty(int(nbytes.value) + 256, dtype=torch.uint8, device=self.device)
        wp = self.ws.data_ptr() + (-self.ws.data_ptr()) % 256
        self.stream = torch.cuda.current_stream(self.device)
        h = ctypes.c_void_p()
        _check(self.lib.topo_umesh_create(ctypes.byref(cp), self.n_nodes, self.n_cells,
                                          coords.ctypes.data, cells.ctypes.data, fixed.ctypes.data,
                                          ctypes.c_void_p(wp), int(nbytes.value),
                                          ctypes.c_void_p(self.stream.cuda_stream),
                                          ctypes.byref(h)), "topo_umesh_create")
        self.h = h
        self.set_loads(torch.as_tensor(np.ascontiguousarray(up.loads), dtype=torch.float64,
                                       device=self.device))

    def _ptr(self, t, numel, name):
        torch = self.torch
        if t is None:
            return None
        if (not isinstance(t, torch.Tensor) or t.device.type != "cuda" or t.dtype != torch.float64
                or not t.is_contiguous() or t.numel() != numel):
            raise TopoError(f"{name} must be a contiguous float64 CUDA tensor of {numel} elements")
        return ctypes.c_void_p(t.data_ptr())

    @property
    def n_dofs(self):
        return self.dim * self.n_nodes

    def vec_numel(self):
        return self.nrhs * self.n_dofs

    def set_loads(self, f):
        _check(self.lib.topo_umesh_set_loads(self.h, self._ptr(f, self.vec_numel(), "f"), self.nrhs),
               "topo_umesh_set_loads")

    def midpoints(self, mid):
        _check(self.lib.topo_umesh_midpoints(self.h, self._ptr(mid, self.dim * self.n_cells, "mid")),
               "topo_umesh_midpoints")

    def volumes(self, vol):
        _check(self.lib.topo_umesh_volumes(self.h, self._ptr(vol, self.n_cells, "vol")),
               "topo_umesh_volumes")

    def apply(self, rho, x, y):
        _check(self.lib.topo_umesh_apply(self.h, self._ptr(rho, self.n_cells, "rho"),
                                         self._ptr(x, self.vec_numel(), "x"),
                                         self._ptr(y, self.vec_numel(), "y")), "topo_umesh_apply")

    def solve(self, rho, u, info=None):
        _check(self.lib.topo_umesh_solve(self.h, self._ptr(rho, self.n_cells, "rho"),
                                         self._ptr(u, self.vec_numel(), "u"),
                                         self._ptr(info, SOLVE_INFO_LEN, "info")), "topo_umesh_solve")

    def sensitivity(self, rho, u, dc, compliance=None):
        _check(self.lib.topo_umesh_sensitivity(self.h, self._ptr(rho, self.n_cells, "rho"),
                                               self._ptr(u, self.vec_numel(), "u"),
                                               self._ptr(dc, self.n_cells, "dc"),
                                               self._ptr(compliance, 1, "compliance")),
               "topo_umesh_sensitivity")

    def iterate(self, rho, u, max_iter: int, edm, log=None):
        """max_iter SIMP iterations; ``edm`` is an EdmFilter built from this
        mesh's midpoints (its CSR weights and row sums)."""
        _check(self.lib.topo_umesh_iterate(self.h, self._ptr(rho, self.n_cells, "rho"),
                                           self._ptr(u, self.vec_numel(), "u"), int(max_iter),
                                           int(edm.nnz), ctypes.c_void_p(edm.rowptr.data_ptr()),
                                           ctypes.c_void_p(edm.col.data_ptr()),
                                           ctypes.c_void_p(edm.w.data_ptr()),
                                           ctypes.c_void_p(edm.R.data_ptr()),
                                           self._ptr(log, int(max_iter) * LOG_LEN, "log")),
               "topo_umesh_iterate")

    def sync(self) -> int:
        st = ctypes.c_int(0)
        _check(self.lib.topo_umesh_sync(self.h, ctypes.byref(st)), "topo_umesh_sync")
        return int(st.value)

    def close(self):
        if getattr(self, "h", None):
            self.lib.topo_umesh_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def oc_update_noalloc(rho, dcf, rho_new, out, volfrac: float, move: float = 0.2,
                      eta: float = 0.5, rho_min: float = 1e-3) -> None:
    """topo_oc_update_noalloc on the current torch stream of rho's device:
    rho, dcf, rho_new float64 [n]; out float64 [4] (lambda, volume, change,
    status).  Allocates nothing; overlapping calls on one GPU race."""
    import torch
    n = int(rho.numel())
    for t, name, size in ((rho, "rho", n), (dcf, "dcf", n), (rho_new, "rho_new", n),
                          (out, "out", 4)):
        if (not isinstance(t, torch.Tensor) or t.device.type != "cuda"
                or t.dtype != torch.float64 or not t.is_contiguous() or t.numel() != size):
            raise TopoError(f"{name} must be a contiguous float64 CUDA tensor of {size} elements")
    lib = load_library()
    st = torch.cuda.current_stream(rho.device)
    with torch.cuda.device(rho.device):
        _check(lib.topo_oc_update_noalloc(n, ctypes.c_void_p(rho.data_ptr()),
                                          ctypes.c_void_p(dcf.data_ptr()),
                                          ctypes.c_void_p(rho_new.data_ptr()), float(volfrac),
                                          float(move), float(eta), float(rho_min),
                                          ctypes.c_void_p(out.data_ptr()),
                                          ctypes.c_void_p(st.cuda_stream)),
               "topo_oc_update_noalloc")


def status_string(code: int) -> str:
    return load_library().topo_status_string(int(code)).decode()


def check_exports(path: Optional[str] = None):
    """Returns the list of declared entry points missing from the library."""
    lib = ctypes.CDLL(path or LIB_PATH)
    missing = []
    for name in EXPORTED:
        try:
            getattr(lib, name)
        except AttributeError:
            missing.append(name)
    return missing
