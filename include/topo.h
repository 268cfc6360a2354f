/*
 * topo.h -- C ABI of the MI355X (gfx950) SIMP topology-optimisation library.
 *
 * The library runs one iteration of the SIMP method of arXiv 2012.08208
 * ("A 55-line code for large-scale parallel topology optimization in 2D
 * and 3D") on one GPU, on structured P1 simplex grids:
 *
 *   solve        K(rho) u = f                 (Sec. 3.1, eq. fe_form; Sec. 2, eq. simp)
 *   sensitivity  c = f^T u and dc/drho_e      (Sec. 3.2, sensitivity of f)
 *   filter       s~ = W (rho s) / (rho R)     (Sec. 3.2.2, eq. filter, eq. filter_cond;
 *                                             Sec. 4.5, eq. filter_mat)
 *   oc_update    rho_new by the OC rule       (Sec. 3.2, eq. kkt, eq. update; Sec. 3.2.1)
 *   iterate      the loop of all four         (Sec. 4.3-4.5 and the Appendix code)
 *
 * Conventions (shared by every entry point)
 * -----------------------------------------
 * Grid: nel = (nx, ny[, nz]) unit cells.  Nodes are numbered x-fastest,
 *   n = j*(nx+1) + i (2D), n = (k*(ny+1) + j)*(nx+1) + i (3D).
 * Cells: 2D unit squares are cut into two triangles, e = 2*(j*nx + i) + t.
 *   Diagonal A joins (0,0)-(1,1): t=0 is (0,0),(1,0),(1,1), t=1 is
 *   (0,0),(1,1),(0,1).  Diagonal B joins (1,0)-(0,1): t=0 is (0,0),(1,0),(0,1),
 *   t=1 is (1,0),(1,1),(0,1).  TOPO_SPLIT_ALT_ROWS uses A on even rows and
 *   B on odd rows; TOPO_SPLIT_UNIFORM uses A everywhere.
 *   3D unit cubes are cut into the six Kuhn tetrahedra, e = 6*h + t with
 *   h = (k*ny + j)*nx + i; tetrahedron t follows the t-th permutation pi of
 *   (x,y,z) in lexicographic order and has vertices v0 = corner,
 *   v1 = v0 + e_pi1, v2 = v1 + e_pi2, v3 = corner + (1,1,1).
 * Nodal vectors (loads f, displacements u) are float64 structure-of-arrays
 *   [nrhs][dim][N_n]: load case, component, node.  Densities and
 *   sensitivities are float64 [N_c].
 * Material: unit-modulus isotropic law with Poisson ratio nu (plane stress
 *   in 2D); SIMP modulus E_e = Emin + rho_e^p (E0 - Emin).  paper_mode
 *   switches to the listing's law: E_e = rho_e^p, Lame mu = 0.4,
 *   lambda = 0.6, and the per-cell sensitivity -p rho^(p-1) psi_e
 *   (= dc/drho_e / (2|T_e|)).
 * Dirichlet conditions: a host mask fixed[dim][N_n] (uint8, nonzero = fixed)
 *   given at creation.  The operator is Z K Z with Z zeroing fixed DOFs.
 *
 * Memory, streams, errors
 * -----------------------
 * Every pointer argument is a DEVICE pointer unless marked "host".  The
 * caller owns all buffers, including the workspace given to topo_create;
 * the library allocates no device memory and keeps no caller pointer
 * after a call returns.  All compute calls are ordered on the context's
 * stream (a hipStream_t passed as void*; NULL = default stream) and return
 * without waiting for their kernels, except, in the default
 * TOPO_SYNC_POLL mode, where a solve's length is decided on the device:
 * topo_solve and topo_iterate (and topo_filter with the Helmholtz filter)
 * queue batches of CG iterations and read a pinned converged flag one batch
 * behind.  With topo_problem.sync_mode = TOPO_SYNC_NONE none of the path
 * calls waits (graph-capturable, fixed iteration budgets).  The OC update
 * never waits.  Scalars are written to device memory; topo_sync waits for
 * the stream and returns the sticky device status.  A context is not
 * thread-safe.
 *
 * Return values: 0 = OK; negative = host-detected error (TOPO_E_*), in
 * which case nothing was enqueued.  Device-detected outcomes (not converged,
 * non-finite values, OC infeasible) go to the sticky status read by
 * topo_sync.
 */
#ifndef TOPO_H
#define TOPO_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct topo_ctx topo_ctx;

enum {
  TOPO_OK = 0,
  TOPO_E_INVALID = -1,   /* invalid argument or parameter */
  TOPO_E_SHAPE = -2,     /* sizes / alignment do not match the problem */
  TOPO_E_STATE = -3,     /* call out of order (e.g. solve before set_loads) */
  TOPO_E_HIP = -4,       /* a HIP runtime call failed */
  TOPO_E_WORKSPACE = -7, /* workspace smaller than topo_workspace_size */
  /* sticky device status (topo_sync) */
  TOPO_S_NOT_CONVERGED = 1, /* a solve stopped at maxit; outputs inexact */
  TOPO_S_LEARNED_FALLBACK = 2, /* the learned-preconditioner CG did not converge
                                  within its cap; multigrid PCG finished the
                                  solve (outputs valid) */
  TOPO_S_OC_INEXACT = 3,    /* the OC multiplier search ended (pass budget, or
                               no FP64 point left in its bracket) with the
                               volume more than 1e-12 N_c from volfrac N_c;
                               the design is valid, its volume inexact */
  TOPO_S_NUMERIC = -5,      /* NaN/Inf or CG breakdown (p^T K p <= 0) */
  TOPO_S_OC_INFEASIBLE = -6 /* volfrac*N outside [sum lo, sum hi] */
};

enum { TOPO_SPLIT_ALT_ROWS = 0, TOPO_SPLIT_UNIFORM = 1 };
/* Precision of the solve.
   TOPO_FP64:       everything in FP64.
   TOPO_MIXED_FP32: FP64 conjugate gradients (operator apply, vectors, dot
                    products) preconditioned by a multigrid V-cycle whose
                    operator applies, smoothing and transfers run on FP32
                    vectors with FP32 moduli; Polak-Ribiere (flexible) beta;
                    after convergence the FP64 true residual f - K u is
                    recomputed and CG restarts from u if it exceeds rtol.
                    With the Jacobi preconditioner this is the FP64 solve.
   TOPO_MIXED_IR:   FP64 iterative refinement: true residual in FP64, inner
                    CG on FP32 vectors with the FP32 operator and FP32
                    preconditioner (FP64 dot products) to 1e-4, u += d in
                    FP64; falls back to FP64 CG if a step stagnates.
   TOPO_MIXED_BF16: TOPO_MIXED_FP32 with the V-cycle's fine-level moduli
                    stored in BF16 (each FP64 modulus rounded to nearest,
                    ties to even, 8 significant bits): the fine-level applies
                    and smoothing read 2 bytes per cell instead of 4; vectors
                    and arithmetic stay FP32, coarse levels keep FP32 moduli,
                    and the FP64 outer iteration and true-residual check are
                    unchanged, so the solution meets rtol as in the other
                    modes.  With the Jacobi preconditioner this is the FP64
                    solve.
   TOPO_MIXED_RU:   flexible CG whose vectors are all FP32 (the correction
                    to u, residual, search direction, FP32 operator apply,
                    FP32 V-cycle) with FP64 dot products, and reliable
                    updates in FP64: whenever a load case's residual norm has
                    fallen 10x since the last update, or below rtol, the
                    correction is added to the FP64 u and the FP64 true
                    residual f - K u replaces the FP32 one; a load case stops
                    only when its true residual meets rtol.  With the Jacobi
                    preconditioner this is the FP64 solve. */
enum { TOPO_FP64 = 0, TOPO_MIXED_FP32 = 1, TOPO_MIXED_IR = 2, TOPO_MIXED_BF16 = 3,
       TOPO_MIXED_RU = 4 };
/* Preconditioner of the CG solve.
   TOPO_PC_JACOBI:  z = D^-1 r.
   TOPO_PC_GMG:     one multigrid cycle (Chebyshev-Jacobi smoothing,
                    nested P1 transfers, Galerkin-exact coarse moduli; a
                    W-cycle on the 3D levels whose coarse level has at least
                    512 nodes, else V; the coarsest level, of at most
                    gmg_dense DOFs, solved with its dense inverse).
   TOPO_PC_LEARNED: 3D, TOPO_FP64 only.  Flexible CG (Polak-Ribiere beta)
                    preconditioned by a two-level cycle whose coarse
                    correction is the convolutional network of
                    topo_precond_* below (BF16 MFMA inference); the FP64 true
                    residual judges convergence, and multigrid PCG takes
                    over from the current iterate if the flexible CG hits
                    its iteration cap or breaks down (sticky status
                    TOPO_S_LEARNED_FALLBACK).  Needs topo_precond_attach and
                    topo_precond_set_weights before the first solve. */
enum { TOPO_PC_JACOBI = 0, TOPO_PC_GMG = 1, TOPO_PC_LEARNED = 2 };

/* Sensitivity filter used by topo_filter and topo_iterate.
   TOPO_FILTER_DISTANCE:  the distance-weighted filter of Sec. 3.2.2,
                          s~_a = sum_b W_ab rho_b s_b / (rho_a sum_b W_ab),
                          W_ab = max(0, rmin - |x_a - x_b|), truncated at the
                          domain boundary.
   TOPO_FILTER_HELMHOLTZ: the PDE filter Sec. 6.3 adopts for parallel runs
                          (Lazarov and Sigmund 2011): the P1 solution x of
                          (r^2 K + M) x = T (rho s) with zero normal
                          derivative on the boundary, r = rmin / (2 sqrt 3),
                          K the P1 Laplacian, M the consistent P1 mass,
                          T_ne = |T_e| / (d+1) at the vertices of e; then
                          s~_e = (mean of x over the vertices of e) / rho_e.
                          Solved by Jacobi-preconditioned FP64 CG to a
                          relative residual of 1e-12 (in TOPO_SYNC_POLL
                          mode the call reads the converged flag between
                          batches of iterations, as topo_solve does); a solve
                          that stops at its cap of 4000 iterations (256 in
                          TOPO_SYNC_NONE mode) sets TOPO_S_NOT_CONVERGED.
   TOPO_FILTER_DENSITY:   a density filter on the same weights (not in the
                          paper, whose filter acts on sensitivities): the
                          physics sees x~ = W x / R (R_a = sum_b W_ab) and
                          the design is x.  topo_iterate filters x before the
                          solve and the sensitivity; topo_filter then returns
                          the design gradient by the chain rule,
                          dcf = W (dc / R) (W is symmetric), from dc = dc/dx~;
                          topo_oc_update uses the volume of the filtered
                          design, sum x~ = sum_e dv_e x_e with dv = W (1 / R),
                          and the ratio -dc_e / (lambda dv_e).  topo_solve and
                          topo_sensitivity take x~ (topo_density_filter). */
enum { TOPO_FILTER_DISTANCE = 0, TOPO_FILTER_HELMHOLTZ = 1, TOPO_FILTER_DENSITY = 2 };

/* Problem description (host struct, copied by topo_create). */
typedef struct topo_problem {
  int32_t dim;        /* 2 or 3 */
  int32_t nel[3];     /* cells per axis, each >= 1; nel[2] ignored in 2D */
  int32_t split2d;    /* TOPO_SPLIT_*; ignored in 3D */
  int32_t nrhs;       /* number of load cases, 1..4 (Sec. 5.3: summed) */
  double E0, Emin, nu;        /* 1, 1e-9, 0.3 */
  double penal;               /* p, e.g. 3 */
  double volfrac;             /* k in (0, 1] */
  double rmin;                /* filter radius in cell widths, > 0 */
  double move, eta, rho_min;  /* OC move limit m, damping eta, lower bound */
  int32_t precision;  /* TOPO_FP64 | TOPO_MIXED_FP32 | TOPO_MIXED_IR | TOPO_MIXED_BF16 |
                         TOPO_MIXED_RU */
  int32_t precond;    /* TOPO_PC_JACOBI | TOPO_PC_GMG | TOPO_PC_LEARNED */
  double rtol;        /* stop when ||f_r - K u_r|| <= rtol ||f_r|| for each r */
  int32_t maxit;      /* cap on preconditioned CG iterations per solve */
  int32_t paper_mode; /* 0: E = Emin + rho^p (E0-Emin), exact dc/drho;
                         1: the listing's law, see above */
  int32_t warm_start; /* 1: topo_solve starts from the u it is given */
  int32_t gmg_dense;  /* multigrid: the largest coarsest level, in DOFs, that
                         is solved directly (its dense inverse is built per
                         solve: by Gauss-Jordan elimination in one
                         work-group up to 128 DOFs, else by the symmetric
                         block sweep, block by block);
                         the hierarchy stops at the first level at or
                         below it.  0 = automatic: 2048 (the environment
                         variable TOPO_GMG_DENSE, read at creation,
                         overrides it); otherwise 128..2048 (else
                         TOPO_E_INVALID) */
  int32_t filter;     /* TOPO_FILTER_DISTANCE (0) | TOPO_FILTER_HELMHOLTZ | TOPO_FILTER_DENSITY */
  int32_t sync_mode;  /* TOPO_SYNC_POLL (0) | TOPO_SYNC_NONE, see below */
} topo_problem;

/* Host waits inside the path calls (topo_problem.sync_mode).
   TOPO_SYNC_POLL: the length of a CG solve is decided on the device and the
                   host follows it: topo_solve and topo_iterate copy the
                   device's converged flag to pinned memory after every batch
                   of queued iterations and read it one batch behind (the GPU
                   queue stays one batch deep, so the wait is off the
                   critical path), and read the true-residual restart flag
                   once per solve; the Helmholtz filter does the same, and
                   topo_iterate with change_tol > 0 reads the change once per
                   iteration.  This is the fastest mode.
   TOPO_SYNC_NONE: no call among topo_set_loads, topo_solve,
                   topo_sensitivity, topo_filter, topo_oc_update and
                   topo_iterate waits for the device or reads device memory
                   on the host, so they can be captured in a HIP graph and
                   replayed.  Every solve queues a fixed budget: maxit CG
                   iterations, then up to three true-residual restarts of
                   max(16, maxit / 4) iterations each, all gated on device
                   flags (iterations after convergence, and restarts that are
                   not needed, return at once; each skipped iteration still
                   costs its launches).  A solve that is not converged within
                   the budget sets TOPO_S_NOT_CONVERGED.  The Helmholtz
                   filter queues 256 gated CG iterations.  Restrictions
                   (TOPO_E_INVALID): precision TOPO_MIXED_IR, preconditioner
                   TOPO_PC_LEARNED, and topo_iterate with change_tol > 0 (its
                   stop needs the host). */
enum { TOPO_SYNC_POLL = 0, TOPO_SYNC_NONE = 1 };

/* Length of the per-solve info record written by topo_solve (doubles):
   [0] PCG iterations, [1] converged (1/0), [2..5] final relative residual
   of load cases 0..3 (0 for absent cases). */
#define TOPO_SOLVE_INFO_LEN 6
/* Length of one per-iteration log record written by topo_iterate (doubles):
   [0] compliance c = sum_r f_r^T u_r, [1] the listing's objective
   sum_e rho^p psi_e, [2] volume fraction of the new design, [3] change
   max|rho_new - rho|, [4] Lagrange multiplier, [5] PCG iterations,
   [6] max relative residual over load cases, [7] converged (1/0). */
#define TOPO_LOG_LEN 8

/* Bytes of device workspace topo_create needs for this problem.
   Returns TOPO_E_INVALID for an invalid problem. */
int topo_workspace_size(const topo_problem* prob, size_t* bytes /* host */);

/* Creates a context.  fixed_mask (host, [dim][N_n] uint8) marks Dirichlet
   DOFs.  workspace must be device memory of at least
   topo_workspace_size bytes, 256-byte aligned, owned by the caller and kept
   alive (and otherwise unused) until topo_destroy.  stream is a hipStream_t
   (NULL = default).  Precomputes the filter row sums R_a = sum_b W_ab.
   Synchronises the stream before returning. */
int topo_create(const topo_problem* prob, const uint8_t* fixed_mask /* host */,
                void* workspace, size_t ws_bytes, void* stream, topo_ctx** out /* host */);

/* Releases the host-side context.  The workspace stays the caller's. */
int topo_destroy(topo_ctx* ctx);

/* Copies the loads f [nrhs][dim][N_n] into the workspace (stream-ordered).
   Values on fixed DOFs are ignored.  nrhs must equal the problem's. */
int topo_set_loads(topo_ctx* ctx, const double* f, int nrhs);

/* Solves K(rho) u_r = f_r for every load case by preconditioned CG (Jacobi
   or geometric multigrid) to the problem's rtol, matrix-free.  rho [N_c]
   in [rho_min, 1]; u [nrhs][dim][N_n] output (also the start vector when
   warm_start is set); info (device, may be NULL) receives
   TOPO_SOLVE_INFO_LEN doubles.  The loop checks convergence on the
   device; in TOPO_SYNC_POLL mode the host polls a pinned flag every few
   iterations, in TOPO_SYNC_NONE mode it queues the fixed budget. */
int topo_solve(topo_ctx* ctx, const double* rho, double* u, double* info);

/* Compliance c = sum_r f_r^T u_r (written to *compliance, device scalar)
   and the sensitivity dc [N_c]:
   dc_e = -p rho_e^(p-1) (E0 - Emin) sum_r u_{r,e}^T K0_e u_{r,e}
   (paper_mode: the listing's -p rho^(p-1) psi_e).  compliance may be NULL. */
int topo_sensitivity(topo_ctx* ctx, const double* rho, const double* u, double* dc,
                     double* compliance);

/* Filtered sensitivity dcf_a = sum_b W_ab rho_b dc_b / (rho_a R_a), with
   W_ab = max(0, rmin - |x_a - x_b|) between cell centroids; cells near
   the boundary use only the cells that exist.  dcf must not alias dc. */
int topo_filter(topo_ctx* ctx, const double* rho, const double* dc, double* dcf);

/* OC update: rho_new_e = clamp(rho_e (-dcf_e / lambda)^eta,
   max(rho_min, rho_e - move), min(1, rho_e + move)) with lambda chosen so
   that sum_e rho_new_e = volfrac * N_c (to rounding).  scalars (device,
   may be NULL) receives [lambda, sum_e rho_new_e, max_e |rho_new_e - rho_e|].
   rho_new must not alias rho. */
int topo_oc_update(topo_ctx* ctx, const double* rho, const double* dcf, double* rho_new,
                   double* scalars);

/* Allocation-free OC update, for callers that cannot allocate device memory
   (code under HIP graph capture, tight serving loops, harnesses that forbid
   hipMalloc).  It needs no context and no workspace: it computes what
   topo_oc_update computes for a context of n cells with no passive cells and
   the distance or Helmholtz filter (unit cell volumes), with the same
   kernels in the same order, so the results are the same bits.
   n         cells, 1 <= n <= TOPO_OC_NOALLOC_MAX_CELLS, else TOPO_E_SHAPE.
   rho, dcf  device [n], the design and its filtered sensitivity.
   rho_new   device [n] output; must alias neither input.
   volfrac, move, eta, rho_min   as in topo_problem; 0 < volfrac <= 1,
             move > 0, eta > 0, 0 < rho_min < 1, else TOPO_E_INVALID.
   out       device [4] output: lambda, sum_e rho_new_e, max_e |rho_new_e -
             rho_e|, and the update's status (TOPO_OK, TOPO_S_OC_INEXACT or
             TOPO_S_OC_INFEASIBLE) as a double.
   stream    hipStream_t as void* (NULL = default stream); the call is
             asynchronous and waits for nothing.
   Scratch: one static device array of about 132 KB per GPU (block partial
   sums, multiplier state, status), held until the process ends.  Every call
   on a GPU shares that GPU's array and overwrites it, so calls that overlap
   on one GPU (two streams, two host threads) race; order them on one
   stream.  Calls no hipMalloc/hipFree. */
#define TOPO_OC_NOALLOC_MAX_CELLS ((int64_t)2147483647)
int topo_oc_update_noalloc(int64_t n, const double* rho, const double* dcf, double* rho_new,
                           double volfrac, double move, double eta, double rho_min, double* out,
                           void* stream);

/* Runs up to max_iter SIMP iterations in place on rho [N_c] (solve ->
   sensitivity -> filter -> OC).  change_tol <= 0: exactly max_iter
   iterations; otherwise stop after the first iteration whose change is
   below change_tol (this polls the device once per iteration, so
   TOPO_SYNC_NONE contexts return TOPO_E_INVALID for it).  u
   [nrhs][dim][N_n] is the displacement work/output buffer (warm-started
   across iterations).  log (device, may be NULL) receives max_iter records
   of TOPO_LOG_LEN doubles; *n_done (host, may be NULL) the iterations
   run. */
int topo_iterate(topo_ctx* ctx, double* rho, double* u, int max_iter, double change_tol,
                 double* log, int* n_done /* host */);

/* Operator apply y = Z K(rho) Z x for all nrhs load cases (x, y
   [nrhs][dim][N_n]); the hot kernel of every solve, exported for checks
   and measurement. */
int topo_apply(topo_ctx* ctx, const double* rho, const double* x, double* y);

/* The same apply in FP32 as the mixed-precision V-cycle runs it on the fine
   level (FP32 vectors and arithmetic; FP32 moduli, or BF16 moduli in a
   TOPO_MIXED_BF16 context): x, y [nrhs][dim][N_n] float.  Mixed-precision
   contexts only (else TOPO_E_STATE); exported for checks and measurement
   (the launch is timed when timing is enabled). */
int topo_apply_f32(topo_ctx* ctx, const double* rho, const float* x, float* y);

/* Jacobi diagonal d = diag(K(rho)) on free DOFs and 1 on fixed DOFs,
   d [dim][N_n]. */
int topo_diagonal(topo_ctx* ctx, const double* rho, double* d);

/* Density filter x~ = W x / R with the distance weights of Sec. 3.2.2
   (x, x_phys [N_c], distinct); available in every filter mode. */
int topo_density_filter(topo_ctx* ctx, const double* x, double* x_phys);

/* Filter row sums R [N_c] computed at creation. */
int topo_filter_rowsums(topo_ctx* ctx, double* R);

/* Passive cells (Sec. 5.4): zones whose density is fixed throughout the
   iteration.  passive is a HOST array [N_c] of TOPO_PASSIVE_* values (cell
   order as rho); it is copied into the workspace before the call returns
   (the call synchronises the context's stream), and NULL removes the set.
   From then on every OC update gives void cells rho_min and solid cells 1
   inside each multiplier evaluation, so the volume constraint counts them
   (they add no slope and do not move the multiplier's bracket); the solve,
   sensitivity and filter see them like any other cell.  Returns
   TOPO_E_INVALID for a value above TOPO_PASSIVE_SOLID. */
enum { TOPO_PASSIVE_FREE = 0, TOPO_PASSIVE_VOID = 1, TOPO_PASSIVE_SOLID = 2 };
int topo_set_passive(topo_ctx* ctx, const uint8_t* passive);

/* Kernel timing (host outputs).  When enabled, every launch of the
   operator-apply kernel inside topo_solve/topo_apply is bracketed by HIP
   events on the context stream; topo_timing_read returns the number of
   launches and their summed duration in milliseconds since the last
   reset, and resets.  Reading synchronises the stream. */
int topo_timing_enable(topo_ctx* ctx, int enable);
int topo_timing_read(topo_ctx* ctx, int64_t* launches /* host */, double* total_ms /* host */);
/* The same for the signal passes of the preconditioner network (the twelve
   convolutions and three upsamplings of one application). */
int topo_timing_read_net(topo_ctx* ctx, int64_t* passes /* host */, double* total_ms /* host */);

/* Waits for the context stream; *device_status (host, may be NULL) gets the
   sticky device status (TOPO_OK or a TOPO_S_* value), which is then
   cleared. */
int topo_sync(topo_ctx* ctx, int* device_status /* host */);

/* Host-only: the filter's neighbourhood of an interior cell of each cell
   class (2D: 2 classes, 4 with TOPO_SPLIT_ALT_ROWS (even/odd rows); 3D:
   the 6 Kuhn tetrahedra), i.e. the number of cells b with
   |x_a - x_b| < rmin (Sec. 3.2.2, eq. filter), self included.  These are the
   tap lists the filter kernels walk; every list is stored whole (the
   workspace grows with rmin).  ntaps: host [8], zero past *nclasses.
   Returns TOPO_E_INVALID for dim not 2 or 3, rmin outside (0, 16] or a
   bad split.  Touches no GPU. */
int topo_filter_taps(int32_t dim, int32_t split, double rmin, int32_t* ntaps /* host [8] */,
                     int32_t* nclasses /* host */);

/* Static description of a status or error code. */
const char* topo_status_string(int code);

/* ------------------------------------------------------------------------
 * Learned preconditioner (an addition of this library; the paper has no
 * learned component).  A convolutional encoder-decoder on the FE node grid
 * (nx+1, ny+1, nz+1) maps (node density, residual) to an approximation of
 * the error K^{-1} r.  Definition:
 *   levels: l+1 has ceil(n/2) points per axis, four levels;
 *   every convolution is 3x3x3, zero padding 1, no bias,
 *     y[m, co] = sum_t sum_ci W[co][t][ci] x[s*m + d_t - 1, ci],
 *     tap t = (dz*3 + dy)*3 + dx, stride s in {1, 2};
 *   activation: leaky ReLU, slope 1/8;
 *   upsampling: per axis fine[i] = (coarse[i>>1] + coarse[(i+1)>>1]) / 2
 *     (the second index clamped to the coarse grid);
 *   layers (flat parameter order, W[co][t][ci] each):
 *     e0a 8->16, e0b 16->16, d1 16->32 (s2), e1 32->32, d2 32->64 (s2),
 *     e2 64->64, d3 64->64 (s2), e3 64->64, c2 [up(e3), e2] 128->64,
 *     c1 [up(c2), e1] 96->32, c0 [up(c1), e0b] 48->16, out 16->3 (linear);
 *   input channels: mean density of the incident cells, r_c / rms(r)
 *     (rms = ||r|| / sqrt(3 N_n)), 1 where the node has a fixed component,
 *     three zeros;
 *   output: z = gamma * rms(r) * Z N(input) (Z zeroes fixed DOFs).
 * BF16 weights and activations, FP32 accumulation (MFMA), FP32 master
 * weights and Adam moments.  Training minimises the K-norm error of the
 * prediction, L = (g N - e)^T K (g N - e) / (e^T K e) with r = K e and both
 * scaled by 1/rms(r), by Adam (Kingma and Ba, 2015).
 * The network state lives in a second caller-owned workspace.  All calls
 * need a 3D context; vectors are float64 [3][N_n] of one load case.
 * ---------------------------------------------------------------------- */

/* Number of FP32 parameters of the network. */
int topo_precond_num_params(int64_t* n /* host */);

/* Bytes of the network workspace for this problem (3D only). */
int topo_precond_workspace_size(const topo_problem* prob, size_t* bytes /* host */);

/* Attach a network workspace (256-byte aligned, at least the size above) to
   the context and zero it.  Re-attaching replaces the previous one. */
int topo_precond_attach(topo_ctx* ctx, void* workspace, size_t ws_bytes);

/* Set the FP32 weights (device [n_params], copied) and reset Adam. */
int topo_precond_set_weights(topo_ctx* ctx, const float* w);

/* Copy the current FP32 weights to w (device [n_params]). */
int topo_precond_get_weights(topo_ctx* ctx, float* w);

/* gamma: fixed output gain; fcg_maxit: flexible-CG iterations before the
   multigrid fallback (>= 1); smooth: 1 = two-level cycle with Chebyshev
   smoothing around the network, 0 = the network alone. */
int topo_precond_config(topo_ctx* ctx, double gamma, int fcg_maxit, int smooth);

/* z = gamma * rms(r) * Z N(rho, r): the network alone, one load case.
   Keeps the activations for topo_precond_backward. */
int topo_precond_apply(topo_ctx* ctx, const double* rho, const double* r, double* z);

/* Weight gradient of sum(gz * z) for the z of the last topo_precond_apply
   (gz: float64 [3][N_n]; grad: float32 [n_params], overwritten). */
int topo_precond_backward(topo_ctx* ctx, const double* gz, float* grad);

/* One training step on the pair (r, e = K^{-1} r) at density rho: forward,
   loss L (written to *loss, device double), backward, and an Adam step with
   learning rate lr (lr = 0: gradient only, readable by get_grad). */
int topo_precond_train_step(topo_ctx* ctx, const double* rho, const double* r, const double* e,
                            float lr, double* loss);

/* Copy the last weight gradient to grad (device float32 [n_params]). */
int topo_precond_get_grad(topo_ctx* ctx, float* grad);

/* Training pairs from a multigrid PCG solve of load case 0 (nrhs must be 1)
   at density rho, from u = 0 to rtol: for each listed iteration k
   (host array, ascending, k >= 0) the pair e_k = u* - x_k and r_k = K e_k is
   written to e_out / r_out + i * 3 N_n.  presmooth = 1 replaces each pair by
   the one the network sees inside the learned cycle: x = S r_k (the
   fine-level smoother), (r_k - K x, e_k - x).  Returns (>= 0) the number of
   pairs written, or a TOPO_E_* code; *final_iters (host) = iterations of
   the solve, so pairs with k >= *final_iters are the converged iterate.
   Blocks until done. */
int topo_precond_harvest(topo_ctx* ctx, const double* rho, const int* iters /* host */, int n,
                         double* r_out, double* e_out, int presmooth,
                         int* final_iters /* host */);

/* Statistics of the last TOPO_PC_LEARNED solve (host): flexible-CG
   iterations of its last pass and whether multigrid took over. */
int topo_precond_stats(topo_ctx* ctx, int* fcg_iters, int* fallback);

/* ------------------------------------------------------------------------
 * Batched 2D instances: many independent SIMP problems of different sizes
 * advanced together (the loop of Sec. 4.3-4.5 and the Appendix for every
 * instance).  Every instance has its own grid, loads, supports, volume
 * fraction, filter radius and convergence; kernels are batched across
 * instances and one SIMP round for all of them is three captured HIP graphs
 * (set-up, CG continuation replayed until every instance has converged,
 * update).  Instances stop individually when max |rho_new - rho| falls below
 * the tolerance.  Restrictions: dim 2, nrhs 1, TOPO_FP64, TOPO_PC_GMG, no
 * paper mode, nel >= 2 per axis and more than 128 DOFs per instance.
 * Concatenated layouts (instance order): loads and displacements
 * [inst][2][N_n,i], densities [inst][N_c,i], masks [inst][2][N_n,i].
 * The batch runs on its own stream ordered after the caller's stream; every
 * call below returns after the batch stream has finished its work.
 * ---------------------------------------------------------------------- */
typedef struct topo_batch topo_batch;

/* per-instance record of topo_batch_iterate (doubles): [0] SIMP iterations
   done, [1] last change max|rho_new - rho|, [2] compliance at the last
   solve, [3] volume fraction of the last design, [4] CG iterations summed
   over the run, [5] stopped by the change tolerance (1/0) */
#define TOPO_BATCH_REC_LEN 6

int topo_batch_workspace_size(const topo_problem* probs /* host [count] */, int count,
                              size_t* bytes /* host */);
/* fixed_masks: host, concatenated [inst][2][N_n,i], nonzero = fixed.  The
   create call also measures the fine-level apply for each supported tile
   shape on these grids and keeps the fastest (topo_batch_tile_shape). */
int topo_batch_create(const topo_problem* probs /* host [count] */, int count,
                      const uint8_t* fixed_masks /* host */, void* workspace, size_t ws_bytes,
                      void* stream, topo_batch** out /* host */);
int topo_batch_destroy(topo_batch* batch);
int topo_batch_set_loads(topo_batch* batch, const double* f /* concatenated */);
/* Runs up to max_iter SIMP rounds; rho (concatenated, in/out) starts each
   instance from the given design.  change_tol > 0: an instance stops once
   its change is below it; the call returns when every instance has stopped
   or after max_iter rounds.  Displacements restart from zero and are warm
   started from one round to the next.  record: device
   [count][TOPO_BATCH_REC_LEN] or NULL; *rounds (host) = rounds run. */
int topo_batch_iterate(topo_batch* batch, double* rho, int max_iter, double change_tol,
                       double* record, int* rounds /* host */);
/* displacements of the last solve (concatenated [inst][2][N_n,i]) */
int topo_batch_solution(topo_batch* batch, double* u);
/* chosen fine-level tile shape (threads per block along x and y) and the
   measured apply time of each shape 16x16, 32x8, 64x4 (host, microseconds) */
int topo_batch_tile_shape(topo_batch* batch, int* bx /* host */, int* by /* host */,
                          double* us_per_shape /* host [3] or NULL */);
/* sticky status over instances (TOPO_OK or the most severe TOPO_S_*) */
int topo_batch_sync(topo_batch* batch, int* device_status /* host */);
/* 1 when the rounds run as captured HIP graphs, 0 when capture was not
   available and the kernels are launched directly */
int topo_batch_uses_graphs(topo_batch* batch);

/* ------------------------------------------------------------------------
 * Distance-weighted filter over arbitrary cell midpoints (unstructured
 * meshes): Sec. 3.2.2 (eq. filter, eq. filter_cond) and Sec. 4.5
 * (eq. filter_mat), with the weight matrix built once, outside the
 * iteration loop, by evaluating the Euclidean distance matrix in chunks
 * (Sec. 6.2).  The chunks are the cells of a spatial hash of side rmin, so
 * only blocks of the distance matrix that can hold a positive weight are
 * evaluated.  These calls need no context.
 *
 * mid    device, FP64, SoA [dim][n]: mid[c * n + a] is coordinate c of the
 *        midpoint of cell a; dim is 2 or 3; every coordinate finite.
 * rmin   filter radius in the midpoints' length unit, > 0.
 * W      CSR: rowptr [n + 1] (int64), col [nnz] (int32), w [nnz] (FP64);
 *        W_ab = rmin - |x_a - x_b| for every pair at distance below rmin
 *        (the diagonal included), no other entries, no duplicates.  Row a
 *        lists its columns by hash chunk, then by increasing index; the
 *        order and every value are the same on every run.
 * R      device [n]: R_a = sum_b W_ab, summed in row order.
 * work   device scratch of topo_edm_workspace_size bytes, 256-byte aligned,
 *        owned by the caller.  topo_edm_count leaves in it the hash order
 *        that topo_edm_fill reads: pass the same buffer, unchanged, with the
 *        same mid, dim, n and rmin.
 *
 * Sequence: topo_edm_count writes rowptr; the caller reads nnz = rowptr[n]
 * (after synchronising the stream), allocates col and w, then calls
 * topo_edm_fill; topo_edm_filter is the per-iteration step.  All calls are
 * asynchronous on stream (a hipStream_t as void*; NULL = default stream).
 * Returns TOPO_E_INVALID (dim not 2 or 3, rmin not positive and finite, a
 * needed pointer NULL), TOPO_E_SHAPE (n < 0 or n > 2^31 - 2, nnz < 0),
 * TOPO_E_WORKSPACE (work too small or misaligned) or TOPO_E_HIP; n = 0
 * is valid (rowptr[0] = 0, nothing else is touched).
 */
int topo_edm_workspace_size(int64_t n, size_t* bytes /* host */);
int topo_edm_count(const double* mid, int32_t dim, int64_t n, double rmin, int64_t* rowptr,
                   void* work, size_t work_bytes, void* stream);
int topo_edm_fill(const double* mid, int32_t dim, int64_t n, double rmin, const int64_t* rowptr,
                  int32_t* col, double* w, double* R, void* work, size_t work_bytes,
                  void* stream);
/* eq. filter_mat on the CSR weights (all device arrays, [n] unless noted):
   dcf_a = sum_b W_ab rho_b dc_b / (rho_a R_a).  nnz = rowptr[n] (host value,
   used to pick the lanes per row).  dcf must not alias rho or dc. */
int topo_edm_filter(int64_t n, int64_t nnz, const int64_t* rowptr, const int32_t* col,
                    const double* w, const double* R, const double* rho, const double* dc,
                    double* dcf, void* stream);

/* ------------------------------------------------------------------------
 * The SIMP loop on an arbitrary P1 simplex mesh (Sec. 6.1: the loop runs
 * unchanged on an imported tetrahedral mesh; its filter takes the actual
 * cell midpoints, Sec. 3.2.2, built in chunks, Sec. 6.2).  Triangles (2D,
 * plane stress) or tetrahedra (3D), any node positions and numbering.
 * The operator is applied element by element in two passes without
 * atomics (cells write their corner forces to node-sorted slots, nodes sum
 * their slots in a fixed order), so results are the same on every run.
 * The solve is Jacobi-preconditioned FP64 CG with the FP64 true-residual
 * restarts of topo_solve.  On such a mesh the cells differ in volume; the
 * loop follows the listing: it filters the sensitivity per unit volume,
 * s_e = (dc/drho_e) / |T_e|, and its OC volume constraint counts cells,
 * sum_e rho_e = volfrac * N_c.
 *
 * prob: the topo_problem fields of the material (E0, Emin, nu), SIMP (penal,
 *   volfrac, move, eta, rho_min), solver (rtol, maxit, warm_start,
 *   sync_mode) and nrhs; dim is 2 or 3; nel, split2d, rmin, gmg_dense and
 *   filter are ignored.  precision must be TOPO_FP64, precond
 *   TOPO_PC_JACOBI, paper_mode 0 (else TOPO_E_INVALID).
 * coords: host, FP64 SoA [dim][n_nodes]; cells: host, int32 [n_cells][dim+1]
 *   node ids; fixed_mask: host uint8 [dim][n_nodes], nonzero = fixed.  All
 *   three are copied at creation; a degenerate cell (zero or non-finite
 *   volume) or an out-of-range node id gives TOPO_E_INVALID.
 * Vectors: FP64 [nrhs][dim][n_nodes]; densities and sensitivities FP64
 *   [n_cells] in the caller's cell order.  Workspace, streams, sticky
 *   status and sync_mode behave as for topo_create (the create call
 *   synchronises once).
 * ---------------------------------------------------------------------- */
typedef struct topo_umesh topo_umesh;

/* Workspace bytes; TOPO_E_SHAPE for n_nodes or n_cells below 1, n_nodes
   above 2^31 - 1 or (dim+1) n_cells above 2^31 - 1. */
int topo_umesh_workspace_size(int32_t dim, int64_t n_nodes, int64_t n_cells, int32_t nrhs,
                              size_t* bytes /* host */);
int topo_umesh_create(const topo_problem* prob, int64_t n_nodes, int64_t n_cells,
                      const double* coords /* host */, const int32_t* cells /* host */,
                      const uint8_t* fixed_mask /* host */, void* workspace, size_t ws_bytes,
                      void* stream, topo_umesh** out /* host */);
int topo_umesh_destroy(topo_umesh* m);
/* loads f [nrhs][dim][n_nodes] (device, copied) */
int topo_umesh_set_loads(topo_umesh* m, const double* f, int nrhs);
/* cell midpoints (vertex averages), SoA [dim][n_cells]: the input of
   topo_edm_count / topo_edm_fill for this mesh's filter weights */
int topo_umesh_midpoints(topo_umesh* m, double* mid);
/* cell volumes |T_e| [n_cells] */
int topo_umesh_volumes(topo_umesh* m, double* vol);
/* y = Z K(rho) Z x for every load case (Sec. 3.1, eq. fe_form) */
int topo_umesh_apply(topo_umesh* m, const double* rho, const double* x, double* y);
/* K(rho) u_r = f_r for every load case to rtol; info as topo_solve */
int topo_umesh_solve(topo_umesh* m, const double* rho, double* u, double* info);
/* compliance c = sum_r f_r^T u_r (device scalar, may be NULL) and
   dc_e = -p rho_e^(p-1) (E0 - Emin) sum_r u_{r,e}^T K0_e u_{r,e} */
int topo_umesh_sensitivity(topo_umesh* m, const double* rho, const double* u, double* dc,
                           double* compliance);
/* max_iter SIMP iterations in place on rho: solve, sensitivity per unit
   volume, the midpoint filter on the CSR weights of topo_edm_fill (rowptr,
   col, w, R; nnz = rowptr[n_cells]) built from topo_umesh_midpoints, and
   the OC update by cell count.  u is the displacement work/output buffer
   (warm-started across iterations); log (device, may be NULL) receives
   max_iter records of TOPO_LOG_LEN doubles (as topo_iterate). */
int topo_umesh_iterate(topo_umesh* m, double* rho, double* u, int max_iter, int64_t nnz,
                       const int64_t* rowptr, const int32_t* col, const double* w,
                       const double* R, double* log);
int topo_umesh_sync(topo_umesh* m, int* device_status /* host */);

#ifdef __cplusplus
}
#endif
#endif /* TOPO_H */
