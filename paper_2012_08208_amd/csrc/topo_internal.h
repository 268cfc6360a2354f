// Internal definitions of the gfx950 SIMP library: device state, workspace
// layout and kernel launchers.  Element-level arithmetic follows the P1
// Galerkin form of Sec. 3.1 (eq. fe_form) with the isotropic law of Sec. 2
// (eq. str_energy) and the SIMP modulus of eq. simp.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "topo.h"

namespace topo {

// Mixed modes whose FP32 V-cycle preconditions the FP64 flexible CG.
inline bool flex_mixed(const topo_problem& p) {
  return p.precision == TOPO_MIXED_FP32 || p.precision == TOPO_MIXED_BF16;
}

constexpr int kMaxRhs = 4;
constexpr int kRedBlocks = 1024;   // fixed block count of grid-stride reductions
constexpr int kMaxFilterClasses = 6;
constexpr int kOcPasses = 32;      // multiplier passes queued per OC update (early exit)
constexpr int kFcgWindow = 8;                 // directions kept by truncated flexible CG
constexpr int kFcgRing = kFcgWindow + 1;      // ring slots (window + the new direction)

// Scalars that live in device memory (part of the workspace).
struct PcgState {
  double rz[kMaxRhs];
  double rz_old[kMaxRhs];
  double pq[kMaxRhs];
  double alpha[kMaxRhs];
  double beta[kMaxRhs];
  double rr[kMaxRhs];
  double ff[kMaxRhs];
  double tol2[kMaxRhs];
  int active[kMaxRhs];
  int done;
  int iters;
  int breakdown;
  int iters_prev;   // iterations of an abandoned learned-preconditioner run
  int iters_sum;    // iterations of the restart passes of one run
};

// Helmholtz filter solve (Jacobi-preconditioned CG on one scalar field)
struct HelmState {
  double rz, rz_old, pq, alpha, beta, rr, bb, tol2;
  int done, iters, breakdown, pad;
};

// Constant cell matrices of the Helmholtz operator r^2 K + M: one cube
// (A[0], corners c = cx + 2 cy + 4 cz), or the two square splits (A[0]
// diagonal A, A[1] diagonal B, corners c = cx + 2 cy); bit t of
// cells_of_corner[s][c] is set when cell t of the cube (square, split s)
// has corner c as a vertex; w_rhs = |T| / (d+1).
struct HelmCoef {
  double A[2][8][8];
  double w_rhs;
  uint8_t cells_of_corner[2][8];
};

struct OcState {
  double target;
  double mu, mu_lo, mu_hi;
  double V, S;
  double sum_lo, sum_hi, sum_a;
  double lam;
  double vol;
  double change;
  int done;
  int passes;
  int infeasible;
  int pad;
};

// Mixed-precision iterative refinement: FP64 true residual per load case.
struct IrState {
  double rr[kMaxRhs], ff[kMaxRhs], tol2[kMaxRhs], rr_prev[kMaxRhs];
  int active[kMaxRhs];
  int done;        // all load cases at rtol (read by the host with the next field)
  int stagnated;   // a refinement step failed to halve a residual norm
  int outer;
  int inner_total;
};

struct DevScalars {
  PcgState pcg;
  IrState ir;
  OcState oc;
  HelmState helm;
  double compliance;
  double c_energy;
  double c_paper;
  double scratch[8];
  int restart;      // mixed-precision CG: true residual above tolerance
  int status;       // sticky device status
  int pass_skip;    // no-wait solves: 1 while no true-residual restart is due
  int ru_skip;      // reliable-update CG: 0 while an FP64 update is due
  double ru_rr_max[kMaxRhs];   // reliable-update CG: ||r||^2 at the last update
  unsigned counters[16];  // last-block-done counters, one per reduction site
  double fcg_pq[kFcgRing][kMaxRhs];       // (p_j, K p_j) of the ring slots
  double fcg_beta[kFcgWindow][kMaxRhs];   // orthogonalisation coefficients
};

enum CounterId {
  CNT_APPLY_DOT = 0,
  CNT_PCG_INIT = 1,
  CNT_PCG_UPDATE = 2,
  CNT_DOT = 3,
  CNT_SENS = 4,
  CNT_OC_INIT = 5,
  CNT_OC_PASS = 6,
  CNT_OC_FINAL = 7,
  CNT_IR = 8,
};

// Filter stencil entry: neighbour cell offset (di, dj, dk) in unit cells,
// neighbour class tb, weight w = rmin - |x_a - x_b| > 0.
struct FilterTap {
  int32_t di, dj, dk, tb;
  double w;
};

// 3D filter tap as an offset into the LDS box of filter3d_tiled_kernel
struct TiledTap {
  int32_t off, pad;
  double w;
};

struct Grid {
  int dim;
  int nx, ny, nz;      // cells per axis (nz = 1 in 2D for sizing convenience)
  int64_t nn;          // nodes
  int64_t nc;          // cells
  int64_t nd;          // dofs per load case = dim * nn
  int split;           // 2D split rule
};

struct Material {
  double lam0, mu0;    // unit-modulus Lame constants of the element law
  double vol;          // cell measure |T| (1/2 or 1/6)
  double E0, Emin, penal;
  int paper;
};

// Geometry and boundary mask of one grid level as seen by the operator
// kernels (the fine grid, or a multigrid level).
struct OpDesc {
  int dim, nx, ny, nz;  // cells per axis (nz = 1 in 2D)
  int64_t nn;           // nodes
  int split_uniform;    // 2D: 1 = diagonal A everywhere
  const uint8_t* mask;  // [nn] fixed-component bits
  int kz;               // z-chunk of the 3D sweep
};

// One multigrid level (level 0 is the fine grid and borrows the context's
// moduli, diagonal and mask; its right-hand side and solution are the CG
// residual and preconditioned residual).
struct GmgLevel {
  OpDesc op;
  int64_t nc;
  double* E;                   // [nc] moduli
  double* invd;                // [dim*nn] inverse diagonal
  float* E32;                  // [nc] FP32 moduli (mixed precision)
  const uint16_t* E16;         // [nc] BF16 moduli (fine level of TOPO_MIXED_BF16, else null)
  float* invd32;               // [dim*nn] FP32 inverse diagonal (mixed precision)
  double *b, *x, *r, *d, *q;   // [nrhs][dim*nn]
  double *pv, *pw;             // [dim*nn] power-iteration vectors
  double* lmax;                // device scalar: lambda_max(D^-1 K) estimate
  double* pscale;              // device scalar: power-iteration scale
  double* Ainv;                // coarsest level: dense inverse [n*n], or [np*np] when np > 0
  float* Ainv32;               // coarsest level with np > 0, mixed precision: FP32 copy [np*np]
  double* gj;                  // coarsest level with np > 0: elimination scratch [64*64 + np*64]
  int np;                      // coarsest level above 128 DOFs: n rounded up to kGjBlock, else 0
  uint8_t* mask;               // [nn]
  size_t off_E, off_invd, off_b, off_x, off_r, off_d, off_q, off_pv, off_pw, off_mask, off_A,
      off_E32, off_invd32, off_A32, off_gj;
};

struct WsLayout {
  size_t mask, f, E, E32, E16, invd, invd32, r, p, q, z, wv, partials, scal, R, taps, ttaps,
      qsoa, dc, dcf, rho_new, rho_tmp, passive, helm, rho_phys, dv, r32, p32, q32, z32, z32b, x32, gmg_scal, pring, qring, total;
  std::vector<GmgLevel> levels;   // offsets only (pointers filled at creation)
};

struct NetState;

// Snapshots of the CG iterate x_k at chosen iterations k (training-data
// harvest): x_k of the i-th listed iteration goes to dst + i * nd.
struct Capture {
  const int* iters;  // host, ascending
  int n;
  int next;
  double* dst;
  long nd;
};

struct LevelDims {
  int nx, ny, nz;
};
// Largest coarsest level (DOFs) that the multigrid hierarchy solves
// directly: topo_problem.gmg_dense, else kDense3 (TOPO_GMG_DENSE overrides
// it).  Up to 128 DOFs the inverse comes from one work-group's Gauss-Jordan
// elimination, above from the symmetric block sweep over the whole GPU.  At most
// kDense3: the dense solve stages 4 FP64 right-hand sides of that length in
// 64 KiB of LDS.
constexpr int kDense3 = 2048;
constexpr int kGjBlock = 64;
int gmg_dense_max(const topo_problem* p);
std::vector<LevelDims> gmg_plan_dims(int dim, int nx, int ny, int nz, int dense_max = 128);
std::vector<uint8_t> coarse_mask_host(const std::vector<uint8_t>& fm, const LevelDims& f,
                                      const LevelDims& d, int dim);

// Smoother parameters (defaults; TOPO_CHEB_DEGREE, TOPO_CHEB_POST, TOPO_CHEB_LOW,
// TOPO_POWER_ITERS and TOPO_POWER_SAFETY override them; read once at context creation)
struct GmgParams {
  int cheb_kind = 1;      // 1: first-kind Chebyshev on [low lmax, lmax]; 4: fourth kind
  bool fused_post = true; // 3D degree-2 post-smoothing in two fused apply kernels
  int cheb_degree = 2;
  int post_degree = -1;   // post-smoothing degree (-1: cheb_degree)
  double cheb_low = 0.09;
  // 6 Rayleigh-quotient steps: on 192x96x96 x 4 load cases 12 / 8 / 6 / 4
  // steps gave 569 / 568 / 567 / 564 CG iterations over 24 SIMP steps and
  // 14.63 / 14.79 / 14.87 / 15.03 SIMP it/s (an earlier hierarchy); 6 keeps
  // a margin on the estimate for other problems
  int power_iters = 6;
  double power_safety = 1.2;
  // W-cycle: levels below wlevels visit their coarse level twice; -1 picks
  // them by size (3D levels whose coarse level has >= kWCoarseNodes nodes)
  int wlevels = -1;
  bool tail = true;       // FP32 cycles down to <= 128 DOFs: the small levels in one work-group
};

GmgParams gmg_params_env();

struct Ctx {
  topo_problem prob;
  Grid g;
  Material m;
  hipStream_t stream;
  char* ws;
  size_t ws_bytes;
  WsLayout L;
  // typed views into the workspace
  uint8_t* mask;      // [nn] bit c set if component c fixed
  double* f;          // [nrhs][dim][nn]
  double* E;          // [nc]
  float* E32;         // [nc] (mixed precision)
  uint16_t* E16;      // [nc] BF16 bits (TOPO_MIXED_BF16)
  double* invd;       // [dim][nn]
  float* invd32;      // [dim][nn]
  double *r, *p, *q, *z, *wv;  // [nrhs][dim][nn]
  double* partials;   // [kRedBlocks * 16]
  DevScalars* scal;
  double* R;          // [nc] filter row sums
  FilterTap* taps;    // [8][tap_stride], then ntaps[8]
  int tap_stride;     // entries per class list (the longest list, rounded up)
  int ntaps[8];
  int nclasses;
  TiledTap* ttaps;    // 3D: [6][tap_stride] offsets into the tiled filter's LDS box
  bool filter_tiled;  // 3D and every tap within the box's halo
  double* qsoa;       // [nc] filter input in class-major order
  double *dc, *dcf, *rho_new, *rho_tmp;  // [nc]
  uint8_t* passive;   // [nc] TOPO_PASSIVE_* per cell
  double *hx, *hr, *hp, *hq, *hinvd;   // Helmholtz filter: [nn] each (else null)
  HelmCoef hcoef;
  double *rho_phys, *dv;   // density filter: x~ = W x / R and dv = W (1 / R), [nc] (else null)
  bool has_passive;   // a passive set is installed (else the OC ignores the array)
  // mixed-precision inner solve buffers [nrhs][dim][nn]
  float *r32, *p32, *q32, *z32, *z32b, *x32;
  double *pring, *qring;   // truncated flexible CG: [kFcgRing][nrhs][dim][nn]
  bool loads_set;
  // host side
  volatile int* pinned;   // pinned host flags
  hipEvent_t ev_poll[2];
  bool timing;
  // HIP events around timed launches: channel 0 = fine-level operator
  // applies, channel 1 = signal passes of the preconditioner network
  std::vector<std::pair<hipEvent_t, hipEvent_t>> tev[2];
  size_t tev_used[2];
  int64_t t_launches;
  double t_ms;
  int apply_kz;       // z-chunk (node planes) of the 3D apply
  GmgParams gp;       // multigrid switches (environment, read at creation)
  int env_nrb;        // TOPO_APPLY_NRB at creation (0: the built-in policy)
  int env_g;          // TOPO_APPLY_G at creation
  std::vector<GmgLevel> lv;   // multigrid hierarchy (empty for Jacobi)
  NetState* net;              // learned preconditioner (attached on request)
  const int* net_stop;        // device flag that makes network kernels return
  const double* cur_rho;      // density of the solve in progress
  Capture* cap;               // harvest of CG iterates (null otherwise)
  bool smooth_always;         // multigrid kernels ignore the CG stop flag
};

// ---- launchers (defined in the .hip files) ----
void launch_simp_modulus(Ctx* c, const double* rho);
void launch_apply(Ctx* c, const double* x, double* y, int nrhs, bool fuse_dot);
void launch_apply_f32(Ctx* c, const float* x, float* y, int nrhs, bool fuse_dot);
OpDesc fine_op(const Ctx* c);
long apply_grid_blocks(const OpDesc& d, int nrhs, int elem_bytes, int env_nrb);
int apply_rhs_per_block(const OpDesc& d, int nrhs, int elem_bytes, int epi, int env_nrb);
void launch_apply_op(Ctx* c, const OpDesc& d, const double* E, const double* x, double* y,
                     int nrhs, bool fuse_dot, bool timed, const int* stop);
void launch_apply_op_f32(Ctx* c, const OpDesc& d, const float* E, const float* x, float* y,
                         int nrhs, bool timed, const int* stop);
void launch_apply_op_bf16(Ctx* c, const OpDesc& d, const uint16_t* E16, const float* x, float* y,
                          int nrhs, bool timed, const int* stop);
void launch_apply_cheb_pre3d_bf16(Ctx* c, const OpDesc& d, const uint16_t* E16, const float* b,
                                  float* x, const float* invd, const double* lmax, double r_cur,
                                  double r_prev, double low, int kind, int nrhs, const int* stop);
void launch_apply_op_f32_dot(Ctx* c, const OpDesc& d, const float* E, const float* x, float* y,
                             int nrhs);
template <typename T>
void launch_apply_cheb_pre3d(Ctx* c, const OpDesc& d, const T* E, const T* b, T* x, const T* invd,
                             const double* lmax, double r_cur, double r_prev, double low, int kind,
                             int nrhs, const int* stop);
template <typename T>
void launch_apply_cheb_post3d(Ctx* c, const OpDesc& d, const T* E, const uint16_t* E16, T* x,
                              const T* b, T* r, T* dd, const T* invd, const double* lmax,
                              double r_cur, double r_prev, double low, int kind, int nrhs,
                              const int* stop);
void launch_to_f32(Ctx* c, float* dst, const double* src, int64_t n);
void launch_to_f64(Ctx* c, double* dst, const float* src, int64_t n);
int pick_kz(int dim, int nx, int ny, int nz);
void launch_diagonal(Ctx* c, double* d, bool inverse);
void launch_diagonal_op(Ctx* c, const OpDesc& od, const double* E, double* d, bool inverse);
void launch_mask_copy(Ctx* c, const double* src, double* dst, int nrhs);
void launch_mask_copy_f32(Ctx* c, const float* src, float* dst, int nrhs);
void launch_fill(Ctx* c, double* dst, double v, int64_t n);
void pcg_solve(Ctx* c, double* u, double* info);
unsigned red_grid(long n);
void gmg_setup(Ctx* c);
void gmg_vcycle(Ctx* c, const double* b, double* x, int nrhs);
void gmg_vcycle_f32(Ctx* c, const float* b, float* x, int nrhs);
void gmg_fine_smooth(Ctx* c, const double* b, double* x, int nrhs, bool from_zero);
void learned_precondition(Ctx* c, const double* r, double* z, int nrhs);
int pcg_harvest(Ctx* c, const double* rho, const int* iters, int n, double* r_out, double* e_out,
                int presmooth, int* final_iters);
void launch_sensitivity(Ctx* c, const double* rho, const double* u, double* dc, double* compliance);
void launch_filter(Ctx* c, const double* rho, const double* dc, double* dcf);
void launch_filter_rowsums(Ctx* c);
void launch_density_filter(Ctx* c, const double* x, double* out);
void launch_density_volume_weights(Ctx* c, double* dv);
void build_helm_coef(Ctx* c);
void launch_helm_diag(Ctx* c);
void launch_filter_helmholtz(Ctx* c, const double* rho, const double* dc, double* dcf);
void build_filter_taps(Ctx* c);
int filter_taps_host(int dim, int split, double rmin, std::vector<FilterTap>& tab, int* ntaps,
                     int* stride);
int filter_tap_stride(int dim, int split, double rmin);
void oc_update(Ctx* c, const double* rho, const double* dcf, double* rho_new, double* scalars);
void oc_update_plain(hipStream_t s, long nc, const double* rho, const double* dcf,
                     double* rho_new, double volfrac, double move, double eta, double rho_min,
                     double* partials, OcState* st, int* status, double* scalars);
void launch_log_record(Ctx* c, double* rec, const double* info);
int timing_begin(Ctx* c, int chan);
void timing_end(Ctx* c, int chan, int slot);

}  // namespace topo

#define TOPO_HIP(call)                                 \
  do {                                                 \
    hipError_t _e = (call);                            \
    if (_e != hipSuccess) return TOPO_E_HIP;           \
  } while (0)
