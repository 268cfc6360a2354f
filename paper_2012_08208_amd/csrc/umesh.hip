// The SIMP loop on an arbitrary P1 simplex mesh (Sec. 6.1): the operator
// K(rho) of Sec. 3.1 (eq. fe_form) with the SIMP modulus of Sec. 2
// (eq. simp) applied element by element over cells given as node lists,
// Jacobi-preconditioned CG, the compliance sensitivity (Sec. 3.2), the
// midpoint filter of Sec. 3.2.2 on caller-built CSR weights (topo_edm_*,
// Sec. 4.5 and Sec. 6.2) and the OC update of Sec. 3.2.1.
//
// Layout: coordinates and vectors are SoA ([dim][N_n], [nrhs][dim][N_n]);
// cells are [N_c][dim+1] node ids.  At creation the host sorts the cell
// corners by node (a counting sort): corner (e, a) owns slot slot[e][a] of
// the node-sorted incidence list, and node n's incidences are
// [iptr[n], iptr[n+1]).  An apply is two passes, both without atomics:
//   cells: gather x at the corners, strain eps = sum_a sym(x_a (x) g_a),
//          stress sig = |T| E (lambda0 tr eps I + 2 mu0 eps), and write each
//          corner force sig g_a to its slot;
//   nodes: y_n = the sum of the node's slots, in slot order (fixed DOFs 0).
// So every y is the same on every run.  The shape gradients g_a and |T| of
// every cell are formed once from the coordinates (inverse Jacobian).
//
// Inside, nodes and cells are renumbered for locality: nodes in the Morton
// order of their coordinates, cells in the Morton order of their
// midpoints, so a cell's corners and its neighbours' sit close in memory
// however the caller numbered them.  Arguments keep the caller's numbering;
// vectors are permuted at the boundary of each call.
//
// On this mesh the cells differ in volume; the loop follows the listing:
// the filtered sensitivity is the derivative per unit volume,
// s_e = (dc/drho_e) / |T_e|, and the OC volume constraint counts cells.
#include <algorithm>
#include <climits>
#include <vector>

#include "common.h"
#include "shared_dev.h"
#include "topo_internal.h"

namespace topo {

struct UState {
  PcgState pcg;
  OcState oc;
  double compliance;   // sum_r f_r^T u_r
  double c_energy;     // sum_e E_e w_e
  double c_paper;      // sum_e E_e w_e / (2 |T_e|)
  int status;
  int restart;
  int pass_skip;
  int bad_cells;       // degenerate cells met at creation
};

struct UMesh {
  topo_problem prob;
  int dim, nv;
  long nn, nc, ninc;
  hipStream_t stream;
  double lam0, mu0;
  uint8_t* mask;
  int32_t* nperm;   // internal node -> caller node
  int32_t* cperm;   // internal cell -> caller cell
  int32_t* cell;
  int32_t* slot;
  int64_t* iptr;
  double *G, *vol, *mid;
  double* F;
  double *f, *r, *p, *q, *invd, *x;
  double *E, *dc, *s, *sf, *rho_new;
  double* partials;
  UState* st;
  bool loads_set;
  volatile int* pinned;
  hipEvent_t ev[2];
};

namespace {

constexpr int kUBatch = 8;   // CG iterations queued between host polls

struct ULayout {
  size_t mask, nperm, cperm, cell, slot, iptr, G, vol, mid, F, f, r, p, q, invd, x, E, dc, s, sf,
      rho_new, partials, st, total;
};

ULayout u_layout(int dim, long nn, long nc, int nrhs) {
  ULayout L;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off += (bytes + 255) & ~(size_t)255;
    return o;
  };
  const long nv = dim + 1, nd = dim * nn;
  L.mask = take((size_t)nn);
  L.nperm = take((size_t)nn * 4);
  L.cperm = take((size_t)nc * 4);
  L.cell = take((size_t)nc * nv * 4);
  L.slot = take((size_t)nc * nv * 4);
  L.iptr = take((size_t)(nn + 1) * 8);
  L.G = take((size_t)nc * nv * dim * 8);
  L.vol = take((size_t)nc * 8);
  L.mid = take((size_t)dim * nc * 8);
  // corner forces; at creation this region also holds the coordinates
  L.F = take(std::max((size_t)nrhs * dim * nc * nv, (size_t)nd) * 8);
  L.f = take((size_t)nrhs * nd * 8);
  L.r = take((size_t)nrhs * nd * 8);
  L.p = take((size_t)nrhs * nd * 8);
  L.q = take((size_t)nrhs * nd * 8);
  L.invd = take((size_t)nd * 8);
  L.x = take((size_t)nrhs * nd * 8);
  L.E = take((size_t)nc * 8);
  L.dc = take((size_t)nc * 8);
  L.s = take((size_t)nc * 8);
  L.sf = take((size_t)nc * 8);
  L.rho_new = take((size_t)nc * 8);
  L.partials = take((size_t)kRedBlocks * kPartStride * 8);
  L.st = take(sizeof(UState));
  L.total = off;
  return L;
}

bool u_valid(const topo_problem* p) {
  if (!p || (p->dim != 2 && p->dim != 3)) return false;
  if (p->nrhs < 1 || p->nrhs > kMaxRhs) return false;
  if (!(p->volfrac > 0.0 && p->volfrac <= 1.0)) return false;
  if (!(p->penal >= 1.0 && p->penal <= 10.0) || !(p->nu > -1.0 && p->nu < 0.5)) return false;
  if (!(p->E0 > 0.0) || !(p->Emin >= 0.0) || !(p->Emin < p->E0)) return false;
  if (!(p->move > 0.0) || !(p->eta > 0.0) || !(p->rho_min > 0.0 && p->rho_min < 1.0)) return false;
  if (!(p->rtol > 0.0) || p->maxit < 1) return false;
  // FP64 Jacobi CG and the modified SIMP law only
  if (p->precision != TOPO_FP64 || p->precond != TOPO_PC_JACOBI || p->paper_mode) return false;
  if (p->sync_mode != TOPO_SYNC_POLL && p->sync_mode != TOPO_SYNC_NONE) return false;
  return true;
}

}  // namespace

// ------------------------------------------------------------ geometry
// Shape gradients g_a (rows of J^-T with J the edge matrix x_a - x_0,
// g_0 = -sum), |T| = |det J| / dim! and the vertex average of every cell.
template <int DIM>
__global__ void ugeom_kernel(const double* __restrict__ X, const int32_t* __restrict__ cell,
                             const int32_t* __restrict__ cperm, long nn, long nc, double* G,
                             double* vol, double* mid, int* bad) {
  constexpr int NV = DIM + 1;
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nc) return;
  double x[NV][DIM];
  for (int a = 0; a < NV; ++a) {
    const long n = cell[e * NV + a];
    for (int c = 0; c < DIM; ++c) x[a][c] = X[c * nn + n];
  }
  double J[DIM][DIM];   // row a-1: x_a - x_0
  for (int a = 1; a < NV; ++a)
    for (int c = 0; c < DIM; ++c) J[a - 1][c] = x[a][c] - x[0][c];
  double inv[DIM][DIM];  // inverse of J
  double det;
  if (DIM == 2) {
    det = J[0][0] * J[1][1] - J[0][1] * J[1][0];
    inv[0][0] = J[1][1] / det;
    inv[0][1] = -J[0][1] / det;
    inv[1][0] = -J[1][0] / det;
    inv[1][1] = J[0][0] / det;
  } else {
    const double c00 = J[1][1] * J[2][2] - J[1][2] * J[2][1];
    const double c01 = J[1][2] * J[2][0] - J[1][0] * J[2][2];
    const double c02 = J[1][0] * J[2][1] - J[1][1] * J[2][0];
    det = J[0][0] * c00 + J[0][1] * c01 + J[0][2] * c02;
    inv[0][0] = c00 / det;
    inv[1][0] = c01 / det;
    inv[2][0] = c02 / det;
    inv[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) / det;
    inv[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) / det;
    inv[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) / det;
    inv[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) / det;
    inv[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) / det;
    inv[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) / det;
  }
  if (!(fabs(det) > 0.0) || !isfinite(det)) atomicAdd(bad, 1);
  // g_a = column a-1 of J^-1 (the barycentric coordinate lambda_a has
  // gradient row a-1 of J^-T)
  double g0[DIM];
  for (int c = 0; c < DIM; ++c) g0[c] = 0.0;
  for (int a = 1; a < NV; ++a)
    for (int c = 0; c < DIM; ++c) {
      const double gv = inv[c][a - 1];
      G[(e * NV + a) * DIM + c] = gv;
      g0[c] -= gv;
    }
  for (int c = 0; c < DIM; ++c) G[(e * NV) * DIM + c] = g0[c];
  vol[e] = fabs(det) / (DIM == 2 ? 2.0 : 6.0);
  for (int c = 0; c < DIM; ++c) {
    double m = 0.0;
    for (int a = 0; a < NV; ++a) m += x[a][c];
    mid[c * nc + cperm[e]] = m / NV;   // caller's cell order
  }
}

__global__ void umod_kernel(double* E, const double* __restrict__ rho,
                            const int32_t* __restrict__ cperm, long nc, double E0, double Emin,
                            double penal) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nc) return;
  const double r = rho[cperm[e]];
  const double rp = (penal == 3.0) ? r * r * r : pow(r, penal);
  E[e] = Emin + rp * (E0 - Emin);
}

// ------------------------------------------------------------ operator
// Pass 1: corner forces of every cell and load case into their slots.
template <int DIM, int NR>
__global__ __launch_bounds__(256) void uforce_kernel(const double* __restrict__ x,
                                                     const double* __restrict__ E,
                                                     const double* __restrict__ G,
                                                     const double* __restrict__ vol,
                                                     const int32_t* __restrict__ cell,
                                                     const int32_t* __restrict__ slot, double* F,
                                                     long nn, long nc, long ninc, double lam0,
                                                     double mu0, const int* stop) {
  if (stop && *stop) return;
  constexpr int NV = DIM + 1;
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nc) return;
  int nd_[NV], sl[NV];
  double g[NV][DIM];
#pragma unroll
  for (int a = 0; a < NV; ++a) {
    nd_[a] = cell[e * NV + a];
    sl[a] = slot[e * NV + a];
#pragma unroll
    for (int c = 0; c < DIM; ++c) g[a][c] = G[(e * NV + a) * DIM + c];
  }
  const double sc = E[e] * vol[e];
  const double lam = lam0 * sc, mu = mu0 * sc;
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    const double* xr = x + (long)r * DIM * nn;
    double H[DIM][DIM];   // grad u = sum_a x_a (x) g_a
#pragma unroll
    for (int i = 0; i < DIM; ++i)
#pragma unroll
      for (int j = 0; j < DIM; ++j) H[i][j] = 0.0;
#pragma unroll
    for (int a = 0; a < NV; ++a)
#pragma unroll
      for (int i = 0; i < DIM; ++i) {
        const double xv = xr[(long)i * nn + nd_[a]];
#pragma unroll
        for (int j = 0; j < DIM; ++j) H[i][j] += xv * g[a][j];
      }
    double tr = 0.0;
#pragma unroll
    for (int i = 0; i < DIM; ++i) tr += H[i][i];
    double S[DIM][DIM];
#pragma unroll
    for (int i = 0; i < DIM; ++i)
#pragma unroll
      for (int j = 0; j < DIM; ++j) S[i][j] = mu * (H[i][j] + H[j][i]) + (i == j ? lam * tr : 0.0);
    double* Fr = F + (long)r * DIM * ninc;
#pragma unroll
    for (int a = 0; a < NV; ++a)
#pragma unroll
      for (int i = 0; i < DIM; ++i) {
        double v = 0.0;
#pragma unroll
        for (int j = 0; j < DIM; ++j) v += S[i][j] * g[a][j];
        Fr[(long)i * ninc + sl[a]] = v;
      }
  }
}

// Pass 2: y_n = sum of node n's slots (fixed DOFs give 0); with dotp, also
// the per-block partial (p, y) of every load case.
template <int DIM, int NR>
__global__ __launch_bounds__(256) void ugather_kernel(const double* __restrict__ F, double* y,
                                                      const int64_t* __restrict__ iptr,
                                                      const uint8_t* __restrict__ mask, long nn,
                                                      long ninc, const double* __restrict__ dotp,
                                                      double* partials, const int* stop) {
  if (stop && *stop) return;
  double acc[kMaxRhs];
#pragma unroll
  for (int r = 0; r < kMaxRhs; ++r) acc[r] = 0.0;
  for (long n = (long)blockIdx.x * blockDim.x + threadIdx.x; n < nn;
       n += (long)gridDim.x * blockDim.x) {
    const long k0 = iptr[n], k1 = iptr[n + 1];
    const int m = mask[n];
#pragma unroll
    for (int r = 0; r < NR; ++r)
#pragma unroll
      for (int c = 0; c < DIM; ++c) {
        const double* Fr = F + ((long)r * DIM + c) * ninc;
        double v = 0.0;
        for (long k = k0; k < k1; ++k) v += Fr[k];
        if ((m >> c) & 1) v = 0.0;
        const long i = ((long)r * DIM + c) * nn + n;
        y[i] = v;
        if (dotp) acc[r] += v * dotp[i];
      }
  }
  if (partials) {
    const double none[1] = {0.0};
    block_partials<kMaxRhs, 0>(acc, none, partials);
  }
}

// Jacobi diagonal: per corner and component E |T| (lambda0 g_c^2 + mu0
// (|g|^2 + g_c^2)) into the slots, then the node pass sums them.
template <int DIM>
__global__ void udiag_kernel(const double* __restrict__ E, const double* __restrict__ G,
                             const double* __restrict__ vol, const int32_t* __restrict__ slot,
                             double* F, long nc, long ninc, double lam0, double mu0) {
  constexpr int NV = DIM + 1;
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nc) return;
  const double sc = E[e] * vol[e];
  for (int a = 0; a < NV; ++a) {
    double g[DIM], gg = 0.0;
    for (int c = 0; c < DIM; ++c) {
      g[c] = G[(e * NV + a) * DIM + c];
      gg += g[c] * g[c];
    }
    const long s = slot[e * NV + a];
    for (int c = 0; c < DIM; ++c) F[(long)c * ninc + s] = sc * (lam0 * g[c] * g[c] + mu0 * (gg + g[c] * g[c]));
  }
}

__global__ void uinvert_kernel(double* d, const uint8_t* __restrict__ mask, long nn, int dim) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nn * dim) return;
  const long n = i % nn;
  const int c = (int)(i / nn);
  d[i] = ((mask[n] >> c) & 1) ? 1.0 : 1.0 / d[i];
}

// ------------------------------------------------------------ CG kernels
template <int NR>
__global__ __launch_bounds__(256) void uinit_kernel(const double* __restrict__ f,
                                                    const double* __restrict__ Ku, double* u,
                                                    double* r, const uint8_t* __restrict__ mask,
                                                    long nn, int dim, int warm, double* partials,
                                                    const int* gate) {
  if (gate && *gate) return;
  const long nd = nn * dim;
  double acc[2 * NR];
#pragma unroll
  for (int k = 0; k < 2 * NR; ++k) acc[k] = 0.0;
  for (long d = (long)blockIdx.x * blockDim.x + threadIdx.x; d < nd; d += (long)gridDim.x * blockDim.x) {
    const bool fixed = (mask[d % nn] >> (d / nn)) & 1;
#pragma unroll
    for (int k = 0; k < NR; ++k) {
      const long i = (long)k * nd + d;
      const double fv = fixed ? 0.0 : f[i];
      double rv = fv;
      if (warm) {
        rv = fixed ? 0.0 : fv - Ku[i];
        if (fixed) u[i] = 0.0;
      } else {
        u[i] = 0.0;
      }
      r[i] = rv;
      acc[k] += rv * rv;
      acc[NR + k] += fv * fv;
    }
  }
  const double none[1] = {0.0};
  block_partials<2 * NR, 0>(acc, none, partials);
}

template <int NR>
__global__ void uinit_fin(const double* partials, long nb, double rtol, PcgState* st,
                          const int* gate) {
  if (gate && *gate) return;
  __shared__ double tot[2 * NR];
  reduce_partials<2 * NR, 0>(partials, nb, tot);
  if (threadIdx.x == 0) pcg_init_finish<NR>(tot, rtol, st);
}

// first direction p = D^-1 r and (r, D^-1 r)
template <int NR>
__global__ __launch_bounds__(256) void ufirst_kernel(double* p, const double* __restrict__ r,
                                                     const double* __restrict__ invd, long nd,
                                                     double* partials, const PcgState* st) {
  if (st->done) return;
  double acc[NR];
#pragma unroll
  for (int k = 0; k < NR; ++k) acc[k] = 0.0;
  for (long d = (long)blockIdx.x * blockDim.x + threadIdx.x; d < nd; d += (long)gridDim.x * blockDim.x) {
    const double id = invd[d];
#pragma unroll
    for (int k = 0; k < NR; ++k) {
      const double rv = r[(long)k * nd + d];
      p[(long)k * nd + d] = id * rv;
      acc[k] += rv * (id * rv);
    }
  }
  const double none[1] = {0.0};
  block_partials<NR, 0>(acc, none, partials);
}

template <int NR>
__global__ void ufirst_fin(const double* partials, long nb, PcgState* st) {
  if (st->done) return;
  __shared__ double tot[NR];
  reduce_partials<NR, 0>(partials, nb, tot);
  if (threadIdx.x == 0) pcg_rz_finish<NR>(tot, 1, st);
}

__global__ void ualpha_fin(const double* partials, long nb, PcgState* st) {
  if (st->done) return;
  __shared__ double tot[kMaxRhs];
  reduce_partials<kMaxRhs, 0>(partials, nb, tot);
  if (threadIdx.x == 0) pcg_alpha_finish(tot, st);
}

// x += alpha p, r -= alpha q; partials (r, r) and (r, D^-1 r)
template <int NR>
__global__ __launch_bounds__(256) void uupdate_kernel(double* x, double* r,
                                                      const double* __restrict__ p,
                                                      const double* __restrict__ q,
                                                      const double* __restrict__ invd, long nd,
                                                      double* partials, const PcgState* st) {
  if (st->done) return;
  double al[NR];
  bool act[NR];
#pragma unroll
  for (int k = 0; k < NR; ++k) { al[k] = st->alpha[k]; act[k] = st->active[k] != 0; }
  double acc[2 * NR];
#pragma unroll
  for (int k = 0; k < 2 * NR; ++k) acc[k] = 0.0;
  for (long d = (long)blockIdx.x * blockDim.x + threadIdx.x; d < nd; d += (long)gridDim.x * blockDim.x) {
    const double id = invd[d];
#pragma unroll
    for (int k = 0; k < NR; ++k) {
      if (!act[k]) continue;
      const long i = (long)k * nd + d;
      x[i] += al[k] * p[i];
      const double rv = r[i] - al[k] * q[i];
      r[i] = rv;
      acc[k] += rv * rv;
      acc[NR + k] += rv * (id * rv);
    }
  }
  const double none[1] = {0.0};
  block_partials<2 * NR, 0>(acc, none, partials);
}

template <int NR>
__global__ void uupdate_fin(const double* partials, long nb, PcgState* st, int* status) {
  if (st->done) return;
  __shared__ double tot[2 * NR];
  reduce_partials<2 * NR, 0>(partials, nb, tot);
  if (threadIdx.x == 0) pcg_update_finish<NR, true>(tot, st, status);
}

// p = D^-1 r + beta p on the load cases still iterating
template <int NR>
__global__ void udir_kernel(double* p, const double* __restrict__ r, const double* __restrict__ invd,
                            long nd, const PcgState* st) {
  if (st->done) return;
  double be[NR];
  bool act[NR];
#pragma unroll
  for (int k = 0; k < NR; ++k) { be[k] = st->beta[k]; act[k] = st->active[k] != 0; }
  for (long d = (long)blockIdx.x * blockDim.x + threadIdx.x; d < nd; d += (long)gridDim.x * blockDim.x) {
    const double id = invd[d];
#pragma unroll
    for (int k = 0; k < NR; ++k) {
      if (!act[k]) continue;
      const long i = (long)k * nd + d;
      p[i] = id * r[i] + be[k] * p[i];
    }
  }
}

// FP64 true residual ||Zf - K u||^2 per load case; restart flag and gate
template <int NR>
__global__ __launch_bounds__(256) void uresid_kernel(const double* __restrict__ f,
                                                     const double* __restrict__ Ku,
                                                     const uint8_t* __restrict__ mask, long nn,
                                                     int dim, double* partials, const int* gate) {
  if (gate && *gate) return;
  const long nd = nn * dim;
  double acc[NR];
#pragma unroll
  for (int k = 0; k < NR; ++k) acc[k] = 0.0;
  for (long d = (long)blockIdx.x * blockDim.x + threadIdx.x; d < nd; d += (long)gridDim.x * blockDim.x) {
    if ((mask[d % nn] >> (d / nn)) & 1) continue;
#pragma unroll
    for (int k = 0; k < NR; ++k) {
      const double rv = f[(long)k * nd + d] - Ku[(long)k * nd + d];
      acc[k] += rv * rv;
    }
  }
  const double none[1] = {0.0};
  block_partials<NR, 0>(acc, none, partials);
}

template <int NR>
__global__ void uresid_fin(const double* partials, long nb, PcgState* st, int* flag, int* skip) {
  if (skip && *skip) return;
  __shared__ double tot[NR];
  reduce_partials<NR, 0>(partials, nb, tot);
  if (threadIdx.x == 0) {
    int again = 0;
    for (int k = 0; k < NR; ++k) {
      st->rr[k] = tot[k];
      if (st->ff[k] > 0.0 && tot[k] > st->tol2[k]) again = 1;
    }
    *flag = again;
    if (skip) *skip = !again;
  }
}

__global__ void uiters_kernel(PcgState* st, int mode, const int* gate) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  if (gate && *gate) return;
  if (mode == 0) st->iters_sum = 0;
  else if (mode == 1) st->iters_sum += st->iters;
  else st->iters = st->iters_sum;
}

__global__ void uset_int(int* p, int v) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *p = v;
}

__global__ void uinfo_kernel(const PcgState* st, double* info, int nr, int* status) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  if (info) {
    info[0] = st->iters;
    info[1] = st->done && !st->breakdown;
    for (int k = 0; k < kMaxRhs; ++k)
      info[2 + k] = (k < nr && st->ff[k] > 0.0) ? sqrt(st->rr[k] / st->ff[k]) : 0.0;
  }
  if (st->breakdown) *status = TOPO_S_NUMERIC;
  else if (!st->done && *status == 0) *status = TOPO_S_NOT_CONVERGED;
}

// ------------------------------------------------------------ sensitivity
// w_e = |T_e| sum_r (lambda0 tr(eps)^2 + 2 mu0 eps:eps) (unit modulus),
// dc_e = -p rho^(p-1) (E0 - Emin) w_e, s_e = dc_e / |T_e|; partial sums of
// E_e w_e and E_e w_e / (2 |T_e|).
template <int DIM, int NR>
__global__ __launch_bounds__(256) void usens_kernel(const double* __restrict__ u,
                                                    const double* __restrict__ rho,
                                                    const double* __restrict__ G,
                                                    const double* __restrict__ vol,
                                                    const int32_t* __restrict__ cell,
                                                    const int32_t* __restrict__ cperm, double* dc,
                                                    double* s, long nn, long nc, double lam0,
                                                    double mu0, double E0, double Emin,
                                                    double penal, double* partials) {
  constexpr int NV = DIM + 1;
  double acc[2] = {0.0, 0.0};
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < nc; e += (long)gridDim.x * blockDim.x) {
    int nd_[NV];
    double g[NV][DIM];
    for (int a = 0; a < NV; ++a) {
      nd_[a] = cell[e * NV + a];
      for (int c = 0; c < DIM; ++c) g[a][c] = G[(e * NV + a) * DIM + c];
    }
    double w = 0.0;
    for (int r = 0; r < NR; ++r) {
      const double* ur = u + (long)r * DIM * nn;
      double H[DIM][DIM];
      for (int i = 0; i < DIM; ++i)
        for (int j = 0; j < DIM; ++j) H[i][j] = 0.0;
      for (int a = 0; a < NV; ++a)
        for (int i = 0; i < DIM; ++i) {
          const double uv = ur[(long)i * nn + nd_[a]];
          for (int j = 0; j < DIM; ++j) H[i][j] += uv * g[a][j];
        }
      double tr = 0.0, ee = 0.0;
      for (int i = 0; i < DIM; ++i) tr += H[i][i];
      for (int i = 0; i < DIM; ++i)
        for (int j = 0; j < DIM; ++j) {
          const double eij = 0.5 * (H[i][j] + H[j][i]);
          ee += eij * eij;
        }
      w += lam0 * tr * tr + 2.0 * mu0 * ee;
    }
    const double v = vol[e];
    w *= v;
    const long ec = cperm[e];   // the caller's cell index
    const double rv = rho[ec];
    const double rp1 = (penal == 3.0) ? rv * rv : pow(rv, penal - 1.0);
    const double d = -penal * rp1 * (E0 - Emin) * w;
    dc[ec] = d;
    s[ec] = d / v;
    const double Ee = Emin + rp1 * rv * (E0 - Emin);
    acc[0] += Ee * w;
    acc[1] += Ee * w / (2.0 * v);
  }
  const double none[1] = {0.0};
  block_partials<2, 0>(acc, none, partials);
}

// sum_r f_r^T u_r (partials slot 2)
template <int NR>
__global__ __launch_bounds__(256) void ufu_kernel(const double* __restrict__ f,
                                                  const double* __restrict__ u, long nd,
                                                  double* partials) {
  double acc[1] = {0.0};
  for (long d = (long)blockIdx.x * blockDim.x + threadIdx.x; d < nd; d += (long)gridDim.x * blockDim.x)
#pragma unroll
    for (int k = 0; k < NR; ++k) acc[0] += f[(long)k * nd + d] * u[(long)k * nd + d];
  const double none[1] = {0.0};
  block_partials<1, 0>(acc, none, partials);
}

__global__ void usens_fin(const double* pe, long nbe, const double* pf, long nbf, UState* st,
                          double* compliance) {
  __shared__ double te[2], tf[1];
  reduce_partials<2, 0>(pe, nbe, te);
  reduce_partials<1, 0>(pf, nbf, tf);
  if (threadIdx.x == 0) {
    st->c_energy = te[0];
    st->c_paper = te[1];
    st->compliance = tf[0];
    if (compliance) *compliance = tf[0];
  }
}

// one record of the iteration log (the structured loop's fields)
__global__ void ulog_kernel(const UState* st, double* rec, long nc, int nr) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  rec[0] = st->compliance;
  rec[1] = st->c_paper;
  rec[2] = st->oc.vol / (double)nc;
  rec[3] = st->oc.change;
  rec[4] = st->oc.lam;
  rec[5] = st->pcg.iters;
  double mx = 0.0;
  for (int k = 0; k < nr; ++k)
    if (st->pcg.ff[k] > 0.0) mx = fmax(mx, sqrt(st->pcg.rr[k] / st->pcg.ff[k]));
  rec[6] = mx;
  rec[7] = st->pcg.done && !st->pcg.breakdown;
}

// ------------------------------------------------------------ host side
static unsigned ublocks(long n) { return (unsigned)std::max<long>((n + 255) / 256, 1); }

// the direction update has no reduction: more blocks than the reductions
static unsigned dir_blocks(long n) {
  return (unsigned)std::min<long>(std::max<long>((n + 255) / 256, 1), 8192);
}

template <int DIM, int NR>
static void u_apply(UMesh* m, const double* x, double* y, const double* dotp, const int* stop) {
  hipStream_t s = m->stream;
  uforce_kernel<DIM, NR><<<ublocks(m->nc), 256, 0, s>>>(x, m->E, m->G, m->vol, m->cell, m->slot,
                                                        m->F, m->nn, m->nc, m->ninc, m->lam0,
                                                        m->mu0, stop);
  ugather_kernel<DIM, NR><<<red_grid(m->nn), 256, 0, s>>>(m->F, y, m->iptr, m->mask, m->nn,
                                                          m->ninc, dotp,
                                                          dotp ? m->partials : nullptr, stop);
}

template <int DIM>
static void u_diag(UMesh* m) {
  hipStream_t s = m->stream;
  udiag_kernel<DIM><<<ublocks(m->nc), 256, 0, s>>>(m->E, m->G, m->vol, m->slot, m->F, m->nc,
                                                   m->ninc, m->lam0, m->mu0);
  ugather_kernel<DIM, 1><<<red_grid(m->nn), 256, 0, s>>>(m->F, m->invd, m->iptr, m->mask, m->nn,
                                                         m->ninc, nullptr, nullptr, nullptr);
  uinvert_kernel<<<ublocks(m->nn * DIM), 256, 0, s>>>(m->invd, m->mask, m->nn, DIM);
}

static bool u_poll(UMesh* m, int b) {
  if (m->prob.sync_mode == TOPO_SYNC_NONE) return false;
  const int sl = b & 1;
  (void)hipMemcpyAsync((void*)&m->pinned[sl], &m->st->pcg.done, sizeof(int), hipMemcpyDeviceToHost,
                       m->stream);
  (void)hipEventRecord(m->ev[sl], m->stream);
  if (b == 0) return false;
  (void)hipEventSynchronize(m->ev[sl ^ 1]);
  return m->pinned[sl ^ 1] != 0;
}

// Jacobi PCG for every load case from u (warm) or 0, FP64; after it the
// FP64 true residual is recomputed and CG restarts from u while it exceeds
// rtol (at most three restarts), as the structured solve does.
template <int DIM, int NR>
static void u_solve(UMesh* m, double* u, double* info, bool warm) {
  hipStream_t s = m->stream;
  PcgState* st = &m->st->pcg;
  const long nd = (long)DIM * m->nn;
  const unsigned gb = red_grid(nd);
  const unsigned gn = red_grid(m->nn);
  const bool nowait = m->prob.sync_mode == TOPO_SYNC_NONE;
  int* skip = nowait ? &m->st->pass_skip : nullptr;
  if (nowait) uset_int<<<1, 1, 0, s>>>(skip, 0);
  u_diag<DIM>(m);
  uiters_kernel<<<1, 1, 0, s>>>(st, 0, nullptr);
  const int maxit = m->prob.maxit;
  for (int pass = 0; pass < 4; ++pass) {
    const bool w = warm || pass > 0;
    const int* gate = pass > 0 ? skip : nullptr;
    const int budget = (nowait && pass > 0) ? std::max(16, maxit / 4) : maxit;
    if (w) u_apply<DIM, NR>(m, u, m->q, nullptr, gate);
    uinit_kernel<NR><<<gb, 256, 0, s>>>(m->f, m->q, u, m->r, m->mask, m->nn, DIM, w, m->partials,
                                        gate);
    uinit_fin<NR><<<1, 256, 0, s>>>(m->partials, gb, m->prob.rtol, st, gate);
    ufirst_kernel<NR><<<gb, 256, 0, s>>>(m->p, m->r, m->invd, nd, m->partials, st);
    ufirst_fin<NR><<<1, 256, 0, s>>>(m->partials, gb, st);
    bool stop = false;
    for (int it = 0, b = 0; it < budget && !stop; ++b) {
      const int nbt = std::min(kUBatch, budget - it);
      for (int k = 0; k < nbt; ++k) {
        u_apply<DIM, NR>(m, m->p, m->q, m->p, &st->done);
        ualpha_fin<<<1, 256, 0, s>>>(m->partials, gn, st);
        uupdate_kernel<NR><<<gb, 256, 0, s>>>(u, m->r, m->p, m->q, m->invd, nd, m->partials, st);
        uupdate_fin<NR><<<1, 256, 0, s>>>(m->partials, gb, st, &m->st->status);
        udir_kernel<NR><<<dir_blocks(nd), 256, 0, s>>>(m->p, m->r, m->invd, nd, st);
      }
      it += nbt;
      stop = u_poll(m, b);
    }
    uiters_kernel<<<1, 1, 0, s>>>(st, 1, gate);
    u_apply<DIM, NR>(m, u, m->q, nullptr, gate);
    uresid_kernel<NR><<<gb, 256, 0, s>>>(m->f, m->q, m->mask, m->nn, DIM, m->partials, gate);
    uresid_fin<NR><<<1, 256, 0, s>>>(m->partials, gb, st, &m->st->restart, skip);
    if (nowait) continue;
    (void)hipMemcpyAsync((void*)&m->pinned[2], &m->st->restart, sizeof(int),
                         hipMemcpyDeviceToHost, s);
    (void)hipStreamSynchronize(s);
    if (!m->pinned[2]) break;
  }
  uiters_kernel<<<1, 1, 0, s>>>(st, 2, nullptr);
  uinfo_kernel<<<1, 64, 0, s>>>(st, info, NR, &m->st->status);
}

template <int DIM, int NR>
static void u_sens(UMesh* m, const double* rho, const double* u, double* dc, double* compliance) {
  hipStream_t s = m->stream;
  const unsigned ge = red_grid(m->nc);
  const long nd = (long)DIM * m->nn;
  const unsigned gf = red_grid(nd);
  const topo_problem& p = m->prob;
  double* pe = m->partials;
  double* pf = m->partials + (size_t)kRedBlocks / 2 * kPartStride;
  usens_kernel<DIM, NR><<<std::min(ge, (unsigned)(kRedBlocks / 2)), 256, 0, s>>>(
      u, rho, m->G, m->vol, m->cell, m->cperm, dc, m->s, m->nn, m->nc, m->lam0, m->mu0, p.E0,
      p.Emin, p.penal, pe);
  ufu_kernel<NR><<<std::min(gf, (unsigned)(kRedBlocks / 2)), 256, 0, s>>>(m->f, u, nd, pf);
  usens_fin<<<1, 256, 0, s>>>(pe, std::min(ge, (unsigned)(kRedBlocks / 2)), pf,
                              std::min(gf, (unsigned)(kRedBlocks / 2)), m->st, compliance);
}

// dispatch on (dim, nrhs)
template <template <int, int> class Op, typename... A>
static void u_dispatch(UMesh* m, A... a) {
  const int nr = m->prob.nrhs;
  if (m->dim == 2) {
    switch (nr) {
      case 1: Op<2, 1>::run(m, a...); break;
      case 2: Op<2, 2>::run(m, a...); break;
      case 3: Op<2, 3>::run(m, a...); break;
      default: Op<2, 4>::run(m, a...); break;
    }
  } else {
    switch (nr) {
      case 1: Op<3, 1>::run(m, a...); break;
      case 2: Op<3, 2>::run(m, a...); break;
      case 3: Op<3, 3>::run(m, a...); break;
      default: Op<3, 4>::run(m, a...); break;
    }
  }
}

template <int DIM, int NR>
struct OpApply {
  static void run(UMesh* m, const double* x, double* y) { u_apply<DIM, NR>(m, x, y, nullptr, nullptr); }
};
template <int DIM, int NR>
struct OpSolve {
  static void run(UMesh* m, double* u, double* info, bool warm) { u_solve<DIM, NR>(m, u, info, warm); }
};
template <int DIM, int NR>
struct OpSens {
  static void run(UMesh* m, const double* rho, const double* u, double* dc, double* c) {
    u_sens<DIM, NR>(m, rho, u, dc, c);
  }
};

// caller-ordered nodal vector -> internal order (fixed DOFs zeroed when
// mask is given)
__global__ void uperm_in_kernel(double* dst, const double* __restrict__ src,
                                const int32_t* __restrict__ nperm, const uint8_t* mask, long nn,
                                int dim, long total) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= total) return;
  const long n = i % nn, rc = i / nn;
  double v = src[rc * nn + nperm[n]];
  if (mask && ((mask[n] >> (int)(rc % dim)) & 1)) v = 0.0;
  dst[i] = v;
}

__global__ void uperm_out_kernel(double* dst, const double* __restrict__ src,
                                 const int32_t* __restrict__ nperm, long nn, long total) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= total) return;
  const long n = i % nn, rc = i / nn;
  dst[rc * nn + nperm[n]] = src[i];
}

__global__ void uperm_cells_out_kernel(double* dst, const double* __restrict__ src,
                                       const int32_t* __restrict__ cperm, long nc) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < nc) dst[cperm[e]] = src[e];
}

static void u_in(UMesh* m, double* dst, const double* src, bool masked) {
  const long total = (long)m->prob.nrhs * m->dim * m->nn;
  uperm_in_kernel<<<ublocks(total), 256, 0, m->stream>>>(dst, src, m->nperm,
                                                        masked ? m->mask : nullptr, m->nn, m->dim,
                                                        total);
}

static void u_out(UMesh* m, double* dst, const double* src) {
  const long total = (long)m->prob.nrhs * m->dim * m->nn;
  uperm_out_kernel<<<ublocks(total), 256, 0, m->stream>>>(dst, src, m->nperm, m->nn, total);
}

// Morton (Z-order) keys of points: 21 bits per axis over the bounding box
static std::vector<int32_t> morton_order(const std::vector<double>& pts, int dim, long n) {
  double lo[3] = {0, 0, 0}, hi[3] = {1, 1, 1};
  for (int c = 0; c < dim; ++c) {
    lo[c] = hi[c] = n > 0 ? pts[(size_t)c * n] : 0.0;
    for (long i = 0; i < n; ++i) {
      lo[c] = std::min(lo[c], pts[(size_t)c * n + i]);
      hi[c] = std::max(hi[c], pts[(size_t)c * n + i]);
    }
  }
  std::vector<std::pair<uint64_t, int32_t>> key((size_t)n);
  for (long i = 0; i < n; ++i) {
    uint64_t k = 0;
    uint32_t q[3] = {0, 0, 0};
    for (int c = 0; c < dim; ++c) {
      const double span = hi[c] > lo[c] ? hi[c] - lo[c] : 1.0;
      const double t = (pts[(size_t)c * n + i] - lo[c]) / span;
      q[c] = (uint32_t)std::min(2097151.0, std::max(0.0, t * 2097151.0));
    }
    for (int b = 20; b >= 0; --b)
      for (int c = 0; c < dim; ++c) k = (k << 1) | ((q[c] >> b) & 1u);
    key[(size_t)i] = {k, (int32_t)i};
  }
  std::sort(key.begin(), key.end());
  std::vector<int32_t> order((size_t)n);
  for (long i = 0; i < n; ++i) order[(size_t)i] = key[(size_t)i].second;
  return order;
}

}  // namespace topo

using namespace topo;

struct topo_umesh : topo::UMesh {};

extern "C" {

int topo_umesh_workspace_size(int32_t dim, int64_t n_nodes, int64_t n_cells, int32_t nrhs,
                              size_t* bytes) {
  if (!bytes || (dim != 2 && dim != 3) || nrhs < 1 || nrhs > kMaxRhs) return TOPO_E_INVALID;
  if (n_nodes < 1 || n_cells < 1 || n_nodes > INT32_MAX || n_cells * (dim + 1) > INT32_MAX)
    return TOPO_E_SHAPE;
  *bytes = u_layout(dim, (long)n_nodes, (long)n_cells, nrhs).total;
  return TOPO_OK;
}

int topo_umesh_create(const topo_problem* prob, int64_t n_nodes, int64_t n_cells,
                      const double* coords, const int32_t* cells, const uint8_t* fixed_mask,
                      void* workspace, size_t ws_bytes, void* stream, topo_umesh** out) {
  if (!out || !coords || !cells || !fixed_mask || !workspace) return TOPO_E_INVALID;
  *out = nullptr;
  if (!u_valid(prob)) return TOPO_E_INVALID;
  size_t need = 0;
  int rc = topo_umesh_workspace_size(prob->dim, n_nodes, n_cells, prob->nrhs, &need);
  if (rc != TOPO_OK) return rc;
  if (ws_bytes < need || ((uintptr_t)workspace & 255)) return TOPO_E_WORKSPACE;
  const int dim = prob->dim, nv = dim + 1;
  const long nn = (long)n_nodes, nc = (long)n_cells, ninc = nc * nv;
  for (long k = 0; k < ninc; ++k)
    if (cells[k] < 0 || cells[k] >= nn) return TOPO_E_INVALID;
  // internal numbering: nodes by the Morton order of their coordinates,
  // cells by the Morton order of their vertex averages
  std::vector<double> pts(coords, coords + (size_t)dim * nn);
  const std::vector<int32_t> nperm = morton_order(pts, dim, nn);   // internal -> caller
  std::vector<int32_t> ninv((size_t)nn);
  for (long i = 0; i < nn; ++i) ninv[(size_t)nperm[(size_t)i]] = (int32_t)i;
  std::vector<double> cmid((size_t)dim * nc, 0.0);
  for (long e = 0; e < nc; ++e)
    for (int c = 0; c < dim; ++c) {
      double acc = 0.0;
      for (int a = 0; a < nv; ++a) acc += pts[(size_t)c * nn + cells[e * nv + a]];
      cmid[(size_t)c * nc + e] = acc / nv;
    }
  const std::vector<int32_t> cperm = morton_order(cmid, dim, nc);  // internal -> caller
  std::vector<int32_t> icell((size_t)ninc);
  for (long e = 0; e < nc; ++e)
    for (int a = 0; a < nv; ++a)
      icell[(size_t)(e * nv + a)] = ninv[(size_t)cells[(size_t)cperm[(size_t)e] * nv + a]];
  std::vector<double> icoord((size_t)dim * nn);
  for (int c = 0; c < dim; ++c)
    for (long i = 0; i < nn; ++i)
      icoord[(size_t)c * nn + i] = pts[(size_t)c * nn + nperm[(size_t)i]];
  // node-sorted incidence list (a counting sort of the cell corners)
  std::vector<int64_t> iptr((size_t)nn + 1, 0);
  for (long k = 0; k < ninc; ++k) iptr[(size_t)icell[(size_t)k] + 1] += 1;
  for (long n = 0; n < nn; ++n) iptr[(size_t)n + 1] += iptr[(size_t)n];
  std::vector<int32_t> slot((size_t)ninc);
  {
    std::vector<int64_t> next(iptr.begin(), iptr.end() - 1);
    for (long k = 0; k < ninc; ++k) slot[(size_t)k] = (int32_t)next[(size_t)icell[(size_t)k]]++;
  }
  std::vector<uint8_t> bits((size_t)nn, 0);
  for (int c = 0; c < dim; ++c)
    for (long i = 0; i < nn; ++i)
      if (fixed_mask[(size_t)c * nn + nperm[(size_t)i]]) bits[(size_t)i] |= (uint8_t)(1u << c);
  topo_umesh* m = new topo_umesh();
  m->prob = *prob;
  m->dim = dim;
  m->nv = nv;
  m->nn = nn;
  m->nc = nc;
  m->ninc = ninc;
  m->stream = static_cast<hipStream_t>(stream);
  m->mu0 = 1.0 / (2.0 * (1.0 + prob->nu));
  m->lam0 = dim == 2 ? prob->nu / (1.0 - prob->nu * prob->nu)      // plane stress
                     : prob->nu / ((1.0 + prob->nu) * (1.0 - 2.0 * prob->nu));
  const ULayout L = u_layout(dim, nn, nc, prob->nrhs);
  char* w = static_cast<char*>(workspace);
  m->mask = (uint8_t*)(w + L.mask);
  m->nperm = (int32_t*)(w + L.nperm);
  m->cperm = (int32_t*)(w + L.cperm);
  m->cell = (int32_t*)(w + L.cell);
  m->slot = (int32_t*)(w + L.slot);
  m->iptr = (int64_t*)(w + L.iptr);
  m->G = (double*)(w + L.G);
  m->vol = (double*)(w + L.vol);
  m->mid = (double*)(w + L.mid);
  m->F = (double*)(w + L.F);
  m->f = (double*)(w + L.f);
  m->r = (double*)(w + L.r);
  m->p = (double*)(w + L.p);
  m->q = (double*)(w + L.q);
  m->invd = (double*)(w + L.invd);
  m->x = (double*)(w + L.x);
  m->E = (double*)(w + L.E);
  m->dc = (double*)(w + L.dc);
  m->s = (double*)(w + L.s);
  m->sf = (double*)(w + L.sf);
  m->rho_new = (double*)(w + L.rho_new);
  m->partials = (double*)(w + L.partials);
  m->st = (UState*)(w + L.st);
  void* pin = nullptr;
  bool ok = hipHostMalloc(&pin, 64, hipHostMallocDefault) == hipSuccess;
  m->pinned = (volatile int*)pin;
  ok = ok && hipEventCreateWithFlags(&m->ev[0], hipEventDisableTiming) == hipSuccess &&
       hipEventCreateWithFlags(&m->ev[1], hipEventDisableTiming) == hipSuccess;
  hipStream_t s = m->stream;
  UState zero{};
  auto up = [&](void* dst, const void* src, size_t bytes) {
    ok = ok && hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, s) == hipSuccess;
  };
  up(m->mask, bits.data(), bits.size());
  up(m->nperm, nperm.data(), (size_t)nn * 4);
  up(m->cperm, cperm.data(), (size_t)nc * 4);
  up(m->cell, icell.data(), (size_t)ninc * 4);
  up(m->slot, slot.data(), (size_t)ninc * 4);
  up(m->iptr, iptr.data(), iptr.size() * 8);
  up(m->F, icoord.data(), (size_t)dim * nn * 8);
  up(m->st, &zero, sizeof(zero));
  if (ok) {
    if (dim == 2)
      ugeom_kernel<2><<<ublocks(nc), 256, 0, s>>>(m->F, m->cell, m->cperm, nn, nc, m->G, m->vol,
                                                  m->mid, &m->st->bad_cells);
    else
      ugeom_kernel<3><<<ublocks(nc), 256, 0, s>>>(m->F, m->cell, m->cperm, nn, nc, m->G, m->vol,
                                                  m->mid, &m->st->bad_cells);
    ok = hipMemcpyAsync((void*)&m->pinned[4], &m->st->bad_cells, sizeof(int), hipMemcpyDeviceToHost,
                        s) == hipSuccess;
    ok = ok && hipStreamSynchronize(s) == hipSuccess && hipGetLastError() == hipSuccess;
  }
  if (!ok || m->pinned[4] != 0) {
    const bool bad = ok;
    (void)hipStreamSynchronize(s);   // no copy from the host arrays left in flight
    topo_umesh_destroy(m);
    return bad ? TOPO_E_INVALID : TOPO_E_HIP;
  }
  *out = m;
  return TOPO_OK;
}

int topo_umesh_destroy(topo_umesh* m) {
  if (!m) return TOPO_E_INVALID;
  if (m->pinned) (void)hipHostFree((void*)m->pinned);
  if (m->ev[0]) (void)hipEventDestroy(m->ev[0]);
  if (m->ev[1]) (void)hipEventDestroy(m->ev[1]);
  delete m;
  return TOPO_OK;
}

int topo_umesh_set_loads(topo_umesh* m, const double* f, int nrhs) {
  if (!m || !f) return TOPO_E_INVALID;
  if (nrhs != m->prob.nrhs) return TOPO_E_SHAPE;
  u_in(m, m->f, f, false);
  m->loads_set = true;
  return TOPO_OK;
}

int topo_umesh_midpoints(topo_umesh* m, double* mid) {
  if (!m || !mid) return TOPO_E_INVALID;
  TOPO_HIP(hipMemcpyAsync(mid, m->mid, (size_t)m->dim * m->nc * 8, hipMemcpyDeviceToDevice,
                          m->stream));
  return TOPO_OK;
}

int topo_umesh_volumes(topo_umesh* m, double* vol) {
  if (!m || !vol) return TOPO_E_INVALID;
  uperm_cells_out_kernel<<<ublocks(m->nc), 256, 0, m->stream>>>(vol, m->vol, m->cperm, m->nc);
  return hipGetLastError() == hipSuccess ? TOPO_OK : TOPO_E_HIP;
}

int topo_umesh_apply(topo_umesh* m, const double* rho, const double* x, double* y) {
  if (!m || !rho || !x || !y || x == y) return TOPO_E_INVALID;
  const topo_problem& p = m->prob;
  umod_kernel<<<ublocks(m->nc), 256, 0, m->stream>>>(m->E, rho, m->cperm, m->nc, p.E0, p.Emin,
                                                     p.penal);
  u_in(m, m->q, x, true);
  u_dispatch<OpApply>(m, (const double*)m->q, m->r);
  u_out(m, y, m->r);
  return hipGetLastError() == hipSuccess ? TOPO_OK : TOPO_E_HIP;
}

int topo_umesh_solve(topo_umesh* m, const double* rho, double* u, double* info) {
  if (!m || !rho || !u) return TOPO_E_INVALID;
  if (!m->loads_set) return TOPO_E_STATE;
  const topo_problem& p = m->prob;
  umod_kernel<<<ublocks(m->nc), 256, 0, m->stream>>>(m->E, rho, m->cperm, m->nc, p.E0, p.Emin,
                                                     p.penal);
  if (p.warm_start) u_in(m, m->x, u, false);
  u_dispatch<OpSolve>(m, m->x, info, p.warm_start != 0);
  u_out(m, u, m->x);
  return hipGetLastError() == hipSuccess ? TOPO_OK : TOPO_E_HIP;
}

int topo_umesh_sensitivity(topo_umesh* m, const double* rho, const double* u, double* dc,
                           double* compliance) {
  if (!m || !rho || !u || !dc) return TOPO_E_INVALID;
  if (!m->loads_set) return TOPO_E_STATE;
  u_in(m, m->x, u, false);
  u_dispatch<OpSens>(m, rho, (const double*)m->x, dc, compliance);
  return hipGetLastError() == hipSuccess ? TOPO_OK : TOPO_E_HIP;
}

int topo_umesh_iterate(topo_umesh* m, double* rho, double* u, int max_iter, int64_t nnz,
                       const int64_t* rowptr, const int32_t* col, const double* w,
                       const double* R, double* log) {
  if (!m || !rho || !u || max_iter < 0 || !rowptr || !col || !w || !R || nnz < 0)
    return TOPO_E_INVALID;
  if (!m->loads_set) return TOPO_E_STATE;
  const topo_problem& p = m->prob;
  hipStream_t s = m->stream;
  if (p.warm_start) u_in(m, m->x, u, false);
  for (int it = 0; it < max_iter; ++it) {
    const bool warm = it > 0 || p.warm_start != 0;
    umod_kernel<<<ublocks(m->nc), 256, 0, s>>>(m->E, rho, m->cperm, m->nc, p.E0, p.Emin, p.penal);
    u_dispatch<OpSolve>(m, m->x, (double*)nullptr, warm);
    u_dispatch<OpSens>(m, (const double*)rho, (const double*)m->x, m->dc, (double*)nullptr);
    // the listing filters the derivative per unit volume
    int rc = topo_edm_filter((int64_t)m->nc, nnz, rowptr, col, w, R, rho, m->s, m->sf, s);
    if (rc != TOPO_OK) return rc;
    oc_update_plain(s, m->nc, rho, m->sf, m->rho_new, p.volfrac, p.move, p.eta, p.rho_min,
                    m->partials, &m->st->oc, &m->st->status, nullptr);
    if (log) ulog_kernel<<<1, 1, 0, s>>>(m->st, log + (size_t)it * TOPO_LOG_LEN, m->nc, p.nrhs);
    TOPO_HIP(hipMemcpyAsync(rho, m->rho_new, (size_t)m->nc * 8, hipMemcpyDeviceToDevice, s));
  }
  if (max_iter > 0) u_out(m, u, m->x);
  return hipGetLastError() == hipSuccess ? TOPO_OK : TOPO_E_HIP;
}

int topo_umesh_sync(topo_umesh* m, int* device_status) {
  if (!m) return TOPO_E_INVALID;
  TOPO_HIP(hipStreamSynchronize(m->stream));
  int st = 0;
  TOPO_HIP(hipMemcpy(&st, &m->st->status, sizeof(int), hipMemcpyDeviceToHost));
  int zero = 0;
  TOPO_HIP(hipMemcpy(&m->st->status, &zero, sizeof(int), hipMemcpyHostToDevice));
  if (device_status) *device_status = st;
  return TOPO_OK;
}

}  // extern "C"
