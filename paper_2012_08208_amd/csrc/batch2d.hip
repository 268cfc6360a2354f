// Batched SIMP loop for many independent 2D problems of different sizes
// (Sec. 4.3-4.5 and the Appendix loop, run for every instance at once).
//
// Every instance keeps its own grid, multigrid hierarchy, CG scalars, filter
// taps, OC multiplier and convergence flags; the kernels are batched across
// instances instead.  An (instance, level) pair is a "slot".  Host-built job
// tables hand each work-group one job: a chunk of up to kBChunk elements of
// one slot, or one apply tile of one slot.  Per-instance reductions stay
// deterministic: the jobs of one instance are contiguous, each job writes
// its partial sums, and a one-block-per-instance finaliser reduces that
// instance's job range in a fixed order.  Instances whose CG has converged,
// or whose SIMP loop has stopped (max |rho_new - rho| < tol), return at the
// top of every kernel.
//
// One SIMP round is three captured HIP graphs replayed on the batch stream:
// setup (moduli, diagonals, multigrid set-up, CG start), a continuation of
// kBCgPerGraph CG iterations replayed until every instance has converged,
// and the update (sensitivity, filter, OC, change, convergence flags).  The
// fine-level apply runs with the tile shape the autotuner measured fastest
// on the batch's own fine grids.
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include <new>
#include <vector>

#include "common.h"
#include "dense_dev.h"
#include "element.h"
#include "shared_dev.h"
#include "topo_internal.h"

namespace topo {

constexpr int kBChunk = 2048;      // elements per job
constexpr int kBChunkNode = 256;   // nodes per job of the restriction, prolongation and
                                   // diagonal tables: their gathers, one node per thread,
                                   // are not serialised over a strided loop
constexpr int kBCgPerGraph = 4;    // CG iterations per continuation replay
constexpr int kBOcPasses = 40;     // OC root passes per round (early exit per instance)
constexpr int kBShapes = 3;        // fine-level apply tile shapes: 16x16, 32x8, 64x4

enum BVec { BV_B = 0, BV_X, BV_R, BV_D, BV_Q, BV_PV, BV_PW, BV_F, BV_U, BV_P, BV_CQ, BV_N };

struct BSlot {
  int inst, level, last, parent, child;
  OpDesc op;
  long nc, nd;
  double lam0, mu0, vol;
  double* E;
  double* invd;
  double* v[BV_N];
  double* Ainv;                // last level: dense inverse [nd*nd], or [np*np] when np > 0
  int np;                      // last level above 128 DOFs: nd rounded up to kGjBlock, else 0
  double* gjP;                 // np > 0: the pivot blocks' inverses of two steps [2*64*64]
  double* gjC;                 // np > 0: the saved column panel [np*64]
  double* gjR;                 // np > 0: the row panel times the pivot inverse [np*64]
  double* lmax;
  double* pscale;
  int j0, j1;  // this slot's jobs in its level's DOF-job table
};

struct BInst {
  int nx, ny;
  long nn, nd, nc, nsq;
  int slot0;
  double *rho, *rho_new, *dc, *dcf, *R, *qcls, *a;
  double E0, Emin, penal, volfrac, move, eta, rho_min, rtol, lam0, mu0, vol;
  int split_uniform, alt, nclasses;
  const FilterTap* taps;
  const int* ntaps;
  int tap_stride;   // entries per class list
  int jd0, jd1;            // fine DOF jobs
  int jc0, jc1;            // fine cell jobs
  int js0, js1;            // fine square jobs
  int jt0[kBShapes], jt1[kBShapes];  // fine tiles per shape
};

struct BState {
  PcgState pcg;
  OcState oc;
  double compliance, c_paper, change;
  long cg_total;
  int active, stepped, iters, cg_last, status, pad;
};

struct BParams {
  double change_tol;
  int max_iter;
  int pad;
};

struct BJob {
  int slot, inst;
  long begin;
  int count, pad;
};

struct BTile {
  int slot, inst, bx, by;
};

__device__ __forceinline__ bool b_live(const BState* st, int inst, bool cg) {
  return st[inst].active && !(cg && st[inst].pcg.done);
}

// ---------------------------------------------------------------- set-up
__global__ void b_modulus(const BJob* jobs, const BInst* I, const BSlot* slots, const BState* st) {
  const BJob j = jobs[blockIdx.x];
  if (!st[j.inst].active) return;
  const BInst& in = I[j.inst];
  double* E = slots[in.slot0].E;
  for (int t = threadIdx.x; t < j.count; t += blockDim.x) {
    const long e = j.begin + t;
    const double r = in.rho[e];
    const double rp = (in.penal == 3.0) ? r * r * r : pow(r, in.penal);
    E[e] = in.Emin + rp * (in.E0 - in.Emin);
  }
}

__global__ void b_diag(const BJob* jobs, const BSlot* slots, const BState* st) {
  const BJob j = jobs[blockIdx.x];
  if (!st[j.inst].active) return;
  const BSlot& s = slots[j.slot];
  for (int t = threadIdx.x; t < j.count; t += blockDim.x)
    diag2d_node(j.begin + t, s.invd, s.E, s.op, s.lam0, s.mu0, s.vol, 1);
}

// moduli of child slot j.slot from its parent
__global__ void b_restrict_E(const BJob* jobs, const BSlot* slots, const BState* st) {
  const BJob j = jobs[blockIdx.x];
  if (!st[j.inst].active) return;
  const BSlot& cs = slots[j.slot];
  const BSlot& fs = slots[cs.parent];
  for (int t = threadIdx.x; t < j.count; t += blockDim.x)
    restrict_E2_square(j.begin + t, cs.E, fs.E, fs.op.nx, fs.op.ny, fs.op.split_uniform, cs.op.nx);
}

__global__ void b_power_init(const BJob* jobs, const BSlot* slots, const BState* st) {
  const BJob j = jobs[blockIdx.x];
  if (!st[j.inst].active) return;
  const BSlot& s = slots[j.slot];
  for (int t = threadIdx.x; t < j.count; t += blockDim.x) {
    const long i = j.begin + t;
    const long n = i % s.op.nn;
    const int c = (int)(i / s.op.nn);
    unsigned h = (unsigned)(i * 2654435761u) ^ 0x9e3779b9u;
    h ^= h >> 16;
    h *= 0x85ebca6bu;
    h ^= h >> 13;
    const double v0 = (double)(h & 0xffffff) / 16777216.0 - 0.5;
    s.v[BV_PV][i] = ((s.op.mask[n] >> c) & 1) ? 0.0 : v0;
  }
  if (j.begin == 0 && threadIdx.x == 0) *s.pscale = 1.0;
}

__global__ __launch_bounds__(256) void b_power_step(const BJob* jobs, const BSlot* slots,
                                                    const BState* st, double* partials) {
  const BJob j = jobs[blockIdx.x];
  double acc[2] = {0.0, 0.0};
  if (st[j.inst].active) {
    const BSlot& s = slots[j.slot];
    const double sc = *s.pscale;
    for (int t = threadIdx.x; t < j.count; t += blockDim.x) {
      const long i = j.begin + t;
      const double id = s.invd[i];
      const double vi = s.v[BV_PV][i], wi = s.v[BV_PW][i];
      acc[0] += vi * wi;
      acc[1] += vi * vi / id;
      s.v[BV_PV][i] = sc * id * wi;
    }
  }
  const double none[1] = {0.0};
  block_partials<2, 0>(acc, none, partials);
}

// one block per slot of the list: Rayleigh quotient, scale, lmax estimate
__global__ void b_power_fin(const int* list, const BSlot* slots, const BState* st,
                            const double* partials, int last, double safety) {
  const BSlot& s = slots[list[blockIdx.x]];
  if (!st[s.inst].active) return;
  __shared__ double tot[2];
  reduce_partials_range<2, 0>(partials, s.j0, s.j1, tot);
  if (threadIdx.x == 0) {
    const double lam = (tot[1] > 0.0) ? tot[0] / tot[1] : 1.0;
    *s.pscale = (lam > 0.0) ? 1.0 / lam : 1.0;
    if (last) *s.lmax = safety * lam;
  }
}

__global__ void b_coarse_assemble(const int* list, const BSlot* slots, const BState* st) {
  const BSlot& s = slots[list[blockIdx.x]];
  if (!st[s.inst].active || s.np > 0) return;
  const int n = (int)(s.op.nn * 2);
  for (int row = threadIdx.x; row < n; row += blockDim.x)
    coarse_assemble_row(row, s.Ainv, s.E, s.op, s.lam0, s.mu0, s.vol);
}

__global__ __launch_bounds__(1024) void b_gauss_jordan(const int* list, const BSlot* slots,
                                                       const BState* st) {
  const BSlot& s = slots[list[blockIdx.x]];
  if (!st[s.inst].active || s.np > 0) return;
  gauss_jordan_block(s.Ainv, (int)(s.op.nn * 2));
}

// last levels above 128 DOFs (np > 0): the block sweep inverse of
// dense_dev.h, one launch per block step for all instances (the list gives
// the slots, blockIdx.y the instance; a slot with fewer blocks returns)
__global__ void b_dense_fill(const int* list, const BSlot* slots, const BState* st) {
  const BSlot& s = slots[list[blockIdx.y]];
  if (!st[s.inst].active || s.np == 0) return;
  dense_fill_range(s.Ainv, (int)s.nd, s.np, (long)blockIdx.x * blockDim.x + threadIdx.x,
                   (long)gridDim.x * blockDim.x);
}

__global__ void b_coarse_assemble_ld(const int* list, const BSlot* slots, const BState* st) {
  const BSlot& s = slots[list[blockIdx.y]];
  if (!st[s.inst].active || s.np == 0) return;
  const int row = blockIdx.x * blockDim.x + threadIdx.x;
  if (row >= (int)s.nd) return;
  coarse_assemble_row(row, s.Ainv, s.E, s.op, s.lam0, s.mu0, s.vol, s.np, false);
}

__global__ __launch_bounds__(kGjPivThreads) void b_gj_pivot(const int* list, const BSlot* slots,
                                                             const BState* st, int k) {
  const BSlot& s = slots[list[blockIdx.x]];
  if (!st[s.inst].active || k >= s.np / kGjB) return;
  gj_pivot_block(s.Ainv, s.np, k, s.gjP + (k & 1) * kGjB * kGjB);
}

__global__ __launch_bounds__(kGjThreads) void b_gj_panel(const int* list, const BSlot* slots,
                                                          const BState* st, int k) {
  const BSlot& s = slots[list[blockIdx.y]];
  const int nb = s.np / kGjB;
  if (!st[s.inst].active || k >= nb || (int)blockIdx.x >= 2 * nb) return;
  sw_panel_block(s.Ainv, s.np, k, s.gjP + (k & 1) * kGjB * kGjB, s.gjC, s.gjR, blockIdx.x);
}

// blockIdx.x numbers the blocks on and above the diagonal (the next
// diagonal block first), blockIdx.y the instance: an instance's blocks are
// dispatched together and share its panels in the caches
__global__ __launch_bounds__(kGjThreads) void b_gj_update(const int* list, const BSlot* slots,
                                                           const BState* st, int k) {
  const BSlot& s = slots[list[blockIdx.y]];
  const int nb = s.np / kGjB;
  if (!st[s.inst].active || k >= nb || (int)blockIdx.x >= nb * (nb + 1) / 2) return;
  int i, j;
  sw_update_index(blockIdx.x, nb, k, i, j);
  sw_update_block(s.Ainv, s.np, k, s.gjP + (k & 1) * kGjB * kGjB, s.gjC, s.gjR, i, j,
                  k + 1 < nb ? s.gjP + ((k + 1) & 1) * kGjB * kGjB : nullptr);
}

__global__ __launch_bounds__(kGjThreads) void b_gj_mirror(const int* list, const BSlot* slots,
                                                           const BState* st) {
  const BSlot& s = slots[list[blockIdx.y]];
  const int nb = s.np / kGjB;
  if (!st[s.inst].active || s.np == 0 || (int)blockIdx.x >= nb * (nb + 1) / 2) return;
  int i, j;
  sw_tri_index(blockIdx.x, i, j);
  sw_mirror_block(s.Ainv, s.np, i, j);
}

// ------------------------------------------------------------- operator
// y = K x on the tiles of the job list; cg: skip converged instances;
// partials: per-tile (x, y) for the CG step length
template <int BX, int BY>
__global__ __launch_bounds__(256) void b_apply(const BTile* jobs, const BSlot* slots, const BState* st,
                                               int src, int dst, int cg, double* partials) {
  const BTile j = jobs[blockIdx.x];
  const bool live = b_live(st, j.inst, cg != 0);
  if (!live && !partials) return;
  const BSlot& s = slots[j.slot];
  const double lam = s.lam0 * s.vol, mu = s.mu0 * s.vol;
  const double dot =
      apply2d_tile<double, double, BX, BY>(live, j.bx, j.by, 0, s.v[src], s.v[dst], s.E, s.op, lam, mu);
  if (partials) {
    double acc[1] = {dot};
    const double none[1] = {0.0};
    block_partials<1, 0>(acc, none, partials);
  }
}

// ------------------------------------------------------------- V-cycle
__global__ void b_cheb_first(const BJob* jobs, const BSlot* slots, const BState* st, int mode,
                             double low) {
  const BJob j = jobs[blockIdx.x];
  if (!b_live(st, j.inst, true)) return;
  const BSlot& s = slots[j.slot];
  double theta, delta;
  cheb_interval(*s.lmax, low, theta, delta);
  const double it = 1.0 / theta;
  double *x = s.v[BV_X], *r = s.v[BV_R], *d = s.v[BV_D];
  const double *b = s.v[BV_B], *q = s.v[BV_Q];
  for (int t = threadIdx.x; t < j.count; t += blockDim.x) {
    const long i = j.begin + t;
    const double rv = mode ? b[i] - q[i] : b[i];
    const double dv = it * s.invd[i] * rv;
    r[i] = rv;
    d[i] = dv;
    x[i] = mode ? x[i] + dv : dv;
  }
}

__global__ void b_cheb_next(const BJob* jobs, const BSlot* slots, const BState* st, ChebCoef cf,
                            double low) {
  const BJob j = jobs[blockIdx.x];
  if (!b_live(st, j.inst, true)) return;
  const BSlot& s = slots[j.slot];
  double theta, delta;
  cheb_interval(*s.lmax, low, theta, delta);
  const double c1 = cf.r_cur * cf.r_prev, c2 = 2.0 * cf.r_cur / delta;
  double *x = s.v[BV_X], *r = s.v[BV_R], *d = s.v[BV_D];
  const double* q = s.v[BV_Q];
  for (int t = threadIdx.x; t < j.count; t += blockDim.x) {
    const long i = j.begin + t;
    const double rv = r[i] - q[i];
    const double dv = c1 * d[i] + c2 * s.invd[i] * rv;
    r[i] = rv;
    d[i] = dv;
    x[i] += dv;
  }
}

// child.b = R (parent.b - parent.q) on the child's nodes
__global__ void b_restrict(const BJob* jobs, const BSlot* slots, const BState* st) {
  const BJob j = jobs[blockIdx.x];
  if (!b_live(st, j.inst, true)) return;
  const BSlot& cs = slots[j.slot];
  const BSlot& fs = slots[cs.parent];
  for (int t = threadIdx.x; t < j.count; t += blockDim.x)
    restrict_node<double>(j.begin + t, cs.v[BV_B], fs.v[BV_B], fs.v[BV_Q], fs.op, cs.op, 1);
}

// slot.x += P child.x on the slot's nodes
__global__ void b_prolong(const BJob* jobs, const BSlot* slots, const BState* st) {
  const BJob j = jobs[blockIdx.x];
  if (!b_live(st, j.inst, true)) return;
  const BSlot& s = slots[j.slot];
  const BSlot& cs = slots[s.child];
  for (int t = threadIdx.x; t < j.count; t += blockDim.x)
    prolong_node<double>(j.begin + t, s.v[BV_X], cs.v[BV_X], s.op, cs.op, 1);
}

__global__ void b_coarse_solve(const int* list, const BSlot* slots, const BState* st) {
  const BSlot& s = slots[list[blockIdx.x]];
  if (s.np > 0 || !b_live(st, s.inst, true)) return;
  coarse_solve_block<double>(s.v[BV_X], s.v[BV_B], s.Ainv, (int)(s.op.nn * 2), 1);
}

// x = Ainv b on the last levels above 128 DOFs (blockIdx.y: the slot)
__global__ __launch_bounds__(64 * kDenseWaves) void b_dense_solve(const int* list,
                                                                  const BSlot* slots,
                                                                  const BState* st) {
  const BSlot& s = slots[list[blockIdx.y]];
  if (s.np == 0 || !b_live(st, s.inst, true)) return;
  const int n = (int)s.nd;
  if ((int)blockIdx.x * kDenseWaves >= n) return;
  dense_solve_rows<double, double>(s.v[BV_X], s.v[BV_B], s.Ainv, n, s.np, 1, blockIdx.x);
}

// ------------------------------------------------------------------ CG
// r = f - K u (masked), partial (r, r) and (f, f)
__global__ __launch_bounds__(256) void b_pcg_init(const BJob* jobs, const BSlot* slots,
                                                  const BState* st, double* partials) {
  const BJob j = jobs[blockIdx.x];
  double acc[2] = {0.0, 0.0};
  if (st[j.inst].active) {
    const BSlot& s = slots[j.slot];
    const long nn = s.op.nn;
    for (int t = threadIdx.x; t < j.count; t += blockDim.x) {
      const long d = j.begin + t;
      const long n = d % nn;
      const int c = (int)(d / nn);
      const bool fixed = (s.op.mask[n] >> c) & 1;
      const double fv = fixed ? 0.0 : s.v[BV_F][d];
      const double rv = fixed ? 0.0 : fv - s.v[BV_CQ][d];
      if (fixed) s.v[BV_U][d] = 0.0;
      s.v[BV_B][d] = rv;
      acc[0] += rv * rv;
      acc[1] += fv * fv;
    }
  }
  const double none[1] = {0.0};
  block_partials<2, 0>(acc, none, partials);
}

__global__ void b_pcg_init_fin(const BInst* I, BState* st, const double* partials) {
  const int i = blockIdx.x;
  if (!st[i].active) return;
  __shared__ double tot[2];
  reduce_partials_range<2, 0>(partials, I[i].jd0, I[i].jd1, tot);
  if (threadIdx.x == 0) pcg_init_finish<1>(tot, I[i].rtol, &st[i].pcg);
}

__global__ void b_alpha_fin(const BInst* I, BState* st, const double* partials, int shape) {
  const int i = blockIdx.x;
  if (!b_live(st, i, true)) return;
  __shared__ double tot[1];
  reduce_partials_range<1, 0>(partials, I[i].jt0[shape], I[i].jt1[shape], tot);
  if (threadIdx.x == 0) {
    const double t4[kMaxRhs] = {tot[0], 0.0, 0.0, 0.0};
    pcg_alpha_finish(t4, &st[i].pcg);
  }
}

// u += alpha p, r -= alpha q; partial (r, r)
__global__ __launch_bounds__(256) void b_update(const BJob* jobs, const BSlot* slots, const BState* st,
                                                double* partials) {
  const BJob j = jobs[blockIdx.x];
  double acc[1] = {0.0};
  if (b_live(st, j.inst, true)) {
    const BSlot& s = slots[j.slot];
    const double al = st[j.inst].pcg.alpha[0];
    double *u = s.v[BV_U], *r = s.v[BV_B];
    const double *p = s.v[BV_P], *q = s.v[BV_CQ];
    for (int t = threadIdx.x; t < j.count; t += blockDim.x) {
      const long d = j.begin + t;
      u[d] += al * p[d];
      const double rv = r[d] - al * q[d];
      r[d] = rv;
      acc[0] += rv * rv;
    }
  }
  const double none[1] = {0.0};
  block_partials<1, 0>(acc, none, partials);
}

__global__ void b_update_fin(const BInst* I, BState* st, const double* partials) {
  const int i = blockIdx.x;
  if (!b_live(st, i, true)) return;
  __shared__ double tot[1];
  reduce_partials_range<1, 0>(partials, I[i].jd0, I[i].jd1, tot);
  if (threadIdx.x == 0) {
    const double t2[2] = {tot[0], 0.0};
    pcg_update_finish<1, false>(t2, &st[i].pcg, &st[i].status);
  }
}

// partial (r, z)
__global__ __launch_bounds__(256) void b_rz(const BJob* jobs, const BSlot* slots, const BState* st,
                                            double* partials) {
  const BJob j = jobs[blockIdx.x];
  double acc[1] = {0.0};
  if (b_live(st, j.inst, true)) {
    const BSlot& s = slots[j.slot];
    for (int t = threadIdx.x; t < j.count; t += blockDim.x) {
      const long d = j.begin + t;
      acc[0] += s.v[BV_B][d] * s.v[BV_X][d];
    }
  }
  const double none[1] = {0.0};
  block_partials<1, 0>(acc, none, partials);
}

__global__ void b_rz_fin(const BInst* I, BState* st, const double* partials, int first) {
  const int i = blockIdx.x;
  if (!b_live(st, i, true)) return;
  __shared__ double tot[1];
  reduce_partials_range<1, 0>(partials, I[i].jd0, I[i].jd1, tot);
  if (threadIdx.x == 0) pcg_rz_finish<1>(tot, first, &st[i].pcg);
}

// p = z + beta p (first: p = z)
__global__ void b_direction(const BJob* jobs, const BSlot* slots, const BState* st, int first) {
  const BJob j = jobs[blockIdx.x];
  if (!b_live(st, j.inst, true)) return;
  const BSlot& s = slots[j.slot];
  const double be = first ? 0.0 : st[j.inst].pcg.beta[0];
  double* p = s.v[BV_P];
  const double* z = s.v[BV_X];
  for (int t = threadIdx.x; t < j.count; t += blockDim.x) {
    const long d = j.begin + t;
    p[d] = first ? z[d] : z[d] + be * p[d];
  }
}

// flag = 1 when no active instance has a CG still running
__global__ void b_all_done(const BState* st, int n, int* flag) {
  __shared__ int any;
  if (threadIdx.x == 0) any = 0;
  __syncthreads();
  for (int i = threadIdx.x; i < n; i += blockDim.x)
    if (st[i].active && !st[i].pcg.done) atomicOr(&any, 1);
  __syncthreads();
  if (threadIdx.x == 0) *flag = !any;
}

// --------------------------------------------------- sensitivity, filter
__global__ __launch_bounds__(256) void b_sens(const BJob* jobs, const BInst* I, const BSlot* slots,
                                              const BState* st, double* partials) {
  const BJob j = jobs[blockIdx.x];
  double acc[2] = {0.0, 0.0};
  if (st[j.inst].active) {
    const BInst& in = I[j.inst];
    const double* u = slots[in.slot0].v[BV_U];
    for (int t = threadIdx.x; t < j.count; t += blockDim.x)
      sens2d_square(j.begin + t, in.rho, u, in.dc, in.nx, in.nn, 1, in.split_uniform, in.lam0, in.mu0,
                    in.vol, in.E0, in.Emin, in.penal, 0, acc);
  }
  const double none[1] = {0.0};
  block_partials<2, 0>(acc, none, partials);
}

__global__ void b_sens_fin(const BInst* I, BState* st, const double* partials) {
  const int i = blockIdx.x;
  if (!st[i].active) return;
  __shared__ double tot[2];
  reduce_partials_range<2, 0>(partials, I[i].js0, I[i].js1, tot);
  if (threadIdx.x == 0) {
    st[i].compliance = tot[0];
    st[i].c_paper = tot[1];
  }
}

// q[t][h] = rho[e] dc[e] (class-major; rowsum: q = 1)
__global__ void b_filter_gather(const BJob* jobs, const BInst* I, const BState* st, int rowsum) {
  const BJob j = jobs[blockIdx.x];
  if (!rowsum && !st[j.inst].active) return;
  const BInst& in = I[j.inst];
  for (int t = threadIdx.x; t < j.count; t += blockDim.x) {
    const long e = j.begin + t;
    const long h = e / 2;
    const int tt = (int)(e % 2);
    in.qcls[(long)tt * in.nsq + h] = rowsum ? 1.0 : in.rho[e] * in.dc[e];
  }
}

__global__ void b_filter(const BJob* jobs, const BInst* I, const BState* st, int rowsum) {
  const BJob j = jobs[blockIdx.x];
  if (!rowsum && !st[j.inst].active) return;
  const BInst& in = I[j.inst];
  double* out = rowsum ? in.R : in.dcf;
  for (int t = threadIdx.x; t < j.count; t += blockDim.x)
    for (int cls = 0; cls < 2; ++cls)
      filter_cell(j.begin + t, cls, out, in.qcls, in.rho, in.R, in.taps, in.ntaps, in.tap_stride, 2,
                  in.nx, in.ny, 1, 2, in.alt, rowsum);
}

// ------------------------------------------------------------------ OC
__global__ __launch_bounds__(256) void b_oc_init(const BJob* jobs, const BInst* I, const BState* st,
                                                 double* partials) {
  const BJob j = jobs[blockIdx.x];
  double acc[3] = {0.0, 0.0, 0.0};
  double mx[1] = {0.0};
  if (st[j.inst].active) {
    const BInst& in = I[j.inst];
    for (int t = threadIdx.x; t < j.count; t += blockDim.x) {
      const long e = j.begin + t;
      const double r = in.rho[e];
      const double a = oc_a(r, in.dcf[e], in.eta);
      in.a[e] = a;
      const double lo = fmax(in.rho_min, r - in.move), hi = fmin(1.0, r + in.move);
      acc[0] += lo;
      acc[1] += (a > 0.0) ? hi : lo;
      acc[2] += a;
      if (a > 0.0) mx[0] = fmax(mx[0], hi / a);
    }
  }
  block_partials<3, 1>(acc, mx, partials);
}

__global__ void b_oc_init_fin(const BInst* I, BState* st, const double* partials) {
  const int i = blockIdx.x;
  if (!st[i].active) return;
  __shared__ double tot[4];
  reduce_partials_range<3, 1>(partials, I[i].jc0, I[i].jc1, tot);
  if (threadIdx.x == 0) oc_init_finish(tot, I[i].nc, I[i].volfrac, &st[i].oc, &st[i].status);
}

__global__ __launch_bounds__(256) void b_oc_pass(const BJob* jobs, const BInst* I, const BState* st,
                                                 double* partials) {
  const BJob j = jobs[blockIdx.x];
  double acc[2] = {0.0, 0.0};
  if (st[j.inst].active && !st[j.inst].oc.done) {
    const BInst& in = I[j.inst];
    const double mu = st[j.inst].oc.mu;
    for (int t = threadIdx.x; t < j.count; t += blockDim.x) {
      const long e = j.begin + t;
      const double r = in.rho[e];
      const double a = in.a[e];
      const double lo = fmax(in.rho_min, r - in.move), hi = fmin(1.0, r + in.move);
      const double v = a * mu;
      acc[0] += fmax(lo, fmin(hi, v));
      acc[1] += (v > lo && v < hi) ? a : 0.0;
    }
  }
  const double none[1] = {0.0};
  block_partials<2, 0>(acc, none, partials);
}

__global__ void b_oc_pass_fin(const BInst* I, BState* st, const double* partials) {
  const int i = blockIdx.x;
  if (!st[i].active || st[i].oc.done) return;
  __shared__ double tot[2];
  reduce_partials_range<2, 0>(partials, I[i].jc0, I[i].jc1, tot);
  if (threadIdx.x == 0) oc_pass_finish(tot, I[i].nc, &st[i].oc);
}

__global__ __launch_bounds__(256) void b_oc_final(const BJob* jobs, const BInst* I, const BState* st,
                                                  double* partials) {
  const BJob j = jobs[blockIdx.x];
  double acc[1] = {0.0};
  double mx[1] = {0.0};
  if (st[j.inst].active) {
    const BInst& in = I[j.inst];
    const double mu = st[j.inst].oc.mu;
    for (int t = threadIdx.x; t < j.count; t += blockDim.x) {
      const long e = j.begin + t;
      const double r = in.rho[e];
      const double lo = fmax(in.rho_min, r - in.move), hi = fmin(1.0, r + in.move);
      const double v = fmax(lo, fmin(hi, in.a[e] * mu));
      in.rho_new[e] = v;
      acc[0] += v;
      mx[0] = fmax(mx[0], fabs(v - r));
    }
  }
  block_partials<1, 1>(acc, mx, partials);
}

__global__ void b_oc_final_fin(const BInst* I, BState* st, const double* partials) {
  const int i = blockIdx.x;
  if (!st[i].active) return;
  __shared__ double tot[2];
  reduce_partials_range<1, 1>(partials, I[i].jc0, I[i].jc1, tot);
  if (threadIdx.x == 0) {
    oc_final_finish(tot, I[i].eta, I[i].nc, &st[i].oc, nullptr, &st[i].status);
    st[i].change = st[i].oc.change;
    st[i].iters += 1;
    st[i].cg_last = st[i].pcg.iters;
    st[i].cg_total += st[i].pcg.iters;
    st[i].stepped = 1;
  }
}

__global__ void b_copy_rho(const BJob* jobs, const BInst* I, const BState* st) {
  const BJob j = jobs[blockIdx.x];
  if (!st[j.inst].stepped) return;
  const BInst& in = I[j.inst];
  for (int t = threadIdx.x; t < j.count; t += blockDim.x) in.rho[j.begin + t] = in.rho_new[j.begin + t];
}

// stop instances whose change fell below the tolerance or that reached the
// iteration cap; flag = 1 while any instance is still active
__global__ void b_next_round(BState* st, int n, const BParams* prm, int* flag) {
  __shared__ int any;
  if (threadIdx.x == 0) any = 0;
  __syncthreads();
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    if (st[i].stepped) {
      const bool conv = prm->change_tol > 0.0 && st[i].change < prm->change_tol;
      if (conv || st[i].iters >= prm->max_iter) st[i].active = 0;
      st[i].stepped = 0;
    }
    if (st[i].active) atomicOr(&any, 1);
  }
  __syncthreads();
  if (threadIdx.x == 0) *flag = any;
}

__global__ void b_reset(BState* st, int n, BParams* prm, double change_tol, int max_iter) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    st[i].active = max_iter > 0 ? 1 : 0;
    st[i].stepped = 0;
    st[i].iters = 0;
    st[i].cg_total = 0;
    st[i].cg_last = 0;
    st[i].change = 0.0;
    st[i].status = 0;
    st[i].pcg.done = 0;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    prm->change_tol = change_tol;
    prm->max_iter = max_iter;
  }
}

// record[i] = [iterations, change, compliance, volume fraction, CG iterations, converged]
__global__ void b_record(const BInst* I, const BState* st, const BParams* prm, int n, double* rec) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    double* r = rec + (long)i * TOPO_BATCH_REC_LEN;
    r[0] = st[i].iters;
    r[1] = st[i].change;
    r[2] = st[i].compliance;
    r[3] = st[i].oc.vol / (double)I[i].nc;
    r[4] = (double)st[i].cg_total;
    r[5] = (prm->change_tol > 0.0 && st[i].iters > 0 && st[i].change < prm->change_tol) ? 1.0 : 0.0;
  }
}

__global__ void b_fill(double* p, double v, long n) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    p[i] = v;
}

__global__ void b_status(const BState* st, int n, int* out) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  int s = 0;
  for (int i = 0; i < n; ++i)
    if (st[i].status != 0 && (s == 0 || st[i].status < 0)) s = st[i].status;
  *out = s;
}

}  // namespace topo

// ======================================================================
// host side
using namespace topo;

namespace {

struct DevTable {
  void* p = nullptr;
  int n = 0;
};

struct BatchCtx {
  int B = 0;
  hipStream_t stream = nullptr;   // internal non-blocking stream (capture needs one)
  hipStream_t caller = nullptr;
  char* ws = nullptr;
  size_t ws_bytes = 0;
  std::vector<BInst> inst;
  std::vector<BSlot> slots;
  int Lmax = 0;
  BInst* d_inst = nullptr;
  BSlot* d_slots = nullptr;
  BState* d_state = nullptr;
  BParams* d_prm = nullptr;
  int* d_flags = nullptr;          // [0] all CG done, [1] any active, [2] status
  double* partials = nullptr;
  // concatenated per-instance arrays
  double *rho = nullptr, *f = nullptr, *u = nullptr;
  long total_cells = 0, total_dofs = 0;
  // job tables
  DevTable fine_cell, fine_sq;
  DevTable fine_tiles[kBShapes];
  std::vector<DevTable> lv_dof, lv_node, lv_child_node, lv_child_sq, lv_tiles, lv_listA, lv_listC;
  std::vector<std::vector<int>> A, C;
  DevTable all_last;
  // last levels above 128 DOFs: the most 64-blocks of any, the most rows,
  // and per level the most rows and the largest padded size
  int gj_nb_max = 0, dense_n_max = 0;
  std::vector<int> lv_dense_rows, lv_dense_np;
  int shape = 0;
  double shape_us[kBShapes] = {0, 0, 0};
  hipGraphExec_t g_setup = nullptr, g_cg = nullptr, g_post = nullptr;
  bool graphs = false;
  volatile int* pinned = nullptr;
  hipEvent_t ev[2] = {nullptr, nullptr};
  hipEvent_t ev_caller = nullptr;
  int maxit = 20000;
};

size_t al(size_t x) { return (x + 255) & ~(size_t)255; }

// carving of the batch workspace: every buffer 256-byte aligned
struct Carver {
  size_t off = 0;
  char* base = nullptr;
  template <typename T>
  T* take(size_t count) {
    const size_t at = off;
    off = al(off + count * sizeof(T));
    return base ? reinterpret_cast<T*>(base + at) : nullptr;
  }
};

bool valid_batch_problem(const topo_problem& p) {
  if (p.dim != 2 || p.nrhs != 1 || p.precision != TOPO_FP64 || p.precond != TOPO_PC_GMG) return false;
  if (p.filter != TOPO_FILTER_DISTANCE) return false;
  if (p.paper_mode) return false;
  if (p.nel[0] < 2 || p.nel[1] < 2 || p.nel[0] > (1 << 15) || p.nel[1] > (1 << 15)) return false;
  if (p.split2d != TOPO_SPLIT_ALT_ROWS && p.split2d != TOPO_SPLIT_UNIFORM) return false;
  if (!(p.volfrac > 0.0 && p.volfrac <= 1.0) || !(p.rmin > 0.0 && p.rmin <= 16.0)) return false;
  if (!(p.penal >= 1.0 && p.penal <= 10.0) || !(p.nu > -1.0 && p.nu < 0.5)) return false;
  if (!(p.E0 > 0.0) || !(p.Emin >= 0.0) || !(p.Emin < p.E0)) return false;
  if (!(p.move > 0.0) || !(p.eta > 0.0) || !(p.rho_min > 0.0 && p.rho_min < 1.0)) return false;
  if (!(p.rtol > 0.0) || p.maxit < 1) return false;
  // at least two multigrid levels (more than the 128 DOFs of a dense solve)
  if (2L * (p.nel[0] + 1) * (p.nel[1] + 1) <= 128) return false;
  return true;
}

const int kShapeBX[kBShapes] = {16, 32, 64};
const int kShapeBY[kBShapes] = {16, 8, 4};

// An instance's levels: down to the first level of at most gmg_dense DOFs
// (2048 by default), solved directly; an instance whose fine level is
// already that small keeps the hierarchy down to 128 DOFs.
static std::vector<LevelDims> batch_plan(const topo_problem& p) {
  int cap = gmg_dense_max(&p);
  if (2L * (p.nel[0] + 1) * (p.nel[1] + 1) <= cap) cap = 128;
  return gmg_plan_dims(2, p.nel[0], p.nel[1], 1, cap);
}

// Plan (and with base != nullptr, carve) the batch; returns total bytes.
size_t plan_batch(const topo_problem* probs, int count, BatchCtx* b, char* base,
                  std::vector<std::vector<LevelDims>>* plans_out,
                  std::vector<std::vector<std::vector<uint8_t>>>* masks_in) {
  Carver cv;
  cv.base = base;
  std::vector<std::vector<LevelDims>> plans(count);
  long cells = 0, dofs = 0;
  for (int i = 0; i < count; ++i) {
    plans[i] = batch_plan(probs[i]);
    cells += 2L * probs[i].nel[0] * probs[i].nel[1];
    dofs += 2L * (probs[i].nel[0] + 1) * (probs[i].nel[1] + 1);
  }
  // concatenated per-instance arrays
  double* rho = cv.take<double>(cells);
  double* rho_new = cv.take<double>(cells);
  double* dc = cv.take<double>(cells);
  double* dcf = cv.take<double>(cells);
  double* R = cv.take<double>(cells);
  double* qcls = cv.take<double>(cells);
  double* aoc = cv.take<double>(cells);
  double* E0 = cv.take<double>(cells);
  double* f = cv.take<double>(dofs);
  double* u = cv.take<double>(dofs);
  double* r = cv.take<double>(dofs);
  double* pp = cv.take<double>(dofs);
  double* q = cv.take<double>(dofs);
  double* z = cv.take<double>(dofs);
  double* invd0 = cv.take<double>(dofs);
  if (b) {
    b->rho = rho;
    b->f = f;
    b->u = u;
    b->total_cells = cells;
    b->total_dofs = dofs;
  }
  long co = 0, dof = 0;
  std::vector<BInst> inst(count);
  std::vector<BSlot> slots;
  int Lmax = 0;
  for (int i = 0; i < count; ++i) {
    const topo_problem& p = probs[i];
    BInst& in = inst[i];
    memset(&in, 0, sizeof(in));
    in.nx = p.nel[0];
    in.ny = p.nel[1];
    in.nn = (long)(in.nx + 1) * (in.ny + 1);
    in.nd = 2 * in.nn;
    in.nsq = (long)in.nx * in.ny;
    in.nc = 2 * in.nsq;
    in.rho = rho ? rho + co : nullptr;
    in.rho_new = rho_new ? rho_new + co : nullptr;
    in.dc = dc ? dc + co : nullptr;
    in.dcf = dcf ? dcf + co : nullptr;
    in.R = R ? R + co : nullptr;
    in.qcls = qcls ? qcls + co : nullptr;
    in.a = aoc ? aoc + co : nullptr;
    in.E0 = p.E0;
    in.Emin = p.Emin;
    in.penal = p.penal;
    in.volfrac = p.volfrac;
    in.move = p.move;
    in.eta = p.eta;
    in.rho_min = p.rho_min;
    in.rtol = p.rtol;
    in.lam0 = p.nu / (1.0 - p.nu * p.nu);
    in.mu0 = 1.0 / (2.0 * (1.0 + p.nu));
    in.vol = 0.5;
    in.split_uniform = p.split2d == TOPO_SPLIT_UNIFORM;
    in.alt = !in.split_uniform;
    in.nclasses = in.alt ? 4 : 2;
    in.tap_stride = filter_tap_stride(2, in.alt ? TOPO_SPLIT_ALT_ROWS : TOPO_SPLIT_UNIFORM, p.rmin);
    in.taps = cv.take<FilterTap>((size_t)4 * in.tap_stride);
    in.ntaps = cv.take<int>(8);
    in.slot0 = (int)slots.size();
    const int L = (int)plans[i].size();
    Lmax = L > Lmax ? L : Lmax;
    for (int l = 0; l < L; ++l) {
      const LevelDims& d = plans[i][l];
      BSlot s;
      memset(&s, 0, sizeof(s));
      s.inst = i;
      s.level = l;
      s.last = l == L - 1;
      s.parent = l > 0 ? (int)slots.size() - 1 : -1;
      s.child = l + 1 < L ? (int)slots.size() + 1 : -1;
      s.op.dim = 2;
      s.op.nx = d.nx;
      s.op.ny = d.ny;
      s.op.nz = 1;
      s.op.nn = (long)(d.nx + 1) * (d.ny + 1);
      s.op.split_uniform = l == 0 ? in.split_uniform : 1;
      s.op.kz = 1;
      s.nc = 2L * d.nx * d.ny;
      s.nd = 2 * s.op.nn;
      s.lam0 = in.lam0;
      s.mu0 = in.mu0;
      s.vol = in.vol;
      s.lmax = cv.take<double>(1);
      s.pscale = cv.take<double>(1);
      if (l == 0) {
        s.op.mask = cv.take<uint8_t>(s.op.nn);
        s.E = E0 ? E0 + co : nullptr;
        s.invd = invd0 ? invd0 + dof : nullptr;
        s.v[BV_F] = f ? f + dof : nullptr;
        s.v[BV_U] = u ? u + dof : nullptr;
        s.v[BV_B] = r ? r + dof : nullptr;     // CG residual: the V-cycle right-hand side
        s.v[BV_P] = pp ? pp + dof : nullptr;
        s.v[BV_CQ] = q ? q + dof : nullptr;
        s.v[BV_X] = z ? z + dof : nullptr;     // preconditioned residual
      } else {
        s.op.mask = cv.take<uint8_t>(s.op.nn);
        s.E = cv.take<double>(s.nc);
        s.v[BV_B] = cv.take<double>(s.nd);
        s.v[BV_X] = cv.take<double>(s.nd);
      }
      if (!s.last) {
        if (l > 0) s.invd = cv.take<double>(s.nd);
        s.v[BV_R] = cv.take<double>(s.nd);
        s.v[BV_D] = cv.take<double>(s.nd);
        s.v[BV_Q] = cv.take<double>(s.nd);
        s.v[BV_PV] = cv.take<double>(s.nd);
        s.v[BV_PW] = cv.take<double>(s.nd);
      } else if (s.nd <= 128) {
        s.Ainv = cv.take<double>((size_t)s.nd * s.nd);
      } else {
        s.np = (int)((s.nd + kGjBlock - 1) / kGjBlock * kGjBlock);
        s.Ainv = cv.take<double>((size_t)s.np * s.np);
        s.gjP = cv.take<double>(2 * (size_t)kGjBlock * kGjBlock);
        s.gjC = cv.take<double>((size_t)s.np * kGjBlock);
        s.gjR = cv.take<double>((size_t)s.np * kGjBlock);
      }
      slots.push_back(s);
    }
    co += in.nc;
    dof += in.nd;
  }
  // job tables
  auto chunks = [](std::vector<BJob>& out, int slot, int inst_id, long n, int cap = kBChunk) {
    for (long b0 = 0; b0 < n; b0 += cap) {
      BJob j;
      j.slot = slot;
      j.inst = inst_id;
      j.begin = b0;
      j.count = (int)((n - b0) < cap ? (n - b0) : cap);
      j.pad = 0;
      out.push_back(j);
    }
  };
  auto tiles = [](std::vector<BTile>& out, int slot, int inst_id, const OpDesc& op, int bx, int by) {
    const int gx = (op.nx + 1 + (bx - 1) - 1) / (bx - 1), gy = (op.ny + 1 + (by - 1) - 1) / (by - 1);
    for (int ty = 0; ty < gy; ++ty)
      for (int tx = 0; tx < gx; ++tx) out.push_back(BTile{slot, inst_id, tx, ty});
  };
  std::vector<BJob> fcell, fsq;
  std::vector<BTile> ftiles[kBShapes];
  for (int i = 0; i < count; ++i) {
    BInst& in = inst[i];
    in.jc0 = (int)fcell.size();
    chunks(fcell, in.slot0, i, in.nc);
    in.jc1 = (int)fcell.size();
    in.js0 = (int)fsq.size();
    chunks(fsq, in.slot0, i, in.nsq);
    in.js1 = (int)fsq.size();
    for (int sh = 0; sh < kBShapes; ++sh) {
      in.jt0[sh] = (int)ftiles[sh].size();
      tiles(ftiles[sh], in.slot0, i, slots[in.slot0].op, kShapeBX[sh], kShapeBY[sh]);
      in.jt1[sh] = (int)ftiles[sh].size();
    }
  }
  std::vector<std::vector<BJob>> ldof(Lmax), lnode(Lmax), lcnode(Lmax), lcsq(Lmax);
  std::vector<std::vector<BTile>> ltiles(Lmax);
  std::vector<std::vector<int>> A(Lmax), C(Lmax);
  std::vector<int> all_last;
  for (int l = 0; l < Lmax; ++l) {
    for (int i = 0; i < count; ++i) {
      const int L = (int)plans[i].size();
      if (l >= L) continue;
      const int sid = inst[i].slot0 + l;
      BSlot& s = slots[sid];
      if (s.last) {
        C[l].push_back(sid);
        all_last.push_back(sid);
        continue;
      }
      A[l].push_back(sid);
      s.j0 = (int)ldof[l].size();
      chunks(ldof[l], sid, i, s.nd);
      s.j1 = (int)ldof[l].size();
      chunks(lnode[l], sid, i, s.op.nn, kBChunkNode);
      const BSlot& cs = slots[s.child];
      chunks(lcnode[l], s.child, i, cs.op.nn, kBChunkNode);
      chunks(lcsq[l], s.child, i, (long)cs.op.nx * cs.op.ny);
      // level 1 (a quarter of the fine grid) in 32 x 8 tiles, fewer halo
      // nodes per tile; the smaller levels in 16 x 16
      if (l > 0) tiles(ltiles[l], sid, i, s.op, l == 1 ? 32 : 16, l == 1 ? 8 : 16);
    }
  }
  for (int i = 0; i < count; ++i) {
    inst[i].jd0 = slots[inst[i].slot0].j0;
    inst[i].jd1 = slots[inst[i].slot0].j1;
  }
  size_t maxjobs = fcell.size();
  for (int sh = 0; sh < kBShapes; ++sh) maxjobs = ftiles[sh].size() > maxjobs ? ftiles[sh].size() : maxjobs;
  for (int l = 0; l < Lmax; ++l) {
    maxjobs = ldof[l].size() > maxjobs ? ldof[l].size() : maxjobs;
    maxjobs = ltiles[l].size() > maxjobs ? ltiles[l].size() : maxjobs;
  }
  // device copies of tables and state
  BInst* d_inst = cv.take<BInst>(count);
  BSlot* d_slots = cv.take<BSlot>(slots.size());
  BState* d_state = cv.take<BState>(count);
  BParams* d_prm = cv.take<BParams>(1);
  int* d_flags = cv.take<int>(8);
  double* partials = cv.take<double>(maxjobs * kPartStride);
  auto put_jobs = [&](const std::vector<BJob>& v) {
    DevTable t;
    t.p = cv.take<BJob>(v.size() > 0 ? v.size() : 1);
    t.n = (int)v.size();
    if (base && !v.empty()) (void)hipMemcpy(t.p, v.data(), v.size() * sizeof(BJob), hipMemcpyHostToDevice);
    return t;
  };
  auto put_tiles = [&](const std::vector<BTile>& v) {
    DevTable t;
    t.p = cv.take<BTile>(v.size() > 0 ? v.size() : 1);
    t.n = (int)v.size();
    if (base && !v.empty()) (void)hipMemcpy(t.p, v.data(), v.size() * sizeof(BTile), hipMemcpyHostToDevice);
    return t;
  };
  auto put_list = [&](const std::vector<int>& v) {
    DevTable t;
    t.p = cv.take<int>(v.size() > 0 ? v.size() : 1);
    t.n = (int)v.size();
    if (base && !v.empty()) (void)hipMemcpy(t.p, v.data(), v.size() * sizeof(int), hipMemcpyHostToDevice);
    return t;
  };
  DevTable t_fcell = put_jobs(fcell), t_fsq = put_jobs(fsq);
  DevTable t_ftiles[kBShapes];
  for (int sh = 0; sh < kBShapes; ++sh) t_ftiles[sh] = put_tiles(ftiles[sh]);
  std::vector<DevTable> t_ldof, t_lnode, t_lcnode, t_lcsq, t_ltiles, t_A, t_C;
  for (int l = 0; l < Lmax; ++l) {
    t_ldof.push_back(put_jobs(ldof[l]));
    t_lnode.push_back(put_jobs(lnode[l]));
    t_lcnode.push_back(put_jobs(lcnode[l]));
    t_lcsq.push_back(put_jobs(lcsq[l]));
    t_ltiles.push_back(put_tiles(ltiles[l]));
    t_A.push_back(put_list(A[l]));
    t_C.push_back(put_list(C[l]));
  }
  DevTable t_last = put_list(all_last);
  if (base && b) {
    // per-instance filter taps and fine masks, then the instance/slot tables
    for (int i = 0; i < count; ++i) {
      std::vector<FilterTap> tab;
      int nt[8] = {0, 0, 0, 0, 0, 0, 0, 0};
      int st = 0;
      filter_taps_host(2, probs[i].split2d == TOPO_SPLIT_UNIFORM ? TOPO_SPLIT_UNIFORM : TOPO_SPLIT_ALT_ROWS,
                       probs[i].rmin, tab, nt, &st);
      (void)hipMemcpy((void*)inst[i].taps, tab.data(), tab.size() * sizeof(FilterTap), hipMemcpyHostToDevice);
      (void)hipMemcpy((void*)inst[i].ntaps, nt, sizeof(nt), hipMemcpyHostToDevice);
      const std::vector<std::vector<uint8_t>>& ms = (*masks_in)[i];
      for (size_t l = 0; l < plans[i].size(); ++l) {
        BSlot& s = slots[inst[i].slot0 + l];
        (void)hipMemcpy((void*)s.op.mask, ms[l].data(), ms[l].size(), hipMemcpyHostToDevice);
      }
    }
    (void)hipMemcpy(d_inst, inst.data(), inst.size() * sizeof(BInst), hipMemcpyHostToDevice);
    (void)hipMemcpy(d_slots, slots.data(), slots.size() * sizeof(BSlot), hipMemcpyHostToDevice);
    b->inst = inst;
    b->slots = slots;
    b->Lmax = Lmax;
    b->d_inst = d_inst;
    b->d_slots = d_slots;
    b->d_state = d_state;
    b->d_prm = d_prm;
    b->d_flags = d_flags;
    b->partials = partials;
    b->fine_cell = t_fcell;
    b->fine_sq = t_fsq;
    for (int sh = 0; sh < kBShapes; ++sh) b->fine_tiles[sh] = t_ftiles[sh];
    b->lv_dof = t_ldof;
    b->lv_node = t_lnode;
    b->lv_child_node = t_lcnode;
    b->lv_child_sq = t_lcsq;
    b->lv_tiles = t_ltiles;
    b->lv_listA = t_A;
    b->lv_listC = t_C;
    b->A = A;
    b->C = C;
    b->all_last = t_last;
    b->gj_nb_max = 0;
    b->dense_n_max = 0;
    b->lv_dense_rows.assign(Lmax, 0);
    b->lv_dense_np.assign(Lmax, 0);
    for (int sid : all_last) {
      const BSlot& s = slots[sid];
      if (s.np == 0) continue;
      const int nb = s.np / kGjBlock, n = (int)s.nd;
      if (nb > b->gj_nb_max) b->gj_nb_max = nb;
      if (n > b->dense_n_max) b->dense_n_max = n;
      if (n > b->lv_dense_rows[s.level]) b->lv_dense_rows[s.level] = n;
      if (s.np > b->lv_dense_np[s.level]) b->lv_dense_np[s.level] = s.np;
    }
  }
  if (plans_out) *plans_out = plans;
  return cv.off;
}

// ------------------------------------------------------------- enqueue
struct Q {
  BatchCtx* b;
  hipStream_t s;
};

void apply_lv(const Q& q, int l, int src, int dst, bool cg, double* partials) {
  BatchCtx* b = q.b;
  const BState* st = b->d_state;
  if (l == 0) {
    const DevTable& t = b->fine_tiles[b->shape];
    if (t.n == 0) return;
    const BTile* jb = (const BTile*)t.p;
    switch (b->shape) {
      case 0: b_apply<16, 16><<<t.n, 256, 0, q.s>>>(jb, b->d_slots, st, src, dst, cg, partials); break;
      case 1: b_apply<32, 8><<<t.n, 256, 0, q.s>>>(jb, b->d_slots, st, src, dst, cg, partials); break;
      default: b_apply<64, 4><<<t.n, 256, 0, q.s>>>(jb, b->d_slots, st, src, dst, cg, partials); break;
    }
  } else {
    const DevTable& t = b->lv_tiles[l];
    if (t.n == 0) return;
    if (l == 1)
      b_apply<32, 8><<<t.n, 256, 0, q.s>>>((const BTile*)t.p, b->d_slots, st, src, dst, cg, partials);
    else
      b_apply<16, 16><<<t.n, 256, 0, q.s>>>((const BTile*)t.p, b->d_slots, st, src, dst, cg, partials);
  }
}

constexpr int kChebDegree = 2;
constexpr double kChebLow = 0.09;
constexpr int kPowerIters = 12;
constexpr double kPowerSafety = 1.2;

void cheb_smooth(const Q& q, int l, bool from_zero) {
  BatchCtx* b = q.b;
  const DevTable& t = b->lv_dof[l];
  if (t.n == 0) return;
  const BJob* jb = (const BJob*)t.p;
  if (!from_zero) apply_lv(q, l, BV_X, BV_Q, true, nullptr);
  b_cheb_first<<<t.n, 256, 0, q.s>>>(jb, b->d_slots, b->d_state, from_zero ? 0 : 1, kChebLow);
  const double sigma = (1.0 + kChebLow) / (1.0 - kChebLow);
  double rho_prev = 1.0 / sigma;
  for (int k = 1; k < kChebDegree; ++k) {
    const double rho = 1.0 / (2.0 * sigma - rho_prev);
    apply_lv(q, l, BV_D, BV_Q, true, nullptr);
    ChebCoef cf{rho, rho_prev, 1, k};
    b_cheb_next<<<t.n, 256, 0, q.s>>>(jb, b->d_slots, b->d_state, cf, kChebLow);
    rho_prev = rho;
  }
}

void vcycle(const Q& q, int l) {
  BatchCtx* b = q.b;
  if (l >= b->Lmax) return;
  if (b->lv_listC[l].n > 0) {
    b_coarse_solve<<<b->lv_listC[l].n, 128, 0, q.s>>>((const int*)b->lv_listC[l].p, b->d_slots,
                                                      b->d_state);
    if (b->lv_dense_rows[l] > 0)
      b_dense_solve<<<dim3((b->lv_dense_rows[l] + kDenseWaves - 1) / kDenseWaves, b->lv_listC[l].n),
                      64 * kDenseWaves, (size_t)b->lv_dense_np[l] * sizeof(double), q.s>>>(
          (const int*)b->lv_listC[l].p, b->d_slots, b->d_state);
  }
  if (b->lv_listA[l].n == 0) return;
  cheb_smooth(q, l, true);
  apply_lv(q, l, BV_X, BV_Q, true, nullptr);
  const DevTable& cn = b->lv_child_node[l];
  b_restrict<<<cn.n, 256, 0, q.s>>>((const BJob*)cn.p, b->d_slots, b->d_state);
  vcycle(q, l + 1);
  const DevTable& nd = b->lv_node[l];
  b_prolong<<<nd.n, 256, 0, q.s>>>((const BJob*)nd.p, b->d_slots, b->d_state);
  cheb_smooth(q, l, false);
}

// moduli, diagonals, multigrid set-up, CG start and first direction
void enqueue_setup(const Q& q) {
  BatchCtx* b = q.b;
  const int B = b->B;
  b_modulus<<<b->fine_cell.n, 256, 0, q.s>>>((const BJob*)b->fine_cell.p, b->d_inst, b->d_slots,
                                            b->d_state);
  for (int l = 0; l + 1 < b->Lmax; ++l)
    if (b->lv_child_sq[l].n > 0)
      b_restrict_E<<<b->lv_child_sq[l].n, 256, 0, q.s>>>((const BJob*)b->lv_child_sq[l].p, b->d_slots,
                                                         b->d_state);
  for (int l = 0; l < b->Lmax; ++l) {
    if (b->lv_listA[l].n == 0) continue;
    const DevTable& nd = b->lv_node[l];
    b_diag<<<nd.n, 256, 0, q.s>>>((const BJob*)nd.p, b->d_slots, b->d_state);
    const DevTable& dj = b->lv_dof[l];
    b_power_init<<<dj.n, 256, 0, q.s>>>((const BJob*)dj.p, b->d_slots, b->d_state);
    for (int it = 0; it < kPowerIters; ++it) {
      apply_lv(q, l, BV_PV, BV_PW, false, nullptr);
      b_power_step<<<dj.n, 256, 0, q.s>>>((const BJob*)dj.p, b->d_slots, b->d_state, b->partials);
      b_power_fin<<<b->lv_listA[l].n, 256, 0, q.s>>>((const int*)b->lv_listA[l].p, b->d_slots,
                                                      b->d_state, b->partials,
                                                      it == kPowerIters - 1, kPowerSafety);
    }
  }
  if (b->all_last.n > 0) {
    b_coarse_assemble<<<b->all_last.n, 128, 0, q.s>>>((const int*)b->all_last.p, b->d_slots, b->d_state);
    b_gauss_jordan<<<b->all_last.n, 1024, 0, q.s>>>((const int*)b->all_last.p, b->d_slots, b->d_state);
    if (b->gj_nb_max > 0) {
      const int nl = b->all_last.n;
      const int* lst = (const int*)b->all_last.p;
      const int ntri = b->gj_nb_max * (b->gj_nb_max + 1) / 2;
      b_dense_fill<<<dim3(256, nl), 256, 0, q.s>>>(lst, b->d_slots, b->d_state);
      b_coarse_assemble_ld<<<dim3((b->dense_n_max + 63) / 64, nl), 64, 0, q.s>>>(lst, b->d_slots,
                                                                                 b->d_state);
      b_gj_pivot<<<nl, kGjPivThreads, 0, q.s>>>(lst, b->d_slots, b->d_state, 0);
      for (int k = 0; k < b->gj_nb_max; ++k) {
        b_gj_panel<<<dim3(2 * b->gj_nb_max, nl), kGjThreads, 0, q.s>>>(lst, b->d_slots, b->d_state, k);
        b_gj_update<<<dim3(ntri, nl), kGjThreads, 0, q.s>>>(lst, b->d_slots, b->d_state, k);
      }
      b_gj_mirror<<<dim3(ntri, nl), kGjThreads, 0, q.s>>>(lst, b->d_slots, b->d_state);
    }
  }
  // CG start from the previous round's u
  apply_lv(q, 0, BV_U, BV_CQ, false, nullptr);
  const DevTable& d0 = b->lv_dof[0];
  b_pcg_init<<<d0.n, 256, 0, q.s>>>((const BJob*)d0.p, b->d_slots, b->d_state, b->partials);
  b_pcg_init_fin<<<B, 256, 0, q.s>>>(b->d_inst, b->d_state, b->partials);
  vcycle(q, 0);
  b_rz<<<d0.n, 256, 0, q.s>>>((const BJob*)d0.p, b->d_slots, b->d_state, b->partials);
  b_rz_fin<<<B, 256, 0, q.s>>>(b->d_inst, b->d_state, b->partials, 1);
  b_direction<<<d0.n, 256, 0, q.s>>>((const BJob*)d0.p, b->d_slots, b->d_state, 1);
}

void enqueue_cg(const Q& q) {
  BatchCtx* b = q.b;
  const int B = b->B;
  const DevTable& d0 = b->lv_dof[0];
  for (int k = 0; k < kBCgPerGraph; ++k) {
    apply_lv(q, 0, BV_P, BV_CQ, true, b->partials);
    b_alpha_fin<<<B, 256, 0, q.s>>>(b->d_inst, b->d_state, b->partials, b->shape);
    b_update<<<d0.n, 256, 0, q.s>>>((const BJob*)d0.p, b->d_slots, b->d_state, b->partials);
    b_update_fin<<<B, 256, 0, q.s>>>(b->d_inst, b->d_state, b->partials);
    vcycle(q, 0);
    b_rz<<<d0.n, 256, 0, q.s>>>((const BJob*)d0.p, b->d_slots, b->d_state, b->partials);
    b_rz_fin<<<B, 256, 0, q.s>>>(b->d_inst, b->d_state, b->partials, 0);
    b_direction<<<d0.n, 256, 0, q.s>>>((const BJob*)d0.p, b->d_slots, b->d_state, 0);
  }
  b_all_done<<<1, 256, 0, q.s>>>(b->d_state, B, &b->d_flags[0]);
}

void enqueue_post(const Q& q) {
  BatchCtx* b = q.b;
  const int B = b->B;
  const BJob* sq = (const BJob*)b->fine_sq.p;
  const BJob* ce = (const BJob*)b->fine_cell.p;
  b_sens<<<b->fine_sq.n, 256, 0, q.s>>>(sq, b->d_inst, b->d_slots, b->d_state, b->partials);
  b_sens_fin<<<B, 256, 0, q.s>>>(b->d_inst, b->d_state, b->partials);
  b_filter_gather<<<b->fine_cell.n, 256, 0, q.s>>>(ce, b->d_inst, b->d_state, 0);
  b_filter<<<b->fine_sq.n, 256, 0, q.s>>>(sq, b->d_inst, b->d_state, 0);
  b_oc_init<<<b->fine_cell.n, 256, 0, q.s>>>(ce, b->d_inst, b->d_state, b->partials);
  b_oc_init_fin<<<B, 256, 0, q.s>>>(b->d_inst, b->d_state, b->partials);
  for (int k = 0; k < kBOcPasses; ++k) {
    b_oc_pass<<<b->fine_cell.n, 256, 0, q.s>>>(ce, b->d_inst, b->d_state, b->partials);
    b_oc_pass_fin<<<B, 256, 0, q.s>>>(b->d_inst, b->d_state, b->partials);
  }
  b_oc_final<<<b->fine_cell.n, 256, 0, q.s>>>(ce, b->d_inst, b->d_state, b->partials);
  b_oc_final_fin<<<B, 256, 0, q.s>>>(b->d_inst, b->d_state, b->partials);
  b_copy_rho<<<b->fine_cell.n, 256, 0, q.s>>>(ce, b->d_inst, b->d_state);
  b_next_round<<<1, 256, 0, q.s>>>(b->d_state, B, b->d_prm, &b->d_flags[1]);
}

bool capture(BatchCtx* b, void (*fn)(const Q&), hipGraphExec_t* out) {
  hipGraph_t g = nullptr;
  if (hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal) != hipSuccess) return false;
  fn(Q{b, b->stream});
  if (hipStreamEndCapture(b->stream, &g) != hipSuccess || !g) {
    (void)hipGetLastError();
    return false;
  }
  const bool ok = hipGraphInstantiate(out, g, nullptr, nullptr, 0) == hipSuccess;
  (void)hipGraphDestroy(g);
  if (!ok) (void)hipGetLastError();
  return ok;
}

void run(BatchCtx* b, void (*fn)(const Q&), hipGraphExec_t g) {
  if (b->graphs && g) (void)hipGraphLaunch(g, b->stream);
  else fn(Q{b, b->stream});
}

// time every fine-level tile shape on the batch's own grids and keep the
// fastest (moduli 1, x = 0: the work does not depend on the values)
void autotune(BatchCtx* b) {
  const Q q{b, b->stream};
  // unit moduli and active instances for the timing runs
  b_reset<<<1, 256, 0, b->stream>>>(b->d_state, b->B, b->d_prm, 0.0, 1);
  long cells = b->total_cells;
  // the fine moduli are one array of all instances
  b_fill<<<1024, 256, 0, b->stream>>>(b->slots[b->inst[0].slot0].E, 1.0, cells);
  b_fill<<<1024, 256, 0, b->stream>>>(b->u, 0.0, b->total_dofs);
  hipEvent_t e0, e1;
  (void)hipEventCreate(&e0);
  (void)hipEventCreate(&e1);
  double best = 1e30;
  for (int sh = 0; sh < kBShapes; ++sh) {
    b->shape = sh;
    for (int w = 0; w < 3; ++w) apply_lv(q, 0, BV_U, BV_CQ, false, nullptr);
    (void)hipEventRecord(e0, b->stream);
    const int reps = 10;
    for (int w = 0; w < reps; ++w) apply_lv(q, 0, BV_U, BV_CQ, false, nullptr);
    (void)hipEventRecord(e1, b->stream);
    (void)hipEventSynchronize(e1);
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, e0, e1);
    b->shape_us[sh] = 1e3 * ms / reps;
    if (b->shape_us[sh] < best) best = b->shape_us[sh];
  }
  for (int sh = 0; sh < kBShapes; ++sh)
    if (b->shape_us[sh] == best) {
      b->shape = sh;
      break;
    }
  // TOPO_BATCH_TILE=0|1|2 pins the shape (the measurements are still made):
  // shapes block the CG dot products differently, so two batches compare
  // bit for bit only with the same shape
  if (const char* e = getenv("TOPO_BATCH_TILE")) {
    const int sh = atoi(e);
    if (sh >= 0 && sh < kBShapes) b->shape = sh;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
}

}  // namespace

struct topo_batch : public BatchCtx {};

extern "C" {

int topo_batch_workspace_size(const topo_problem* probs, int count, size_t* bytes) {
  if (!probs || count < 1 || count > 4096 || !bytes) return TOPO_E_INVALID;
  for (int i = 0; i < count; ++i)
    if (!valid_batch_problem(probs[i])) return TOPO_E_INVALID;
  *bytes = plan_batch(probs, count, nullptr, nullptr, nullptr, nullptr);
  return TOPO_OK;
}

int topo_batch_create(const topo_problem* probs, int count, const uint8_t* fixed_masks, void* ws,
                      size_t ws_bytes, void* stream, topo_batch** out) {
  if (!out) return TOPO_E_INVALID;
  *out = nullptr;
  size_t need = 0;
  int rc = topo_batch_workspace_size(probs, count, &need);
  if (rc != TOPO_OK) return rc;
  if (!fixed_masks || !ws) return TOPO_E_INVALID;
  if (((uintptr_t)ws & 255) != 0) return TOPO_E_SHAPE;
  if (ws_bytes < need) return TOPO_E_WORKSPACE;
  topo_batch* b = new (std::nothrow) topo_batch();
  if (!b) return TOPO_E_INVALID;
  b->B = count;
  b->ws = (char*)ws;
  b->ws_bytes = ws_bytes;
  b->caller = (hipStream_t)stream;
  b->maxit = 1;
  for (int i = 0; i < count; ++i) b->maxit = probs[i].maxit > b->maxit ? probs[i].maxit : b->maxit;
  if (hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking) != hipSuccess) {
    delete b;
    return TOPO_E_HIP;
  }
  // node masks of every level of every instance (host), from the fine masks
  std::vector<std::vector<std::vector<uint8_t>>> masks(count);
  const uint8_t* fm = fixed_masks;
  for (int i = 0; i < count; ++i) {
    const std::vector<LevelDims> plan = batch_plan(probs[i]);
    const long nn = (long)(probs[i].nel[0] + 1) * (probs[i].nel[1] + 1);
    std::vector<uint8_t> bits((size_t)nn, 0);
    for (int c = 0; c < 2; ++c)
      for (long n = 0; n < nn; ++n)
        if (fm[(size_t)c * nn + n]) bits[n] |= (uint8_t)(1u << c);
    fm += 2 * nn;
    masks[i].push_back(bits);
    for (size_t l = 1; l < plan.size(); ++l)
      masks[i].push_back(coarse_mask_host(masks[i][l - 1], plan[l - 1], plan[l], 2));
  }
  // zero the workspace, then carve and upload tables
  b_fill<<<1024, 256, 0, b->stream>>>((double*)ws, 0.0, (long)(need / 8));
  if (hipStreamSynchronize(b->stream) != hipSuccess) {
    (void)hipStreamDestroy(b->stream);
    delete b;
    return TOPO_E_HIP;
  }
  plan_batch(probs, count, b, (char*)ws, nullptr, &masks);
  void* pin = nullptr;
  if (hipHostMalloc(&pin, 64, hipHostMallocDefault) != hipSuccess) {
    (void)hipStreamDestroy(b->stream);
    delete b;
    return TOPO_E_HIP;
  }
  b->pinned = (volatile int*)pin;
  memset(pin, 0, 64);
  (void)hipEventCreateWithFlags(&b->ev[0], hipEventDisableTiming);
  (void)hipEventCreateWithFlags(&b->ev[1], hipEventDisableTiming);
  (void)hipEventCreateWithFlags(&b->ev_caller, hipEventDisableTiming);
  // filter row sums (rho-independent)
  b_filter_gather<<<b->fine_cell.n, 256, 0, b->stream>>>((const BJob*)b->fine_cell.p, b->d_inst,
                                                        b->d_state, 1);
  b_filter<<<b->fine_sq.n, 256, 0, b->stream>>>((const BJob*)b->fine_sq.p, b->d_inst, b->d_state, 1);
  autotune(b);
  // TOPO_BATCH_EAGER=1 launches the same kernels directly (for comparison)
  const char* eager = getenv("TOPO_BATCH_EAGER");
  b->graphs = !(eager && atoi(eager) == 1) && capture(b, enqueue_setup, &b->g_setup) &&
              capture(b, enqueue_cg, &b->g_cg) && capture(b, enqueue_post, &b->g_post);
  if (hipStreamSynchronize(b->stream) != hipSuccess || hipGetLastError() != hipSuccess) {
    (void)hipHostFree(pin);
    (void)hipStreamDestroy(b->stream);
    delete b;
    return TOPO_E_HIP;
  }
  *out = b;
  return TOPO_OK;
}

int topo_batch_destroy(topo_batch* b) {
  if (!b) return TOPO_E_INVALID;
  (void)hipStreamSynchronize(b->stream);
  if (b->g_setup) (void)hipGraphExecDestroy(b->g_setup);
  if (b->g_cg) (void)hipGraphExecDestroy(b->g_cg);
  if (b->g_post) (void)hipGraphExecDestroy(b->g_post);
  for (hipEvent_t e : {b->ev[0], b->ev[1], b->ev_caller})
    if (e) (void)hipEventDestroy(e);
  (void)hipHostFree((void*)b->pinned);
  (void)hipStreamDestroy(b->stream);
  delete b;
  return TOPO_OK;
}

int topo_batch_set_loads(topo_batch* b, const double* f) {
  if (!b || !f) return TOPO_E_INVALID;
  TOPO_HIP(hipEventRecord(b->ev_caller, b->caller));
  TOPO_HIP(hipStreamWaitEvent(b->stream, b->ev_caller, 0));
  TOPO_HIP(hipMemcpyAsync(b->f, f, (size_t)b->total_dofs * 8, hipMemcpyDeviceToDevice, b->stream));
  TOPO_HIP(hipStreamSynchronize(b->stream));
  return TOPO_OK;
}

int topo_batch_iterate(topo_batch* b, double* rho, int max_iter, double change_tol, double* record,
                       int* rounds) {
  if (!b || !rho || max_iter < 0) return TOPO_E_INVALID;
  hipStream_t s = b->stream;
  TOPO_HIP(hipEventRecord(b->ev_caller, b->caller));
  TOPO_HIP(hipStreamWaitEvent(s, b->ev_caller, 0));
  TOPO_HIP(hipMemcpyAsync(b->rho, rho, (size_t)b->total_cells * 8, hipMemcpyDeviceToDevice, s));
  b_reset<<<1, 256, 0, s>>>(b->d_state, b->B, b->d_prm, change_tol, max_iter);
  b_fill<<<1024, 256, 0, s>>>(b->u, 0.0, b->total_dofs);
  int done_rounds = 0;
  for (int it = 0; it < max_iter; ++it) {
    run(b, enqueue_setup, b->g_setup);
    // CG continuation until every active instance has converged; the flag
    // is polled one replay behind the queue
    const int cap = (b->maxit + kBCgPerGraph - 1) / kBCgPerGraph;
    bool stop = false;
    for (int k = 0; k < cap && !stop; ++k) {
      run(b, enqueue_cg, b->g_cg);
      const int sl = k & 1;
      TOPO_HIP(hipMemcpyAsync((void*)&b->pinned[sl], &b->d_flags[0], sizeof(int), hipMemcpyDeviceToHost, s));
      TOPO_HIP(hipEventRecord(b->ev[sl], s));
      if (k > 0) {
        TOPO_HIP(hipEventSynchronize(b->ev[sl ^ 1]));
        if (b->pinned[sl ^ 1]) stop = true;
      }
    }
    run(b, enqueue_post, b->g_post);
    ++done_rounds;
    TOPO_HIP(hipMemcpyAsync((void*)&b->pinned[4], &b->d_flags[1], sizeof(int), hipMemcpyDeviceToHost, s));
    TOPO_HIP(hipStreamSynchronize(s));
    if (!b->pinned[4]) break;
  }
  TOPO_HIP(hipMemcpyAsync(rho, b->rho, (size_t)b->total_cells * 8, hipMemcpyDeviceToDevice, s));
  if (record) b_record<<<1, 256, 0, s>>>(b->d_inst, b->d_state, b->d_prm, b->B, record);
  TOPO_HIP(hipStreamSynchronize(s));
  if (rounds) *rounds = done_rounds;
  return hipGetLastError() == hipSuccess ? TOPO_OK : TOPO_E_HIP;
}

int topo_batch_solution(topo_batch* b, double* u) {
  if (!b || !u) return TOPO_E_INVALID;
  TOPO_HIP(hipMemcpyAsync(u, b->u, (size_t)b->total_dofs * 8, hipMemcpyDeviceToDevice, b->stream));
  TOPO_HIP(hipStreamSynchronize(b->stream));
  return TOPO_OK;
}

int topo_batch_tile_shape(topo_batch* b, int* bx, int* by, double* us_per_shape) {
  if (!b) return TOPO_E_INVALID;
  if (bx) *bx = kShapeBX[b->shape];
  if (by) *by = kShapeBY[b->shape];
  if (us_per_shape)
    for (int sh = 0; sh < kBShapes; ++sh) us_per_shape[sh] = b->shape_us[sh];
  return TOPO_OK;
}

int topo_batch_sync(topo_batch* b, int* device_status) {
  if (!b) return TOPO_E_INVALID;
  b_status<<<1, 1, 0, b->stream>>>(b->d_state, b->B, &b->d_flags[2]);
  int st = 0;
  TOPO_HIP(hipMemcpyAsync(&st, &b->d_flags[2], sizeof(int), hipMemcpyDeviceToHost, b->stream));
  TOPO_HIP(hipStreamSynchronize(b->stream));
  if (device_status) *device_status = st;
  return TOPO_OK;
}

int topo_batch_uses_graphs(topo_batch* b) { return b ? (b->graphs ? 1 : 0) : TOPO_E_INVALID; }

}  // extern "C"
