// Preconditioned conjugate gradients for K(rho) u_r = f_r, one independent
// CG per load case r with FP64 scalars (the paper solves the same system by
// sparse LU, Sec. 4.2.4; the iteration here is the textbook PCG).
//
// Per iteration three kernels run on the context stream:
//   apply:   q = K p, and alpha_r = (r,z)_r / (p,q)_r (fused reduction)
//   update:  u += alpha p, r -= alpha q, z = M r; beta_r and the
//            convergence test ||r_r|| <= rtol ||f_r|| (fused reduction)
//   direction: p = z + beta p
// All reductions are single-pass and deterministic (fixed block order).
// Once every load case has converged the kernels return immediately; the
// host polls a pinned copy of the done flag one batch behind the queue, so
// the device never waits for the host.
#include "common.h"
#include "topo_internal.h"

namespace topo {

template <int NR>
__global__ __launch_bounds__(256) void pcg_init_kernel(const double* __restrict__ f,
                                                       const double* __restrict__ Ku, double* u,
                                                       double* r, double* p,
                                                       const double* __restrict__ invd,
                                                       const uint8_t* __restrict__ mask, long nn,
                                                       int dim, double rtol, int warm,
                                                       double* partials, unsigned* counter,
                                                       PcgState* st) {
  const long nd = nn * dim;
  double acc[3 * NR];
#pragma unroll
  for (int k = 0; k < 3 * NR; ++k) acc[k] = 0.0;
  for (long d = (long)blockIdx.x * blockDim.x + threadIdx.x; d < nd; d += (long)gridDim.x * blockDim.x) {
    const long n = d % nn;
    const int c = (int)(d / nn);
    const bool fixed = (mask[n] >> c) & 1;
    const double id = invd[d];
#pragma unroll
    for (int q = 0; q < NR; ++q) {
      const long i = (long)q * nd + d;
      const double fv = fixed ? 0.0 : f[i];
      double rv = fv;
      if (warm) rv = fixed ? 0.0 : fv - Ku[i];
      else u[i] = 0.0;
      if (fixed && warm) u[i] = 0.0;
      const double zv = id * rv;
      r[i] = rv;
      p[i] = zv;
      acc[q] += rv * zv;
      acc[NR + q] += rv * rv;
      acc[2 * NR + q] += fv * fv;
    }
  }
  double dummy[1] = {0.0};
  __shared__ double tot[3 * NR];
  if (grid_reduce<3 * NR, 0>(acc, dummy, partials, counter, tot)) {
    if (threadIdx.x == 0) {
      int any = 0;
      for (int q = 0; q < NR; ++q) {
        st->rz[q] = tot[q];
        st->rr[q] = tot[NR + q];
        st->ff[q] = tot[2 * NR + q];
        st->tol2[q] = rtol * rtol * tot[2 * NR + q];
        st->active[q] = (tot[2 * NR + q] > 0.0) && (tot[NR + q] > st->tol2[q]);
        st->alpha[q] = 0.0;
        st->beta[q] = 0.0;
        any |= st->active[q];
      }
      for (int q = NR; q < kMaxRhs; ++q) { st->active[q] = 0; st->rr[q] = 0; st->ff[q] = 0; }
      st->done = !any;
      st->iters = 0;
      st->breakdown = 0;
    }
  }
}

template <int NR>
__global__ __launch_bounds__(256) void pcg_update_kernel(double* u, double* r,
                                                         const double* __restrict__ p,
                                                         const double* __restrict__ q,
                                                         const double* __restrict__ invd, long nd,
                                                         double* partials, unsigned* counter,
                                                         PcgState* st, int* status) {
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
      u[i] += al[k] * p[i];
      const double rv = r[i] - al[k] * q[i];
      r[i] = rv;
      acc[k] += rv * (id * rv);
      acc[NR + k] += rv * rv;
    }
  }
  double dummy[1] = {0.0};
  __shared__ double tot[2 * NR];
  if (grid_reduce<2 * NR, 0>(acc, dummy, partials, counter, tot)) {
    if (threadIdx.x == 0) {
      int any = 0;
      for (int k = 0; k < NR; ++k) {
        if (!st->active[k]) continue;
        st->rz_old[k] = st->rz[k];
        st->rz[k] = tot[k];
        st->rr[k] = tot[NR + k];
        st->beta[k] = tot[k] / st->rz_old[k];
        if (!(tot[NR + k] > st->tol2[k])) st->active[k] = 0;
        if (!isfinite(tot[NR + k])) { st->breakdown = 1; st->active[k] = 0; }
        any |= st->active[k];
      }
      st->iters += 1;
      if (st->breakdown) { *status = TOPO_S_NUMERIC; any = 0; }
      st->done = !any;
    }
  }
}

template <int NR>
__global__ __launch_bounds__(256) void pcg_direction_kernel(double* p, const double* __restrict__ r,
                                                            const double* __restrict__ invd,
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

__global__ void pcg_info_kernel(const PcgState* st, double* info, int nr, int* status) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const int conv = st->done && !st->breakdown;
  if (info) {
    info[0] = st->iters;
    info[1] = conv;
    for (int k = 0; k < kMaxRhs; ++k)
      info[2 + k] = (k < nr && st->ff[k] > 0.0) ? sqrt(st->rr[k] / st->ff[k]) : 0.0;
  }
  if (st->breakdown) *status = TOPO_S_NUMERIC;
  else if (!st->done && *status == 0) *status = TOPO_S_NOT_CONVERGED;
}

static unsigned red_grid(long n) {
  long b = (n + 255) / 256;
  return (unsigned)(b < kRedBlocks ? (b < 1 ? 1 : b) : kRedBlocks);
}

void pcg_solve(Ctx* c, double* u, double* info) {
  const int nr = c->prob.nrhs;
  const long nd = c->g.nd;
  PcgState* st = &c->scal->pcg;
  int* status = &c->scal->status;
  const bool warm = c->prob.warm_start != 0;
  if (warm) launch_apply(c, u, c->q, nr, false);
  const unsigned gb = red_grid(nd);
#define INIT(NR) pcg_init_kernel<NR><<<gb, 256, 0, c->stream>>>(c->f, c->q, u, c->r, c->p, c->invd, c->mask, c->g.nn, c->g.dim, c->prob.rtol, warm, c->partials, &c->scal->counters[CNT_PCG_INIT], st)
  switch (nr) { case 1: INIT(1); break; case 2: INIT(2); break; case 3: INIT(3); break; default: INIT(4); }
#undef INIT
  const int batch = 8;
  const int maxit = c->prob.maxit;
  int it = 0, b = 0;
  bool stop = false;
  while (it < maxit && !stop) {
    const int nb = (maxit - it < batch) ? (maxit - it) : batch;
    for (int k = 0; k < nb; ++k) {
      launch_apply(c, c->p, c->q, nr, true);
#define UPD(NR) pcg_update_kernel<NR><<<gb, 256, 0, c->stream>>>(u, c->r, c->p, c->q, c->invd, nd, c->partials, &c->scal->counters[CNT_PCG_UPDATE], st, status)
      switch (nr) { case 1: UPD(1); break; case 2: UPD(2); break; case 3: UPD(3); break; default: UPD(4); }
#undef UPD
#define DIR(NR) pcg_direction_kernel<NR><<<gb, 256, 0, c->stream>>>(c->p, c->r, c->invd, nd, st)
      switch (nr) { case 1: DIR(1); break; case 2: DIR(2); break; case 3: DIR(3); break; default: DIR(4); }
#undef DIR
    }
    it += nb;
    // poll the previous batch's flag while this batch runs
    const int s = b & 1;
    (void)hipMemcpyAsync((void*)&c->pinned[s], &st->done, sizeof(int), hipMemcpyDeviceToHost, c->stream);
    (void)hipEventRecord(c->ev_poll[s], c->stream);
    if (b > 0) {
      (void)hipEventSynchronize(c->ev_poll[s ^ 1]);
      if (c->pinned[s ^ 1]) stop = true;
    }
    ++b;
  }
  pcg_info_kernel<<<1, 64, 0, c->stream>>>(st, info, nr, status);
}

}  // namespace topo
