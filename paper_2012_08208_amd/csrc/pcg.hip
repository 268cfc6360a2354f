// Preconditioned conjugate gradients for K(rho) u_r = f_r, one independent
// CG per load case r with FP64 scalars.  (The paper solves the same system
// by sparse LU, Sec. 4.2.4; the iteration here is the textbook PCG.)
//
// One iteration on the context stream:
//   apply      q = K p and per-block (p,q)        -> alpha_fin: alpha = (r,z)/(p,q)
//   update     u += alpha p, r -= alpha q, (r,r)  -> update_fin: convergence test
//              (Jacobi: also (r, D^-1 r) and beta, fused)
//   precond    z = M r (multigrid V-cycle)        -> rz, rz_fin: beta = (r,z)/(r,z)_old
//   direction  p = z + beta p
// Wide kernels write per-block partials; one-block "fin" kernels reduce them
// in a fixed order, so results are deterministic.  After every load case
// has converged all kernels return at once; the host polls a pinned copy of
// the done flag one batch behind the queue, so the device never idles.
#include "common.h"
#include "topo_internal.h"

namespace topo {

template <int NR>
__global__ __launch_bounds__(256) void pcg_init_kernel(const double* __restrict__ f,
                                                       const double* __restrict__ Ku, double* u,
                                                       double* r, const uint8_t* __restrict__ mask,
                                                       long nn, int dim, int warm,
                                                       double* partials) {
  const long nd = nn * dim;
  double acc[2 * NR];
#pragma unroll
  for (int k = 0; k < 2 * NR; ++k) acc[k] = 0.0;
  for (long d = (long)blockIdx.x * blockDim.x + threadIdx.x; d < nd; d += (long)gridDim.x * blockDim.x) {
    const long n = d % nn;
    const int c = (int)(d / nn);
    const bool fixed = (mask[n] >> c) & 1;
#pragma unroll
    for (int q = 0; q < NR; ++q) {
      const long i = (long)q * nd + d;
      const double fv = fixed ? 0.0 : f[i];
      double rv = fv;
      if (warm) {
        rv = fixed ? 0.0 : fv - Ku[i];
        if (fixed) u[i] = 0.0;
      } else {
        u[i] = 0.0;
      }
      r[i] = rv;
      acc[q] += rv * rv;
      acc[NR + q] += fv * fv;
    }
  }
  const double none[1] = {0.0};
  block_partials<2 * NR, 0>(acc, none, partials);
}

template <int NR>
__global__ void pcg_init_fin(const double* partials, long nb, double rtol, PcgState* st) {
  __shared__ double tot[2 * NR];
  reduce_partials<2 * NR, 0>(partials, nb, tot);
  if (threadIdx.x == 0) {
    int any = 0;
    for (int q = 0; q < kMaxRhs; ++q) {
      const bool has = q < NR;
      st->rr[q] = has ? tot[q] : 0.0;
      st->ff[q] = has ? tot[NR + q] : 0.0;
      st->tol2[q] = rtol * rtol * st->ff[q];
      st->active[q] = has && (st->ff[q] > 0.0) && (st->rr[q] > st->tol2[q]);
      st->alpha[q] = 0.0;
      st->beta[q] = 0.0;
      st->rz[q] = 0.0;
      any |= st->active[q];
    }
    st->done = !any;
    st->iters = 0;
    st->breakdown = 0;
  }
}

// z = D^-1 r (Jacobi) written explicitly, used for the first direction
template <int NR>
__global__ __launch_bounds__(256) void jacobi_kernel(double* z, const double* __restrict__ r,
                                                     const double* __restrict__ invd, long nd) {
  for (long d = (long)blockIdx.x * blockDim.x + threadIdx.x; d < nd; d += (long)gridDim.x * blockDim.x) {
    const double id = invd[d];
#pragma unroll
    for (int k = 0; k < NR; ++k) z[(long)k * nd + d] = id * r[(long)k * nd + d];
  }
}

// partial (r, z) per load case
template <int NR>
__global__ __launch_bounds__(256) void pcg_rz_kernel(const double* __restrict__ r,
                                                     const double* __restrict__ z, long nd,
                                                     double* partials, const PcgState* st) {
  if (st->done) return;
  double acc[NR];
#pragma unroll
  for (int k = 0; k < NR; ++k) acc[k] = 0.0;
  for (long d = (long)blockIdx.x * blockDim.x + threadIdx.x; d < nd; d += (long)gridDim.x * blockDim.x) {
#pragma unroll
    for (int k = 0; k < NR; ++k) acc[k] += r[(long)k * nd + d] * z[(long)k * nd + d];
  }
  const double none[1] = {0.0};
  block_partials<NR, 0>(acc, none, partials);
}

template <int NR>
__global__ void pcg_rz_fin(const double* partials, long nb, int first, PcgState* st) {
  if (st->done) return;
  __shared__ double tot[NR];
  reduce_partials<NR, 0>(partials, nb, tot);
  if (threadIdx.x == 0) {
    for (int k = 0; k < NR; ++k) {
      if (!st->active[k]) continue;
      if (first) {
        st->rz[k] = tot[k];
        st->beta[k] = 0.0;
      } else {
        st->rz_old[k] = st->rz[k];
        st->rz[k] = tot[k];
        st->beta[k] = tot[k] / st->rz_old[k];
      }
      if (!(tot[k] > 0.0)) { st->breakdown = 1; st->active[k] = 0; }
    }
    if (st->breakdown) st->done = 1;
  }
}

__global__ void pcg_alpha_fin(const double* partials, long nb, PcgState* st) {
  if (st->done) return;
  __shared__ double tot[kMaxRhs];
  reduce_partials<kMaxRhs, 0>(partials, nb, tot);
  if (threadIdx.x == 0) {
    for (int r = 0; r < kMaxRhs; ++r) {
      st->pq[r] = tot[r];
      if (st->active[r]) {
        if (!(tot[r] > 0.0)) { st->breakdown = 1; st->alpha[r] = 0.0; }
        else st->alpha[r] = st->rz[r] / tot[r];
      } else {
        st->alpha[r] = 0.0;
      }
    }
  }
}

// u += alpha p, r -= alpha q; partial (r,r) and, for Jacobi, (r, D^-1 r)
template <int NR, bool JAC>
__global__ __launch_bounds__(256) void pcg_update_kernel(double* u, double* r,
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
    const double id = JAC ? invd[d] : 0.0;
#pragma unroll
    for (int k = 0; k < NR; ++k) {
      if (!act[k]) continue;
      const long i = (long)k * nd + d;
      u[i] += al[k] * p[i];
      const double rv = r[i] - al[k] * q[i];
      r[i] = rv;
      acc[k] += rv * rv;
      if (JAC) acc[NR + k] += rv * (id * rv);
    }
  }
  const double none[1] = {0.0};
  block_partials<2 * NR, 0>(acc, none, partials);
}

template <int NR, bool JAC>
__global__ void pcg_update_fin(const double* partials, long nb, PcgState* st, int* status) {
  if (st->done) return;
  __shared__ double tot[2 * NR];
  reduce_partials<2 * NR, 0>(partials, nb, tot);
  if (threadIdx.x == 0) {
    int any = 0;
    for (int k = 0; k < NR; ++k) {
      if (!st->active[k]) continue;
      st->rr[k] = tot[k];
      if (JAC) {
        st->rz_old[k] = st->rz[k];
        st->rz[k] = tot[NR + k];
        st->beta[k] = tot[NR + k] / st->rz_old[k];
      }
      if (!(tot[k] > st->tol2[k])) st->active[k] = 0;
      if (!isfinite(tot[k])) { st->breakdown = 1; st->active[k] = 0; }
      any |= st->active[k];
    }
    st->iters += 1;
    if (st->breakdown) { *status = TOPO_S_NUMERIC; any = 0; }
    st->done = !any;
  }
}

// p = z + beta p (Jacobi: z = D^-1 r on the fly); first: p = z
template <int NR, bool JAC>
__global__ __launch_bounds__(256) void pcg_direction_kernel(double* p, const double* __restrict__ z,
                                                            const double* __restrict__ r,
                                                            const double* __restrict__ invd,
                                                            long nd, const PcgState* st,
                                                            int first) {
  if (st->done) return;
  double be[NR];
  bool act[NR];
#pragma unroll
  for (int k = 0; k < NR; ++k) { be[k] = first ? 0.0 : st->beta[k]; act[k] = st->active[k] != 0; }
  for (long d = (long)blockIdx.x * blockDim.x + threadIdx.x; d < nd; d += (long)gridDim.x * blockDim.x) {
    const double id = JAC ? invd[d] : 0.0;
#pragma unroll
    for (int k = 0; k < NR; ++k) {
      if (!act[k]) continue;
      const long i = (long)k * nd + d;
      const double zv = JAC ? id * r[i] : z[i];
      p[i] = first ? zv : zv + be[k] * p[i];
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

unsigned red_grid(long n) {
  long b = (n + 255) / 256;
  return (unsigned)(b < kRedBlocks ? (b < 1 ? 1 : b) : kRedBlocks);
}

template <int NR>
static void pcg_run(Ctx* c, double* u, double* info) {
  const long nd = c->g.nd;
  PcgState* st = &c->scal->pcg;
  int* status = &c->scal->status;
  hipStream_t s = c->stream;
  const bool warm = c->prob.warm_start != 0;
  const bool gmg = c->prob.precond == TOPO_PC_GMG;
  const unsigned gb = red_grid(nd);
  const long nb_apply = apply_grid_blocks(fine_op(c), NR);
  if (warm) launch_apply(c, u, c->q, NR, false);
  pcg_init_kernel<NR><<<gb, 256, 0, s>>>(c->f, c->q, u, c->r, c->mask, c->g.nn, c->g.dim, warm,
                                         c->partials);
  pcg_init_fin<NR><<<1, 256, 0, s>>>(c->partials, gb, c->prob.rtol, st);
  // first direction p = M r
  if (gmg) {
    gmg_vcycle(c, c->r, c->z, NR);
    pcg_rz_kernel<NR><<<gb, 256, 0, s>>>(c->r, c->z, nd, c->partials, st);
    pcg_rz_fin<NR><<<1, 256, 0, s>>>(c->partials, gb, 1, st);
    pcg_direction_kernel<NR, false><<<gb, 256, 0, s>>>(c->p, c->z, c->r, c->invd, nd, st, 1);
  } else {
    jacobi_kernel<NR><<<gb, 256, 0, s>>>(c->p, c->r, c->invd, nd);
    pcg_rz_kernel<NR><<<gb, 256, 0, s>>>(c->r, c->p, nd, c->partials, st);
    pcg_rz_fin<NR><<<1, 256, 0, s>>>(c->partials, gb, 1, st);
  }
  const int batch = gmg ? 2 : 8;
  const int maxit = c->prob.maxit;
  int it = 0, b = 0;
  bool stop = false;
  while (it < maxit && !stop) {
    const int nbt = (maxit - it < batch) ? (maxit - it) : batch;
    for (int k = 0; k < nbt; ++k) {
      launch_apply(c, c->p, c->q, NR, true);
      pcg_alpha_fin<<<1, 256, 0, s>>>(c->partials, nb_apply, st);
      if (gmg) {
        pcg_update_kernel<NR, false><<<gb, 256, 0, s>>>(u, c->r, c->p, c->q, c->invd, nd,
                                                        c->partials, st);
        pcg_update_fin<NR, false><<<1, 256, 0, s>>>(c->partials, gb, st, status);
        gmg_vcycle(c, c->r, c->z, NR);
        pcg_rz_kernel<NR><<<gb, 256, 0, s>>>(c->r, c->z, nd, c->partials, st);
        pcg_rz_fin<NR><<<1, 256, 0, s>>>(c->partials, gb, 0, st);
        pcg_direction_kernel<NR, false><<<gb, 256, 0, s>>>(c->p, c->z, c->r, c->invd, nd, st, 0);
      } else {
        pcg_update_kernel<NR, true><<<gb, 256, 0, s>>>(u, c->r, c->p, c->q, c->invd, nd,
                                                       c->partials, st);
        pcg_update_fin<NR, true><<<1, 256, 0, s>>>(c->partials, gb, st, status);
        pcg_direction_kernel<NR, true><<<gb, 256, 0, s>>>(c->p, nullptr, c->r, c->invd, nd, st, 0);
      }
    }
    it += nbt;
    // poll the previous batch's flag while this batch runs
    const int sl = b & 1;
    (void)hipMemcpyAsync((void*)&c->pinned[sl], &st->done, sizeof(int), hipMemcpyDeviceToHost, s);
    (void)hipEventRecord(c->ev_poll[sl], s);
    if (b > 0) {
      (void)hipEventSynchronize(c->ev_poll[sl ^ 1]);
      if (c->pinned[sl ^ 1]) stop = true;
    }
    ++b;
  }
  pcg_info_kernel<<<1, 64, 0, s>>>(st, info, NR, status);
}

void pcg_solve(Ctx* c, double* u, double* info) {
  if (c->prob.precond == TOPO_PC_GMG) gmg_setup(c);
  switch (c->prob.nrhs) {
    case 1: pcg_run<1>(c, u, info); break;
    case 2: pcg_run<2>(c, u, info); break;
    case 3: pcg_run<3>(c, u, info); break;
    default: pcg_run<4>(c, u, info); break;
  }
}

}  // namespace topo
