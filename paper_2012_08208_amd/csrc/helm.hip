// Helmholtz-type PDE sensitivity filter (the filter Sec. 6.3 switches to for
// parallel runs, after Lazarov and Sigmund 2011):
//   (r^2 K + M) x = T (rho s),   s~_e = mean of x over the vertices of e / rho_e,
// with K the P1 Laplacian stiffness, M the consistent P1 mass and
// T_ne = |T_e| / (d+1) for the vertices n of cell e, on the elasticity mesh
// (zero normal derivative on the whole boundary), r = rmin / (2 sqrt 3).
//
// The operator has constant coefficients: every cube (square) carries the
// same 8 x 8 (4 x 4) matrix, summed on the host from the element matrices of
// its tetrahedra (triangles).  Kernels work per node and gather from the
// cubes (squares) that exist around it, so the truncated boundary needs no
// special case.  The solve is Jacobi-preconditioned CG in FP64 with the
// deterministic two-stage reductions of the elasticity solver; the host
// polls the converged flag between batches of iterations.
#include <math.h>
#include <string.h>

#include "common.h"
#include "topo_internal.h"

namespace topo {

constexpr double kHelmRtol = 1e-12;   // relative residual of the filter solve
constexpr int kHelmMaxit = 4000;
constexpr int kHelmNoWaitIters = 256;   // iterations queued per filter call without host waits

static inline unsigned cdivu(long a, long b) { return (unsigned)((a + b - 1) / b); }

// ------------------------------------------------------ host: coefficients

// P1 gradients of a simplex with vertices X[0..d] (d = 2 or 3) from the
// inverse Jacobian; returns the measure.
static double simplex_grads(int d, const double (*X)[3], double (*g)[3]) {
  double J[3][3] = {{0}}, Ji[3][3] = {{0}};
  for (int a = 0; a < d; ++a)
    for (int i = 0; i < d; ++i) J[a][i] = X[a + 1][i] - X[0][i];   // row a: x_{a+1} - x_0
  double det;
  if (d == 2) {
    det = J[0][0] * J[1][1] - J[0][1] * J[1][0];
    Ji[0][0] = J[1][1] / det;  Ji[0][1] = -J[0][1] / det;
    Ji[1][0] = -J[1][0] / det; Ji[1][1] = J[0][0] / det;
  } else {
    det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) -
          J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
          J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        const int i1 = (j + 1) % 3, i2 = (j + 2) % 3, j1 = (i + 1) % 3, j2 = (i + 2) % 3;
        Ji[i][j] = (J[i1][j1] * J[i2][j2] - J[i1][j2] * J[i2][j1]) / det;
      }
  }
  // with x = x_0 + J^T xi, grad N_a (a >= 1) is column a-1 of J^-1
  for (int a = 1; a <= d; ++a)
    for (int i = 0; i < d; ++i) g[a][i] = Ji[i][a - 1];
  for (int i = 0; i < d; ++i) {
    g[0][i] = 0.0;
    for (int a = 1; a <= d; ++a) g[0][i] -= g[a][i];
  }
  return fabs(det) / (d == 2 ? 2.0 : 6.0);
}

// Adds r^2 |T| grad N_a . grad N_b + |T| (1 + delta_ab) / ((d+1)(d+2)) of
// one simplex (vertices = cell corners cs[]) into the cell matrix A.
static void add_simplex(int d, const int* cs, double r2, double (*A)[8], double* vol_out) {
  double X[4][3] = {{0}};
  for (int a = 0; a <= d; ++a)
    for (int i = 0; i < d; ++i) X[a][i] = (cs[a] >> i) & 1;
  double g[4][3];
  const double vol = simplex_grads(d, X, g);
  const double mdiv = (double)((d + 1) * (d + 2));
  for (int a = 0; a <= d; ++a)
    for (int b = 0; b <= d; ++b) {
      double gg = 0.0;
      for (int i = 0; i < d; ++i) gg += g[a][i] * g[b][i];
      A[cs[a]][cs[b]] += r2 * vol * gg + vol * (a == b ? 2.0 : 1.0) / mdiv;
    }
  *vol_out = vol;
}

void build_helm_coef(Ctx* c) {
  HelmCoef& h = c->hcoef;
  memset(&h, 0, sizeof(h));
  const double r = c->prob.rmin / (2.0 * sqrt(3.0));
  const double r2 = r * r;
  double vol = 0.0;
  if (c->g.dim == 3) {
    // Kuhn tetrahedron t: corners 0, 1<<p0, (1<<p0)|(1<<p1), 7
    const int perm[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
    for (int t = 0; t < 6; ++t) {
      const int c1 = 1 << perm[t][0];
      const int c2 = c1 | (1 << perm[t][1]);
      const int cs[4] = {0, c1, c2, 7};
      add_simplex(3, cs, r2, h.A[0], &vol);
      for (int v = 0; v < 4; ++v) h.cells_of_corner[0][cs[v]] |= (uint8_t)(1 << t);
    }
    h.w_rhs = vol / 4.0;
  } else {
    // corners 0 = (0,0), 1 = (1,0), 2 = (0,1), 3 = (1,1); diagonal A joins
    // 0-3 (triangles {0,1,3}, {0,3,2}), diagonal B joins 1-2 ({0,1,2}, {1,3,2})
    const int tri[2][2][3] = {{{0, 1, 3}, {0, 3, 2}}, {{0, 1, 2}, {1, 3, 2}}};
    for (int s = 0; s < 2; ++s)
      for (int t = 0; t < 2; ++t) {
        add_simplex(2, tri[s][t], r2, h.A[s], &vol);
        for (int v = 0; v < 3; ++v) h.cells_of_corner[s][tri[s][t][v]] |= (uint8_t)(1 << t);
      }
    h.w_rhs = vol / 3.0;
  }
}

// ------------------------------------------------------------- kernels

__device__ __forceinline__ bool helm_sq_a(int uniform, int hj) { return uniform || ((hj & 1) == 0); }

// diagonal of r^2 K + M, inverted
__global__ void helm_diag_kernel(double* invd, int dim, int nx, int ny, int nz, int uniform,
                                 HelmCoef hc, long nn) {
  const long n = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= nn) return;
  const int i = (int)(n % (nx + 1));
  const int j = (int)((n / (nx + 1)) % (ny + 1));
  const int k = dim == 3 ? (int)(n / ((long)(nx + 1) * (ny + 1))) : 0;
  double d = 0.0;
  for (int sz = (dim == 3 ? -1 : 0); sz <= 0; ++sz)
    for (int sy = -1; sy <= 0; ++sy)
      for (int sx = -1; sx <= 0; ++sx) {
        const int hi = i + sx, hj = j + sy, hk = k + sz;
        if (hi < 0 || hi >= nx || hj < 0 || hj >= ny || (dim == 3 && (hk < 0 || hk >= nz))) continue;
        const int cn = (-sx) + 2 * (-sy) + 4 * (-sz);
        d += hc.A[dim == 3 ? 0 : (helm_sq_a(uniform, hj) ? 0 : 1)][cn][cn];
      }
  invd[n] = 1.0 / d;
}

// b = T (rho s) at node n; then x = 0, r = b, p = D^-1 b, partials (r, D^-1 r), (b, b)
template <int DIM>
__global__ __launch_bounds__(256) void helm_init_kernel(const double* __restrict__ rho,
                                                        const double* __restrict__ s, double* x,
                                                        double* r, double* p,
                                                        const double* __restrict__ invd, int nx,
                                                        int ny, int nz, int uniform, HelmCoef hc,
                                                        long nn, double* partials) {
  double acc[2] = {0.0, 0.0};
  const long plane = (long)(nx + 1) * (ny + 1);
  for (long n = (long)blockIdx.x * blockDim.x + threadIdx.x; n < nn; n += (long)gridDim.x * blockDim.x) {
    const int i = (int)(n % (nx + 1));
    const int j = (int)((n / (nx + 1)) % (ny + 1));
    const int k = DIM == 3 ? (int)(n / plane) : 0;
    double b = 0.0;
#pragma unroll
    for (int sz = (DIM == 3 ? -1 : 0); sz <= 0; ++sz)
#pragma unroll
      for (int sy = -1; sy <= 0; ++sy)
#pragma unroll
        for (int sx = -1; sx <= 0; ++sx) {
          const int hi = i + sx, hj = j + sy, hk = k + sz;
          if (hi < 0 || hi >= nx || hj < 0 || hj >= ny || (DIM == 3 && (hk < 0 || hk >= nz))) continue;
          const int cn = (-sx) + 2 * (-sy) + 4 * (-sz);
          if (DIM == 3) {
            const long h = ((long)hk * ny + hj) * nx + hi;
            const int bits = hc.cells_of_corner[0][cn];
#pragma unroll
            for (int t = 0; t < 6; ++t)
              if ((bits >> t) & 1) b += rho[6 * h + t] * s[6 * h + t];
          } else {
            const long h = (long)hj * nx + hi;
            const int bits = hc.cells_of_corner[helm_sq_a(uniform, hj) ? 0 : 1][cn];
#pragma unroll
            for (int t = 0; t < 2; ++t)
              if ((bits >> t) & 1) b += rho[2 * h + t] * s[2 * h + t];
          }
        }
    b *= hc.w_rhs;
    const double z = invd[n] * b;
    x[n] = 0.0;
    r[n] = b;
    p[n] = z;
    acc[0] += b * z;
    acc[1] += b * b;
  }
  const double none[1] = {0.0};
  block_partials<2, 0>(acc, none, partials);
}

// q = (r^2 K + M) p, partial (p, q)
template <int DIM>
__global__ __launch_bounds__(256) void helm_apply_kernel(const double* __restrict__ p,
                                                         double* __restrict__ q,
                                                         int nx, int ny, int nz, int uniform,
                                                         HelmCoef hc, long nn, double* partials,
                                                         const HelmState* st) {
  if (st->done) return;
  double acc[1] = {0.0};
  const long row = nx + 1;
  const long plane = row * (ny + 1);
  for (long n = (long)blockIdx.x * blockDim.x + threadIdx.x; n < nn; n += (long)gridDim.x * blockDim.x) {
    const int i = (int)(n % (nx + 1));
    const int j = (int)((n / (nx + 1)) % (ny + 1));
    const int k = DIM == 3 ? (int)(n / plane) : 0;
    // neighbour values (zero outside the grid), index (dx+1) + 3 (dy+1) + 9 (dz+1)
    double pv[DIM == 3 ? 27 : 9];
#pragma unroll
    for (int dz = (DIM == 3 ? -1 : 0); dz <= (DIM == 3 ? 1 : 0); ++dz)
#pragma unroll
      for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
        for (int dx = -1; dx <= 1; ++dx) {
          const bool in = i + dx >= 0 && i + dx <= nx && j + dy >= 0 && j + dy <= ny &&
                          (DIM == 2 || (k + dz >= 0 && k + dz <= nz));
          const long m = in ? n + dx + dy * row + dz * plane : n;
          const double v = p[m];
          pv[(dx + 1) + 3 * (dy + 1) + (DIM == 3 ? 9 * (dz + 1) : 0)] = in ? v : 0.0;
        }
    double y = 0.0;
#pragma unroll
    for (int sz = (DIM == 3 ? -1 : 0); sz <= 0; ++sz)
#pragma unroll
      for (int sy = -1; sy <= 0; ++sy)
#pragma unroll
        for (int sx = -1; sx <= 0; ++sx) {
          const int hi = i + sx, hj = j + sy, hk = k + sz;
          const bool ex = hi >= 0 && hi < nx && hj >= 0 && hj < ny && (DIM == 2 || (hk >= 0 && hk < nz));
          const int cn = (-sx) + 2 * (-sy) + 4 * (-sz);
          const bool sa = DIM == 3 || helm_sq_a(uniform, hj);
          double part = 0.0;
#pragma unroll
          for (int c2 = 0; c2 < (DIM == 3 ? 8 : 4); ++c2) {
            const int ox = sx + (c2 & 1), oy = sy + ((c2 >> 1) & 1), oz = sz + (c2 >> 2);
            const double a = sa ? hc.A[0][cn][c2] : hc.A[1][cn][c2];
            part += a * pv[(ox + 1) + 3 * (oy + 1) + (DIM == 3 ? 9 * (oz + 1) : 0)];
          }
          y += ex ? part : 0.0;
        }
    q[n] = y;
    acc[0] += pv[DIM == 3 ? 13 : 4] * y;
  }
  const double none[1] = {0.0};
  block_partials<1, 0>(acc, none, partials);
}

__global__ void helm_init_fin(const double* partials, long nb, double rtol, HelmState* st) {
  __shared__ double tot[2];
  reduce_partials<2, 0>(partials, nb, tot);
  if (threadIdx.x == 0) {
    st->rz = tot[0];
    st->bb = tot[1];
    st->rr = tot[1];
    st->tol2 = rtol * rtol * tot[1];
    st->iters = 0;
    st->breakdown = 0;
    st->done = !(tot[1] > 0.0);   // b = 0: x = 0 is the solution
  }
}

__global__ void helm_alpha_fin(const double* partials, long nb, HelmState* st) {
  if (st->done) return;
  __shared__ double tot[1];
  reduce_partials<1, 0>(partials, nb, tot);
  if (threadIdx.x == 0) {
    st->pq = tot[0];
    if (!(tot[0] > 0.0)) {
      st->breakdown = 1;
      st->done = 1;
      st->alpha = 0.0;
    } else {
      st->alpha = st->rz / tot[0];
    }
  }
}

// x += alpha p, r -= alpha q, partials (r, D^-1 r), (r, r)
__global__ __launch_bounds__(256) void helm_update_kernel(double* __restrict__ x,
                                                          double* __restrict__ r,
                                                          const double* __restrict__ p,
                                                          const double* __restrict__ q,
                                                          const double* __restrict__ invd, long nn,
                                                          double* partials, const HelmState* st) {
  if (st->done) return;
  const double alpha = st->alpha;
  double acc[2] = {0.0, 0.0};
  // distinct vectors (restrict): the next node's loads may pass this one's
  // stores
#pragma unroll 2
  for (long n = (long)blockIdx.x * blockDim.x + threadIdx.x; n < nn; n += (long)gridDim.x * blockDim.x) {
    x[n] += alpha * p[n];
    const double rv = r[n] - alpha * q[n];
    r[n] = rv;
    acc[0] += rv * invd[n] * rv;
    acc[1] += rv * rv;
  }
  const double none[1] = {0.0};
  block_partials<2, 0>(acc, none, partials);
}

__global__ void helm_beta_fin(const double* partials, long nb, int maxit, HelmState* st,
                              int* status) {
  if (st->done) return;
  __shared__ double tot[2];
  reduce_partials<2, 0>(partials, nb, tot);
  if (threadIdx.x == 0) {
    st->iters += 1;
    st->rz_old = st->rz;
    st->rz = tot[0];
    st->rr = tot[1];
    st->beta = tot[0] / st->rz_old;
    if (tot[1] <= st->tol2) {
      st->done = 1;
    } else if (st->iters >= maxit) {
      st->done = 1;
      if (*status == 0) *status = TOPO_S_NOT_CONVERGED;
    }
  }
}

// p = D^-1 r + beta p
__global__ __launch_bounds__(256) void helm_dir_kernel(double* p, const double* __restrict__ r,
                                                       const double* __restrict__ invd, long nn,
                                                       const HelmState* st) {
  if (st->done) return;
  const double beta = st->beta;
  for (long n = (long)blockIdx.x * blockDim.x + threadIdx.x; n < nn; n += (long)gridDim.x * blockDim.x)
    p[n] = invd[n] * r[n] + beta * p[n];
}

// s~_e = (mean of x over the vertices of e) / rho_e, one cube (square) per thread
template <int DIM>
__global__ __launch_bounds__(256) void helm_out_kernel(const double* __restrict__ x,
                                                       const double* __restrict__ rho,
                                                       double* out, int nx, int ny, int nz,
                                                       int uniform, HelmCoef hc, long ncube,
                                                       const HelmState* st, int* status) {
  const long h = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (h == 0 && st->breakdown) *status = TOPO_S_NUMERIC;
  if (h >= ncube) return;
  const int i = (int)(h % nx);
  const int j = (int)((h / nx) % ny);
  const int k = DIM == 3 ? (int)(h / ((long)nx * ny)) : 0;
  const long row = nx + 1, plane = row * (ny + 1);
  const long n0 = (long)k * plane + (long)j * row + i;
  constexpr int NC = DIM == 3 ? 8 : 4;
  double xc[NC];
#pragma unroll
  for (int cn = 0; cn < NC; ++cn) xc[cn] = x[n0 + (cn & 1) + ((cn >> 1) & 1) * row + (cn >> 2) * plane];
  const int s = (DIM == 3 || helm_sq_a(uniform, j)) ? 0 : 1;
  constexpr int NT = DIM == 3 ? 6 : 2;
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    double sum = 0.0;
#pragma unroll
    for (int cn = 0; cn < NC; ++cn)
      if ((hc.cells_of_corner[s][cn] >> t) & 1) sum += xc[cn];
    const long e = NT * h + t;
    out[e] = sum / (double)(DIM + 1) / rho[e];
  }
}

// ------------------------------------------------------------- launchers

void launch_helm_diag(Ctx* c) {
  const Grid& g = c->g;
  helm_diag_kernel<<<cdivu(g.nn, 256), 256, 0, c->stream>>>(
      c->hinvd, g.dim, g.nx, g.ny, g.nz, g.split == TOPO_SPLIT_UNIFORM, c->hcoef, g.nn);
}

void launch_filter_helmholtz(Ctx* c, const double* rho, const double* dc, double* dcf) {
  const Grid& g = c->g;
  const long nn = g.nn;
  const unsigned nb = red_grid(nn);
  const int uni = g.split == TOPO_SPLIT_UNIFORM;
  hipStream_t s = c->stream;
  HelmState* st = &c->scal->helm;
  int* status = &c->scal->status;
  double *x = c->hx, *r = c->hr, *p = c->hp, *q = c->hq;
  const double* invd = c->hinvd;
  const HelmCoef& hc = c->hcoef;
  if (g.dim == 3)
    helm_init_kernel<3><<<nb, 256, 0, s>>>(rho, dc, x, r, p, invd, g.nx, g.ny, g.nz, uni, hc, nn,
                                           c->partials);
  else
    helm_init_kernel<2><<<nb, 256, 0, s>>>(rho, dc, x, r, p, invd, g.nx, g.ny, 1, uni, hc, nn,
                                           c->partials);
  helm_init_fin<<<1, 256, 0, s>>>(c->partials, nb, kHelmRtol, st);
  // no-wait contexts queue a fixed budget of gated iterations
  const bool nowait = c->prob.sync_mode == TOPO_SYNC_NONE;
  const int maxit = nowait ? kHelmNoWaitIters : kHelmMaxit;
  const int batch = 8;
  bool stop = false;
  int b = 0;
  for (int it = 0; it < maxit && !stop; it += batch, ++b) {
    for (int k = 0; k < batch; ++k) {
      if (g.dim == 3)
        helm_apply_kernel<3><<<nb, 256, 0, s>>>(p, q, g.nx, g.ny, g.nz, uni, hc, nn, c->partials, st);
      else
        helm_apply_kernel<2><<<nb, 256, 0, s>>>(p, q, g.nx, g.ny, 1, uni, hc, nn, c->partials, st);
      helm_alpha_fin<<<1, 256, 0, s>>>(c->partials, nb, st);
      helm_update_kernel<<<nb, 256, 0, s>>>(x, r, p, q, invd, nn, c->partials, st);
      helm_beta_fin<<<1, 256, 0, s>>>(c->partials, nb, maxit, st, status);
      helm_dir_kernel<<<nb, 256, 0, s>>>(p, r, invd, nn, st);
    }
    if (nowait) continue;
    // poll the previous batch's flag while this batch runs
    const int sl = b & 1;
    (void)hipMemcpyAsync((void*)&c->pinned[14 + sl], &st->done, sizeof(int), hipMemcpyDeviceToHost, s);
    (void)hipEventRecord(c->ev_poll[sl], s);
    if (b > 0) {
      (void)hipEventSynchronize(c->ev_poll[sl ^ 1]);
      if (c->pinned[14 + (sl ^ 1)]) stop = true;
    }
  }
  const long ncube = (long)g.nx * g.ny * (g.dim == 3 ? g.nz : 1);
  if (g.dim == 3)
    helm_out_kernel<3><<<cdivu(ncube, 256), 256, 0, s>>>(x, rho, dcf, g.nx, g.ny, g.nz, uni, hc, ncube,
                                                        st, status);
  else
    helm_out_kernel<2><<<cdivu(ncube, 256), 256, 0, s>>>(x, rho, dcf, g.nx, g.ny, 1, uni, hc, ncube,
                                                        st, status);
}

}  // namespace topo
