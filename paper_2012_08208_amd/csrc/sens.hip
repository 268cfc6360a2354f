// Compliance and its sensitivity (Sec. 3.2: sensitivity of f; multiple load
// cases summed as in Sec. 5.3).
//   c      = sum_r f_r^T u_r
//   dc_e   = -p rho_e^(p-1) (E0 - Emin) sum_r u_{r,e}^T K0_e u_{r,e}
// with u_e^T K0_e u_e = |T| (lambda tr(eps)^2 + 2 mu eps:eps) at unit modulus.
// The listing's per-cell value (paper mode) is -p rho^(p-1) psi_e, i.e. the
// same expression divided by 2|T| with E = rho^p.
// The kernel also reduces sum_e E_e w_e (= c, an energy cross-check) and the
// listing's objective sum_e E_e w_e / (2|T|).
#include "common.h"
#include "element.h"
#include "shared_dev.h"
#include "topo_internal.h"

namespace topo {

__global__ __launch_bounds__(256) void sens2d_kernel(const double* __restrict__ rho,
                                                     const double* __restrict__ u, double* dc,
                                                     int nx, int ny, long nn, int nr,
                                                     int split_uniform, double lam0, double mu0,
                                                     double vol, double E0, double Emin,
                                                     double penal, int paper, double* partials) {
  const long nsq = (long)nx * ny;
  double acc[2] = {0.0, 0.0};
  for (long s = (long)blockIdx.x * blockDim.x + threadIdx.x; s < nsq; s += (long)gridDim.x * blockDim.x)
    sens2d_square(s, rho, u, dc, nx, nn, nr, split_uniform, lam0, mu0, vol, E0, Emin, penal, paper,
                  acc);
  const double none[1] = {0.0};
  block_partials<2, 0>(acc, none, partials);
}

__global__ __launch_bounds__(256) void sens3d_kernel(const double* __restrict__ rho,
                                                     const double* __restrict__ u, double* dc,
                                                     int nx, int ny, int nz, long nn, int nr,
                                                     double lam0, double mu0, double vol,
                                                     double E0, double Emin, double penal,
                                                     int paper, double* partials) {
  const long nh = (long)nx * ny * nz;
  double acc[2] = {0.0, 0.0};
  for (long h = (long)blockIdx.x * blockDim.x + threadIdx.x; h < nh; h += (long)gridDim.x * blockDim.x) {
    const int i = (int)(h % nx);
    const int j = (int)((h / nx) % ny);
    const int k = (int)(h / ((long)nx * ny));
    double w[6] = {0, 0, 0, 0, 0, 0};
    for (int r = 0; r < nr; ++r) {
      double uc[8][3];
#pragma unroll
      for (int c = 0; c < 8; ++c) {
        const long n = ((long)(k + (c >> 2)) * (ny + 1) + j + ((c >> 1) & 1)) * (nx + 1) + i + (c & 1);
#pragma unroll
        for (int a = 0; a < 3; ++a) uc[c][a] = u[((long)r * 3 + a) * nn + n];
      }
      double wt[6];
      cube_energy<double>(uc, lam0, mu0, wt);
#pragma unroll
      for (int t = 0; t < 6; ++t) w[t] += wt[t];
    }
#pragma unroll
    for (int t = 0; t < 6; ++t) {
      const long e = 6 * h + t;
      const double ws = w[t] * vol;
      const double rv = rho[e];
      const double rp1 = (penal == 3.0) ? rv * rv : pow(rv, penal - 1.0);
      const double Ee = paper ? rp1 * rv : Emin + rp1 * rv * (E0 - Emin);
      dc[e] = paper ? -penal * rp1 * ws / (2.0 * vol) : -penal * rp1 * (E0 - Emin) * ws;
      acc[0] += Ee * ws;
      acc[1] += Ee * ws / (2.0 * vol);
    }
  }
  const double none[1] = {0.0};
  block_partials<2, 0>(acc, none, partials);
}

__global__ void sens_fin(const double* partials, long nb, DevScalars* sc) {
  __shared__ double tot[2];
  reduce_partials<2, 0>(partials, nb, tot);
  if (threadIdx.x == 0) {
    sc->c_energy = tot[0];
    sc->c_paper = tot[1];
  }
}

__global__ __launch_bounds__(256) void dot_kernel(const double* __restrict__ a,
                                                  const double* __restrict__ b, long n,
                                                  double* partials) {
  double acc[1] = {0.0};
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    acc[0] += a[i] * b[i];
  const double none[1] = {0.0};
  block_partials<1, 0>(acc, none, partials);
}

__global__ void dot_fin(const double* partials, long nb, double* out1, double* out2) {
  __shared__ double tot[1];
  reduce_partials<1, 0>(partials, nb, tot);
  if (threadIdx.x == 0) {
    if (out1) *out1 = tot[0];
    if (out2) *out2 = tot[0];
  }
}

void launch_sensitivity(Ctx* c, const double* rho, const double* u, double* dc,
                        double* compliance) {
  const Grid& g = c->g;
  const Material& m = c->m;
  const long ncells = g.dim == 2 ? (long)g.nx * g.ny : (long)g.nx * g.ny * g.nz;
  const unsigned nb = red_grid(ncells);
  const int nr = c->prob.nrhs;
  if (g.dim == 2)
    sens2d_kernel<<<nb, 256, 0, c->stream>>>(rho, u, dc, g.nx, g.ny, g.nn, nr,
                                            g.split == TOPO_SPLIT_UNIFORM, m.lam0, m.mu0, m.vol,
                                            m.E0, m.Emin, m.penal, m.paper, c->partials);
  else
    sens3d_kernel<<<nb, 256, 0, c->stream>>>(rho, u, dc, g.nx, g.ny, g.nz, g.nn, nr, m.lam0,
                                            m.mu0, m.vol, m.E0, m.Emin, m.penal, m.paper,
                                            c->partials);
  sens_fin<<<1, 256, 0, c->stream>>>(c->partials, nb, c->scal);
  const long n = (long)nr * g.nd;
  const unsigned nb2 = red_grid(n);
  dot_kernel<<<nb2, 256, 0, c->stream>>>(c->f, u, n, c->partials);
  dot_fin<<<1, 256, 0, c->stream>>>(c->partials, nb2, compliance, &c->scal->compliance);
}

}  // namespace topo
