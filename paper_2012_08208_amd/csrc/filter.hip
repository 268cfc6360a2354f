// Distance-weighted sensitivity filter in stencil form (Sec. 3.2.2, eq. filter
// and eq. filter_cond; Sec. 4.4, eq. filter_mat):
//   dcf_a = sum_b W_ab rho_b dc_b / (rho_a R_a),
//   W_ab  = max(0, rmin - |x_a - x_b|),   R_a = sum_b W_ab.
// On the structured grid W_ab depends only on the two cell classes and the
// integer offset between their squares/cubes, so the dense matrix the paper
// builds from a Euclidean distance matrix becomes a per-class tap table
// (offset, neighbour class, weight), built once on the host at context
// creation with the same midpoint distances.  Cells near the boundary keep
// only the taps that land inside the grid, so their R_a is smaller.
//
// The kernel runs one block row per cell class t, so all lanes of a wave
// walk the same tap list (uniform table reads); the filter input rho*dc is
// first gathered into class-major order so neighbour reads are coalesced.
#include <math.h>

#include "common.h"
#include "shared_dev.h"
#include "topo_internal.h"

namespace topo {

// Host tap table of every cell class: (offset, neighbour class, weight),
// kMaxFilterTaps entries per class; returns the number of classes.
int filter_taps_host(int dim, int split, double rmin, std::vector<FilterTap>& tab, int* ntaps) {
  const int reach = (int)ceil(rmin) + 1;
  int nclasses = 0;
  tab.clear();
  if (dim == 3) {
    static const int perm[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
    double cen[6][3];
    for (int t = 0; t < 6; ++t) {
      cen[t][perm[t][0]] = 0.75;
      cen[t][perm[t][1]] = 0.5;
      cen[t][perm[t][2]] = 0.25;
    }
    nclasses = 6;
    for (int ta = 0; ta < 6; ++ta) {
      int n = 0;
      for (int dk = -reach; dk <= reach; ++dk)
        for (int dj = -reach; dj <= reach; ++dj)
          for (int di = -reach; di <= reach; ++di)
            for (int tb = 0; tb < 6; ++tb) {
              const double dx = di + cen[tb][0] - cen[ta][0];
              const double dy = dj + cen[tb][1] - cen[ta][1];
              const double dz = dk + cen[tb][2] - cen[ta][2];
              const double w = rmin - sqrt(dx * dx + dy * dy + dz * dz);
              if (w > 0.0 && n < kMaxFilterTaps) {
                tab.push_back({di, dj, dk, tb, w});
                ++n;
              }
            }
      ntaps[ta] = n;
      tab.resize((size_t)(ta + 1) * kMaxFilterTaps);
    }
  } else {
    // centroids (relative to the square corner) of the two triangles of
    // diagonal A and diagonal B
    const double cA[2][2] = {{2.0 / 3.0, 1.0 / 3.0}, {1.0 / 3.0, 2.0 / 3.0}};
    const double cB[2][2] = {{1.0 / 3.0, 1.0 / 3.0}, {2.0 / 3.0, 2.0 / 3.0}};
    const bool alt = split == TOPO_SPLIT_ALT_ROWS;
    nclasses = alt ? 4 : 2;
    for (int cls = 0; cls < nclasses; ++cls) {
      const int ta = cls & 1, par = cls >> 1;  // row parity of the target
      const double* ca = (alt && par) ? cB[ta] : cA[ta];
      int n = 0;
      for (int dj = -reach; dj <= reach; ++dj)
        for (int di = -reach; di <= reach; ++di)
          for (int tb = 0; tb < 2; ++tb) {
            const int pb = (par + (dj & 1)) & 1;
            const double* cb = (alt && pb) ? cB[tb] : cA[tb];
            const double dx = di + cb[0] - ca[0];
            const double dy = dj + cb[1] - ca[1];
            const double w = rmin - sqrt(dx * dx + dy * dy);
            if (w > 0.0 && n < kMaxFilterTaps) {
              tab.push_back({di, dj, 0, tb, w});
              ++n;
            }
          }
      ntaps[cls] = n;
      tab.resize((size_t)(cls + 1) * kMaxFilterTaps);
    }
  }
  return nclasses;
}

void build_filter_taps(Ctx* c) {
  std::vector<FilterTap> tab;
  c->nclasses = filter_taps_host(c->g.dim, c->g.split, c->prob.rmin, tab, c->ntaps);
  (void)hipMemcpy(c->taps, tab.data(), tab.size() * sizeof(FilterTap), hipMemcpyHostToDevice);
  (void)hipMemcpy(c->taps + (size_t)8 * kMaxFilterTaps, c->ntaps, sizeof(c->ntaps),
                  hipMemcpyHostToDevice);
}

// q[t][h] = rho[e] * dc[e] (class-major); with rho == nullptr, q = 1.
__global__ void filter_gather_kernel(double* q, const double* rho, const double* dc, long ncell,
                                     int ncls, long nblk) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= ncell) return;
  const long h = e / ncls;
  const int t = (int)(e % ncls);
  q[(long)t * nblk + h] = rho ? rho[e] * dc[e] : 1.0;
}

// one thread per (block-cell h, class t = blockIdx.y)
__global__ __launch_bounds__(256) void filter_kernel(double* out, const double* __restrict__ q,
                                                     const double* __restrict__ rho,
                                                     const double* __restrict__ R,
                                                     const FilterTap* __restrict__ taps,
                                                     const int* __restrict__ ntaps, int dim, int nx,
                                                     int ny, int nz, int ncls, int alt, int rowsum) {
  const long nblk = (long)nx * ny * nz;
  const long h = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (h >= nblk) return;
  filter_cell(h, blockIdx.y, out, q, rho, R, taps, ntaps, dim, nx, ny, nz, ncls, alt, rowsum);
}

static void filter_launch(Ctx* c, const double* rho, const double* dc, double* out, bool rowsum) {
  const Grid& g = c->g;
  const int ncls = g.dim == 2 ? 2 : 6;
  const int nz = g.dim == 2 ? 1 : g.nz;
  const long nblk = (long)g.nx * g.ny * nz;
  const long ncell = nblk * ncls;
  filter_gather_kernel<<<(unsigned)((ncell + 255) / 256), 256, 0, c->stream>>>(
      c->qsoa, rowsum ? nullptr : rho, dc, ncell, ncls, nblk);
  dim3 grid((unsigned)((nblk + 255) / 256), ncls);
  filter_kernel<<<grid, 256, 0, c->stream>>>(out, c->qsoa, rho, c->R, c->taps,
                                             (const int*)(c->taps + (size_t)8 * kMaxFilterTaps),
                                             g.dim, g.nx, g.ny, nz, ncls,
                                             g.split == TOPO_SPLIT_ALT_ROWS, rowsum ? 1 : 0);
}

void launch_filter_rowsums(Ctx* c) { filter_launch(c, nullptr, nullptr, c->R, true); }

void launch_filter(Ctx* c, const double* rho, const double* dc, double* dcf) {
  filter_launch(c, rho, dc, dcf, false);
}

}  // namespace topo
