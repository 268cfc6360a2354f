// Distance-weighted sensitivity filter in stencil form (Sec. 3.2.2, eq. filter
// and eq. filter_cond; Sec. 4.5, eq. filter_mat):
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
#include <stdlib.h>

#include <algorithm>

#include "common.h"
#include "shared_dev.h"
#include "topo_internal.h"

namespace topo {

// Host tap table of every cell class: (offset, neighbour class, weight).
// Every tap with a positive weight is kept; the classes' lists are laid out
// *stride entries apart, where *stride is the longest list rounded up to a
// multiple of 16 (at least 16).  Returns the number of classes.
int filter_taps_host(int dim, int split, double rmin, std::vector<FilterTap>& tab, int* ntaps,
                     int* stride) {
  const int reach = (int)ceil(rmin) + 1;
  std::vector<std::vector<FilterTap>> lists;
  if (dim == 3) {
    static const int perm[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
    double cen[6][3];
    for (int t = 0; t < 6; ++t) {
      cen[t][perm[t][0]] = 0.75;
      cen[t][perm[t][1]] = 0.5;
      cen[t][perm[t][2]] = 0.25;
    }
    lists.resize(6);
    for (int ta = 0; ta < 6; ++ta)
      for (int dk = -reach; dk <= reach; ++dk)
        for (int dj = -reach; dj <= reach; ++dj)
          for (int di = -reach; di <= reach; ++di)
            for (int tb = 0; tb < 6; ++tb) {
              const double dx = di + cen[tb][0] - cen[ta][0];
              const double dy = dj + cen[tb][1] - cen[ta][1];
              const double dz = dk + cen[tb][2] - cen[ta][2];
              const double w = rmin - sqrt(dx * dx + dy * dy + dz * dz);
              if (w > 0.0) lists[ta].push_back({di, dj, dk, tb, w});
            }
  } else {
    // centroids (relative to the square corner) of the two triangles of
    // diagonal A and diagonal B
    const double cA[2][2] = {{2.0 / 3.0, 1.0 / 3.0}, {1.0 / 3.0, 2.0 / 3.0}};
    const double cB[2][2] = {{1.0 / 3.0, 1.0 / 3.0}, {2.0 / 3.0, 2.0 / 3.0}};
    const bool alt = split == TOPO_SPLIT_ALT_ROWS;
    lists.resize(alt ? 4 : 2);
    for (int cls = 0; cls < (int)lists.size(); ++cls) {
      const int ta = cls & 1, par = cls >> 1;  // row parity of the target
      const double* ca = (alt && par) ? cB[ta] : cA[ta];
      for (int dj = -reach; dj <= reach; ++dj)
        for (int di = -reach; di <= reach; ++di)
          for (int tb = 0; tb < 2; ++tb) {
            const int pb = (par + (dj & 1)) & 1;
            const double* cb = (alt && pb) ? cB[tb] : cA[tb];
            const double dx = di + cb[0] - ca[0];
            const double dy = dj + cb[1] - ca[1];
            const double w = rmin - sqrt(dx * dx + dy * dy);
            if (w > 0.0) lists[cls].push_back({di, dj, 0, tb, w});
          }
    }
  }
  size_t longest = 0;
  for (const auto& l : lists) longest = std::max(longest, l.size());
  const int st = (int)std::max<size_t>(16, (longest + 15) / 16 * 16);
  tab.assign((size_t)lists.size() * st, FilterTap{0, 0, 0, 0, 0.0});
  for (size_t cls = 0; cls < lists.size(); ++cls) {
    ntaps[cls] = (int)lists[cls].size();
    std::copy(lists[cls].begin(), lists[cls].end(), tab.begin() + cls * st);
  }
  if (stride) *stride = st;
  return (int)lists.size();
}

int filter_tap_stride(int dim, int split, double rmin) {
  std::vector<FilterTap> tab;
  int nt[8], st = 0;
  filter_taps_host(dim, split, rmin, tab, nt, &st);
  return st;
}

// The 3D filter on LDS boxes: a block owns kFtX x kFtY x kFtZ cubes (all six
// cell classes) and stages rho*dc of those cubes and a kFtH-cube halo,
// zero outside the grid; each cell then sums its taps from LDS.  A tap is a
// precomputed box offset and a weight, read uniformly by the wave (the
// wave's cells share a class).  Taps landing outside the grid read a staged
// zero, so the sums are those of the checked loop, term by term.
constexpr int kFtX = 8, kFtY = 4, kFtZ = 4, kFtH = 2;
constexpr int kFtIX = kFtX + 2 * kFtH, kFtIY = kFtY + 2 * kFtH, kFtIZ = kFtZ + 2 * kFtH;
constexpr int kFtV = kFtIX * kFtIY * kFtIZ;

void build_filter_taps(Ctx* c) {
  std::vector<FilterTap> tab;
  int st = 0;
  c->nclasses = filter_taps_host(c->g.dim, c->g.split, c->prob.rmin, tab, c->ntaps, &st);
  // the workspace was sized for exactly this stride (filter_tap_stride)
  c->tap_stride = st;
  (void)hipMemcpy(c->taps, tab.data(), tab.size() * sizeof(FilterTap), hipMemcpyHostToDevice);
  (void)hipMemcpy(c->taps + (size_t)8 * st, c->ntaps, sizeof(c->ntaps), hipMemcpyHostToDevice);
  c->filter_tiled = false;
  if (c->g.dim == 3 && c->ttaps) {
    int reach = 0;
    for (int t = 0; t < 6; ++t)
      for (int s = 0; s < c->ntaps[t]; ++s) {
        const FilterTap& f = tab[(size_t)t * st + s];
        reach = std::max(reach, std::max(std::abs(f.di), std::max(std::abs(f.dj), std::abs(f.dk))));
      }
    if (reach <= kFtH) {
      std::vector<TiledTap> tt((size_t)6 * st, TiledTap{0, 0, 0.0});
      for (int t = 0; t < 6; ++t)
        for (int s = 0; s < c->ntaps[t]; ++s) {
          const FilterTap& f = tab[(size_t)t * st + s];
          tt[(size_t)t * st + s] =
              TiledTap{((f.dk * kFtIY + f.dj) * kFtIX + f.di) * 6 + f.tb, 0, f.w};
        }
      (void)hipMemcpy(c->ttaps, tt.data(), tt.size() * sizeof(TiledTap), hipMemcpyHostToDevice);
      c->filter_tiled = true;
    }
  }
}

// Filter modes (what is summed over the taps, and the divisor):
//   FM_SENS      q = rho dc, out = sum / (rho_e R_e)   sensitivity filter
//   FM_ROWSUM    q = 1,      out = sum                  row sums R
//   FM_DENSITY   q = dc,     out = sum / R_e            density filter x~ = W x / R
//   FM_TRANSPOSE q = dc / R (1 / R when dc is null), out = sum
//                                                      its adjoint W (g / R) (W is symmetric)
enum FilterMode { FM_SENS = 0, FM_ROWSUM = 1, FM_DENSITY = 2, FM_TRANSPOSE = 3 };

__device__ __forceinline__ double filter_input(int mode, long e, const double* rho, const double* dc,
                                               const double* R) {
  if (mode == FM_SENS) return rho[e] * dc[e];
  if (mode == FM_ROWSUM) return 1.0;
  if (mode == FM_DENSITY) return dc[e];
  return (dc ? dc[e] : 1.0) / R[e];
}

// out[e] = sum_taps w q, divided as the mode says
__global__ __launch_bounds__(256) void filter3d_tiled_kernel(double* out, const double* __restrict__ rho,
                                                             const double* __restrict__ dc,
                                                             const double* __restrict__ R,
                                                             const TiledTap* __restrict__ tt,
                                                             const int* __restrict__ ntaps,
                                                             int stride, int nx, int ny, int nz,
                                                             int mode) {
  __shared__ double q[kFtV * 6];
  const int tid = threadIdx.x;
  const int gx = (nx + kFtX - 1) / kFtX, gy = (ny + kFtY - 1) / kFtY;
  const int b = blockIdx.x;
  const int X0 = (b % gx) * kFtX, Y0 = ((b / gx) % gy) * kFtY, Z0 = (b / (gx * gy)) * kFtZ;
  for (int idx = tid; idx < kFtV * 6; idx += 256) {
    const int v = idx / 6, t = idx - v * 6;
    const int gi = X0 - kFtH + v % kFtIX, gj = Y0 - kFtH + (v / kFtIX) % kFtIY,
              gk = Z0 - kFtH + v / (kFtIX * kFtIY);
    double val = 0.0;
    if (gi >= 0 && gi < nx && gj >= 0 && gj < ny && gk >= 0 && gk < nz) {
      const long e = (((long)gk * ny + gj) * nx + gi) * 6 + t;
      val = filter_input(mode, e, rho, dc, R);
    }
    q[idx] = val;
  }
  __syncthreads();
  const int cbx = tid & (kFtX * kFtY * kFtZ - 1);   // 128 cubes
  const int half = __builtin_amdgcn_readfirstlane(tid >> 7);
  const int x = cbx % kFtX, y = (cbx / kFtX) % kFtY, z = cbx / (kFtX * kFtY);
  const int base = (((z + kFtH) * kFtIY + (y + kFtH)) * kFtIX + (x + kFtH)) * 6;
  const int gi = X0 + x, gj = Y0 + y, gk = Z0 + z;
  const bool in = gi < nx && gj < ny && gk < nz;
  const long h = ((long)gk * ny + gj) * nx + gi;
#pragma unroll 1
  for (int r = 0; r < 3; ++r) {
    const int t = half + 2 * r;   // uniform over the wave
    const TiledTap* tp = tt + (long)t * stride;
    const int nt = ntaps[t];
    double acc = 0.0;
    for (int s = 0; s < nt; ++s) acc += tp[s].w * q[base + tp[s].off];
    if (in) {
      const long e = h * 6 + t;
      out[e] = mode == FM_SENS ? acc / (rho[e] * R[e]) : mode == FM_DENSITY ? acc / R[e] : acc;
    }
  }
}

// q[t][h] = the mode's filter input of cell e (class-major)
__global__ void filter_gather_kernel(double* q, const double* rho, const double* dc,
                                     const double* R, int mode, long ncell, int ncls, long nblk) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= ncell) return;
  const long h = e / ncls;
  const int t = (int)(e % ncls);
  q[(long)t * nblk + h] = filter_input(mode, e, rho, dc, R);
}

// one thread per (block-cell h, class t = blockIdx.y)
__global__ __launch_bounds__(256) void filter_kernel(double* out, const double* __restrict__ q,
                                                     const double* __restrict__ rho,
                                                     const double* __restrict__ R,
                                                     const FilterTap* __restrict__ taps,
                                                     const int* __restrict__ ntaps, int stride,
                                                     int dim, int nx, int ny, int nz, int ncls,
                                                     int alt, int out_mode) {
  const long nblk = (long)nx * ny * nz;
  const long h = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (h >= nblk) return;
  filter_cell(h, blockIdx.y, out, q, rho, R, taps, ntaps, stride, dim, nx, ny, nz, ncls, alt,
              out_mode);
}

static void filter_launch(Ctx* c, const double* rho, const double* dc, double* out, int mode) {
  const Grid& g = c->g;
  if (g.dim == 3 && c->filter_tiled) {
    const long tiles = (long)((g.nx + kFtX - 1) / kFtX) * ((g.ny + kFtY - 1) / kFtY) *
                       ((g.nz + kFtZ - 1) / kFtZ);
    filter3d_tiled_kernel<<<(unsigned)tiles, 256, 0, c->stream>>>(
        out, rho, dc, c->R, c->ttaps, (const int*)(c->taps + (size_t)8 * c->tap_stride),
        c->tap_stride, g.nx, g.ny, g.nz, mode);
    return;
  }
  const int ncls = g.dim == 2 ? 2 : 6;
  const int nz = g.dim == 2 ? 1 : g.nz;
  const long nblk = (long)g.nx * g.ny * nz;
  const long ncell = nblk * ncls;
  filter_gather_kernel<<<(unsigned)((ncell + 255) / 256), 256, 0, c->stream>>>(
      c->qsoa, rho, dc, c->R, mode, ncell, ncls, nblk);
  dim3 grid((unsigned)((nblk + 255) / 256), ncls);
  filter_kernel<<<grid, 256, 0, c->stream>>>(out, c->qsoa, rho, c->R, c->taps,
                                             (const int*)(c->taps + (size_t)8 * c->tap_stride),
                                             c->tap_stride, g.dim, g.nx, g.ny, nz, ncls,
                                             g.split == TOPO_SPLIT_ALT_ROWS,
                                             mode == FM_SENS ? 0 : mode == FM_DENSITY ? 2 : 1);
}

void launch_filter_rowsums(Ctx* c) { filter_launch(c, nullptr, nullptr, c->R, FM_ROWSUM); }

void launch_density_filter(Ctx* c, const double* x, double* out) {
  filter_launch(c, nullptr, x, out, FM_DENSITY);
}

// volume sensitivity of the density filter: dv = W (1 / R)
void launch_density_volume_weights(Ctx* c, double* dv) {
  filter_launch(c, nullptr, nullptr, dv, FM_TRANSPOSE);
}

void launch_filter(Ctx* c, const double* rho, const double* dc, double* dcf) {
  if (c->prob.filter == TOPO_FILTER_HELMHOLTZ) {
    launch_filter_helmholtz(c, rho, dc, dcf);
    return;
  }
  if (c->prob.filter == TOPO_FILTER_DENSITY) {
    // chain rule through x~ = W x / R: dc/dx = W (dc/dx~ / R)
    filter_launch(c, nullptr, dc, dcf, FM_TRANSPOSE);
    return;
  }
  filter_launch(c, rho, dc, dcf, FM_SENS);
}

}  // namespace topo
