// Matrix-free P1 operator apply y = Z K(rho) Z x on structured grids
// (Sec. 3.1, eq. fe_form, with the SIMP modulus of Sec. 2, eq. simp).
//
// Work decomposition (owner computes, no atomics, deterministic):
// a 256-thread block owns a 15 x 15 column of nodes in the x-y plane and
// computes the 16 x 16 cells (squares / cubes) that touch it, one cell per
// thread.  Node values of the 17 x 17 node patch are staged in LDS.  Cell
// forces are combined into nodes in two steps: along x with a cross-lane
// shift inside each 16-lane row, along y through a small LDS exchange.
// In 3D the block sweeps a chunk of z-planes; the cube layer below a node
// plane hands its top-corner forces to the layer above in registers.
// Only owned nodes are written, so every y entry is stored exactly once.
#include "common.h"
#include "element.h"
#include "topo_internal.h"

namespace topo {

constexpr int TILE = 15;       // owned nodes per tile edge
constexpr int PATCH = 17;      // staged node patch edge
constexpr int PATCH2 = PATCH * PATCH;

template <typename T>
__device__ __forceinline__ T shift_down1(T v) {
  return __shfl_down(v, 1, 16);
}

// -------------------------------------------------------------- 2D apply
template <typename T, typename TE, int NR>
__global__ __launch_bounds__(256) void apply2d_kernel(const T* __restrict__ x, T* __restrict__ y,
                                                      const TE* __restrict__ E,
                                                      const uint8_t* __restrict__ mask, int nx,
                                                      int ny, long nn, int split_uniform, T lam0,
                                                      T mu0, double* partials, unsigned* counter,
                                                      PcgState* st) {
  __shared__ T xs[NR][2][PATCH2];
  __shared__ T ex[2][256];
  const int tid = threadIdx.x;
  const int tx = tid & 15, ty = tid >> 4;
  const int i0 = blockIdx.x * TILE, j0 = blockIdx.y * TILE;
  if (st && st->done) return;
  for (int idx = tid; idx < PATCH2; idx += 256) {
    const int a = idx % PATCH, b = idx / PATCH;
    const int gi = i0 - 1 + a, gj = j0 - 1 + b;
    const bool ok = gi >= 0 && gi <= nx && gj >= 0 && gj <= ny;
    const long n = (long)gj * (nx + 1) + gi;
    const int m = ok ? mask[n] : 3;
#pragma unroll
    for (int r = 0; r < NR; ++r)
#pragma unroll
      for (int c = 0; c < 2; ++c)
        xs[r][c][idx] = ((m >> c) & 1) ? T(0) : x[((long)r * 2 + c) * nn + n];
  }
  __syncthreads();
  const int hi = i0 - 1 + tx, hj = j0 - 1 + ty;
  const bool cell_ok = hi >= 0 && hi < nx && hj >= 0 && hj < ny;
  T l0 = 0, m0 = 0, l1 = 0, m1 = 0;
  if (cell_ok) {
    const long e = 2 * ((long)hj * nx + hi);
    const T e0 = T(E[e]), e1 = T(E[e + 1]);
    l0 = lam0 * e0; m0 = mu0 * e0; l1 = lam0 * e1; m1 = mu0 * e1;
  }
  const bool diag_a = split_uniform || ((hj & 1) == 0);
  const int oi = i0 + tx, oj = j0 + ty;
  const bool owner = tx < TILE && ty < TILE && oi <= nx && oj <= ny;
  const long on = (long)oj * (nx + 1) + oi;
  const int om = owner ? mask[on] : 3;
  double dot[NR];
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    T u[4][2], f[4][2];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int li = (ty + (c >> 1)) * PATCH + tx + (c & 1);
      u[c][0] = xs[r][0][li];
      u[c][1] = xs[r][1][li];
      f[c][0] = 0; f[c][1] = 0;
    }
    square_force<T>(diag_a, u, l0, m0, l1, m1, f);
    T X[2][2];
#pragma unroll
    for (int cy = 0; cy < 2; ++cy)
#pragma unroll
      for (int c = 0; c < 2; ++c) X[cy][c] = f[1 + 2 * cy][c] + shift_down1(f[2 * cy][c]);
    if (r > 0) __syncthreads();
    ex[0][tid] = X[0][0];
    ex[1][tid] = X[0][1];
    __syncthreads();
    dot[r] = 0.0;
    if (owner) {
      const int lc = (ty + 1) * PATCH + tx + 1;
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        T v = X[1][c] + ex[c][tid + 16];
        if ((om >> c) & 1) v = 0;
        y[((long)r * 2 + c) * nn + on] = v;
        dot[r] += (double)v * (double)xs[r][c][lc];
      }
    }
  }
  if (partials) {
    double dummy[1] = {0.0};
    __shared__ double tot[NR];
    if (grid_reduce<NR, 0>(dot, dummy, partials, counter, tot)) {
      if (tid == 0) {
        for (int r = 0; r < NR; ++r) {
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
  }
}

// -------------------------------------------------------------- 3D apply
template <typename T, typename TE, int NR>
__global__ __launch_bounds__(256) void apply3d_kernel(const T* __restrict__ x, T* __restrict__ y,
                                                      const TE* __restrict__ E,
                                                      const uint8_t* __restrict__ mask, int nx,
                                                      int ny, int nz, long nn, int kz, T lam0,
                                                      T mu0, double* partials, unsigned* counter,
                                                      PcgState* st) {
  __shared__ T xs[2][NR][3][PATCH2];
  __shared__ T ex[6][256];
  const int tid = threadIdx.x;
  const int tx = tid & 15, ty = tid >> 4;
  const int i0 = blockIdx.x * TILE, j0 = blockIdx.y * TILE;
  if (st && st->done) return;
  const int k0 = blockIdx.z * kz;
  const int k1 = min(k0 + kz, nz + 1);
  const long plane = (long)(nx + 1) * (ny + 1);

  auto load_plane = [&](int kk) {
    const int s = kk & 1;
    for (int idx = tid; idx < PATCH2; idx += 256) {
      const int a = idx % PATCH, b = idx / PATCH;
      const int gi = i0 - 1 + a, gj = j0 - 1 + b;
      const bool ok = gi >= 0 && gi <= nx && gj >= 0 && gj <= ny && kk >= 0 && kk <= nz;
      const long n = (long)kk * plane + (long)gj * (nx + 1) + gi;
      const int m = ok ? mask[n] : 7;
#pragma unroll
      for (int r = 0; r < NR; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c)
          xs[s][r][c][idx] = ((m >> c) & 1) ? T(0) : x[((long)r * 3 + c) * nn + n];
    }
  };

  const int hi = i0 - 1 + tx, hj = j0 - 1 + ty;
  const bool col_ok = hi >= 0 && hi < nx && hj >= 0 && hj < ny;
  const int oi = i0 + tx, oj = j0 + ty;
  const bool owner = tx < TILE && ty < TILE && oi <= nx && oj <= ny;
  T carry[NR][3];
#pragma unroll
  for (int r = 0; r < NR; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c) carry[r][c] = 0;
  double dot[NR];
#pragma unroll
  for (int r = 0; r < NR; ++r) dot[r] = 0.0;

  load_plane(k0 - 1);
  for (int kh = k0 - 1; kh < k1; ++kh) {
    // the slot being refilled held plane kh - 1, read until the end of the
    // previous step
    if (kh > k0 - 1) __syncthreads();
    load_plane(kh + 1);
    __syncthreads();
    const bool cell_ok = col_ok && kh >= 0 && kh < nz;
    T lam[6], mu[6];
    if (cell_ok) {
      const long h = ((long)kh * ny + hj) * nx + hi;
#pragma unroll
      for (int t = 0; t < 6; ++t) {
        const T e = T(E[6 * h + t]);
        lam[t] = lam0 * e;
        mu[t] = mu0 * e;
      }
    } else {
#pragma unroll
      for (int t = 0; t < 6; ++t) { lam[t] = 0; mu[t] = 0; }
    }
    const int sb = kh & 1, st_ = (kh + 1) & 1;
    const bool store = owner && kh >= k0 && kh <= nz;
    const long on = (long)kh * plane + (long)oj * (nx + 1) + oi;
    const int om = store ? mask[on] : 7;
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      T u[8][3], f[8][3];
#pragma unroll
      for (int c = 0; c < 8; ++c) {
        const int li = (ty + ((c >> 1) & 1)) * PATCH + tx + (c & 1);
        const int s = (c >> 2) ? st_ : sb;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          u[c][a] = xs[s][r][a][li];
          f[c][a] = 0;
        }
      }
      cube_force<T>(u, lam, mu, f);
      T X[2][2][3];
#pragma unroll
      for (int cy = 0; cy < 2; ++cy)
#pragma unroll
        for (int cz = 0; cz < 2; ++cz)
#pragma unroll
          for (int a = 0; a < 3; ++a)
            X[cy][cz][a] = f[1 + 2 * cy + 4 * cz][a] + shift_down1(f[2 * cy + 4 * cz][a]);
      __syncthreads();
#pragma unroll
      for (int cz = 0; cz < 2; ++cz)
#pragma unroll
        for (int a = 0; a < 3; ++a) ex[cz * 3 + a][tid] = X[0][cz][a];
      __syncthreads();
      if (owner) {
        const int lc = (ty + 1) * PATCH + tx + 1;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          T yb = carry[r][a] + X[1][0][a] + ex[a][tid + 16];
          carry[r][a] = X[1][1][a] + ex[3 + a][tid + 16];
          if (store) {
            if ((om >> a) & 1) yb = 0;
            y[((long)r * 3 + a) * nn + on] = yb;
            dot[r] += (double)yb * (double)xs[sb][r][a][lc];
          }
        }
      }
    }
  }
  if (partials) {
    double dummy[1] = {0.0};
    __shared__ double tot[NR];
    if (grid_reduce<NR, 0>(dot, dummy, partials, counter, tot)) {
      if (tid == 0) {
        for (int r = 0; r < NR; ++r) {
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
  }
}

// ------------------------------------------------------------- diagonal
// diag K at node a, component c: sum over cells of
// |T| E (lambda g_c^2 + mu (g_c^2 + |g|^2)) with g = grad N_a.
__device__ __forceinline__ void diag_add(double (&d)[3], int dim, const int* g, double lam,
                                         double mu) {
  double gg = 0.0;
  for (int a = 0; a < dim; ++a) gg += g[a] * g[a];
  for (int c = 0; c < dim; ++c) d[c] += lam * g[c] * g[c] + mu * (g[c] * g[c] + gg);
}

__global__ void diag2d_kernel(double* d, const double* E, const uint8_t* mask, int nx, int ny,
                              long nn, int split_uniform, double lam0, double mu0, double vol,
                              int inverse) {
  const long n = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= nn) return;
  const int i = (int)(n % (nx + 1)), j = (int)(n / (nx + 1));
  // (corner, gx, gy) of the three vertices of each triangle type
  const int tri[4][3][3] = {{{0, -1, 0}, {1, 1, -1}, {3, 0, 1}},
                            {{0, 0, -1}, {2, -1, 1}, {3, 1, 0}},
                            {{0, -1, -1}, {1, 1, 0}, {2, 0, 1}},
                            {{3, 1, 1}, {1, 0, -1}, {2, -1, 0}}};
  double acc[3] = {0, 0, 0};
  for (int sy = -1; sy <= 0; ++sy)
    for (int sx = -1; sx <= 0; ++sx) {
      const int hi = i + sx, hj = j + sy;
      if (hi < 0 || hi >= nx || hj < 0 || hj >= ny) continue;
      const int corner = (-sx) + 2 * (-sy);
      const bool a = split_uniform || ((hj & 1) == 0);
      for (int t = 0; t < 2; ++t) {
        const int type = (a ? 0 : 2) + t;
        const double e = E[2 * ((long)hj * nx + hi) + t] * vol;
        for (int v = 0; v < 3; ++v)
          if (tri[type][v][0] == corner) {
            const int g[2] = {tri[type][v][1], tri[type][v][2]};
            diag_add(acc, 2, g, lam0 * e, mu0 * e);
          }
      }
    }
  const int m = mask[n];
  for (int c = 0; c < 2; ++c) {
    double v = ((m >> c) & 1) ? 1.0 : acc[c];
    d[c * nn + n] = inverse ? 1.0 / v : v;
  }
}

__global__ void diag3d_kernel(double* d, const double* E, const uint8_t* mask, int nx, int ny,
                              int nz, long nn, double lam0, double mu0, double vol, int inverse) {
  const long n = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= nn) return;
  const int i = (int)(n % (nx + 1));
  const int j = (int)((n / (nx + 1)) % (ny + 1));
  const int k = (int)(n / ((long)(nx + 1) * (ny + 1)));
  const int perm[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
  double acc[3] = {0, 0, 0};
  for (int sz = -1; sz <= 0; ++sz)
    for (int sy = -1; sy <= 0; ++sy)
      for (int sx = -1; sx <= 0; ++sx) {
        const int hi = i + sx, hj = j + sy, hk = k + sz;
        if (hi < 0 || hi >= nx || hj < 0 || hj >= ny || hk < 0 || hk >= nz) continue;
        const int corner = (-sx) + 2 * (-sy) + 4 * (-sz);
        const long h = ((long)hk * ny + hj) * nx + hi;
        for (int t = 0; t < 6; ++t) {
          const int c1 = 1 << perm[t][0];
          const int c2 = c1 | (1 << perm[t][1]);
          const int cs[4] = {0, c1, c2, 7};
          for (int v = 0; v < 4; ++v) {
            if (cs[v] != corner) continue;
            int g[3] = {0, 0, 0};
            if (v == 0) g[perm[t][0]] = -1;
            if (v == 1) { g[perm[t][0]] += 1; g[perm[t][1]] -= 1; }
            if (v == 2) { g[perm[t][1]] += 1; g[perm[t][2]] -= 1; }
            if (v == 3) g[perm[t][2]] = 1;
            const double e = E[6 * h + t] * vol;
            diag_add(acc, 3, g, lam0 * e, mu0 * e);
          }
        }
      }
  const int m = mask[n];
  for (int c = 0; c < 3; ++c) {
    double v = ((m >> c) & 1) ? 1.0 : acc[c];
    d[c * nn + n] = inverse ? 1.0 / v : v;
  }
}

// ---------------------------------------------------- elementwise helpers
__global__ void simp_modulus_kernel(double* E, float* E32, const double* rho, long nc, double E0,
                                    double Emin, double penal, int paper) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nc) return;
  const double r = rho[e];
  const double rp = (penal == 3.0) ? r * r * r : pow(r, penal);
  const double v = paper ? rp : Emin + rp * (E0 - Emin);
  E[e] = v;
  if (E32) E32[e] = (float)v;
}

__global__ void mask_copy_kernel(const double* src, double* dst, const uint8_t* mask, long nn,
                                 int dim, long total) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= total) return;
  const long n = i % nn;
  const int c = (int)((i / nn) % dim);
  dst[i] = ((mask[n] >> c) & 1) ? 0.0 : src[i];
}

__global__ void fill_kernel(double* dst, double v, long n) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = v;
}

// ------------------------------------------------------------ launchers
static inline unsigned cdiv(long a, long b) { return (unsigned)((a + b - 1) / b); }

void launch_simp_modulus(Ctx* c, const double* rho) {
  simp_modulus_kernel<<<cdiv(c->g.nc, 256), 256, 0, c->stream>>>(
      c->E, c->prob.precision == TOPO_MIXED_FP32 ? c->E32 : nullptr, rho, c->g.nc, c->m.E0,
      c->m.Emin, c->m.penal, c->m.paper);
}

template <typename T, typename TE>
static void apply_dispatch(Ctx* c, const T* x, T* y, const TE* E, int nrhs, bool fuse_dot) {
  const Grid& g = c->g;
  double* part = fuse_dot ? c->partials : nullptr;
  unsigned* cnt = &c->scal->counters[CNT_APPLY_DOT];
  PcgState* st = fuse_dot ? &c->scal->pcg : nullptr;
  const T lam = T(c->m.lam0 * c->m.vol), mu = T(c->m.mu0 * c->m.vol);
  if (g.dim == 2) {
    dim3 grid(cdiv(g.nx + 1, TILE), cdiv(g.ny + 1, TILE));
    const int su = g.split == TOPO_SPLIT_UNIFORM;
#define A2(NR) apply2d_kernel<T, TE, NR><<<grid, 256, 0, c->stream>>>(x, y, E, c->mask, g.nx, g.ny, g.nn, su, lam, mu, part, cnt, st)
    switch (nrhs) { case 1: A2(1); break; case 2: A2(2); break; case 3: A2(3); break; default: A2(4); }
#undef A2
  } else {
    const int kz = c->apply_kz;
    dim3 grid(cdiv(g.nx + 1, TILE), cdiv(g.ny + 1, TILE), cdiv(g.nz + 1, kz));
#define A3(NR) apply3d_kernel<T, TE, NR><<<grid, 256, 0, c->stream>>>(x, y, E, c->mask, g.nx, g.ny, g.nz, g.nn, kz, lam, mu, part, cnt, st)
    switch (nrhs) { case 1: A3(1); break; case 2: A3(2); break; case 3: A3(3); break; default: A3(4); }
#undef A3
  }
}

void launch_apply(Ctx* c, const double* x, double* y, int nrhs, bool fuse_dot) {
  int slot = c->timing ? timing_begin(c, nullptr) : -1;
  apply_dispatch<double, double>(c, x, y, c->E, nrhs, fuse_dot);
  if (slot >= 0) timing_end(c, slot);
}

void launch_apply_f32(Ctx* c, const float* x, float* y, int nrhs, bool fuse_dot) {
  int slot = c->timing ? timing_begin(c, nullptr) : -1;
  apply_dispatch<float, float>(c, x, y, c->E32, nrhs, fuse_dot);
  if (slot >= 0) timing_end(c, slot);
}

void launch_diagonal(Ctx* c, double* d, bool inverse) {
  const Grid& g = c->g;
  if (g.dim == 2)
    diag2d_kernel<<<cdiv(g.nn, 256), 256, 0, c->stream>>>(
        d, c->E, c->mask, g.nx, g.ny, g.nn, g.split == TOPO_SPLIT_UNIFORM, c->m.lam0, c->m.mu0,
        c->m.vol, inverse);
  else
    diag3d_kernel<<<cdiv(g.nn, 256), 256, 0, c->stream>>>(
        d, c->E, c->mask, g.nx, g.ny, g.nz, g.nn, c->m.lam0, c->m.mu0, c->m.vol, inverse);
}

void launch_mask_copy(Ctx* c, const double* src, double* dst, int nrhs) {
  const long total = (long)nrhs * c->g.nd;
  mask_copy_kernel<<<cdiv(total, 256), 256, 0, c->stream>>>(src, dst, c->mask, c->g.nn, c->g.dim,
                                                            total);
}

void launch_fill(Ctx* c, double* dst, double v, int64_t n) {
  fill_kernel<<<cdiv(n, 256), 256, 0, c->stream>>>(dst, v, n);
}

}  // namespace topo
