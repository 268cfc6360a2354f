// Element- and node-level device code shared by the single-grid kernels and
// the batched 2D kernels: the 2D operator tile, the diagonal, the multigrid
// transfers and coarse solve, and the Chebyshev interval.  (Device functions
// are shared through this header because every .hip file is compiled as
// its own code object.)
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>

#include "common.h"
#include "element.h"
#include "topo_internal.h"

namespace topo {

// Value held by the next lane of the same tile row (tx + 1).  Rows of 16
// lanes use the DPP row shift (row_shl:1), rows of 32 or 64 lanes the DPP
// wave shift (wave_shl:1, which crosses the 16-lane rows), other widths a
// permute through LDS.  The last lane of a row receives no neighbour value;
// callers do not use it.
template <int BX>
__device__ __forceinline__ int next_lane_b32(int v) {
  if constexpr (BX == 16) return __builtin_amdgcn_update_dpp(v, v, 0x101, 0xf, 0xf, false);
  else if constexpr (BX == 32 || BX == 64)
    return __builtin_amdgcn_update_dpp(v, v, 0x130, 0xf, 0xf, false);
  else return __shfl_down(v, 1, BX);
}

template <int BX>
__device__ __forceinline__ float next_lane(float v) {
  return __int_as_float(next_lane_b32<BX>(__float_as_int(v)));
}

template <int BX>
__device__ __forceinline__ double next_lane(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = next_lane_b32<BX>((int)b), hi = next_lane_b32<BX>((int)(b >> 32));
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

// One tile of a BX x BY thread block (BX * BY = 256): the block owns
// (BX-1) x (BY-1) nodes and computes the BX x BY squares touching them.
// Returns this thread's share of (x, y) over owned nodes.
template <typename T, typename TE, int BX, int BY>
__device__ inline double apply2d_tile(bool live, int bx, int by, int rhs,
                                               const T* __restrict__ x, T* __restrict__ y,
                                               const TE* __restrict__ E, const OpDesc& d, T lam0,
                                               T mu0) {
  constexpr int PX = BX + 1, PY = BY + 1, OX = BX - 1, OY = BY - 1;
  __shared__ T xs[2][PX * PY];
  __shared__ T ex[2][BX * BY];
  const int tid = threadIdx.x;
  const int tx = tid % BX, ty = tid / BX;
  const int nx = d.nx, ny = d.ny;
  const long nn = d.nn;
  const int i0 = bx * OX, j0 = by * OY;
  const T* xr = x + (long)rhs * 2 * nn;
  double dot = 0.0;
  if (live) {
    for (int idx = tid; idx < PX * PY; idx += BX * BY) {
      const int a = idx % PX, b = idx / PX;
      const int gi = i0 - 1 + a, gj = j0 - 1 + b;
      const int ci = min(max(gi, 0), nx), cj = min(max(gj, 0), ny);
      const long n = (long)cj * (nx + 1) + ci;
      xs[0][idx] = xr[n];
      xs[1][idx] = xr[nn + n];
    }
  }
  const int hi = i0 - 1 + tx, hj = j0 - 1 + ty;
  const bool cell_ok = live && hi >= 0 && hi < nx && hj >= 0 && hj < ny;
  T l0 = 0, m0 = 0, l1 = 0, m1 = 0;
  if (cell_ok) {
    const long e = 2 * ((long)hj * nx + hi);
    const T e0 = T(E[e]), e1 = T(E[e + 1]);
    l0 = lam0 * e0; m0 = mu0 * e0; l1 = lam0 * e1; m1 = mu0 * e1;
  }
  lds_barrier();
  if (live) {
    const bool diag_a = d.split_uniform || ((hj & 1) == 0);
    const int oi = i0 + tx, oj = j0 + ty;
    const bool owner = tx < OX && ty < OY && oi <= nx && oj <= ny;
    const long on = (long)oj * (nx + 1) + oi;
    const int om = owner ? d.mask[on] : 3;
    T u[4][2], f[4][2];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int li = (ty + (c >> 1)) * PX + tx + (c & 1);
      u[c][0] = xs[0][li];
      u[c][1] = xs[1][li];
      f[c][0] = 0; f[c][1] = 0;
    }
    square_force<T>(diag_a, u, l0, m0, l1, m1, f);
    T X[2][2];
#pragma unroll
    for (int cy = 0; cy < 2; ++cy)
#pragma unroll
      for (int c = 0; c < 2; ++c) X[cy][c] = f[1 + 2 * cy][c] + next_lane<BX>(f[2 * cy][c]);
    ex[0][tid] = X[0][0];
    ex[1][tid] = X[0][1];
    lds_barrier();
    if (owner) {
      T* yr = y + (long)rhs * 2 * nn;
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        T v = X[1][c] + ex[c][tid + BX];
        if ((om >> c) & 1) v = 0;
        yr[c * nn + on] = v;
        dot += (double)v * (double)u[3][c];
      }
    }
  } else {
    lds_barrier();
  }
  return dot;
}

// diag K at node a, component c: sum over cells of
// |T| E (lambda g_c^2 + mu (g_c^2 + |g|^2)) with g = grad N_a.
__device__ inline void diag_add(double (&d)[3], int dim, const int* g, double lam,
                                         double mu) {
  double gg = 0.0;
  for (int a = 0; a < dim; ++a) gg += g[a] * g[a];
  for (int c = 0; c < dim; ++c) d[c] += lam * g[c] * g[c] + mu * (g[c] * g[c] + gg);
}

__device__ inline void diag2d_node(long n, double* d, const double* E, const OpDesc& od, double lam0,
                            double mu0, double vol, int inverse) {
  const int nx = od.nx, ny = od.ny;
  const long nn = od.nn;
  const int split_uniform = od.split_uniform;
  const uint8_t* mask = od.mask;
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

// ------------------------------------------------------ coarse moduli (2D)
__device__ inline void restrict_E2_square(long S, double* Ec, const double* __restrict__ Ef, int nxf,
                                   int nyf, int uniform_f, int nxc) {
  const int I = (int)(S % nxc), J = (int)(S / nxc);
  double acc[2] = {0, 0};
  for (int dy = 0; dy < 2; ++dy)
    for (int dx = 0; dx < 2; ++dx) {
      const int fi = 2 * I + dx, fj = 2 * J + dy;
      if (fi >= nxf || fj >= nyf) continue;
      const bool a = uniform_f || ((fj & 1) == 0);
      // triangle centroids x3: A: (2,1), (1,2); B: (1,1), (2,2)
      const int cx[2] = {a ? 2 : 1, a ? 1 : 2};
      const int cy[2] = {a ? 1 : 1, a ? 2 : 2};
      for (int t = 0; t < 2; ++t) {
        const double e = Ef[2 * ((long)fj * nxf + fi) + t];
        const int qx = 3 * dx + cx[t], qy = 3 * dy + cy[t];
        if (qx > qy) acc[0] += e;
        else if (qx < qy) acc[1] += e;
        else { acc[0] += 0.5 * e; acc[1] += 0.5 * e; }
      }
    }
  Ec[2 * S] = acc[0] * 0.25;
  Ec[2 * S + 1] = acc[1] * 0.25;
}

// ----------------------------------------------- transfer operators
// b_c = R (b_f - q_f): restriction of the fine residual
template <typename T>
__device__ inline void restrict_node(long C, T* bc, const T* __restrict__ bf, const T* __restrict__ qf,
                              const OpDesc& fo, const OpDesc& co, int nrhs) {
  const int dim = co.dim;
  const int nxc1 = co.nx + 1, nyc1 = co.ny + 1;
  const int I = (int)(C % nxc1), J = (int)((C / nxc1) % nyc1), K = dim == 3 ? (int)(C / ((long)nxc1 * nyc1)) : 0;
  const int nxf1 = fo.nx + 1, nyf1 = fo.ny + 1;
  const int nzf = dim == 3 ? fo.nz : 0;
  const int cm = co.mask[C];
  const int ndir = dim == 3 ? 7 : 3;
  for (int r = 0; r < nrhs; ++r)
    for (int c = 0; c < dim; ++c) {
      const long off = ((long)r * dim + c) * fo.nn;
      T acc = 0;
      {
        const int fi = 2 * I, fj = 2 * J, fk = 2 * K;
        if (fi <= fo.nx && fj <= fo.ny && fk <= nzf) {
          const long n = ((long)fk * nyf1 + fj) * nxf1 + fi;
          acc += bf[off + n] - qf[off + n];
        }
      }
      for (int dd = 1; dd <= ndir; ++dd) {
        const int dx = dd & 1, dy = (dd >> 1) & 1, dz = (dd >> 2) & 1;
        for (int sgn = -1; sgn <= 1; sgn += 2) {
          const int fi = 2 * I + sgn * dx, fj = 2 * J + sgn * dy, fk = 2 * K + sgn * dz;
          if (fi < 0 || fj < 0 || fk < 0 || fi > fo.nx || fj > fo.ny || fk > nzf) continue;
          const long n = ((long)fk * nyf1 + fj) * nxf1 + fi;
          acc += T(0.5) * (bf[off + n] - qf[off + n]);
        }
      }
      bc[((long)r * dim + c) * co.nn + C] = ((cm >> c) & 1) ? T(0) : acc;
    }
}

// x_f += P x_c (fixed fine DOFs untouched)
template <typename T>
__device__ inline void prolong_node(long n, T* xf, const T* __restrict__ xc, const OpDesc& fo,
                             const OpDesc& co, int nrhs) {
  const int dim = fo.dim;
  const int nxf1 = fo.nx + 1, nyf1 = fo.ny + 1;
  const int i = (int)(n % nxf1), j = (int)((n / nxf1) % nyf1), k = dim == 3 ? (int)(n / ((long)nxf1 * nyf1)) : 0;
  const int nxc1 = co.nx + 1, nyc1 = co.ny + 1;
  const long c0 = ((long)(k >> 1) * nyc1 + (j >> 1)) * nxc1 + (i >> 1);
  const long c1 = ((long)((k + 1) >> 1) * nyc1 + ((j + 1) >> 1)) * nxc1 + ((i + 1) >> 1);
  const bool even = ((i | j | k) & 1) == 0;
  const int fm = fo.mask[n];
  for (int r = 0; r < nrhs; ++r)
    for (int c = 0; c < dim; ++c) {
      if ((fm >> c) & 1) continue;
      const T* xcr = xc + ((long)r * dim + c) * co.nn;
      const T e = even ? xcr[c0] : T(0.5) * (xcr[c0] + xcr[c1]);
      xf[((long)r * dim + c) * fo.nn + n] += e;
    }
}

// ------------------------------------------------------- smoother
// Chebyshev smoothing of D^-1 K, d_0 = s D^-1 r_0, d_i = c1 d_(i-1) + c2 D^-1 r_i.
// kind 1: first-kind polynomial on [low lmax, lmax] (rho_k, rho_(k-1) of its
// three-term recurrence); kind 4: the fourth-kind polynomial on (0, lmax]
// (Lottes 2023), s = 4 / (3 lmax), c1 = (2i-1)/(2i+3), c2 = (8i+4)/((2i+3) lmax),
// which needs no lower bound of the spectrum.
struct ChebCoef {
  double r_cur, r_prev;
  int kind;   // 1 or 4
  int step;   // i >= 1
};

__device__ inline void cheb_interval(double lmax, double low, double& theta,
                                              double& delta) {
  const double hi = lmax, lo = low * lmax;
  theta = 0.5 * (hi + lo);
  delta = 0.5 * (hi - lo);
}

__device__ inline double cheb_first_scale(double lmax, double low, int kind) {
  if (kind == 4) return 4.0 / (3.0 * lmax);
  double theta, delta;
  cheb_interval(lmax, low, theta, delta);
  return 1.0 / theta;
}

__device__ inline void cheb_next_coef(double lmax, double low, const ChebCoef& cf, double& c1,
                                      double& c2) {
  if (cf.kind == 4) {
    const double i = (double)cf.step;
    c1 = (2.0 * i - 1.0) / (2.0 * i + 3.0);
    c2 = (8.0 * i + 4.0) / ((2.0 * i + 3.0) * lmax);
    return;
  }
  double theta, delta;
  cheb_interval(lmax, low, theta, delta);
  c1 = cf.r_cur * cf.r_prev;
  c2 = 2.0 * cf.r_cur / delta;
}

// ---------------------------------------------------- coarsest level
// Dense A (row-major with leading dimension ld, n = dim * nn): row i =
// c * nn + node, built by the thread that owns the row from the element
// matrices K_e[(a,i),(b,j)] = |T| E (lambda g_a,i g_b,j + mu (g_a,j g_b,i +
// delta_ij g_a.g_b)).  ld = 0 means ld = n; with zero = false the row must
// already hold zeros.
__device__ inline void coarse_assemble_row(int row, double* A, const double* __restrict__ E,
                                    const OpDesc& o, double lam0, double mu0, double vol,
                                    long ld = 0, bool zero = true) {
  const int n = (int)(o.nn * o.dim);
  const int dim = o.dim;
  const int node = row % (int)o.nn, ci = row / (int)o.nn;
  double* Ar = A + (long)row * (ld > 0 ? ld : n);
  if (zero)
    for (int j = 0; j < n; ++j) Ar[j] = 0.0;
  const int nx1 = o.nx + 1, ny1 = o.ny + 1;
  const int i = node % nx1, jj = (node / nx1) % ny1, k = dim == 3 ? node / (nx1 * ny1) : 0;
  if ((o.mask[node] >> ci) & 1) {
    Ar[row] = 1.0;
    return;
  }
  auto add_cell = [&](int nv, const int* nodes, const int (*g)[3], int av, double e) {
    const double l = lam0 * e * vol, m = mu0 * e * vol;
    const int* ga = g[av];
    double gaga_dummy = 0.0;
    (void)gaga_dummy;
    for (int bv = 0; bv < nv; ++bv) {
      const int* gb = g[bv];
      double dot = 0.0;
      for (int a = 0; a < dim; ++a) dot += ga[a] * gb[a];
      for (int cj = 0; cj < dim; ++cj) {
        const int col = cj * (int)o.nn + nodes[bv];
        if ((o.mask[nodes[bv]] >> cj) & 1) continue;
        Ar[col] += l * ga[ci] * gb[cj] + m * (ga[cj] * gb[ci] + (ci == cj ? dot : 0.0));
      }
    }
  };
  if (dim == 3) {
    const int perm[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
    for (int sz = -1; sz <= 0; ++sz)
      for (int sy = -1; sy <= 0; ++sy)
        for (int sx = -1; sx <= 0; ++sx) {
          const int hi = i + sx, hj = jj + sy, hk = k + sz;
          if (hi < 0 || hi >= o.nx || hj < 0 || hj >= o.ny || hk < 0 || hk >= o.nz) continue;
          const int corner = (-sx) + 2 * (-sy) + 4 * (-sz);
          const long h = ((long)hk * o.ny + hj) * o.nx + hi;
          for (int t = 0; t < 6; ++t) {
            const int c1 = 1 << perm[t][0];
            const int c2 = c1 | (1 << perm[t][1]);
            const int cs[4] = {0, c1, c2, 7};
            int av = -1;
            for (int v = 0; v < 4; ++v)
              if (cs[v] == corner) av = v;
            if (av < 0) continue;
            int g[4][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
            g[0][perm[t][0]] = -1;
            g[1][perm[t][0]] += 1;
            g[1][perm[t][1]] -= 1;
            g[2][perm[t][1]] += 1;
            g[2][perm[t][2]] -= 1;
            g[3][perm[t][2]] = 1;
            int nodes[4];
            for (int v = 0; v < 4; ++v) {
              const int cc = cs[v];
              nodes[v] = ((hk + (cc >> 2)) * ny1 + hj + ((cc >> 1) & 1)) * nx1 + hi + (cc & 1);
            }
            add_cell(4, nodes, g, av, E[6 * h + t]);
          }
        }
  } else {
    // (corner, gx, gy) of the three vertices of each triangle type
    const int tri[4][3][3] = {{{0, -1, 0}, {1, 1, -1}, {3, 0, 1}},
                              {{0, 0, -1}, {2, -1, 1}, {3, 1, 0}},
                              {{0, -1, -1}, {1, 1, 0}, {2, 0, 1}},
                              {{3, 1, 1}, {1, 0, -1}, {2, -1, 0}}};
    for (int sy = -1; sy <= 0; ++sy)
      for (int sx = -1; sx <= 0; ++sx) {
        const int hi = i + sx, hj = jj + sy;
        if (hi < 0 || hi >= o.nx || hj < 0 || hj >= o.ny) continue;
        const int corner = (-sx) + 2 * (-sy);
        const bool da = o.split_uniform || ((hj & 1) == 0);
        for (int t = 0; t < 2; ++t) {
          const int type = (da ? 0 : 2) + t;
          int av = -1;
          for (int v = 0; v < 3; ++v)
            if (tri[type][v][0] == corner) av = v;
          if (av < 0) continue;
          int g[3][3];
          int nodes[3];
          for (int v = 0; v < 3; ++v) {
            g[v][0] = tri[type][v][1];
            g[v][1] = tri[type][v][2];
            g[v][2] = 0;
            const int cc = tri[type][v][0];
            nodes[v] = (hj + (cc >> 1)) * nx1 + hi + (cc & 1);
          }
          add_cell(3, nodes, g, av, E[2 * ((long)hj * o.nx + hi) + t]);
        }
      }
  }
}

// In-place Gauss-Jordan inversion of the SPD matrix A (n x n, row-major),
// one work-group; column k of the eliminated rows is saved first.
// (blockDim.x must be a multiple of 128)
__device__ inline void gauss_jordan_block(double* A, int n) {
  // the whole matrix (n <= 128: at most 128 KiB) lives in LDS during the
  // n elimination steps, so each step's update is an LDS pass, not a
  // global read-modify-write (n = 108: 428 -> tens of microseconds)
  __shared__ double As[128 * 128];
  __shared__ double rowk[128];
  __shared__ double colk[128];
  for (int t = threadIdx.x; t < n * n; t += blockDim.x) As[t] = A[t];
  __syncthreads();
  for (int k = 0; k < n; ++k) {
    const double piv = As[k * n + k];
    __syncthreads();
    for (int t = threadIdx.x; t < n; t += blockDim.x) {
      colk[t] = As[t * n + k];
      rowk[t] = ((t == k) ? 1.0 : As[k * n + t]) / piv;
    }
    __syncthreads();
    // thread (column j, first row i0) walks its column in steps of the
    // block's row count: no per-entry index division
    const int j = threadIdx.x % 128, i0 = threadIdx.x / 128, di = blockDim.x / 128;
    if (j < n) {
      const double rj = rowk[j];
      for (int i = i0; i < n; i += di) {
        const int t = i * n + j;
        if (i == k) {
          As[t] = rj;
        } else {
          const double base = (j == k) ? 0.0 : As[t];
          As[t] = base - colk[i] * rj;
        }
      }
    }
    __syncthreads();
  }
  for (int t = threadIdx.x; t < n * n; t += blockDim.x) A[t] = As[t];
}

// x = A^-1 b for every load case (n <= 128, nrhs <= 4), accumulated in
// FP64, by one work-group: b is staged in LDS, thread t computes row
// i = t % n of load case t / n, and since the inverse of the symmetric
// coarse matrix is symmetric it reads column i (consecutive threads read
// consecutive addresses).
template <typename T>
__device__ inline void coarse_solve_block(T* x, const T* __restrict__ b,
                                          const double* __restrict__ Ainv, int n, int nrhs) {
  __shared__ double bs[kMaxRhs * 128];
  for (int t = threadIdx.x; t < n * nrhs; t += blockDim.x) bs[t] = (double)b[t];
  __syncthreads();
  for (int t = threadIdx.x; t < n * nrhs; t += blockDim.x) {
    const int r = t / n, i = t - r * n;
    const double* br = bs + r * n;
    double acc0 = 0.0, acc1 = 0.0;
    int j = 0;
    for (; j + 1 < n; j += 2) {
      acc0 += Ainv[(long)j * n + i] * br[j];
      acc1 += Ainv[(long)(j + 1) * n + i] * br[j + 1];
    }
    if (j < n) acc0 += Ainv[(long)j * n + i] * br[j];
    x[t] = T(acc0 + acc1);
  }
}

// ------------------------------------------------ CG scalar updates
// rr and the reference norm ff from the totals; tol2 = rtol^2 ff
template <int NR>
__device__ inline void pcg_init_finish(const double* tot, double rtol, PcgState* st) {
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

// alpha = (r, z) / (p, K p) per active load case
__device__ inline void pcg_alpha_finish(const double* tot, PcgState* st) {
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

// convergence test after x += alpha p, r -= alpha q (Jacobi: also beta)
template <int NR, bool JAC>
__device__ inline void pcg_update_finish(const double* tot, PcgState* st, int* status) {
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

// beta = (r, z) / (r, z)_old (first iteration: beta = 0)
template <int NR>
__device__ inline void pcg_rz_finish(const double* tot, int first, PcgState* st) {
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

// ------------------------------------------------ OC scalar updates
__device__ inline double oc_a(double rho, double s, double eta) {
  const double ns = s < 0.0 ? -s : 0.0;
  return rho * (eta == 0.5 ? sqrt(ns) : pow(ns, eta));
}

// target, bracket and first multiplier from the totals (sum lo, volume at
// large mu, sum a, largest useful mu); infeasible targets are flagged
__device__ inline void oc_init_finish(const double* tot, long nc, double volfrac, OcState* st,
                                      int* status) {
  const double target = volfrac * (double)nc;
  st->target = target;
  st->sum_lo = tot[0];
  st->sum_hi = tot[1];
  st->sum_a = tot[2];
  st->passes = 0;
  st->infeasible = 0;
  st->mu_lo = 0.0;
  st->mu_hi = tot[3];
  const double tol = 1e-13 * (double)nc;
  if (target < tot[0] - tol || target > tot[1] + tol || !(tot[2] > 0.0)) {
    st->infeasible = 1;
    st->mu = (target < tot[0]) ? 0.0 : tot[3];
    st->done = 1;
    *status = TOPO_S_OC_INFEASIBLE;
  } else {
    double mu = target / tot[2];
    if (!(mu < st->mu_hi)) mu = 0.5 * st->mu_hi;
    st->mu = mu;
    st->done = 0;
  }
}

// one safeguarded Newton step on V(mu) - target from V and its slope S
__device__ inline void oc_pass_finish(const double* tot, long nc, OcState* st) {
  const double mu = st->mu;
  const double V = tot[0], S = tot[1], T = st->target;
  st->V = V;
  st->S = S;
  st->passes += 1;
  const double err = V - T;
  const double tol = 1e-14 * (double)nc;
  if (fabs(err) <= tol || st->passes >= 200) {
    st->done = 1;
    return;
  }
  if (err < 0.0) st->mu_lo = mu; else st->mu_hi = mu;
  double next = 0.5 * (st->mu_lo + st->mu_hi);
  if (S > 0.0) {
    const double nw = mu - err / S;
    if (nw > st->mu_lo && nw < st->mu_hi) next = nw;
  }
  if (!(next > st->mu_lo && next < st->mu_hi)) {
    // the bracket cannot be split further in FP64: keep the last point
    st->done = 1;
    return;
  }
  st->mu = next;
}

// volume, change and lambda = mu^(-1/eta) of the new design.  A feasible
// update whose volume misses volfrac * N by more than 1e-12 N (the pass
// budget ran out, or the bracket could not be split further) sets the
// sticky TOPO_S_OC_INEXACT: the design is valid, its volume inexact.
__device__ inline void oc_final_finish(const double* tot, double eta, long nc, OcState* st,
                                       double* scalars, int* status) {
  const double mu = st->mu;
  if (!st->infeasible && !(fabs(tot[0] - st->target) <= 1e-12 * (double)nc) && *status == 0)
    *status = TOPO_S_OC_INEXACT;
  st->vol = tot[0];
  st->change = tot[1];
  st->lam = (mu > 0.0) ? pow(mu, -1.0 / eta) : INFINITY;
  if (scalars) {
    scalars[0] = st->lam;
    scalars[1] = tot[0];
    scalars[2] = tot[1];
  }
}

// ------------------------------------------------ 2D sensitivity
// energies of the two triangles of square s over the load cases, their
// sensitivities, and the compliance sums (sum E w, listing objective)
__device__ inline void sens2d_square(long s, const double* __restrict__ rho, const double* __restrict__ u,
                                     double* dc, int nx, long nn, int nr, int split_uniform,
                                     double lam0, double mu0, double vol, double E0, double Emin,
                                     double penal, int paper, double (&acc)[2]) {
  const int i = (int)(s % nx), j = (int)(s / nx);
  const bool a = split_uniform || ((j & 1) == 0);
  double w0 = 0.0, w1 = 0.0;
  for (int r = 0; r < nr; ++r) {
    double uc[4][2];
    for (int c = 0; c < 4; ++c) {
      const long n = (long)(j + (c >> 1)) * (nx + 1) + i + (c & 1);
      uc[c][0] = u[((long)r * 2 + 0) * nn + n];
      uc[c][1] = u[((long)r * 2 + 1) * nn + n];
    }
    double e0, e1;
    square_energy<double>(a, uc, lam0, mu0, e0, e1);
    w0 += e0;
    w1 += e1;
  }
  const double ws[2] = {w0 * vol, w1 * vol};
  for (int t = 0; t < 2; ++t) {
    const long e = 2 * s + t;
    const double rv = rho[e];
    const double rp1 = (penal == 3.0) ? rv * rv : pow(rv, penal - 1.0);
    const double Ee = paper ? rp1 * rv : Emin + rp1 * rv * (E0 - Emin);
    dc[e] = paper ? -penal * rp1 * ws[t] / (2.0 * vol) : -penal * rp1 * (E0 - Emin) * ws[t];
    acc[0] += Ee * ws[t];
    acc[1] += Ee * ws[t] / (2.0 * vol);
  }
}

// ------------------------------------------------ filter
// one cell (block-cell h, class t): sum over the class's taps inside the grid
__device__ inline void filter_cell(long h, int t, double* out, const double* __restrict__ q,
                                   const double* __restrict__ rho, const double* __restrict__ R,
                                   const FilterTap* __restrict__ taps, const int* __restrict__ ntaps,
                                   int stride, int dim, int nx, int ny, int nz, int ncls, int alt, int out_mode) {
  const long nblk = (long)nx * ny * nz;
  const int i = (int)(h % nx);
  const int j = (int)((h / nx) % ny);
  const int k = (int)(h / ((long)nx * ny));
  const int cls = (dim == 2 && alt) ? t + 2 * (j & 1) : t;
  const FilterTap* tp = taps + (long)cls * stride;
  const int nt = ntaps[cls];
  double acc = 0.0;
  for (int s = 0; s < nt; ++s) {
    const FilterTap tap = tp[s];
    const int ii = i + tap.di, jj = j + tap.dj, kk = k + tap.dk;
    if (ii < 0 || ii >= nx || jj < 0 || jj >= ny || kk < 0 || kk >= nz) continue;
    const long hb = ((long)kk * ny + jj) * nx + ii;
    acc += tap.w * q[(long)tap.tb * nblk + hb];
  }
  const long e = h * ncls + t;
  // out_mode 0: sensitivity filter, divide by rho_e R_e; 1: the plain sum;
  // 2: divide by R_e (density filter)
  if (out_mode == 1) out[e] = acc;
  else if (out_mode == 2) out[e] = acc / R[e];
  else out[e] = acc / (rho[e] * R[e]);
}

}  // namespace topo
