// Geometric multigrid V-cycle used as the CG preconditioner.
//
// Hierarchy: level l+1 has ceil(n_l / 2) cells per axis and cell size 2^(l+1).
// In 3D every Kuhn tetrahedron of a coarse cube is exactly the union of 8
// Kuhn tetrahedra of the fine grid (Freudenthal refinement), and in 2D the
// same holds for diagonal-A triangles.  The coarse P1 space is therefore
// nested in the fine one, prolongation is linear interpolation on the coarse
// simplices, fine(x) = coarse(x/2) at even nodes and the mean of
// coarse(floor(x/2)) and coarse(ceil(x/2)) otherwise, restriction is its
// transpose, and the Galerkin coarse operator P^T K P is the coarse P1
// operator with each coarse modulus the mean of its 8 (2D: 4) children's
// moduli -- fine cells outside an odd-sized grid count as void.  The coarse
// levels re-use the fine-level apply kernels, which assume unit cells.  A P1
// element matrix scales as (cell volume) x (gradient)^2, i.e. as h^(dim-2):
// unchanged in 2D, doubled per level in 3D.  So the 3D coarse moduli stored
// for the unit-cell kernels are twice the children's mean (without the
// factor every level is half its Galerkin operator, the coarse corrections
// overshoot by 2 per level and the CG iterations grow with the depth).  A coarse DOF is fixed when
// any fine DOF of the same component in the support of its basis function
// is fixed (this keeps every level non-singular).
//
// Smoother: Chebyshev polynomial of degree K in D^-1 K on
// [0.09 lmax, lmax], lmax from a Rayleigh-quotient power iteration with a
// safety factor; the same polynomial is used before and after the coarse
// correction, so the V-cycle is a symmetric positive definite operator.
// Coarsest level (the first of at most 2048 DOFs, or the size the problem
// asks for): dense matrix assembled per solve and inverted, by Gauss-Jordan
// elimination in one work-group up to 128 DOFs, else by the symmetric block
// sweep over the whole GPU.
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include <type_traits>
#include <vector>

#include "common.h"
#include "dense_dev.h"
#include "element.h"
#include "shared_dev.h"
#include "topo_internal.h"

namespace topo {

// A revisit of a smaller coarse level costs more in launches than it saves
// in iterations: on 192x96x96 x 4 load cases (7 levels, the last three in
// the one-block tail) W on the top 2 levels gave 12.8 SIMP it/s (38 CG
// iterations per solve), the top 3 14.0 (29), the top 4 14.2 (25), the
// top 5 13.4 (24).  This threshold selects the top 4 there (coarse levels
// of 230k, 31k, 4.2k and 637 nodes).
constexpr long kWCoarseNodes = 512;

GmgParams gmg_params_env() {
  GmgParams p;
  if (const char* e = getenv("TOPO_CHEB_DEGREE")) p.cheb_degree = atoi(e) > 0 ? atoi(e) : p.cheb_degree;
  if (const char* e = getenv("TOPO_CHEB_LOW")) p.cheb_low = atof(e) > 0 ? atof(e) : p.cheb_low;
  if (const char* e = getenv("TOPO_POWER_ITERS")) p.power_iters = atoi(e) > 0 ? atoi(e) : p.power_iters;
  if (const char* e = getenv("TOPO_POWER_SAFETY")) p.power_safety = atof(e) > 0 ? atof(e) : p.power_safety;
  if (const char* e = getenv("TOPO_CHEB_POST")) p.post_degree = atoi(e);
  if (const char* e = getenv("TOPO_CHEB_KIND")) p.cheb_kind = atoi(e) == 4 ? 4 : 1;
  if (const char* e = getenv("TOPO_CHEB_POST_FUSED")) p.fused_post = atoi(e) != 0;
  if (const char* e = getenv("TOPO_GMG_WLEVELS")) p.wlevels = atoi(e) > 0 ? atoi(e) : 0;
  if (const char* e = getenv("TOPO_GMG_TAIL")) p.tail = atoi(e) != 0;
  if (p.post_degree < 0) p.post_degree = p.cheb_degree;
  return p;
}

static inline unsigned cdivu(long a, long b) { return (unsigned)((a + b - 1) / b); }

// ------------------------------------------------------ coarse moduli
__global__ void restrict_E3_kernel(double* Ec, const double* __restrict__ Ef, int nxf, int nyf,
                                   int nzf, int nxc, int nyc, int nzc) {
  const long H = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const long nh = (long)nxc * nyc * nzc;
  if (H >= nh) return;
  const int I = (int)(H % nxc), J = (int)((H / nxc) % nyc), K = (int)(H / ((long)nxc * nyc));
  const int perm[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
  double acc[6] = {0, 0, 0, 0, 0, 0};
  for (int dz = 0; dz < 2; ++dz)
    for (int dy = 0; dy < 2; ++dy)
      for (int dx = 0; dx < 2; ++dx) {
        const int fi = 2 * I + dx, fj = 2 * J + dy, fk = 2 * K + dz;
        if (fi >= nxf || fj >= nyf || fk >= nzf) continue;
        const long hf = ((long)fk * nyf + fj) * nxf + fi;
        const int dlt[3] = {dx, dy, dz};
        for (int s = 0; s < 6; ++s) {
          // centroid of the fine tetrahedron in coarse-cube units of 1/8
          int q[3];
          q[perm[s][0]] = 3;
          q[perm[s][1]] = 2;
          q[perm[s][2]] = 1;
          for (int a = 0; a < 3; ++a) q[a] += 4 * dlt[a];
          int p0 = 0;
          if (q[1] > q[p0]) p0 = 1;
          if (q[2] > q[p0]) p0 = 2;
          int p2 = 0;
          if (q[1] < q[p2]) p2 = 1;
          if (q[2] < q[p2]) p2 = 2;
          const int p1 = 3 - p0 - p2;
          const int t = 2 * p0 + (p1 > p2 ? 1 : 0);
          acc[t] += Ef[6 * hf + s];
        }
      }
  // mean of the 8 children (x 1/8), times 2 for the doubled cell size
  for (int t = 0; t < 6; ++t) Ec[6 * H + t] = acc[t] * 0.25;
}

__global__ void restrict_E2_kernel(double* Ec, const double* __restrict__ Ef, int nxf, int nyf,
                                   int uniform_f, int nxc, int nyc) {
  const long S = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (S >= (long)nxc * nyc) return;
  restrict_E2_square(S, Ec, Ef, nxf, nyf, uniform_f, nxc);
}

// ----------------------------------------------- transfer operators
// 3D restriction tiled through LDS: a block owns an 8 x 8 x 4 tile of coarse
// nodes; for each (load case, component) it stages the 17 x 17 x 9 fine
// nodes of (b - q) that the tile's basis supports cover (coalesced along x),
// then every thread sums its coarse node's 15 support points (the centre
// with weight 1, the 7 lattice directions d in {0,1}^3 \ 0 at +-d with
// weight 1/2) from LDS.  Same arithmetic and summation order as
// restrict_node.
constexpr int kRcx = 8, kRcy = 8, kRcz = 4;
constexpr int kRfx = 2 * kRcx + 1, kRfy = 2 * kRcy + 1, kRfz = 2 * kRcz + 1;

template <typename T>
__global__ __launch_bounds__(256) void restrict3d_tiled_kernel(T* bc, const T* __restrict__ bf,
                                                               const T* __restrict__ qf, OpDesc fo,
                                                               OpDesc co, int nrhs, const int* stop) {
  if (stop && *stop) return;
  __shared__ T tile[kRfz * kRfy * kRfx];
  const int tid = threadIdx.x;
  const int gx = (co.nx + 1 + kRcx - 1) / kRcx, gy = (co.ny + 1 + kRcy - 1) / kRcy;
  // blockIdx.y = load case * 3 + component: one staged field per block
  const int b = blockIdx.x;
  const int I0 = (b % gx) * kRcx, J0 = ((b / gx) % gy) * kRcy, K0 = (b / (gx * gy)) * kRcz;
  const int tx = tid % kRcx, ty = (tid / kRcx) % kRcy, tz = tid / (kRcx * kRcy);
  const int I = I0 + tx, J = J0 + ty, K = K0 + tz;
  const bool own = I <= co.nx && J <= co.ny && K <= co.nz;
  const long C = ((long)K * (co.ny + 1) + J) * (co.nx + 1) + I;
  const int cm = own ? co.mask[C] : 7;
  const int fx0 = 2 * I0 - 1, fy0 = 2 * J0 - 1, fz0 = 2 * K0 - 1;
  const int nxf1 = fo.nx + 1, nyf1 = fo.ny + 1;
  {
    {
      const int r = blockIdx.y / 3, c = blockIdx.y % 3;
      const long off = ((long)r * 3 + c) * fo.nn;
      for (int idx = tid; idx < kRfz * kRfy * kRfx; idx += 256) {
        const int a = idx % kRfx, bb = (idx / kRfx) % kRfy, cc = idx / (kRfx * kRfy);
        const int fi = fx0 + a, fj = fy0 + bb, fk = fz0 + cc;
        T v = T(0);
        if (fi >= 0 && fj >= 0 && fk >= 0 && fi <= fo.nx && fj <= fo.ny && fk <= fo.nz) {
          const long n = ((long)fk * nyf1 + fj) * nxf1 + fi;
          v = bf[off + n] - qf[off + n];
        }
        tile[idx] = v;
      }
      lds_barrier();
      if (own) {
        // local fine coordinates of the centre 2I, 2J, 2K
        const int li = 2 * tx + 1, lj = 2 * ty + 1, lk = 2 * tz + 1;
        T acc = tile[(lk * kRfy + lj) * kRfx + li];
        for (int dd = 1; dd <= 7; ++dd) {
          const int dx = dd & 1, dy = (dd >> 1) & 1, dz = (dd >> 2) & 1;
          for (int sgn = -1; sgn <= 1; sgn += 2)
            acc += T(0.5) * tile[((lk + sgn * dz) * kRfy + lj + sgn * dy) * kRfx + li + sgn * dx];
        }
        bc[((long)r * 3 + c) * co.nn + C] = ((cm >> c) & 1) ? T(0) : acc;
      }
    }
  }
  (void)nrhs;
}

// 3D restriction b_c = P^T (b - q) as a z-sweep: a block owns 32 x 8 coarse
// nodes of kRsZ coarse planes for one (load case, component); the fine
// residuals of its 65 x 17 fine columns pass through a ring of three fine
// planes in LDS, two new planes per coarse plane, rows loaded whole
// (coalesced).  Sums in the order of restrict_node.
constexpr int kRsX = 32, kRsY = 8, kRsZ = 8;
constexpr int kRsFx = 2 * kRsX + 1, kRsFy = 2 * kRsY + 1;
constexpr int kRsPlane = kRsFx * kRsFy;

template <typename T>
__global__ __launch_bounds__(256) void restrict3d_sweep_kernel(T* bc, const T* __restrict__ bf,
                                                               const T* __restrict__ qf, OpDesc fo,
                                                               OpDesc co, const int* stop) {
  if (stop && *stop) return;
  __shared__ T ring[3][kRsPlane];
  const int tid = threadIdx.x;
  const int gx = (co.nx + kRsX) / kRsX, gy = (co.ny + kRsY) / kRsY;
  const int b = blockIdx.x;
  const int I0 = (b % gx) * kRsX, J0 = ((b / gx) % gy) * kRsY, K0 = (b / (gx * gy)) * kRsZ;
  const int K1 = min(K0 + kRsZ, co.nz + 1);
  const int r = blockIdx.y / 3, c = blockIdx.y % 3;
  const long off = ((long)r * 3 + c) * fo.nn;
  const int nxf1 = fo.nx + 1, nyf1 = fo.ny + 1;
  const int fx0 = 2 * I0 - 1, fy0 = 2 * J0 - 1;
  // a fine plane in registers: b and q of the thread's plane slots
  constexpr int NQ = (kRsPlane + 255) / 256;
  struct Pl {
    T b[NQ], q[NQ];
  };
  auto fetch = [&](int fk, Pl& v) {
    const bool kin = fk >= 0 && fk <= fo.nz;
#pragma unroll
    for (int j = 0; j < NQ; ++j) {
      const int idx = tid + 256 * j;
      const int a = idx % kRsFx, bb = idx / kRsFx;
      const int fi = fx0 + a, fj = fy0 + bb;
      v.b[j] = T(0);
      v.q[j] = T(0);
      if (idx < kRsPlane && kin && fi >= 0 && fj >= 0 && fi <= fo.nx && fj <= fo.ny) {
        const long n = ((long)fk * nyf1 + fj) * nxf1 + fi;
        v.b[j] = bf[off + n];
        v.q[j] = qf[off + n];
      }
    }
  };
  auto store = [&](int fk, const Pl& v) {
    T* pl = ring[(fk + 3) % 3];
#pragma unroll
    for (int j = 0; j < NQ; ++j) {
      const int idx = tid + 256 * j;
      if (idx < kRsPlane) pl[idx] = v.b[j] - v.q[j];
    }
  };
  const int tx = tid % kRsX, ty = tid / kRsX;
  const int I = I0 + tx, J = J0 + ty;
  const bool colok = I <= co.nx && J <= co.ny;
  Pl va, vb;
  fetch(2 * K0 - 1, va);
  store(2 * K0 - 1, va);
  fetch(2 * K0, va);
  fetch(2 * K0 + 1, vb);
  for (int K = K0; K < K1; ++K) {
    store(2 * K, va);
    store(2 * K + 1, vb);
    __syncthreads();
    if (K + 1 < K1) {   // the next two planes load while this one is summed
      fetch(2 * K + 2, va);
      fetch(2 * K + 3, vb);
    }
    if (colok) {
      const int li = 2 * tx + 1, lj = 2 * ty + 1;
      const T* pm = ring[(2 * K - 1 + 3) % 3];
      const T* p0 = ring[(2 * K) % 3];
      const T* pp = ring[(2 * K + 1) % 3];
      T acc = p0[lj * kRsFx + li];
#pragma unroll
      for (int dd = 1; dd <= 7; ++dd) {
        const int dx = dd & 1, dy = (dd >> 1) & 1, dz = (dd >> 2) & 1;
        const T* lo = dz ? pm : p0;
        const T* hi = dz ? pp : p0;
        acc += T(0.5) * lo[(lj - dy) * kRsFx + li - dx];
        acc += T(0.5) * hi[(lj + dy) * kRsFx + li + dx];
      }
      const long C = ((long)K * (co.ny + 1) + J) * (co.nx + 1) + I;
      const int cm = co.mask[C];
      bc[((long)r * 3 + c) * co.nn + C] = ((cm >> c) & 1) ? T(0) : acc;
    }
    __syncthreads();   // the plane 2K+1 stays; the other two are overwritten next
  }
}

template <typename T>
__global__ void restrict_kernel(T* bc, const T* __restrict__ bf, const T* __restrict__ qf,
                                OpDesc fo, OpDesc co, int nrhs, const int* stop) {
  if (stop && *stop) return;
  const long C = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (C >= co.nn) return;
  restrict_node<T>(C, bc, bf, qf, fo, co, nrhs);
}

// x_f += P x_c, one thread per fine node (large grids): the same
// interpolation as prolong_node with the load-case and component loops
// unrolled, so all of a node's loads are in flight together
template <typename T, int NR, int DIM>
__global__ void prolong_add_kernel(T* __restrict__ xf, const T* __restrict__ xc, OpDesc fo,
                                   OpDesc co, const int* stop) {
  if (stop && *stop) return;
  const long n = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= fo.nn) return;
  const int nxf1 = fo.nx + 1, nyf1 = fo.ny + 1;
  const int i = (int)(n % nxf1), j = (int)((n / nxf1) % nyf1);
  const int k = DIM == 3 ? (int)(n / ((long)nxf1 * nyf1)) : 0;
  const int nxc1 = co.nx + 1, nyc1 = co.ny + 1;
  const long c0 = ((long)(k >> 1) * nyc1 + (j >> 1)) * nxc1 + (i >> 1);
  const long c1 = ((long)((k + 1) >> 1) * nyc1 + ((j + 1) >> 1)) * nxc1 + ((i + 1) >> 1);
  const bool even = ((i | j | k) & 1) == 0;
  const int fm = fo.mask[n];
  T a0[NR * DIM], a1[NR * DIM], xv[NR * DIM];
#pragma unroll
  for (int rc = 0; rc < NR * DIM; ++rc) {
    const T* xcr = xc + (long)rc * co.nn;
    a0[rc] = xcr[c0];
    a1[rc] = xcr[c1];
    xv[rc] = xf[(long)rc * fo.nn + n];
  }
#pragma unroll
  for (int rc = 0; rc < NR * DIM; ++rc) {
    if ((fm >> (rc % DIM)) & 1) continue;
    const T e = even ? a0[rc] : T(0.5) * (a0[rc] + a1[rc]);
    xf[(long)rc * fo.nn + n] = xv[rc] + e;
  }
}

template <typename T, int DIM>
static void prolong_large(hipStream_t s, T* xf, const T* xc, const OpDesc& fo, const OpDesc& co,
                          int nrhs, const int* stop) {
  const unsigned nb = cdivu(fo.nn, 256);
  switch (nrhs) {
    case 1: prolong_add_kernel<T, 1, DIM><<<nb, 256, 0, s>>>(xf, xc, fo, co, stop); break;
    case 2: prolong_add_kernel<T, 2, DIM><<<nb, 256, 0, s>>>(xf, xc, fo, co, stop); break;
    case 3: prolong_add_kernel<T, 3, DIM><<<nb, 256, 0, s>>>(xf, xc, fo, co, stop); break;
    default: prolong_add_kernel<T, 4, DIM><<<nb, 256, 0, s>>>(xf, xc, fo, co, stop); break;
  }
}

// x_f += P x_c, one thread per (fine node, load case and component
// = blockIdx.y): the same interpolation as prolong_node, each value in a
// thread of its own, for small grids where one thread per node leaves the
// chip nearly idle
template <typename T>
__global__ void prolong_add_split_kernel(T* xf, const T* __restrict__ xc, OpDesc fo, OpDesc co,
                                   const int* stop) {
  if (stop && *stop) return;
  const long n = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= fo.nn) return;
  const int dim = fo.dim;
  const int rc = blockIdx.y;   // r * dim + c
  const int c = rc % dim;
  if ((fo.mask[n] >> c) & 1) return;
  const int nxf1 = fo.nx + 1, nyf1 = fo.ny + 1;
  const int i = (int)(n % nxf1), j = (int)((n / nxf1) % nyf1);
  const int k = dim == 3 ? (int)(n / ((long)nxf1 * nyf1)) : 0;
  const int nxc1 = co.nx + 1, nyc1 = co.ny + 1;
  const long c0 = ((long)(k >> 1) * nyc1 + (j >> 1)) * nxc1 + (i >> 1);
  const long c1 = ((long)((k + 1) >> 1) * nyc1 + ((j + 1) >> 1)) * nxc1 + ((i + 1) >> 1);
  const bool even = ((i | j | k) & 1) == 0;
  const T* xcr = xc + (long)rc * co.nn;
  const T e = even ? xcr[c0] : T(0.5) * (xcr[c0] + xcr[c1]);
  xf[(long)rc * fo.nn + n] += e;
}

// ------------------------------------------------------- smoother
// mode 0: x = 0 on entry (r = b);  mode 1: r = b - q with q = K x
template <typename T>
__global__ void cheb_first_kernel(T* __restrict__ x, T* __restrict__ r, T* __restrict__ d,
                                  const T* __restrict__ b, const T* __restrict__ q,
                                  const T* __restrict__ invd, const double* lmax, long nd, int nrhs,
                                  int mode, double low, int kind, const int* stop) {
  if (stop && *stop) return;
  const T it = T(cheb_first_scale(*lmax, low, kind));
  // distinct vectors (restrict): the next element's loads may pass this
  // one's stores
#pragma unroll 2
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < nd; i += (long)gridDim.x * blockDim.x) {
    const T id = invd[i];
    for (int k = 0; k < nrhs; ++k) {
      const long j = (long)k * nd + i;
      const T rv = mode ? b[j] - q[j] : b[j];
      const T dv = it * id * rv;
      r[j] = rv;
      d[j] = dv;
      x[j] = mode ? x[j] + dv : dv;
    }
  }
}

template <typename T>
__global__ void cheb_next_kernel(T* __restrict__ x, T* __restrict__ r, T* __restrict__ d,
                                 const T* __restrict__ q, const T* __restrict__ invd,
                                 const double* lmax, long nd, int nrhs, ChebCoef cf, double low,
                                 const int* stop) {
  if (stop && *stop) return;
  double c1d, c2d;
  cheb_next_coef(*lmax, low, cf, c1d, c2d);
  const T c1 = T(c1d), c2 = T(c2d);
#pragma unroll 2
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < nd; i += (long)gridDim.x * blockDim.x) {
    const T id = invd[i];
    for (int k = 0; k < nrhs; ++k) {
      const long j = (long)k * nd + i;
      const T rv = r[j] - q[j];
      const T dv = c1 * d[j] + c2 * id * rv;
      r[j] = rv;
      d[j] = dv;
      x[j] += dv;
    }
  }
}

// ------------------------------------------------- lmax estimation
__global__ void power_init_kernel(double* v, const uint8_t* mask, long nn, int dim) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nn * dim) return;
  const long n = i % nn;
  const int c = (int)(i / nn);
  unsigned h = (unsigned)(i * 2654435761u) ^ 0x9e3779b9u;
  h ^= h >> 16;
  h *= 0x85ebca6bu;
  h ^= h >> 13;
  const double v0 = (double)(h & 0xffffff) / 16777216.0 - 0.5;
  v[i] = ((mask[n] >> c) & 1) ? 0.0 : v0;
}

// partial sums of v.(Kv) and v.(D v); then v <- scale * D^-1 (K v)
__global__ __launch_bounds__(256) void power_step_kernel(double* v, const double* __restrict__ w,
                                                         const double* __restrict__ invd, long nd,
                                                         const double* scale, double* partials) {
  const double sc = *scale;
  double acc[2] = {0.0, 0.0};
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < nd; i += (long)gridDim.x * blockDim.x) {
    const double id = invd[i];
    const double vi = v[i], wi = w[i];
    acc[0] += vi * wi;
    acc[1] += vi * vi / id;
    v[i] = sc * id * wi;
  }
  const double none[1] = {0.0};
  block_partials<2, 0>(acc, none, partials);
}

__global__ void power_fin_kernel(const double* partials, long nb, double* scale, double* lmax,
                                 int last, double safety) {
  __shared__ double tot[2];
  reduce_partials<2, 0>(partials, nb, tot);
  if (threadIdx.x == 0) {
    const double lam = (tot[1] > 0.0) ? tot[0] / tot[1] : 1.0;
    *scale = (lam > 0.0) ? 1.0 / lam : 1.0;
    if (last) *lmax = safety * lam;
  }
}

__global__ void set_scalar_kernel(double* p, double v) { *p = v; }

// ---------------------------------------------------- coarsest level
__global__ void coarse_assemble_kernel(double* A, const double* __restrict__ E, OpDesc o,
                                       double lam0, double mu0, double vol) {
  const int row = blockIdx.x * blockDim.x + threadIdx.x;
  if (row >= (int)(o.nn * o.dim)) return;
  coarse_assemble_row(row, A, E, o, lam0, mu0, vol);
}

__global__ __launch_bounds__(1024) void gauss_jordan_kernel(double* A, int n) {
  gauss_jordan_block(A, n);
}

template <typename T>
__global__ __launch_bounds__(512) void coarse_solve_kernel(T* x, const T* __restrict__ b,
                                                           const double* __restrict__ Ainv, int n,
                                                           int nrhs, const int* stop) {
  if (stop && *stop) return;
  coarse_solve_block<T>(x, b, Ainv, n, nrhs);
}

// ------------------------------------------ larger coarsest level (> 128 DOFs)
// The coarsest level of a deep hierarchy (12 x 6 x 6 cells, 1911 DOFs, on
// 192 x 96 x 96) is solved directly too: its padded matrix is assembled and
// inverted per solve by the symmetric block sweep of dense_dev.h, and each
// visit is one dense matrix-vector product over the whole GPU.  A revisit of a level solved exactly would change nothing, so
// the level above it never revisits (W) and the tail kernel is not used
// with it.
__global__ void dense_fill_kernel(double* A, int n, int np) {
  dense_fill_range(A, n, np, (long)blockIdx.x * blockDim.x + threadIdx.x,
                   (long)gridDim.x * blockDim.x);
}

__global__ void coarse_assemble_ld_kernel(double* A, const double* __restrict__ E, OpDesc o,
                                          double lam0, double mu0, double vol, int np) {
  const int row = blockIdx.x * blockDim.x + threadIdx.x;
  if (row >= (int)(o.nn * o.dim)) return;
  coarse_assemble_row(row, A, E, o, lam0, mu0, vol, np, false);
}

__global__ __launch_bounds__(kGjPivThreads) void gj_pivot_kernel(const double* __restrict__ A,
                                                                  int np, int k, double* P) {
  gj_pivot_block(A, np, k, P);
}

__global__ __launch_bounds__(kGjThreads) void sw_panel_kernel(const double* A, int np, int k,
                                                               const double* __restrict__ P,
                                                               double* C, double* R) {
  sw_panel_block(A, np, k, P, C, R, blockIdx.x);
}

// one work-group per block on or above the diagonal
__global__ __launch_bounds__(kGjThreads) void sw_update_kernel(double* A, int np, int k,
                                                                const double* __restrict__ P,
                                                                const double* __restrict__ C,
                                                                const double* __restrict__ R,
                                                                double* Pnext) {
  int i, j;
  sw_update_index(blockIdx.x, np / kGjB, k, i, j);
  sw_update_block(A, np, k, P, C, R, i, j, Pnext);
}

__global__ __launch_bounds__(kGjThreads) void sw_mirror_kernel(double* A, int np) {
  int i, j;
  sw_tri_index(blockIdx.x, i, j);
  sw_mirror_block(A, np, i, j);
}

template <typename T, typename TA>
__global__ __launch_bounds__(64 * kDenseWaves) void dense_solve_kernel(
    T* x, const T* __restrict__ b, const TA* __restrict__ Ainv, int n, int np, int nrhs,
    const int* stop) {
  if (stop && *stop) return;
  dense_solve_rows<T, TA>(x, b, Ainv, n, np, nrhs, blockIdx.x);
}

__global__ void to_f32_kernel(float* dst, const double* __restrict__ src, long n) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    dst[i] = (float)src[i];
}

// ------------------------------------------------------------ drivers
static const int* stop_flag(Ctx* c) { return c->smooth_always ? nullptr : &c->scal->pcg.done; }

void gmg_setup(Ctx* c) {
  hipStream_t s = c->stream;
  const int L = (int)c->lv.size();
  for (int l = 1; l < L; ++l) {
    const GmgLevel& f = c->lv[l - 1];
    GmgLevel& g = c->lv[l];
    if (g.op.dim == 3)
      restrict_E3_kernel<<<cdivu((long)g.op.nx * g.op.ny * g.op.nz, 256), 256, 0, s>>>(
          g.E, f.E, f.op.nx, f.op.ny, f.op.nz, g.op.nx, g.op.ny, g.op.nz);
    else
      restrict_E2_kernel<<<cdivu((long)g.op.nx * g.op.ny, 256), 256, 0, s>>>(
          g.E, f.E, f.op.nx, f.op.ny, f.op.split_uniform, g.op.nx, g.op.ny);
  }
  for (int l = 0; l + 1 < L; ++l) {
    GmgLevel& g = c->lv[l];
    launch_diagonal_op(c, g.op, g.E, g.invd, true);
    const long nd = g.op.nn * g.op.dim;
    const unsigned nb = red_grid(nd);
    power_init_kernel<<<cdivu(nd, 256), 256, 0, s>>>(g.pv, g.op.mask, g.op.nn, g.op.dim);
    set_scalar_kernel<<<1, 1, 0, s>>>(g.pscale, 1.0);
    const GmgParams& gp = c->gp;
    for (int it = 0; it < gp.power_iters; ++it) {
      launch_apply_op(c, g.op, g.E, g.pv, g.pw, 1, false, false, nullptr);
      power_step_kernel<<<nb, 256, 0, s>>>(g.pv, g.pw, g.invd, nd, g.pscale, c->partials);
      power_fin_kernel<<<1, 256, 0, s>>>(c->partials, nb, g.pscale, g.lmax,
                                         it == gp.power_iters - 1, gp.power_safety);
    }
  }
  if (c->prob.precision != TOPO_FP64) {
    for (int l = 0; l < L; ++l) {
      GmgLevel& g = c->lv[l];
      const long nd = g.op.nn * g.op.dim;
      if (l > 0) to_f32_kernel<<<red_grid(g.nc), 256, 0, s>>>(g.E32, g.E, g.nc);
      if (l + 1 < L) to_f32_kernel<<<red_grid(nd), 256, 0, s>>>(g.invd32, g.invd, nd);
    }
  }
  GmgLevel& cl = c->lv[L - 1];
  const int n = (int)(cl.op.nn * cl.op.dim);
  if (cl.np == 0) {
    coarse_assemble_kernel<<<cdivu(n, 128), 128, 0, s>>>(cl.Ainv, cl.E, cl.op, c->m.lam0, c->m.mu0,
                                                        c->m.vol);
    gauss_jordan_kernel<<<1, 1024, 0, s>>>(cl.Ainv, n);
    return;
  }
  const int np = cl.np, nb = np / kGjB;
  // two pivot inverses (step k reads one while its update writes the next)
  double* P2 = cl.gj;
  double* C = cl.gj + 2 * kGjB * kGjB;
  double* R = C + (long)np * kGjB;
  dense_fill_kernel<<<red_grid((long)np * np), 256, 0, s>>>(cl.Ainv, n, np);
  coarse_assemble_ld_kernel<<<cdivu(n, 64), 64, 0, s>>>(cl.Ainv, cl.E, cl.op, c->m.lam0, c->m.mu0,
                                                       c->m.vol, np);
  gj_pivot_kernel<<<1, kGjPivThreads, 0, s>>>(cl.Ainv, np, 0, P2);
  for (int k = 0; k < nb; ++k) {
    double* P = P2 + (k & 1) * kGjB * kGjB;
    double* Pn = k + 1 < nb ? P2 + ((k + 1) & 1) * kGjB * kGjB : nullptr;
    sw_panel_kernel<<<2 * nb, kGjThreads, 0, s>>>(cl.Ainv, np, k, P, C, R);
    sw_update_kernel<<<nb * (nb + 1) / 2, kGjThreads, 0, s>>>(cl.Ainv, np, k, P, C, R, Pn);
  }
  sw_mirror_kernel<<<nb * (nb + 1) / 2, kGjThreads, 0, s>>>(cl.Ainv, np);
  if (cl.Ainv32) to_f32_kernel<<<red_grid((long)np * np), 256, 0, s>>>(cl.Ainv32, cl.Ainv, (long)np * np);
}

// per-precision views of a level's operator data
template <typename T>
struct LevelOps;
template <>
struct LevelOps<double> {
  static const double* E(const GmgLevel& g) { return g.E; }
  static const double* invd(const GmgLevel& g) { return g.invd; }
  static void apply(Ctx* c, const GmgLevel& g, const double* x, double* y, int nrhs,
                    const int* stop) {
    launch_apply_op(c, g.op, g.E, x, y, nrhs, false, false, stop);
  }
};
template <>
struct LevelOps<float> {
  static const float* E(const GmgLevel& g) { return g.E32; }
  static const float* invd(const GmgLevel& g) { return g.invd32; }
  static void apply(Ctx* c, const GmgLevel& g, const float* x, float* y, int nrhs,
                    const int* stop) {
    // fine-level FP32 applies are the timed kernel of the mixed solves
    if (g.E16)
      launch_apply_op_bf16(c, g.op, g.E16, x, y, nrhs, g.op.nn == c->g.nn, stop);
    else
      launch_apply_op_f32(c, g.op, g.E32, x, y, nrhs, g.op.nn == c->g.nn, stop);
  }
};

template <typename T>
static void cheb_smooth(Ctx* c, GmgLevel& g, const T* b, T* x, int nrhs, bool from_zero) {
  hipStream_t s = c->stream;
  const long nd = g.op.nn * g.op.dim;
  const unsigned nb = red_grid(nd);
  const int* stop = stop_flag(c);
  T* gr = reinterpret_cast<T*>(g.r);
  T* gd = reinterpret_cast<T*>(g.d);
  T* gq = reinterpret_cast<T*>(g.q);
  const T* invd = LevelOps<T>::invd(g);
  const GmgParams& gp = c->gp;
  if (from_zero && g.op.dim == 3 && gp.cheb_degree == 2) {
    // the whole degree-2 smoothing from zero in one kernel
    const double sigma = (1.0 + gp.cheb_low) / (1.0 - gp.cheb_low);
    const double rho_prev = 1.0 / sigma, rho = 1.0 / (2.0 * sigma - rho_prev);
    if constexpr (std::is_same<T, float>::value) {
      if (g.E16) {
        launch_apply_cheb_pre3d_bf16(c, g.op, g.E16, b, x, invd, g.lmax, rho, rho_prev,
                                     gp.cheb_low, gp.cheb_kind, nrhs, stop);
        return;
      }
    }
    launch_apply_cheb_pre3d<T>(c, g.op, LevelOps<T>::E(g), b, x, invd, g.lmax, rho, rho_prev,
                               gp.cheb_low, gp.cheb_kind, nrhs, stop);
    return;
  }
  const int degree = from_zero ? gp.cheb_degree : gp.post_degree;
  if (degree == 0) return;
  if (!from_zero && g.op.dim == 3 && degree == 2 && gp.fused_post) {
    // degree-2 smoothing from the given x in two fused kernels
    const double sigma = (1.0 + gp.cheb_low) / (1.0 - gp.cheb_low);
    const double rho_prev = 1.0 / sigma, rho = 1.0 / (2.0 * sigma - rho_prev);
    const uint16_t* e16 = nullptr;
    if constexpr (std::is_same<T, float>::value) e16 = g.E16;
    launch_apply_cheb_post3d<T>(c, g.op, LevelOps<T>::E(g), e16, x, b, gr, gd, invd, g.lmax, rho,
                                rho_prev, gp.cheb_low, gp.cheb_kind, nrhs, stop);
    return;
  }
  if (!from_zero) LevelOps<T>::apply(c, g, x, gq, nrhs, stop);
  cheb_first_kernel<T><<<nb, 256, 0, s>>>(x, gr, gd, b, gq, invd, g.lmax, nd, nrhs,
                                          from_zero ? 0 : 1, gp.cheb_low, gp.cheb_kind, stop);
  const double sigma = (1.0 + gp.cheb_low) / (1.0 - gp.cheb_low);
  double rho_prev = 1.0 / sigma;
  for (int k = 1; k < degree; ++k) {
    const double rho = 1.0 / (2.0 * sigma - rho_prev);
    LevelOps<T>::apply(c, g, gd, gq, nrhs, stop);
    ChebCoef cf{rho, rho_prev, gp.cheb_kind, k};
    cheb_next_kernel<T><<<nb, 256, 0, s>>>(x, gr, gd, gq, invd, g.lmax, nd, nrhs, cf, gp.cheb_low,
                                           stop);
    rho_prev = rho;
  }
}

// Whether level l visits its coarse level a second time (W-cycle).
static bool revisits(const Ctx* c, int l, int wlevels) {
  const int L = (int)c->lv.size();
  if (l + 2 >= L) return false;   // the coarsest level is solved directly
  const GmgLevel& h = c->lv[l + 1];
  return wlevels >= 0 ? l < wlevels : (h.op.dim == 3 && h.op.nn >= kWCoarseNodes);
}

// ------------------------------------------------ coarse tail, one work-group
// From the first 3D coarse level whose vectors fit in LDS down to the
// coarsest, a level's kernels last a few microseconds each and the gaps
// between dependent launches cost as much again.  There the FP32 cycle
// runs in one work-group per load case (the cycle acts on each load case
// on its own), with every vector, the moduli, D^-1 and the masks of those
// levels staged in LDS: smoothing, residual and restriction, the direct
// coarsest solve, prolongation and any W revisits, one phase after another
// with work-group barriers in between.  The phases compute what the
// per-level kernels compute, in the same order, except the operator's node
// sums: a cube pass writes each cube's 8 corner forces (the same
// cube_force) to LDS, then a node pass adds the forces of a node's cubes in
// corner order.  Every result is the same on every run.
constexpr int kTailMaxLevels = 8;
constexpr int kTailMaxOps = 192;
constexpr int kTailLdsFloats = 36864;   // 144 KiB, and 8 KiB for the coarsest solve's partial sums
constexpr int kTailCoarseSplit = 8;     // partial sums per coarsest-level row
constexpr int kTailThreads = 1024;
enum TailOpKind : uint8_t { kTailSmooth0, kTailSmoothX, kTailRestrict, kTailCoarse, kTailProlong };
struct TailOp {
  uint8_t kind, level;   // level relative to the tail's first level
};

// one level of one load case, pointers into LDS
struct TailLevel {
  int nx, ny, nz, nn;
  float rnx, rnxy, rnx1, rpl;   // 1/nx, 1/(nx ny), 1/(nx+1), 1/((nx+1)(ny+1))
  const uint8_t* mask;
  const float* E;      // [6 * cubes] moduli of the unit-cell kernels
  const float* invd;   // [3 * nn]
  float *b, *x, *r, *d, *q;   // [3][nn] (r, d, q unused on the coarsest level)
};

struct TailLevelSrc {
  int nx, ny, nz, nn;
  float rnx, rnxy, rnx1, rpl;
  const uint8_t* mask;   // global
  const float* E;
  const float* invd;
  const double* lmax;
  // LDS offsets in floats (mask: in bytes)
  int o_mask, o_E, o_invd, o_b, o_x, o_r, o_d, o_q;
};

struct TailArgs {
  TailLevelSrc lv[kTailMaxLevels];
  int nlev;
  const float* b0;      // first level's right-hand side, [nrhs][3][nn] (global)
  float* x0;            // and its solution
  int x0_zero;          // start from x = 0
  const double* Ainv;   // coarsest level: dense inverse
  int o_F;              // LDS corner forces [24][cubes of the first level]
  float lam, mu;        // lambda0 |T|, mu0 |T| of the unit cell
  double low;
  double rc[8], rp[8];  // first-kind recurrence coefficients of steps 1..7
  int kind, deg0, degx; // Chebyshev kind, degree from zero, degree from x
  int ncoarse, nops;
  TailOp ops[kTailMaxOps];
};

__device__ inline TailLevel tail_view(const TailArgs& A, int l, float* lds) {
  const TailLevelSrc& s = A.lv[l];
  TailLevel v;
  v.nx = s.nx;
  v.ny = s.ny;
  v.nz = s.nz;
  v.nn = s.nn;
  v.rnx = s.rnx;
  v.rnxy = s.rnxy;
  v.rnx1 = s.rnx1;
  v.rpl = s.rpl;
  v.mask = reinterpret_cast<const uint8_t*>(lds) + s.o_mask;
  v.E = lds + s.o_E;
  v.invd = lds + s.o_invd;
  v.b = lds + s.o_b;
  v.x = lds + s.o_x;
  v.r = lds + s.o_r;
  v.d = lds + s.o_d;
  v.q = lds + s.o_q;
  return v;
}

// floor(a / b) for 0 <= a < 2^22 from the rounded reciprocal rb = 1/b:
// a/b + 0.5/b stays at least 0.5/b away from an integer
__device__ __forceinline__ int tail_div(int a, float rb) {
  return (int)(((float)a + 0.5f) * rb);
}

// node (i, j, k) of index n on a level
__device__ __forceinline__ void tail_node_ijk(const TailLevel& L, int n, int& i, int& j, int& k) {
  k = tail_div(n, L.rpl);
  const int rem = n - k * (L.nx + 1) * (L.ny + 1);
  j = tail_div(rem, L.rnx1);
  i = rem - j * (L.nx + 1);
}

// K v on one level (v is zero on fixed DOFs; fixed rows give 0), the whole
// block.  3D: cubes of six Kuhn tetrahedra (cube_force, 24 corner values);
// 2D: squares of two diagonal-A triangles, as on every coarse 2D level
// (square_force, 8 corner values).  What the node pass does with K v at its
// node:
//   EPI 0: q = K v;
//   EPI 1 (first Chebyshev step from x, v = x): r = b - K x, d = s D^-1 r, x += d;
//   EPI 2 (next Chebyshev step, v = d): r -= K d, d = c1 d + c2 D^-1 r, x += d.
// The node pass writes v only at its own node, after the barrier that ends
// the cell pass, so the in-place updates are safe.
template <int DIM, int EPI>
__device__ void tail_apply(const TailLevel& L, const float* v, float* F, float lam0, float mu0,
                           float s1 = 0.f, float s2 = 0.f) {
  constexpr int NC = DIM == 3 ? 8 : 4;   // corners per cell
  const int nx = L.nx, ny = L.ny, nz = DIM == 3 ? L.nz : 1, nn = L.nn;
  const int ncell = nx * ny * nz, nx1 = nx + 1, pl = (nx + 1) * (ny + 1);
  for (int h = threadIdx.x; h < ncell; h += blockDim.x) {
    int i, j, k;
    if (DIM == 3) {
      k = tail_div(h, L.rnxy);
      const int rem = h - k * nx * ny;
      j = tail_div(rem, L.rnx);
      i = rem - j * nx;
    } else {
      k = 0;
      j = tail_div(h, L.rnx);
      i = h - j * nx;
    }
    float u[NC][DIM], f[NC][DIM];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      const int node = (k + (c >> 2)) * pl + (j + ((c >> 1) & 1)) * nx1 + i + (c & 1);
#pragma unroll
      for (int a = 0; a < DIM; ++a) u[c][a] = v[a * nn + node];
    }
    if constexpr (DIM == 3) {
      float lam[6], mu[6];
#pragma unroll
      for (int t = 0; t < 6; ++t) {
        const float e = L.E[6 * h + t];
        lam[t] = lam0 * e;
        mu[t] = mu0 * e;
      }
      cube_force<float>(u, lam, mu, f);
    } else {
      const float e0 = L.E[2 * h], e1 = L.E[2 * h + 1];
#pragma unroll
      for (int c = 0; c < NC; ++c) f[c][0] = f[c][1] = 0.f;
      square_force<float>(true, u, lam0 * e0, mu0 * e0, lam0 * e1, mu0 * e1, f);
    }
#pragma unroll
    for (int c = 0; c < NC; ++c)
#pragma unroll
      for (int a = 0; a < DIM; ++a) F[(c * DIM + a) * ncell + h] = f[c][a];
  }
  __syncthreads();
  for (int n = threadIdx.x; n < nn; n += blockDim.x) {
    int i, j, k;
    tail_node_ijk(L, n, i, j, k);
    const int m = L.mask[n];
    float acc[DIM];
#pragma unroll
    for (int a = 0; a < DIM; ++a) acc[a] = 0.f;
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      // the node is corner c of the cell at (i, j, k) - c
      const int ci = i - (c & 1), cj = j - ((c >> 1) & 1), ck = k - (c >> 2);
      if (ci < 0 || cj < 0 || ck < 0 || ci >= nx || cj >= ny || ck >= nz) continue;
      const int h = (ck * ny + cj) * nx + ci;
#pragma unroll
      for (int a = 0; a < DIM; ++a) acc[a] += F[(c * DIM + a) * ncell + h];
    }
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
      const int e = a * nn + n;
      const float kv = ((m >> a) & 1) ? 0.f : acc[a];
      if (EPI == 0) {
        L.q[e] = kv;
      } else if (EPI == 1) {
        const float rv = L.b[e] - kv;
        const float dv = s1 * L.invd[e] * rv;
        L.r[e] = rv;
        L.d[e] = dv;
        L.x[e] = L.x[e] + dv;
      } else {
        const float rv = L.r[e] - kv;
        const float dv = s1 * L.d[e] + s2 * L.invd[e] * rv;
        L.r[e] = rv;
        L.d[e] = dv;
        L.x[e] += dv;
      }
    }
  }
  __syncthreads();
}

// Chebyshev smoothing of one level from x = 0 or from x (the steps of
// cheb_first_kernel and cheb_next_kernel)
template <int DIM>
__device__ void tail_smooth(const TailArgs& A, const TailLevel& L, double lmax, float* F,
                            bool from_zero) {
  const int degree = from_zero ? A.deg0 : A.degx;
  if (degree == 0) return;
  const float it = float(cheb_first_scale(lmax, A.low, A.kind));
  if (from_zero) {
    for (int j = threadIdx.x; j < DIM * L.nn; j += blockDim.x) {
      const float rv = L.b[j];
      const float dv = it * L.invd[j] * rv;
      L.r[j] = rv;
      L.d[j] = dv;
      L.x[j] = dv;
    }
    __syncthreads();
  } else {
    tail_apply<DIM, 1>(L, L.x, F, A.lam, A.mu, it);
  }
  for (int k = 1; k < degree; ++k) {
    double c1d, c2d;
    cheb_next_coef(lmax, A.low, ChebCoef{A.rc[k], A.rp[k], A.kind, k}, c1d, c2d);
    tail_apply<DIM, 2>(L, L.d, F, A.lam, A.mu, float(c1d), float(c2d));
  }
}

// coarse b = P^T (b - K x) of the fine level (restrict_node's sums: the
// centre, then the lattice directions d in {0,1}^DIM \ 0 at -d and +d)
template <int DIM>
__device__ void tail_restrict(const TailArgs& A, const TailLevel& Fl, const TailLevel& Cl, float* F) {
  tail_apply<DIM, 0>(Fl, Fl.x, F, A.lam, A.mu);
  constexpr int NDIR = DIM == 3 ? 7 : 3;
  const int nxf1 = Fl.nx + 1, nyf1 = Fl.ny + 1, nzf = DIM == 3 ? Fl.nz : 0;
  for (int C = threadIdx.x; C < Cl.nn; C += blockDim.x) {
    int I, J, K;
    tail_node_ijk(Cl, C, I, J, K);
    const int cm = Cl.mask[C];
#pragma unroll
    for (int c = 0; c < DIM; ++c) {
      const float* bf = Fl.b + c * Fl.nn;
      const float* qf = Fl.q + c * Fl.nn;
      float acc = 0.f;
      if (2 * I <= Fl.nx && 2 * J <= Fl.ny && 2 * K <= nzf) {
        const int n = ((2 * K) * nyf1 + 2 * J) * nxf1 + 2 * I;
        acc += bf[n] - qf[n];
      }
      for (int dd = 1; dd <= NDIR; ++dd) {
        const int dx = dd & 1, dy = (dd >> 1) & 1, dz = (dd >> 2) & 1;
        for (int sgn = -1; sgn <= 1; sgn += 2) {
          const int fi = 2 * I + sgn * dx, fj = 2 * J + sgn * dy, fk = 2 * K + sgn * dz;
          if (fi < 0 || fj < 0 || fk < 0 || fi > Fl.nx || fj > Fl.ny || fk > nzf) continue;
          const int n = (fk * nyf1 + fj) * nxf1 + fi;
          acc += 0.5f * (bf[n] - qf[n]);
        }
      }
      Cl.b[c * Cl.nn + C] = ((cm >> c) & 1) ? 0.f : acc;
    }
  }
  __syncthreads();
}

// fine x += P (coarse x) (prolong_add_split_kernel's interpolation)
template <int DIM>
__device__ void tail_prolong(const TailLevel& Fl, const TailLevel& Cl) {
  const int nxc1 = Cl.nx + 1, nyc1 = Cl.ny + 1;
  for (int n = threadIdx.x; n < Fl.nn; n += blockDim.x) {
    int i, j, k;
    tail_node_ijk(Fl, n, i, j, k);
    const int m = Fl.mask[n];
    const int c0 = ((k >> 1) * nyc1 + (j >> 1)) * nxc1 + (i >> 1);
    const int c1 = (((k + 1) >> 1) * nyc1 + ((j + 1) >> 1)) * nxc1 + ((i + 1) >> 1);
    const bool even = ((i | j | k) & 1) == 0;
#pragma unroll
    for (int c = 0; c < DIM; ++c) {
      if ((m >> c) & 1) continue;
      const float* xcr = Cl.x + c * Cl.nn;
      const float e = even ? xcr[c0] : 0.5f * (xcr[c0] + xcr[c1]);
      Fl.x[c * Fl.nn + n] += e;
    }
  }
  __syncthreads();
}

// x = Ainv b on the coarsest level (n <= 128): each row's dot product in
// kTailCoarseSplit strided partial sums, then their sum in order
__device__ void tail_coarse(const double* __restrict__ Ainv, int n, float* x, const float* b,
                            double* red) {
  for (int t = threadIdx.x; t < n * kTailCoarseSplit; t += blockDim.x) {
    const int i = t % n, p = t / n;
    double acc = 0.0;
    for (int j = p; j < n; j += kTailCoarseSplit) acc += Ainv[(long)j * n + i] * (double)b[j];
    red[p * n + i] = acc;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    double acc = 0.0;
    for (int p = 0; p < kTailCoarseSplit; ++p) acc += red[p * n + i];
    x[i] = float(acc);
  }
  __syncthreads();
}

// one work-group per load case (blockIdx.x)
template <int DIM>
__global__ __launch_bounds__(kTailThreads) void gmg_tail_kernel(TailArgs A, const int* stop) {
  if (stop && *stop) return;
  __shared__ float lds[kTailLdsFloats];
  __shared__ double red[kTailCoarseSplit * 128];
  const int r = blockIdx.x;
  uint8_t* lmask = reinterpret_cast<uint8_t*>(lds);
  // stage the levels' moduli, D^-1 and masks, and the first level's b (and x)
  for (int l = 0; l < A.nlev; ++l) {
    const TailLevelSrc& s = A.lv[l];
    const int nE = DIM == 3 ? 6 * s.nx * s.ny * s.nz : 2 * s.nx * s.ny;
    for (int n = threadIdx.x; n < s.nn; n += blockDim.x) lmask[s.o_mask + n] = s.mask[n];
    if (l + 1 < A.nlev) {
      for (int i = threadIdx.x; i < nE; i += blockDim.x) lds[s.o_E + i] = s.E[i];
      for (int i = threadIdx.x; i < DIM * s.nn; i += blockDim.x) lds[s.o_invd + i] = s.invd[i];
    }
  }
  {
    const TailLevelSrc& s = A.lv[0];
    const long off = (long)r * DIM * s.nn;
    for (int i = threadIdx.x; i < DIM * s.nn; i += blockDim.x) {
      lds[s.o_b + i] = A.b0[off + i];
      if (!A.x0_zero) lds[s.o_x + i] = A.x0[off + i];
    }
  }
  __syncthreads();
  float* F = lds + A.o_F;
  for (int o = 0; o < A.nops; ++o) {
    const TailOp op = A.ops[o];
    const TailLevel L = tail_view(A, op.level, lds);
    switch (op.kind) {
      case kTailSmooth0: tail_smooth<DIM>(A, L, *A.lv[op.level].lmax, F, true); break;
      case kTailSmoothX: tail_smooth<DIM>(A, L, *A.lv[op.level].lmax, F, false); break;
      case kTailRestrict: tail_restrict<DIM>(A, L, tail_view(A, op.level + 1, lds), F); break;
      case kTailProlong: tail_prolong<DIM>(L, tail_view(A, op.level + 1, lds)); break;
      default: tail_coarse(A.Ainv, A.ncoarse, L.x, L.b, red); break;
    }
  }
  {
    const TailLevelSrc& s = A.lv[0];
    const long off = (long)r * DIM * s.nn;
    for (int i = threadIdx.x; i < DIM * s.nn; i += blockDim.x) A.x0[off + i] = lds[s.o_x + i];
  }
}

// LDS layout of the levels from l0 down (floats; false if it does not fit)
static bool tail_layout(const Ctx* c, int l0, TailArgs& A) {
  const int L = (int)c->lv.size();
  if (L - l0 > kTailMaxLevels) return false;
  int mask_bytes = 0;
  for (int l = l0; l < L; ++l) mask_bytes += (int)c->lv[l].op.nn;
  int o = (mask_bytes + 15) / 16 * 4;   // masks first, 16-byte aligned
  int mb = 0;
  A.nlev = L - l0;
  for (int l = l0; l < L; ++l) {
    const OpDesc& d = c->lv[l].op;
    TailLevelSrc& s = A.lv[l - l0];
    const int nn = (int)d.nn, nd = d.dim * nn;
    const int nE = d.dim == 3 ? 6 * d.nx * d.ny * d.nz : 2 * d.nx * d.ny;
    const bool last = l + 1 == L;
    s.o_mask = mb;
    mb += nn;
    s.o_b = o;
    o += nd;
    s.o_x = o;
    o += nd;
    if (!last) {
      s.o_r = o;
      o += nd;
      s.o_d = o;
      o += nd;
      s.o_q = o;
      o += nd;
      s.o_E = o;
      o += nE;
      s.o_invd = o;
      o += nd;
    }
  }
  const OpDesc& d0 = c->lv[l0].op;
  A.o_F = o;
  o += d0.dim == 3 ? 24 * d0.nx * d0.ny * d0.nz : 8 * d0.nx * d0.ny;
  return o <= kTailLdsFloats;
}

// first level of the one-block tail (FP32 cycles), or -1
static int tail_level(const Ctx* c) {
  const int L = (int)c->lv.size();
  if (L < 2 || !c->gp.tail || c->lv[L - 1].np > 0) return -1;
  static thread_local TailArgs probe;
  for (int l = 1; l + 1 < L; ++l)
    if (tail_layout(c, l, probe)) return l;
  return -1;
}

// the tail's phases, in the order of vcycle_level's recursion
static bool tail_program(const Ctx* c, int l, int l0, bool x_zero, int wlevels,
                         std::vector<TailOp>& ops) {
  const int L = (int)c->lv.size();
  const uint8_t rl = (uint8_t)(l - l0);
  if (l == L - 1) {
    ops.push_back({kTailCoarse, rl});
    return true;
  }
  ops.push_back({x_zero ? (uint8_t)kTailSmooth0 : (uint8_t)kTailSmoothX, rl});
  ops.push_back({kTailRestrict, rl});
  if (!tail_program(c, l + 1, l0, true, wlevels, ops)) return false;
  if (revisits(c, l, wlevels) && !tail_program(c, l + 1, l0, false, wlevels, ops)) return false;
  ops.push_back({kTailProlong, rl});
  ops.push_back({kTailSmoothX, rl});
  return (int)ops.size() <= kTailMaxOps;
}

// the cycle of levels l0.. from x_zero, then (visits = 2) once more from
// its result, in one launch
static bool launch_tail(Ctx* c, int l0, const float* b, float* x, int nrhs, bool x_zero,
                        int wlevels, int visits) {
  std::vector<TailOp> ops;
  if (!tail_program(c, l0, l0, x_zero, wlevels, ops)) return false;
  if (visits == 2 && !tail_program(c, l0, l0, false, wlevels, ops)) return false;
  const int L = (int)c->lv.size();
  const GmgParams& gp = c->gp;
  if (gp.cheb_degree > 8 || gp.post_degree > 8) return false;
  TailArgs A;
  memset(&A, 0, sizeof(A));
  if (!tail_layout(c, l0, A)) return false;
  for (int l = l0; l < L; ++l) {
    const GmgLevel& g = c->lv[l];
    TailLevelSrc& s = A.lv[l - l0];
    s.nx = g.op.nx;
    s.ny = g.op.ny;
    s.nz = g.op.nz;
    s.nn = (int)g.op.nn;
    s.rnx = float(1.0 / s.nx);
    s.rnxy = float(1.0 / ((double)s.nx * s.ny));
    s.rnx1 = float(1.0 / (s.nx + 1));
    s.rpl = float(1.0 / ((double)(s.nx + 1) * (s.ny + 1)));
    s.mask = g.op.mask;
    s.E = g.E32;
    s.invd = g.invd32;
    s.lmax = g.lmax;
  }
  A.b0 = b;
  A.x0 = x;
  A.x0_zero = x_zero ? 1 : 0;
  A.Ainv = c->lv[L - 1].Ainv;
  A.lam = float(c->m.lam0 * c->m.vol);
  A.mu = float(c->m.mu0 * c->m.vol);
  A.low = gp.cheb_low;
  const double sigma = (1.0 + gp.cheb_low) / (1.0 - gp.cheb_low);
  double rho_prev = 1.0 / sigma;
  for (int k = 1; k < 8; ++k) {
    const double rho = 1.0 / (2.0 * sigma - rho_prev);
    A.rc[k] = rho;
    A.rp[k] = rho_prev;
    rho_prev = rho;
  }
  A.kind = gp.cheb_kind;
  A.deg0 = gp.cheb_degree;
  A.degx = gp.post_degree;
  const int dim = c->lv[l0].op.dim;
  A.ncoarse = (int)(c->lv[L - 1].op.nn * dim);
  if (A.ncoarse > 128) return false;
  A.nops = (int)ops.size();
  for (size_t i = 0; i < ops.size(); ++i) A.ops[i] = ops[i];
  if (dim == 3)
    gmg_tail_kernel<3><<<nrhs, kTailThreads, 0, c->stream>>>(A, stop_flag(c));
  else
    gmg_tail_kernel<2><<<nrhs, kTailThreads, 0, c->stream>>>(A, stop_flag(c));
  return true;
}

// One cycle at level l for K x = b, from x = 0 (x_zero) or from the given x.
// Levels below wlevels (wlevels < 0: 3D levels whose coarse level has at
// least kWCoarseNodes nodes) visit their coarse level twice, a W-cycle on
// those levels; the second visit starts from the first one's result.  Every
// level's operator is the Galerkin one, so a cycle's error operator is
// K-symmetric with spectrum in [0, 1) and the repeated coarse correction
// stays positive definite.  The coarsest level is solved directly and never
// revisited.
template <typename T>
static void vcycle_level(Ctx* c, int l, const T* b, T* x, int nrhs, bool x_zero, int wlevels) {
  hipStream_t s = c->stream;
  const int L = (int)c->lv.size();
  GmgLevel& g = c->lv[l];
  const int* stop = stop_flag(c);
  if (l == L - 1) {
    // the direct coarsest solve does not depend on the start
    const int n = (int)(g.op.nn * g.op.dim);
    if (g.np == 0) {
      coarse_solve_kernel<T><<<1, 512, 0, s>>>(x, b, g.Ainv, n, nrhs, stop);
    } else if constexpr (std::is_same<T, float>::value) {
      dense_solve_kernel<float, float><<<cdivu(n, kDenseWaves), 64 * kDenseWaves,
                                         (size_t)nrhs * g.np * sizeof(float), s>>>(
          x, b, g.Ainv32, n, g.np, nrhs, stop);
    } else {
      dense_solve_kernel<double, double><<<cdivu(n, kDenseWaves), 64 * kDenseWaves,
                                           (size_t)nrhs * g.np * sizeof(double), s>>>(
          x, b, g.Ainv, n, g.np, nrhs, stop);
    }
    return;
  }
  if constexpr (std::is_same<T, float>::value) {
    if (l == tail_level(c) && launch_tail(c, l, b, x, nrhs, x_zero, wlevels, 1)) return;
  }
  GmgLevel& h = c->lv[l + 1];
  T* hb = reinterpret_cast<T*>(h.b);
  T* hx = reinterpret_cast<T*>(h.x);
  T* gq = reinterpret_cast<T*>(g.q);
  cheb_smooth<T>(c, g, b, x, nrhs, x_zero);
  LevelOps<T>::apply(c, g, x, gq, nrhs, stop);
  if (g.op.dim == 3 && h.op.nn >= 65536) {
    // large coarse grids: the z-sweep (fine planes read once, whole rows)
    const long tiles = (long)cdivu(h.op.nx + 1, kRsX) * cdivu(h.op.ny + 1, kRsY) * cdivu(h.op.nz + 1, kRsZ);
    restrict3d_sweep_kernel<T><<<dim3((unsigned)tiles, 3 * nrhs), 256, 0, s>>>(hb, b, gq, g.op, h.op,
                                                                              stop);
  } else if (g.op.dim == 3) {
    // small coarse grids: one 8 x 8 x 4 tile per block, more blocks
    const long tiles = (long)cdivu(h.op.nx + 1, kRcx) * cdivu(h.op.ny + 1, kRcy) * cdivu(h.op.nz + 1, kRcz);
    restrict3d_tiled_kernel<T><<<dim3((unsigned)tiles, 3 * nrhs), 256, 0, s>>>(hb, b, gq, g.op, h.op,
                                                                              nrhs, stop);
  } else {
    restrict_kernel<T><<<cdivu(h.op.nn, 256), 256, 0, s>>>(hb, b, gq, g.op, h.op, nrhs, stop);
  }
  const bool twice = revisits(c, l, wlevels);
  bool in_tail = false;
  if constexpr (std::is_same<T, float>::value) {
    // both visits of a tail level in one launch
    if (l + 1 == tail_level(c)) in_tail = launch_tail(c, l + 1, hb, hx, nrhs, true, wlevels, twice ? 2 : 1);
  }
  if (!in_tail) {
    vcycle_level<T>(c, l + 1, hb, hx, nrhs, true, wlevels);
    if (twice) vcycle_level<T>(c, l + 1, hb, hx, nrhs, false, wlevels);
  }
  if (g.op.nn >= 262144) {
    if (g.op.dim == 3) prolong_large<T, 3>(s, x, hx, g.op, h.op, nrhs, stop);
    else prolong_large<T, 2>(s, x, hx, g.op, h.op, nrhs, stop);
  } else
    prolong_add_split_kernel<T><<<dim3(cdivu(g.op.nn, 256), g.op.dim * nrhs), 256, 0, s>>>(
        x, hx, g.op, h.op, stop);
  cheb_smooth<T>(c, g, b, x, nrhs, false);
}

void gmg_vcycle(Ctx* c, const double* b, double* x, int nrhs) {
  vcycle_level<double>(c, 0, b, x, nrhs, true, c->gp.wlevels);
}

void gmg_vcycle_f32(Ctx* c, const float* b, float* x, int nrhs) {
  vcycle_level<float>(c, 0, b, x, nrhs, true, c->gp.wlevels);
}

// the fine-level Chebyshev-Jacobi smoother on its own (FP64)
void gmg_fine_smooth(Ctx* c, const double* b, double* x, int nrhs, bool from_zero) {
  cheb_smooth<double>(c, c->lv[0], b, x, nrhs, from_zero);
}

}  // namespace topo
