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
// Input contract: x is zero on fixed DOFs (every internal vector is; the
// exported apply masks its input first).  Cells outside the grid get a zero
// modulus, so the clamped halo reads never reach an owned node.
#include "common.h"
#include "element.h"
#include "shared_dev.h"
#include "topo_internal.h"

namespace topo {

constexpr int TILE = 15;       // owned nodes per tile edge
constexpr int PATCH = 17;      // staged node patch edge
constexpr int PATCH2 = PATCH * PATCH;

static inline unsigned cdiv(long a, long b) { return (unsigned)((a + b - 1) / b); }


// Block -> (tile, load case) map.  Work-groups are handed to the 8 XCDs
// round-robin by linear id, so id % 8 selects the XCD.  Each XCD gets a
// contiguous range of tiles (neighbouring tiles share halo nodes in the
// same L2), and the nrhs blocks of one tile are consecutive on that XCD (they
// read the same moduli while they are still in L2).
struct TileMap {
  int gx, gy, gz;     // tiles per axis
  int per_xcd;        // tiles per XCD
  int nrhs;
};

__device__ __forceinline__ bool map_block(const TileMap& tm, int& bx, int& by, int& bz, int& rhs) {
  const int b = blockIdx.x;
  const int xcd = b & 7;
  const int k = b >> 3;
  rhs = k % tm.nrhs;
  const int tl = k / tm.nrhs;
  if (tl >= tm.per_xcd) return false;
  const int tile = xcd * tm.per_xcd + tl;
  const int ntiles = tm.gx * tm.gy * tm.gz;
  if (tile >= ntiles) return false;
  bx = tile % tm.gx;
  by = (tile / tm.gx) % tm.gy;
  bz = tile / (tm.gx * tm.gy);
  return true;
}

__device__ __forceinline__ void dot_partials(double dot, int rhs, double* partials) {
  double acc[kMaxRhs];
#pragma unroll
  for (int r = 0; r < kMaxRhs; ++r) acc[r] = (r == rhs) ? dot : 0.0;
  const double none[1] = {0.0};
  block_partials<kMaxRhs, 0>(acc, none, partials);
}

// -------------------------------------------------------------- 2D apply
template <typename T, typename TE>
__global__ __launch_bounds__(256) void apply2d_kernel(const T* __restrict__ x, T* __restrict__ y,
                                                      const TE* __restrict__ E, OpDesc d,
                                                      TileMap tm, T lam0, T mu0, double* partials,
                                                      const int* stop) {
  if (stop && *stop) return;
  int bx, by, bz, rhs;
  const bool live = map_block(tm, bx, by, bz, rhs);
  if (!live && !partials) return;
  const double dot = apply2d_tile<T, TE, 16, 16>(live, bx, by, rhs, x, y, E, d, lam0, mu0);
  if (partials) dot_partials(dot, live ? rhs : 0, partials);
}

// -------------------------------------------------------------- 3D apply
// One block: one tile of 15 x 15 node columns, one z-chunk, and NRB load
// cases (all of them on the fine level), so each layer's moduli, mask and
// D^-1 are read once for every load case the block handles.  Per cube
// layer: the next node plane of every load case is committed from registers
// to LDS, the plane after it is fetched from memory while the layer is
// computed, and each load case's cube forces are combined into owned nodes.
// The load cases pass through the LDS exchange in groups of G (G = NRB in
// FP32; at most 2 in FP64, to bound LDS), each group behind one LDS-only
// barrier.  All loads use clamped (always valid) addresses so they are
// issued unconditionally.  A plane's loads are kept raw until the commit one
// layer later (validity selects, the D^-1 b product of the pre-smoothing),
// so no wait for them falls inside the layer that issued them.
template <typename T, int NRB>
struct PlaneBuf {
  T v[NRB][2][3];
  T w[2][3];  // EPI 2: D^-1 at the staged nodes (v holds b)
  int m[2];
  bool ok[2];
};

// EPI = 2: the whole degree-2 Chebyshev smoothing from x = 0 in one kernel.
// The operator input is d0 = D^-1 b / theta, formed while staging the
// patch; at each owned node the epilogue forms r = b - K d0,
// d1 = c1 d0 + c2 D^-1 r and writes x = d0 + d1 (r and the increments are
// not needed afterwards), so r and d are never stored.
// EPI = 3 and 4: degree-2 smoothing from a given x in two kernels.  EPI 3
// takes x as the operator input and writes r = b - K x and d1 = s D^-1 r at
// owned nodes (x itself is left alone: other blocks still read it as halo).
// EPI 4 takes d1 as the operator input and, at owned nodes, forms
// r - K d1, d2 = c1 d1 + c2 D^-1 (r - K d1) and writes x = (x + d1) + d2.
template <typename T>
struct ChebEpi {
  T* x;
  const T* invd;
  const T* b;
  const double* lmax;
  double r_cur, r_prev, low;
  int kind;   // Chebyshev kind (1 or 4)
  T* r;       // EPI 3: residual out; EPI 4: residual in
  T* d;       // EPI 3: first increment out
};

template <typename T, typename TE, int EPI, int NRB, int G>
__global__ __launch_bounds__(256) void apply3d_kernel(const T* __restrict__ x, T* __restrict__ y,
                                                      const TE* __restrict__ E, OpDesc d,
                                                      TileMap tm, T lam0, T mu0, double* partials,
                                                      const int* stop, ChebEpi<T> ce) {
  static_assert(NRB % G == 0, "load-case groups must tile the block's load cases");
  __shared__ T xs[2][NRB][3][PATCH2];
  __shared__ T ex[G][6][256];
  __shared__ uint8_t ms[2][PATCH2];
  const int tid = threadIdx.x;
  const int tx = tid & 15, ty = tid >> 4;
  if (stop && *stop) return;
  int bx, by, bz, rb;
  const bool live = map_block(tm, bx, by, bz, rb);
  if (!live && !partials) return;
  const int rhs0 = rb * NRB;
  double dot[NRB];
#pragma unroll
  for (int r = 0; r < NRB; ++r) dot[r] = 0.0;
  if (live) {
    const int nx = d.nx, ny = d.ny, nz = d.nz;
    const long nn = d.nn;
    const int i0 = bx * TILE, j0 = by * TILE;
    const int k0 = bz * d.kz;
    const int k1 = min(k0 + d.kz, nz + 1);
    const long plane = (long)(nx + 1) * (ny + 1);
    const long rs = 3 * nn;   // stride between load cases
    const T* xr = x + (long)rhs0 * rs;
    T* yr = y + (long)rhs0 * rs;
    const T* br = (EPI == 2 || EPI == 3) ? ce.b + (long)rhs0 * rs : nullptr;
    T* rr_ = (EPI == 3 || EPI == 4) ? ce.r + (long)rhs0 * rs : nullptr;
    T* dd_ = EPI == 3 ? ce.d + (long)rhs0 * rs : nullptr;
    T it0 = 0;
    if (EPI == 2 || EPI == 3) it0 = T(cheb_first_scale(*ce.lmax, ce.low, ce.kind));

    // plane staging: thread handles patch nodes idx = tid and tid + 256
    long poff[2];
    bool pin[2];
    bool pidx[2];
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int idx = tid + 256 * q;
      const int a = idx % PATCH, b = idx / PATCH;
      const int gi = i0 - 1 + a, gj = j0 - 1 + b;
      pidx[q] = idx < PATCH2;
      pin[q] = pidx[q] && gi >= 0 && gi <= nx && gj >= 0 && gj <= ny;
      const int ci = min(max(gi, 0), nx), cj = min(max(gj, 0), ny);
      poff[q] = (long)cj * (nx + 1) + ci;
    }
    auto fetch = [&](int kk, PlaneBuf<T, NRB>& pb) {
      const bool kin = kk >= 0 && kk <= nz;
      const long base = (long)min(max(kk, 0), nz) * plane;
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        const long n = base + poff[q];
        pb.m[q] = d.mask[n];
        pb.ok[q] = pin[q] && kin;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          if (EPI == 2) pb.w[q][c] = ce.invd[c * nn + n];
#pragma unroll
          for (int r = 0; r < NRB; ++r)
            pb.v[r][q][c] = EPI == 2 ? br[r * rs + c * nn + n] : xr[r * rs + c * nn + n];
        }
      }
    };
    auto commit = [&](int kk, const PlaneBuf<T, NRB>& pb) {
      const int s = kk & 1;
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        const int idx = tid + 256 * q;
        if (pidx[q]) {
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            const T sc = EPI == 2 ? it0 * pb.w[q][c] : T(0);
#pragma unroll
            for (int r = 0; r < NRB; ++r)
              xs[s][r][c][idx] = EPI == 2 ? sc * pb.v[r][q][c] : pb.v[r][q][c];
          }
          ms[s][idx] = pb.ok[q] ? (uint8_t)pb.m[q] : (uint8_t)7;
        }
      }
    };

    const int hi = i0 - 1 + tx, hj = j0 - 1 + ty;
    const bool col_ok = hi >= 0 && hi < nx && hj >= 0 && hj < ny;
    const long hcol = (long)min(max(hj, 0), ny - 1) * nx + min(max(hi, 0), nx - 1);
    // raw moduli; the validity select is applied where they are used
    auto fetch_E = [&](int kk, T (&en)[6]) {
      const long h = (long)min(max(kk, 0), nz - 1) * ny * nx + hcol;
      if constexpr (sizeof(TE) == 2) {
        // BF16 moduli: the cube's six are 12 bytes, read as three dwords
        const uint32_t* w = reinterpret_cast<const uint32_t*>(E + 6 * h);
#pragma unroll
        for (int q = 0; q < 3; ++q) {
          const uint32_t v = w[q];
          en[2 * q] = T(__uint_as_float(v << 16));
          en[2 * q + 1] = T(__uint_as_float(v & 0xffff0000u));
        }
      } else {
#pragma unroll
        for (int t = 0; t < 6; ++t) en[t] = T(E[6 * h + t]);
      }
    };
    const int oi = i0 + tx, oj = j0 + ty;
    const bool owner = tx < TILE && ty < TILE && oi <= nx && oj <= ny;
    const long ocol = (long)oj * (nx + 1) + oi;
    const int oli = (ty + 1) * PATCH + tx + 1;   // the owned node in the patch (mask)
    T carry[NRB][3];
#pragma unroll
    for (int r = 0; r < NRB; ++r)
#pragma unroll
      for (int a = 0; a < 3; ++a) carry[r][a] = 0;
    T c1 = 0, c2 = 0;
    T* ex_ = nullptr;
    if (EPI == 2 || EPI == 4) {
      double c1d, c2d;
      cheb_next_coef(*ce.lmax, ce.low, ChebCoef{ce.r_cur, ce.r_prev, ce.kind, 1}, c1d, c2d);
      c1 = T(c1d);
      c2 = T(c2d);
      ex_ = ce.x + (long)rhs0 * rs;
    }

    PlaneBuf<T, NRB> pb;
    fetch(k0 - 1, pb);
    commit(k0 - 1, pb);
    fetch(k0, pb);
    for (int kh = k0 - 1; kh < k1; ++kh) {
      // this layer's moduli: issued first, their latency hides behind the
      // plane commit and the barrier
      T ev[6];
      fetch_E(kh, ev);
      // smoothing epilogue: this layer's b (or r, x) and D^-1 at the owned
      // node, issued now so their latency hides behind the layer's arithmetic
      T pb_[NRB][3], pi[3], px[NRB][3];
      if (EPI >= 2) {
        const long on = (long)min(max(kh, 0), nz) * plane + (owner ? ocol : 0);
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          pi[a] = ce.invd[a * nn + on];
#pragma unroll
          for (int r = 0; r < NRB; ++r) {
            pb_[r][a] = EPI == 4 ? rr_[r * rs + a * nn + on] : br[r * rs + a * nn + on];
            if (EPI == 4) px[r][a] = ex_[r * rs + a * nn + on];
          }
        }
      }
      commit(kh + 1, pb);
      lds_barrier();
      // unconditional: past the chunk's end this re-reads its last plane
      // (still in cache), which is never committed
      fetch(min(kh + 2, k1), pb);
      const bool eok = col_ok && kh >= 0 && kh < nz;
      T lam[6], mu[6];
#pragma unroll
      for (int t = 0; t < 6; ++t) {
        const T e = eok ? ev[t] : T(0);
        lam[t] = lam0 * e;
        mu[t] = mu0 * e;
      }
      const int sb = kh & 1, stp = (kh + 1) & 1;
      const int om = owner ? ms[sb][oli] : 0;
      const bool store = owner && kh >= k0;
      const long on = (long)kh * plane + ocol;
#pragma unroll
      for (int g0 = 0; g0 < NRB; g0 += G) {
        T X1[G][2][3], U3[G][3];
#pragma unroll
        for (int gr = 0; gr < G; ++gr) {
          const int r = g0 + gr;
          T u[8][3], f[8][3];
#pragma unroll
          for (int c = 0; c < 8; ++c) {
            const int li = (ty + ((c >> 1) & 1)) * PATCH + tx + (c & 1);
            const int s = (c >> 2) ? stp : sb;
#pragma unroll
            for (int a = 0; a < 3; ++a) u[c][a] = xs[s][r][a][li];
          }
          cube_force<T>(u, lam, mu, f);
          // corner 3 of this cube is the owned node (its operator input is
          // kept here: the next layer's commit overwrites this LDS plane)
#pragma unroll
          for (int a = 0; a < 3; ++a) U3[gr][a] = u[3][a];
#pragma unroll
          for (int cz = 0; cz < 2; ++cz)
#pragma unroll
            for (int a = 0; a < 3; ++a) {
              ex[gr][cz * 3 + a][tid] = f[1 + 4 * cz][a] + next_lane<16>(f[4 * cz][a]);
              X1[gr][cz][a] = f[3 + 4 * cz][a] + next_lane<16>(f[2 + 4 * cz][a]);
            }
        }
        lds_barrier();
        if (owner) {
#pragma unroll
          for (int gr = 0; gr < G; ++gr) {
            const int r = g0 + gr;
#pragma unroll
            for (int a = 0; a < 3; ++a) {
              T yb = carry[r][a] + X1[gr][0][a] + ex[gr][a][tid + 16];
              carry[r][a] = X1[gr][1][a] + ex[gr][3 + a][tid + 16];
              if (store) {
                if ((om >> a) & 1) yb = 0;
                const long ia = r * rs + a * nn + on;
                const T uo = U3[gr][a];   // operator input at the owned node
                if (EPI == 0) {
                  yr[ia] = yb;
                  if (partials) dot[r] += (double)yb * (double)uo;
                } else if (EPI == 2) {
                  // uo = d0 at the owned node; r = b - K d0
                  const T rv = pb_[r][a] - yb;
                  ex_[ia] = uo + (c1 * uo + c2 * pi[a] * rv);
                } else if (EPI == 3) {
                  const T rv = pb_[r][a] - yb;
                  rr_[ia] = rv;
                  dd_[ia] = it0 * pi[a] * rv;
                } else {
                  // uo = d1 at the owned node, pb_ = r, px = x
                  const T rv = pb_[r][a] - yb;
                  const T dv = c1 * uo + c2 * pi[a] * rv;
                  ex_[ia] = (px[r][a] + uo) + dv;
                }
              }
            }
          }
        }
        // the next group reuses the exchange buffer
        if (g0 + G < NRB) lds_barrier();
      }
    }
  }
  if (partials) {
    double acc[kMaxRhs];
#pragma unroll
    for (int r = 0; r < kMaxRhs; ++r) acc[r] = 0.0;
#pragma unroll
    for (int k = 0; k < kMaxRhs; ++k)
#pragma unroll
      for (int r = 0; r < NRB; ++r)
        if (rhs0 + r == k) acc[k] = dot[r];
    const double none[1] = {0.0};
    block_partials<kMaxRhs, 0>(acc, none, partials);
  }
}

// ------------------------------------------------------------- diagonal
__global__ void diag2d_kernel(double* d, const double* E, OpDesc od, double lam0, double mu0,
                              double vol, int inverse) {
  const long n = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= od.nn) return;
  diag2d_node(n, d, E, od, lam0, mu0, vol, inverse);
}

__global__ void diag3d_kernel(double* d, const double* E, OpDesc od, double lam0, double mu0,
                              double vol, int inverse) {
  const int nx = od.nx, ny = od.ny, nz = od.nz;
  const long nn = od.nn;
  const uint8_t* mask = od.mask;
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
__global__ void simp_modulus_kernel(double* E, float* E32, uint16_t* E16, const double* rho, long nc,
                                    double E0, double Emin, double penal, int paper) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nc) return;
  const double r = rho[e];
  const double rp = (penal == 3.0) ? r * r * r : pow(r, penal);
  const double v = paper ? rp : Emin + rp * (E0 - Emin);
  E[e] = v;
  if (E32) E32[e] = (float)v;
  if (E16) E16[e] = bf16_from_f64(v);
}

template <typename T>
__global__ void mask_copy_kernel(const T* src, T* dst, const uint8_t* mask, long nn, int dim,
                                 long total) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= total) return;
  const long n = i % nn;
  const int c = (int)((i / nn) % dim);
  dst[i] = ((mask[n] >> c) & 1) ? T(0) : src[i];
}

__global__ void fill_kernel(double* dst, double v, long n) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = v;
}

// ------------------------------------------------------------ launchers

void launch_simp_modulus(Ctx* c, const double* rho) {
  simp_modulus_kernel<<<cdiv(c->g.nc, 256), 256, 0, c->stream>>>(
      c->E, c->prob.precision != TOPO_FP64 ? c->E32 : nullptr, c->E16, rho, c->g.nc, c->m.E0,
      c->m.Emin, c->m.penal, c->m.paper);
}

static TileMap make_tilemap(const OpDesc& d, int nrhs) {
  TileMap tm;
  tm.gx = (int)cdiv(d.nx + 1, TILE);
  tm.gy = (int)cdiv(d.ny + 1, TILE);
  tm.gz = d.dim == 3 ? (int)cdiv(d.nz + 1, d.kz) : 1;
  const long ntiles = (long)tm.gx * tm.gy * tm.gz;
  tm.per_xcd = (int)((ntiles + 7) / 8);
  tm.nrhs = nrhs;
  return tm;
}

// Load cases per block of the 3D apply (a divisor of nrhs).  A block that
// handles all load cases reads the moduli, mask and D^-1 once for all of them
// (the byte saving of batched load cases); blocks that split them hold fewer
// registers and keep more blocks in flight.  Measured at 192 x 96 x 96 with
// 4 load cases (the kernels are bound by arithmetic and latency, not HBM):
// FP32, all cases per block 128 us against 125 us for one case per block;
// FP64, 280 us against 216 us (256 VGPRs, one wave per SIMD).  So FP32 grids
// with 1024 or more tiles take all load cases per block; FP64 applies and
// smaller grids take one.  env_nrb (TOPO_APPLY_NRB at context creation)
// overrides the choice when it divides nrhs.
int apply_rhs_per_block(const OpDesc& d, int nrhs, int elem_bytes, int epi, int env_nrb) {
  if (d.dim != 3 || nrhs <= 1) return 1;
  if (env_nrb >= 1 && env_nrb <= nrhs && nrhs % env_nrb == 0) return env_nrb;
  if (elem_bytes != 4) return 1;
  const TileMap tm = make_tilemap(d, 1);
  if (8L * tm.per_xcd < 1024) return 1;
  // the plain apply of four load cases runs two per block (192x96x96:
  // 93.6 us against 101.4 us with four, 93.2 us with one); the smoothing
  // kernels keep all four (pre-smoothing 127.5 us against 134.7 with two)
  return (epi == 0 && nrhs == 4) ? 2 : nrhs;
}

long apply_grid_blocks(const OpDesc& d, int nrhs, int elem_bytes, int env_nrb) {
  const int nrb = apply_rhs_per_block(d, nrhs, elem_bytes, 0, env_nrb);
  TileMap tm = make_tilemap(d, nrhs / nrb);
  return 8L * tm.per_xcd * (nrhs / nrb);
}

// launches apply3d_kernel<T, TE, EPI, NRB> with NRB = the block's load cases
template <typename T, typename TE, int EPI>
static void launch_apply3d(Ctx* c, const OpDesc& d, const TE* E, const T* x, T* y, int nrhs,
                           double* part, const int* stop, const ChebEpi<T>& ce) {
  const T lam = T(c->m.lam0 * c->m.vol), mu = T(c->m.mu0 * c->m.vol);
  const int nrb = apply_rhs_per_block(d, nrhs, (int)sizeof(T), EPI, c->env_nrb);
  const TileMap tm = make_tilemap(d, nrhs / nrb);
  const unsigned blocks = (unsigned)(8L * tm.per_xcd * (nrhs / nrb));
  hipStream_t s = c->stream;
  const int g = c->env_g;
#define TOPO_APPLY3D(NRB_, G_) \
  apply3d_kernel<T, TE, EPI, NRB_, G_><<<blocks, 256, 0, s>>>(x, y, E, d, tm, lam, mu, part, stop, ce)
  if (nrb == 4 && g == 4) TOPO_APPLY3D(4, 4);
  else if (nrb == 4 && g == 2) TOPO_APPLY3D(4, 2);
  else if (nrb == 4) TOPO_APPLY3D(4, 1);
  else if (nrb == 2 && g >= 2) TOPO_APPLY3D(2, 2);
  else if (nrb == 2) TOPO_APPLY3D(2, 1);
  else if (nrb == 3) TOPO_APPLY3D(3, 1);
  else TOPO_APPLY3D(1, 1);
#undef TOPO_APPLY3D
}

OpDesc fine_op(const Ctx* c) {
  OpDesc d;
  d.dim = c->g.dim;
  d.nx = c->g.nx;
  d.ny = c->g.ny;
  d.nz = c->g.dim == 3 ? c->g.nz : 1;
  d.nn = c->g.nn;
  d.split_uniform = c->g.split == TOPO_SPLIT_UNIFORM;
  d.mask = c->mask;
  d.kz = c->apply_kz;
  return d;
}

template <typename T, typename TE>
static void apply_dispatch(Ctx* c, const OpDesc& d, const TE* E, const T* x, T* y, int nrhs,
                           bool fuse_dot, const int* stop) {
  double* part = fuse_dot ? c->partials : nullptr;
  const int* st = stop;
  const T lam = T(c->m.lam0 * c->m.vol), mu = T(c->m.mu0 * c->m.vol);
  const TileMap tm = make_tilemap(d, nrhs);
  const unsigned blocks = (unsigned)(8L * tm.per_xcd * nrhs);
  if (d.dim == 2)
    apply2d_kernel<T, TE><<<blocks, 256, 0, c->stream>>>(x, y, E, d, tm, lam, mu, part, st);
  else
    launch_apply3d<T, TE, 0>(c, d, E, x, y, nrhs, part, st, ChebEpi<T>{});
}

// degree-2 smoothing from x = 0 (3D): x = d0 + c1 d0 + c2 D^-1 (b - K d0),
// d0 = D^-1 b / theta
template <typename T, typename TE>
static void cheb_pre3d(Ctx* c, const OpDesc& d, const TE* E, const T* b, T* x, const T* invd,
                       const double* lmax, double r_cur, double r_prev, double low, int kind,
                       int nrhs, const int* stop) {
  ChebEpi<T> ce{x, invd, b, lmax, r_cur, r_prev, low, kind};
  launch_apply3d<T, TE, 2>(c, d, E, nullptr, nullptr, nrhs, nullptr, stop, ce);
}

// degree-2 smoothing from a given x (3D), two kernels (EPI 3, EPI 4); the
// coefficients are those of the first and second step of the separate
// smoothing kernels, so the result is the same arithmetic
template <typename T, typename TE>
static void cheb_post3d(Ctx* c, const OpDesc& d, const TE* E, T* x, const T* b, T* r, T* dd,
                        const T* invd, const double* lmax, double r_cur, double r_prev, double low,
                        int kind, int nrhs, const int* stop) {
  ChebEpi<T> ce{x, invd, b, lmax, r_cur, r_prev, low, kind, r, dd};
  launch_apply3d<T, TE, 3>(c, d, E, x, nullptr, nrhs, nullptr, stop, ce);
  launch_apply3d<T, TE, 4>(c, d, E, dd, nullptr, nrhs, nullptr, stop, ce);
}

template <typename T>
void launch_apply_cheb_post3d(Ctx* c, const OpDesc& d, const T* E, const uint16_t* E16, T* x,
                              const T* b, T* r, T* dd, const T* invd, const double* lmax,
                              double r_cur, double r_prev, double low, int kind, int nrhs,
                              const int* stop) {
  if constexpr (sizeof(T) == 4) {
    if (E16) {
      cheb_post3d<T, bf16m>(c, d, reinterpret_cast<const bf16m*>(E16), x, b, r, dd, invd, lmax,
                            r_cur, r_prev, low, kind, nrhs, stop);
      return;
    }
  }
  cheb_post3d<T, T>(c, d, E, x, b, r, dd, invd, lmax, r_cur, r_prev, low, kind, nrhs, stop);
}

template void launch_apply_cheb_post3d<float>(Ctx*, const OpDesc&, const float*, const uint16_t*,
                                              float*, const float*, float*, float*, const float*,
                                              const double*, double, double, double, int, int,
                                              const int*);
template void launch_apply_cheb_post3d<double>(Ctx*, const OpDesc&, const double*, const uint16_t*,
                                               double*, const double*, double*, double*,
                                               const double*, const double*, double, double, double,
                                               int, int, const int*);

template <typename T>
void launch_apply_cheb_pre3d(Ctx* c, const OpDesc& d, const T* E, const T* b, T* x, const T* invd,
                             const double* lmax, double r_cur, double r_prev, double low, int kind,
                             int nrhs, const int* stop) {
  cheb_pre3d<T, T>(c, d, E, b, x, invd, lmax, r_cur, r_prev, low, kind, nrhs, stop);
}

void launch_apply_cheb_pre3d_bf16(Ctx* c, const OpDesc& d, const uint16_t* E16, const float* b,
                                  float* x, const float* invd, const double* lmax, double r_cur,
                                  double r_prev, double low, int kind, int nrhs, const int* stop) {
  cheb_pre3d<float, bf16m>(c, d, reinterpret_cast<const bf16m*>(E16), b, x, invd, lmax, r_cur,
                           r_prev, low, kind, nrhs, stop);
}

template void launch_apply_cheb_pre3d<float>(Ctx*, const OpDesc&, const float*, const float*, float*,
                                             const float*, const double*, double, double, double, int,
                                             int, const int*);
template void launch_apply_cheb_pre3d<double>(Ctx*, const OpDesc&, const double*, const double*,
                                              double*, const double*, const double*, double, double,
                                              double, int, int, const int*);

void launch_apply_op(Ctx* c, const OpDesc& d, const double* E, const double* x, double* y,
                     int nrhs, bool fuse_dot, bool timed, const int* stop) {
  int slot = (timed && c->timing) ? timing_begin(c, 0) : -1;
  apply_dispatch<double, double>(c, d, E, x, y, nrhs, fuse_dot, stop);
  if (slot >= 0) timing_end(c, 0, slot);
}

void launch_apply_op_f32(Ctx* c, const OpDesc& d, const float* E, const float* x, float* y,
                         int nrhs, bool timed, const int* stop) {
  int slot = (timed && c->timing) ? timing_begin(c, 0) : -1;
  apply_dispatch<float, float>(c, d, E, x, y, nrhs, false, stop);
  if (slot >= 0) timing_end(c, 0, slot);
}

void launch_apply_op_bf16(Ctx* c, const OpDesc& d, const uint16_t* E16, const float* x, float* y,
                          int nrhs, bool timed, const int* stop) {
  int slot = (timed && c->timing) ? timing_begin(c, 0) : -1;
  apply_dispatch<float, bf16m>(c, d, reinterpret_cast<const bf16m*>(E16), x, y, nrhs, false, stop);
  if (slot >= 0) timing_end(c, 0, slot);
}

void launch_apply_op_f32_dot(Ctx* c, const OpDesc& d, const float* E, const float* x, float* y,
                             int nrhs) {
  int slot = c->timing ? timing_begin(c, 0) : -1;
  apply_dispatch<float, float>(c, d, E, x, y, nrhs, true, &c->scal->pcg.done);
  if (slot >= 0) timing_end(c, 0, slot);
}

__global__ void to_f32_cast_kernel(float* dst, const double* __restrict__ src, long n) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    dst[i] = (float)src[i];
}

void launch_to_f32(Ctx* c, float* dst, const double* src, int64_t n) {
  long b = (n + 255) / 256;
  if (b > 4096) b = 4096;
  to_f32_cast_kernel<<<(unsigned)(b < 1 ? 1 : b), 256, 0, c->stream>>>(dst, src, n);
}

// Timed launches are the fine-level applies in the solve's working
// precision (FP64 solve: FP64 applies; mixed solves: the FP32 applies).
__global__ void to_f64_cast_kernel(double* dst, const float* __restrict__ src, long n) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    dst[i] = (double)src[i];
}

void launch_to_f64(Ctx* c, double* dst, const float* src, int64_t n) {
  long b = (n + 255) / 256;
  if (b > 4096) b = 4096;
  to_f64_cast_kernel<<<(unsigned)(b < 1 ? 1 : b), 256, 0, c->stream>>>(dst, src, n);
}

void launch_apply(Ctx* c, const double* x, double* y, int nrhs, bool fuse_dot) {
  launch_apply_op(c, fine_op(c), c->E, x, y, nrhs, fuse_dot, c->prob.precision == TOPO_FP64,
                  fuse_dot ? &c->scal->pcg.done : nullptr);
}

void launch_apply_f32(Ctx* c, const float* x, float* y, int nrhs, bool fuse_dot) {
  (void)fuse_dot;
  launch_apply_op_f32(c, fine_op(c), c->E32, x, y, nrhs, true, nullptr);
}

void launch_diagonal_op(Ctx* c, const OpDesc& od, const double* E, double* d, bool inverse) {
  if (od.dim == 2)
    diag2d_kernel<<<cdiv(od.nn, 256), 256, 0, c->stream>>>(d, E, od, c->m.lam0, c->m.mu0, c->m.vol,
                                                          inverse);
  else
    diag3d_kernel<<<cdiv(od.nn, 256), 256, 0, c->stream>>>(d, E, od, c->m.lam0, c->m.mu0, c->m.vol,
                                                          inverse);
}

void launch_diagonal(Ctx* c, double* d, bool inverse) {
  launch_diagonal_op(c, fine_op(c), c->E, d, inverse);
}

void launch_mask_copy(Ctx* c, const double* src, double* dst, int nrhs) {
  const long total = (long)nrhs * c->g.nd;
  mask_copy_kernel<double><<<cdiv(total, 256), 256, 0, c->stream>>>(src, dst, c->mask, c->g.nn,
                                                                    c->g.dim, total);
}

void launch_mask_copy_f32(Ctx* c, const float* src, float* dst, int nrhs) {
  const long total = (long)nrhs * c->g.nd;
  mask_copy_kernel<float><<<cdiv(total, 256), 256, 0, c->stream>>>(src, dst, c->mask, c->g.nn,
                                                                   c->g.dim, total);
}

void launch_fill(Ctx* c, double* dst, double v, int64_t n) {
  fill_kernel<<<cdiv(n, 256), 256, 0, c->stream>>>(dst, v, n);
}

}  // namespace topo
