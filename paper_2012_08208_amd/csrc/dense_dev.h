// Dense direct solve of a multigrid coarsest level above 128 DOFs: the
// block sweep inverse and the dense matrix-vector product, as
// device functions shared by the single-context solver and the batch.
//
// The matrix, padded to np = a whole number of 64-blocks with identity rows
// and columns, is inverted in FP64 by block elimination without pivoting
// (the matrix is SPD, so every pivot block is SPD), in the symmetric form
// of the sweep operator (Goodnight, The American Statistician 33(3), 1979)
// applied block by block: per block step k, with P = A_kk^-1,
//   A_ij <- A_ij - A_ik P A_kj,  A_ik <- A_ik P,  A_kj <- P A_kj  (i, j != k),
//   A_kk <- -P,
// which keeps the matrix symmetric and ends at -A^-1.  Only the blocks on
// and above the diagonal are updated (half the work of the unsymmetric
// Gauss-Jordan form); a last pass negates and mirrors them.
// The work-group of every function below has kGjThreads (256) threads,
// except dense_solve_rows (64 * kDenseWaves); each returns, if it returns
// early, for the whole work-group.
#pragma once

#include <type_traits>

#include "common.h"
#include "topo_internal.h"

namespace topo {

// A: zeros, with identity rows and columns past n (the padding), by the
// threads t0, t0 + dt, ... of a grid
__device__ inline void dense_fill_range(double* A, int n, int np, long t0, long dt) {
  const long tot = (long)np * np;
  for (long t = t0; t < tot; t += dt) {
    const int i = (int)(t / np), j = (int)(t - (long)i * np);
    A[t] = (i == j && i >= n) ? 1.0 : 0.0;
  }
}

constexpr int kGjB = kGjBlock;
constexpr int kGjPad = kGjB + 1;   // LDS row pitch (doubles)

// P = inverse of the diagonal block k by in-place Gauss-Jordan elimination,
// itself blocked by 16: for each 16 x 16 diagonal sub-block one wave
// inverts it in registers (lane l holds column l & 15, rows (l >> 4) + 4m;
// the pivot row and column come from lane shuffles, so its 16 steps need no
// barrier), then the work-group forms the sub-block row panel and updates
// the other 48 rows, as the blocked elimination over the whole matrix
// does.  Four sub-blocks, three barriers each, instead of 64 barrier-
// separated steps.
constexpr int kGjPivThreads = 256;
constexpr int kGjSub = 16;
// S: the block in LDS (row pitch kGjPad), overwritten; every thread of the
// work-group has stored its part of S and passed a barrier before the call
__device__ __forceinline__ void gj_pivot_lds(double* S, double* P) {
  __shared__ double Cb[(kGjB - kGjSub) * (kGjSub + 1)];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  for (int kb = 0; kb < kGjB / kGjSub; ++kb) {
    const int o = kb * kGjSub;
    if (wave == 0) {
      const int j = lane & 15, g = lane >> 4;
      double v[4];
#pragma unroll
      for (int m = 0; m < 4; ++m) v[m] = S[(o + g + 4 * m) * kGjPad + o + j];
#pragma unroll
      for (int p = 0; p < kGjSub; ++p) {
        const int rp = p >> 2, lp = (p & 3) << 4;
        const double piv = __shfl(v[rp], lp | p);
        const double rowv = __shfl(v[rp], lp | j);
        double colv[4];
#pragma unroll
        for (int m = 0; m < 4; ++m) colv[m] = __shfl(v[m], (lane & 0x30) | p);
        double r = __builtin_amdgcn_rcp(piv);
        r = fma(r, fma(-piv, r, 1.0), r);
        const double rj = (j == p ? 1.0 : rowv) * r;
#pragma unroll
        for (int m = 0; m < 4; ++m) {
          const int i = g + 4 * m;
          v[m] = (i == p) ? rj : ((j == p) ? 0.0 : v[m]) - colv[m] * rj;
        }
      }
#pragma unroll
      for (int m = 0; m < 4; ++m) S[(o + g + 4 * m) * kGjPad + o + j] = v[m];
    }
    __syncthreads();
    // row panel (16 rows x 48 columns) from the sub-block inverse; the
    // other rows' sub-block columns saved for the update
    double col[kGjSub];
    const int cc = t % 48, r0 = t / 48;
    const int c = cc < o ? cc : cc + kGjSub;
    if (t < 192) {
#pragma unroll
      for (int q = 0; q < kGjSub; ++q) col[q] = S[(o + q) * kGjPad + c];
    }
    for (int e = t; e < (kGjB - kGjSub) * kGjSub; e += kGjPivThreads) {
      const int ri = e / kGjSub, q = e % kGjSub;
      const int i = ri < o ? ri : ri + kGjSub;
      Cb[ri * (kGjSub + 1) + q] = S[i * kGjPad + o + q];
    }
    __syncthreads();
    if (t < 192) {
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int r = r0 + 4 * u;
        double acc = 0.0;
#pragma unroll
        for (int q = 0; q < kGjSub; ++q) acc = fma(S[(o + r) * kGjPad + o + q], col[q], acc);
        S[(o + r) * kGjPad + c] = acc;
      }
    }
    __syncthreads();
    // every other row: A_ic -= C_i (row panel)_c, and the sub-block columns
    // become -C_i P16 (the same product: those columns of the sub-block rows
    // hold P16)
    {
      const int c2 = t & 63, g2 = t >> 6;
      double rc[kGjSub];
#pragma unroll
      for (int q = 0; q < kGjSub; ++q) rc[q] = S[(o + q) * kGjPad + c2];
      const bool diag = c2 >= o && c2 < o + kGjSub;
#pragma unroll
      for (int u = 0; u < 12; ++u) {
        const int ri = g2 + 4 * u;
        const int i = ri < o ? ri : ri + kGjSub;
        double acc = 0.0;
#pragma unroll
        for (int q = 0; q < kGjSub; ++q) acc = fma(Cb[ri * (kGjSub + 1) + q], rc[q], acc);
        double& y = S[i * kGjPad + c2];
        y = diag ? -acc : y - acc;
      }
    }
    __syncthreads();
  }
  for (int e = t; e < kGjB * kGjB; e += kGjPivThreads) P[e] = S[(e / kGjB) * kGjPad + e % kGjB];
}

__device__ inline void gj_pivot_block(const double* __restrict__ A, int np, int k, double* P) {
  __shared__ double S[kGjB * kGjPad];
  const int t = threadIdx.x;
  const long base = ((long)k * np + k) * kGjB;
  constexpr int PER = kGjB * kGjB / kGjPivThreads;
  double v[PER];
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    const int e = t + u * kGjPivThreads;
    v[u] = A[base + (long)(e / kGjB) * np + e % kGjB];
  }
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    const int e = t + u * kGjPivThreads;
    S[(e / kGjB) * kGjPad + e % kGjB] = v[u];
  }
  __syncthreads();
  gj_pivot_lds(S, P);
}

// acc = X Y for 64 x 64 blocks staged in LDS, on the FP64 matrix cores:
// wave w owns the 32 x 32 quadrant (32 (w / 2), 32 (w % 2)) as 2 x 2 tiles
// of v_mfma_f64_16x16x4_f64.  Lane layout of that instruction (checked on
// gfx950): lane l supplies A[l % 16][l / 16] and B[l / 16][l % 16], and
// register r of its result holds D[l / 16 + 4 r][l % 16].
typedef double gj_d4 __attribute__((ext_vector_type(4)));
__device__ inline void gj_block_product(const double* Xs, const double* Ys, gj_d4 acc[2][2]) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int r0 = 32 * (w >> 1), c0 = 32 * (w & 1);
  const int li = lane & 15, lk = lane >> 4;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = gj_d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
  for (int k0 = 0; k0 < kGjB; k0 += 4) {
    double xa[2], yb[2];
#pragma unroll
    for (int a = 0; a < 2; ++a) xa[a] = Xs[(r0 + 16 * a + li) * kGjPad + k0 + lk];
#pragma unroll
    for (int b = 0; b < 2; ++b) yb[b] = Ys[(k0 + lk) * kGjPad + c0 + 16 * b + li];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b)
        acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(xa[a], yb[b], acc[a][b], 0, 0, 0);
  }
}

// the entry (row, column) of the block that register r of acc[a][b] holds
__device__ inline int gj_acc_row(int a, int r) {
  return 32 * ((threadIdx.x >> 6) >> 1) + 16 * a + ((threadIdx.x & 63) >> 4) + 4 * r;
}
__device__ inline int gj_acc_col(int b) {
  return 32 * ((threadIdx.x >> 6) & 1) + 16 * b + (threadIdx.x & 15);
}

// stage two 64 x 64 blocks (leading dimensions lx, ly) into LDS, every
// load of the 256 threads issued before the first store
constexpr int kGjThreads = 256;
static_assert(kGjThreads == kGjPivThreads, "the update work-group also inverts the next pivot");
__device__ inline void gj_stage2(double* dx, const double* __restrict__ sx, long lx, double* dy,
                                 const double* __restrict__ sy, long ly) {
  constexpr int PER = kGjB * kGjB / kGjThreads;
  double vx[PER], vy[PER];
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    const int t = threadIdx.x + u * kGjThreads;
    vx[u] = sx[(long)(t / kGjB) * lx + t % kGjB];
    vy[u] = sy[(long)(t / kGjB) * ly + t % kGjB];
  }
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    const int t = threadIdx.x + u * kGjThreads;
    dx[(t / kGjB) * kGjPad + t % kGjB] = vx[u];
    dy[(t / kGjB) * kGjPad + t % kGjB] = vy[u];
  }
}

// The elimination keeps the matrix symmetric (the block sweep operator):
// per block step k, with P = A_kk^-1,
//   A_ij -= A_ik P A_kj,  A_ik <- A_ik P,  A_kj <- P A_kj  (i, j != k),
//   A_kk <- -P,
// and after the last step the matrix is -A^-1.  Only the blocks (i, j) with
// i <= j are kept; a block below the diagonal is the transpose of its
// mirror.  Per step the panel saves the old column, C_i = A_ik, and the row
// panel R_j = P A_kj (both as 64 x 64 blocks of scratch, leading dimension
// 64), the update rewrites the upper blocks, and a last pass mirrors the
// upper blocks and negates.

// the 64 x 64 block (bi, bj) of the symmetric matrix held in its upper
// blocks, into LDS (row pitch kGjPad): coalesced loads from the stored block,
// transposed on the LDS store when the block lies below the diagonal
__device__ inline void sw_stage_block(double* Ls, const double* A, int np, int bi, int bj) {
  constexpr int PER = kGjB * kGjB / kGjThreads;
  const bool tr = bi > bj;
  const double* src = tr ? A + ((long)bj * np + bi) * kGjB : A + ((long)bi * np + bj) * kGjB;
  double v[PER];
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    const int t = threadIdx.x + u * kGjThreads;
    v[u] = src[(long)(t / kGjB) * np + t % kGjB];
  }
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    const int t = threadIdx.x + u * kGjThreads;
    const int r = t / kGjB, c = t % kGjB;
    Ls[tr ? c * kGjPad + r : r * kGjPad + c] = v[u];
  }
}

// a contiguous 64 x 64 block into LDS (row pitch kGjPad)
__device__ inline void sw_stage_dense(double* Ls, const double* __restrict__ src) {
  constexpr int PER = kGjB * kGjB / kGjThreads;
  double v[PER];
#pragma unroll
  for (int u = 0; u < PER; ++u) v[u] = src[threadIdx.x + u * kGjThreads];
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    const int t = threadIdx.x + u * kGjThreads;
    Ls[(t / kGjB) * kGjPad + t % kGjB] = v[u];
  }
}

// work-group blk < nb: R_j = P A_kj (j = blk != k) into R; blk in [nb, 2 nb):
// C_i = A_ik (i = blk - nb != k) into C
__device__ inline void sw_panel_block(const double* A, int np, int k,
                                      const double* __restrict__ P, double* C, double* R,
                                      int blk) {
  __shared__ double Xs[kGjB * kGjPad], Ys[kGjB * kGjPad];
  constexpr int PER = kGjB * kGjB / kGjThreads;
  const int nb = np / kGjB;
  if (blk >= nb) {
    const int i = blk - nb;
    if (i == k) return;
    sw_stage_block(Xs, A, np, i, k);
    __syncthreads();
    double* dst = C + (long)i * kGjB * kGjB;
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int t = threadIdx.x + u * kGjThreads;
      dst[t] = Xs[(t / kGjB) * kGjPad + t % kGjB];
    }
    return;
  }
  const int j = blk;
  if (j == k) return;
  sw_stage_dense(Xs, P);
  sw_stage_block(Ys, A, np, k, j);
  __syncthreads();
  gj_d4 acc[2][2];
  gj_block_product(Xs, Ys, acc);
  double* dst = R + (long)j * kGjB * kGjB;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) dst[gj_acc_row(a, r) * kGjB + gj_acc_col(b)] = acc[a][b][r];
}

// the upper block (i, j), i <= j, numbered tri = j (j + 1) / 2 + i
__device__ inline void sw_tri_index(int tri, int& i, int& j) {
  j = (int)((sqrtf(8.0f * (float)tri + 1.0f) - 1.0f) * 0.5f);
  while (j * (j + 1) / 2 > tri) --j;
  while ((j + 1) * (j + 2) / 2 <= tri) ++j;
  i = tri - j * (j + 1) / 2;
}

// the upper block of work-group blk (< nb (nb + 1) / 2) in a step-k update:
// the numbering starts at the next diagonal block, the one whose
// work-group also inverts it, so that it is dispatched first
__device__ inline void sw_update_index(int blk, int nb, int k, int& i, int& j) {
  const int ntri = nb * (nb + 1) / 2;
  int t = blk + (k + 1 < nb ? (k + 1) * (k + 2) / 2 + k + 1 : 0);
  if (t >= ntri) t -= ntri;
  sw_tri_index(t, i, j);
}

// upper block (i, j), i <= j: A_ij -= C_i R_j; A_ik = C_i P; A_kj = R_j;
// A_kk = -P.  Pnext (if not null): the work-group of the next diagonal
// block, which this step completes, goes on to invert it for the next
// step (so no pivot launch stands between two steps); Pnext must not be P,
// which the other work-groups are still reading.
__device__ inline void sw_update_block(double* A, int np, int k, const double* __restrict__ P,
                                       const double* __restrict__ C, const double* __restrict__ R,
                                       int i, int j, double* Pnext) {
  __shared__ double Xs[kGjB * kGjPad], Ys[kGjB * kGjPad];
  constexpr int PER = kGjB * kGjB / kGjThreads;
  double* Aij = A + ((long)i * np + j) * kGjB;
  if (i == k) {
    // row block k: A_kk = -P, A_kj = R_j
    const double* src = j == k ? P : R + (long)j * kGjB * kGjB;
    const double sg = j == k ? -1.0 : 1.0;
    double v[PER];
#pragma unroll
    for (int u = 0; u < PER; ++u) v[u] = src[threadIdx.x + u * kGjThreads];
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int t = threadIdx.x + u * kGjThreads;
      Aij[(long)(t / kGjB) * np + t % kGjB] = sg * v[u];
    }
    return;
  }
  // the block's own entries are requested first: their latency hides
  // behind the staging and the product
  const bool upd = j != k;
  double yv[2][2][4];
  if (upd) {
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int r = 0; r < 4; ++r) yv[a][b][r] = Aij[(long)gj_acc_row(a, r) * np + gj_acc_col(b)];
  }
  gj_stage2(Xs, C + (long)i * kGjB * kGjB, kGjB, Ys, upd ? R + (long)j * kGjB * kGjB : P, kGjB);
  __syncthreads();
  gj_d4 acc[2][2];
  gj_block_product(Xs, Ys, acc);
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        yv[a][b][r] = upd ? yv[a][b][r] - acc[a][b][r] : acc[a][b][r];
        Aij[(long)gj_acc_row(a, r) * np + gj_acc_col(b)] = yv[a][b][r];
      }
  if (Pnext && i == k + 1 && j == k + 1) {
    __syncthreads();   // every wave is done reading Xs
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int r = 0; r < 4; ++r) Xs[gj_acc_row(a, r) * kGjPad + gj_acc_col(b)] = yv[a][b][r];
    __syncthreads();
    gj_pivot_lds(Xs, Pnext);
  }
}

// after the last step: A^-1 = -(the upper blocks and their mirrors); upper
// block (i, j) by one work-group, its mirror written through LDS so that
// both stores are coalesced
__device__ inline void sw_mirror_block(double* A, int np, int i, int j) {
  __shared__ double Xs[kGjB * kGjPad];
  constexpr int PER = kGjB * kGjB / kGjThreads;
  double* Aij = A + ((long)i * np + j) * kGjB;
  double* Aji = A + ((long)j * np + i) * kGjB;
  double v[PER];
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    const int t = threadIdx.x + u * kGjThreads;
    v[u] = Aij[(long)(t / kGjB) * np + t % kGjB];
  }
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    const int t = threadIdx.x + u * kGjThreads;
    const int r = t / kGjB, c = t % kGjB;
    Aij[(long)r * np + c] = -v[u];
    Xs[c * kGjPad + r] = -v[u];
  }
  if (i == j) return;
  __syncthreads();
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    const int t = threadIdx.x + u * kGjThreads;
    const int r = t / kGjB, c = t % kGjB;
    Aji[(long)r * np + c] = Xs[r * kGjPad + c];
  }
}

// x = Ainv b for every load case: one wave per row, 8 waves per work-group
// with b staged in LDS (zero-padded to np), each lane streaming 16-byte
// pieces of its row, 8 loads in flight; FP64 sums reduced in a fixed order.
// Rows are np entries long and np is a multiple of 64, so every piece is
// aligned and the padded columns (zero) need no bounds test.
constexpr int kDenseWaves = 8;
static_assert(kDense3 <= 4 * 64 * kDenseWaves, "the b staging covers np <= 4 * blockDim");
// (work-group rb: rows rb * kDenseWaves ...; nrhs * np * sizeof(T) bytes of
// dynamic LDS)
template <typename T, typename TA>
__device__ inline void dense_solve_rows(T* x, const T* __restrict__ b, const TA* __restrict__ Ainv,
                                        int n, int np, int nrhs, int rb) {
  extern __shared__ double dsm[];
  T* bs = reinterpret_cast<T*>(dsm);   // [nrhs][np]
  constexpr int V = 16 / (int)sizeof(TA);
  using VA = typename std::conditional<sizeof(TA) == 4, float4, double2>::type;
  using VB = typename std::conditional<sizeof(T) == 4, float4, double2>::type;
  const int lane = threadIdx.x & 63;
  const int row = rb * kDenseWaves + (threadIdx.x >> 6);
  const int nv = np / V;
  // the row's first pieces are requested before b is staged (rows past n
  // read row 0, in bounds, and are not used)
  const VA* Ar = reinterpret_cast<const VA*>(Ainv + (long)(row < n ? row : 0) * np);
  VA a[8];
#pragma unroll
  for (int u = 0; u < 8; ++u) {
    const int q = lane + 64 * u;
    if (q < nv) a[u] = Ar[q];
  }
  // b staged with every load issued before the stores (np <= 4 * blockDim)
  {
    T v[kMaxRhs][4];
#pragma unroll
    for (int r = 0; r < kMaxRhs; ++r)
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int j = threadIdx.x + u * (int)blockDim.x;
        v[r][u] = (r < nrhs && j < n) ? b[(long)r * n + j] : T(0);
      }
#pragma unroll
    for (int r = 0; r < kMaxRhs; ++r)
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int j = threadIdx.x + u * (int)blockDim.x;
        if (r < nrhs && j < np) bs[(long)r * np + j] = v[r][u];
      }
  }
  __syncthreads();
  if (row >= n) return;
  double acc[kMaxRhs] = {0.0, 0.0, 0.0, 0.0};
  for (int q0 = lane; q0 < nv; q0 += 64 * 8) {
    if (q0 != lane) {
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int q = q0 + 64 * u;
        if (q < nv) a[u] = Ar[q];
      }
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int q = q0 + 64 * u;
      if (q >= nv) break;
      const TA* av = reinterpret_cast<const TA*>(&a[u]);
#pragma unroll
      for (int r = 0; r < kMaxRhs; ++r) {
        if (r >= nrhs) break;
        const T* br = bs + (long)r * np + q * V;
        T bv[V];
#pragma unroll
        for (int e = 0; e < V; e += 16 / (int)sizeof(T)) {
          const VB w = *reinterpret_cast<const VB*>(br + e);
          const T* wv = reinterpret_cast<const T*>(&w);
#pragma unroll
          for (int f = 0; f < 16 / (int)sizeof(T); ++f) bv[e + f] = wv[f];
        }
#pragma unroll
        for (int e = 0; e < V; ++e) acc[r] = fma((double)av[e], (double)bv[e], acc[r]);
      }
    }
  }
#pragma unroll
  for (int r = 0; r < kMaxRhs; ++r) {
    const double v = wave_sum(acc[r]);
    if (lane == 0 && r < nrhs) x[(long)r * n + row] = T(v);
  }
}


}  // namespace topo
