// Distance-weighted sensitivity filter over arbitrary cell midpoints
// (Sec. 3.2.2, eq. filter and eq. filter_cond; Sec. 4.5, eq. filter_mat).
//
// The paper forms the weights W_ab = max(0, rmin - |x_a - x_b|) from the
// Euclidean distance matrix of the midpoints, computes W and its row sums
// once outside the iteration loop, and for large meshes advises evaluating
// that matrix chunk by chunk (Sec. 6.2).  Here the chunks are cells of a
// spatial hash of side rmin: a midpoint's nonzero weights can only come from
// the 3^dim hash cells around its own, so only those blocks of the distance
// matrix are evaluated; every other block is zero by eq. filter_cond.
//
//   1. key:   slot of every midpoint in a power-of-two hash table
//             (collisions only merge chunks; every pair is still tested by
//             its distance), slot histogram;
//   2. sort:  stable radix sort of (slot, index) pairs, so each slot's
//             members are contiguous and in increasing index order, and an
//             exclusive scan of the histogram gives the slot starts;
//   3. count: per row, the number of members of the neighbouring slots
//             with a positive weight; an inclusive scan gives the CSR rows;
//   4. fill:  the same traversal writes column, weight and the row sum in a
//             fixed order (deterministic);
//   5. filter (every call): s~_a = sum_b W_ab rho_b s_b / (rho_a R_a) with a
//             lane group per row and a fixed-order butterfly reduction.
//
// Rows are processed in hash order in steps 3 and 4 so that the threads of a
// wave scan the same slots; the filter runs rows in their own order.

#include <hip/hip_runtime.h>
#include <hipcub/hipcub.hpp>

#include <algorithm>
#include <cmath>
#include <cstdint>

#include "topo.h"

namespace {

constexpr int64_t kMaxPoints = 0x7ffffffe;  // column indices are int32
constexpr size_t kAlign = 256;

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

uint32_t table_bits(int64_t n) {
  uint32_t b = 6;
  while ((int64_t(1) << b) < n && b < 30) ++b;
  return b;
}

struct EdmLayout {
  uint32_t bits = 0;
  size_t keys_in = 0, keys_out = 0, idx_in = 0, idx_out = 0, counts = 0, starts = 0, rowcnt = 0,
         temp = 0, temp_bytes = 0, total = 0;
};

hipError_t edm_layout(int64_t n, EdmLayout& L) {
  L.bits = table_bits(n);
  const size_t T = size_t(1) << L.bits;
  const size_t nn = size_t(n > 0 ? n : 1);
  size_t sort_bytes = 0, scan_a = 0, scan_b = 0;
  hipError_t e = hipcub::DeviceRadixSort::SortPairs(nullptr, sort_bytes, (uint32_t*)nullptr,
                                                    (uint32_t*)nullptr, (int32_t*)nullptr,
                                                    (int32_t*)nullptr, (int)nn, 0, (int)L.bits);
  if (e != hipSuccess) return e;
  e = hipcub::DeviceScan::ExclusiveSum(nullptr, scan_a, (int32_t*)nullptr, (int32_t*)nullptr,
                                       (int)(T + 1));
  if (e != hipSuccess) return e;
  e = hipcub::DeviceScan::InclusiveSum(nullptr, scan_b, (int64_t*)nullptr, (int64_t*)nullptr,
                                       (int)nn);
  if (e != hipSuccess) return e;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off += align_up(bytes);
    return o;
  };
  L.keys_in = take(nn * 4);
  L.keys_out = take(nn * 4);
  L.idx_in = take(nn * 4);
  L.idx_out = take(nn * 4);
  L.counts = take((T + 1) * 4);
  L.starts = take((T + 1) * 4);
  L.rowcnt = take(nn * 8);
  L.temp_bytes = std::max(sort_bytes, std::max(scan_a, scan_b));
  L.temp = take(L.temp_bytes);
  L.total = off;
  return hipSuccess;
}

struct Cloud {
  const double* mid;  // SoA [dim][n]
  int64_t n;
  int dim;
  double rmin, inv_h;
  uint32_t mask;
};

__device__ __forceinline__ int64_t hash_coord(double v, double inv_h) {
  // bounded so that the conversion is defined for any finite midpoint
  const double f = fmin(fmax(floor(v * inv_h), -1.0e15), 1.0e15);
  return (int64_t)f;
}

__device__ __forceinline__ uint32_t slot_of(int64_t ix, int64_t iy, int64_t iz, uint32_t mask) {
  uint64_t h = (uint64_t)ix * 0x9E3779B97F4A7C15ull;
  h ^= (uint64_t)iy * 0xC2B2AE3D27D4EB4Full;
  h ^= (uint64_t)iz * 0x165667B19E3779F9ull;
  h ^= h >> 29;
  h *= 0xBF58476D1CE4E5B9ull;
  h ^= h >> 32;
  return (uint32_t)h & mask;
}

// eq. filter_cond: the weight of a pair; the one expression serves the count
// and the fill, so both see the same set of positive weights.
__device__ __forceinline__ double pair_weight(const Cloud& c, int64_t a, int64_t b, double xa,
                                              double ya, double za) {
  const double dx = c.mid[b] - xa;
  const double dy = c.mid[c.n + b] - ya;
  double d2 = __fma_rn(dy, dy, dx * dx);
  if (c.dim == 3) {
    const double dz = c.mid[2 * c.n + b] - za;
    d2 = __fma_rn(dz, dz, d2);
  }
  return c.rmin - sqrt(d2);
}

__global__ void edm_key_kernel(Cloud c, uint32_t* keys, int32_t* idx, int32_t* counts) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= c.n) return;
  const int64_t ix = hash_coord(c.mid[i], c.inv_h);
  const int64_t iy = hash_coord(c.mid[c.n + i], c.inv_h);
  const int64_t iz = c.dim == 3 ? hash_coord(c.mid[2 * c.n + i], c.inv_h) : 0;
  const uint32_t s = slot_of(ix, iy, iz, c.mask);
  keys[i] = s;
  idx[i] = (int32_t)i;
  atomicAdd(&counts[s], 1);  // integer: the histogram does not depend on order
}

__global__ void zero_i32_kernel(int32_t* p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

__global__ void rowptr_head_kernel(int64_t* rowptr) { rowptr[0] = 0; }

// Steps 3 and 4.  FILL = false: rowcnt[a] = number of positive weights of
// row a.  FILL = true: writes the row's columns and weights from rowptr[a]
// and its row sum R[a].
template <bool FILL>
__global__ __launch_bounds__(256) void edm_rows_kernel(Cloud c, const int32_t* __restrict__ order,
                                                       const int32_t* __restrict__ starts,
                                                       int64_t* rowcnt, const int64_t* rowptr,
                                                       int32_t* col, double* w, double* R) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= c.n) return;
  const int64_t a = order[t];
  const double xa = c.mid[a], ya = c.mid[c.n + a];
  const double za = c.dim == 3 ? c.mid[2 * c.n + a] : 0.0;
  const int64_t ix = hash_coord(xa, c.inv_h), iy = hash_coord(ya, c.inv_h);
  const int64_t iz = c.dim == 3 ? hash_coord(za, c.inv_h) : 0;
  const int nz = c.dim == 3 ? 3 : 1;
  uint32_t seen[27];
  int nseen = 0;
  int64_t k = FILL ? rowptr[a] : 0;
  const int64_t kend = FILL ? rowptr[a + 1] : 0;
  int64_t cnt = 0;
  double rsum = 0.0;
  for (int oz = 0; oz < nz; ++oz)
    for (int oy = 0; oy < 3; ++oy)
      for (int ox = 0; ox < 3; ++ox) {
        const uint32_t s =
            slot_of(ix + ox - 1, iy + oy - 1, c.dim == 3 ? iz + oz - 1 : 0, c.mask);
        // two neighbouring chunks that share a slot are scanned once
        bool dup = false;
        for (int q = 0; q < nseen; ++q) dup |= seen[q] == s;
        if (dup) continue;
        seen[nseen++] = s;
        const int32_t p1 = starts[s + 1];
        for (int32_t p = starts[s]; p < p1; ++p) {
          const int64_t b = order[p];
          const double wv = pair_weight(c, a, b, xa, ya, za);
          if (wv > 0.0) {
            if (FILL) {
              if (k < kend) {
                col[k] = (int32_t)b;
                w[k] = wv;
                ++k;
              }
              rsum += wv;
            } else {
              ++cnt;
            }
          }
        }
      }
  if (FILL) {
    // the count used the same expression, so k == kend here; should it not,
    // the row is padded with zero weights on its own column, never left
    // holding unwritten column indices
    for (; k < kend; ++k) {
      col[k] = (int32_t)a;
      w[k] = 0.0;
    }
    R[a] = rsum;
  }
  else
    rowcnt[a] = cnt;
}

// Step 5: G lanes per row, G in {16, 32, 64}.  Rows are split into 8
// contiguous ranges, one per XCD (consecutive blocks go to consecutive
// XCDs), so each XCD's L2 holds the rho and s window of its own range only;
// within a range, rows are taken in a block-stride loop, and a row's lanes
// always share the loop condition.  Column indices and weights are read
// once, with non-temporal loads, so that they do not evict that window.
// gridDim.x is a multiple of 8.
template <int G>
__global__ __launch_bounds__(256) void edm_filter_kernel(int64_t n, const int64_t* __restrict__ rowptr,
                                                         const int32_t* __restrict__ col,
                                                         const double* __restrict__ w,
                                                         const double* __restrict__ R,
                                                         const double* __restrict__ rho,
                                                         const double* __restrict__ dc,
                                                         double* __restrict__ dcf) {
  constexpr int kRows = 256 / G;
  constexpr int kU = 8;
  const int lane = threadIdx.x & (G - 1);
  const int64_t xcd = blockIdx.x & 7, q = blockIdx.x >> 3;
  const int64_t per_xcd = gridDim.x >> 3;
  const int64_t chunk = (n + 7) >> 3;
  const int64_t r1 = min(n, (xcd + 1) * chunk);
  for (int64_t g = xcd * chunk + q * kRows + threadIdx.x / G; g < r1; g += per_xcd * kRows) {
    double acc = 0.0;
    const int64_t k1 = rowptr[g + 1];
    // kU entries per lane in flight: their column and weight loads are
    // issued together, then the gathers; entries past the row's end read
    // the row's own cell with a zero weight
    for (int64_t k = rowptr[g] + lane; k < k1; k += kU * G) {
      int32_t b[kU];
      double wv[kU];
#pragma unroll
      for (int u = 0; u < kU; ++u) {
        const int64_t kk = k + u * G;
        const bool ok = kk < k1;
        b[u] = ok ? __builtin_nontemporal_load(col + kk) : (int32_t)g;
        wv[u] = ok ? __builtin_nontemporal_load(w + kk) : 0.0;
      }
#pragma unroll
      for (int u = 0; u < kU; ++u) acc += wv[u] * (rho[b[u]] * dc[b[u]]);
    }
#pragma unroll
    for (int m = G / 2; m > 0; m >>= 1) acc += __shfl_xor(acc, m, G);
    if (lane == 0) dcf[g] = acc / (rho[g] * R[g]);
  }
}

int grid_of(int64_t work, int block) { return (int)((work + block - 1) / block); }

bool bad_cloud(const double* mid, int32_t dim, int64_t n, double rmin) {
  return (dim != 2 && dim != 3) || !(rmin > 0.0) || !std::isfinite(rmin) || (n > 0 && !mid);
}

}  // namespace

extern "C" {

int topo_edm_workspace_size(int64_t n, size_t* bytes) {
  if (!bytes) return TOPO_E_INVALID;
  if (n < 0 || n > kMaxPoints) return TOPO_E_SHAPE;
  EdmLayout L;
  if (edm_layout(n, L) != hipSuccess) return TOPO_E_HIP;
  *bytes = L.total;
  return TOPO_OK;
}

int topo_edm_count(const double* mid, int32_t dim, int64_t n, double rmin, int64_t* rowptr,
                   void* work, size_t work_bytes, void* stream) {
  if (bad_cloud(mid, dim, n, rmin) || !rowptr || (n > 0 && !work)) return TOPO_E_INVALID;
  if (n < 0 || n > kMaxPoints) return TOPO_E_SHAPE;
  if (reinterpret_cast<uintptr_t>(work) % kAlign) return TOPO_E_WORKSPACE;
  EdmLayout L;
  if (edm_layout(n, L) != hipSuccess) return TOPO_E_HIP;
  if (work_bytes < L.total) return TOPO_E_WORKSPACE;
  hipStream_t st = (hipStream_t)stream;
  rowptr_head_kernel<<<1, 1, 0, st>>>(rowptr);
  if (n == 0) return hipGetLastError() == hipSuccess ? TOPO_OK : TOPO_E_HIP;
  char* base = static_cast<char*>(work);
  auto* keys_in = reinterpret_cast<uint32_t*>(base + L.keys_in);
  auto* keys_out = reinterpret_cast<uint32_t*>(base + L.keys_out);
  auto* idx_in = reinterpret_cast<int32_t*>(base + L.idx_in);
  auto* idx_out = reinterpret_cast<int32_t*>(base + L.idx_out);
  auto* counts = reinterpret_cast<int32_t*>(base + L.counts);
  auto* starts = reinterpret_cast<int32_t*>(base + L.starts);
  auto* rowcnt = reinterpret_cast<int64_t*>(base + L.rowcnt);
  void* temp = base + L.temp;
  const int64_t T = int64_t(1) << L.bits;
  const Cloud c{mid, n, dim, rmin, 1.0 / rmin, (uint32_t)(T - 1)};
  zero_i32_kernel<<<grid_of(T + 1, 256), 256, 0, st>>>(counts, T + 1);
  edm_key_kernel<<<grid_of(n, 256), 256, 0, st>>>(c, keys_in, idx_in, counts);
  size_t tb = L.temp_bytes;
  if (hipcub::DeviceRadixSort::SortPairs(temp, tb, keys_in, keys_out, idx_in, idx_out, (int)n, 0,
                                         (int)L.bits, st) != hipSuccess)
    return TOPO_E_HIP;
  tb = L.temp_bytes;
  if (hipcub::DeviceScan::ExclusiveSum(temp, tb, counts, starts, (int)(T + 1), st) != hipSuccess)
    return TOPO_E_HIP;
  edm_rows_kernel<false><<<grid_of(n, 256), 256, 0, st>>>(c, idx_out, starts, rowcnt, nullptr,
                                                          nullptr, nullptr, nullptr);
  tb = L.temp_bytes;
  if (hipcub::DeviceScan::InclusiveSum(temp, tb, rowcnt, rowptr + 1, (int)n, st) != hipSuccess)
    return TOPO_E_HIP;
  return hipGetLastError() == hipSuccess ? TOPO_OK : TOPO_E_HIP;
}

int topo_edm_fill(const double* mid, int32_t dim, int64_t n, double rmin, const int64_t* rowptr,
                  int32_t* col, double* w, double* R, void* work, size_t work_bytes,
                  void* stream) {
  if (bad_cloud(mid, dim, n, rmin) || !rowptr) return TOPO_E_INVALID;
  if (n < 0 || n > kMaxPoints) return TOPO_E_SHAPE;
  if (n == 0) return TOPO_OK;
  if (!col || !w || !R || !work) return TOPO_E_INVALID;
  if (reinterpret_cast<uintptr_t>(work) % kAlign) return TOPO_E_WORKSPACE;
  EdmLayout L;
  if (edm_layout(n, L) != hipSuccess) return TOPO_E_HIP;
  if (work_bytes < L.total) return TOPO_E_WORKSPACE;
  char* base = static_cast<char*>(work);
  const int64_t T = int64_t(1) << L.bits;
  const Cloud c{mid, n, dim, rmin, 1.0 / rmin, (uint32_t)(T - 1)};
  edm_rows_kernel<true><<<grid_of(n, 256), 256, 0, (hipStream_t)stream>>>(
      c, reinterpret_cast<const int32_t*>(base + L.idx_out),
      reinterpret_cast<const int32_t*>(base + L.starts), nullptr, rowptr, col, w, R);
  return hipGetLastError() == hipSuccess ? TOPO_OK : TOPO_E_HIP;
}

int topo_edm_filter(int64_t n, int64_t nnz, const int64_t* rowptr, const int32_t* col,
                    const double* w, const double* R, const double* rho, const double* dc,
                    double* dcf, void* stream) {
  if (n < 0 || n > kMaxPoints || nnz < 0) return TOPO_E_SHAPE;
  if (n == 0) return TOPO_OK;
  if (!rowptr || !R || !rho || !dc || !dcf || (nnz > 0 && (!col || !w))) return TOPO_E_INVALID;
  hipStream_t st = (hipStream_t)stream;
  const double avg = double(nnz) / double(n);
  // up to 65536 blocks of 256 threads (a multiple of 8: one share per XCD);
  // longer inputs loop
  auto blocks = [&](int rows_per_block) {
    const int64_t b = std::min<int64_t>((n + rows_per_block - 1) / rows_per_block, 65536);
    return (int)((b + 7) / 8 * 8);
  };
  if (avg >= 48.0)
    edm_filter_kernel<64><<<blocks(4), 256, 0, st>>>(n, rowptr, col, w, R, rho, dc, dcf);
  else if (avg >= 24.0)
    edm_filter_kernel<32><<<blocks(8), 256, 0, st>>>(n, rowptr, col, w, R, rho, dc, dcf);
  else
    edm_filter_kernel<16><<<blocks(16), 256, 0, st>>>(n, rowptr, col, w, R, rho, dc, dcf);
  return hipGetLastError() == hipSuccess ? TOPO_OK : TOPO_E_HIP;
}

}  // extern "C"
