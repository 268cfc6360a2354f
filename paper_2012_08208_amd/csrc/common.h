// Device helpers shared by the kernels: deterministic block reductions and
// the single-pass "last block finalises" grid reduction.
#pragma once

#include <hip/hip_runtime.h>

namespace topo {

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}

__device__ inline double wave_max(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_down(v, off, 64));
  return v;
}

// Sums NV values over the block in a fixed order; result valid in thread 0
// (and returned via the shared array red_out to every thread after the
// barrier).  blockDim.x must be a multiple of 64 and at most 1024.
template <int NV>
__device__ inline void block_sum(double (&v)[NV], double (&red_out)[NV]) {
  __shared__ double wsum[16][NV];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int nw = blockDim.x >> 6;
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    double s = wave_sum(v[k]);
    if (lane == 0) wsum[wid][k] = s;
  }
  __syncthreads();
  if (threadIdx.x < NV) {
    double s = 0.0;
    for (int w = 0; w < nw; ++w) s += wsum[w][threadIdx.x];
    red_out[threadIdx.x] = s;
  }
  __syncthreads();
}

// Writes this block's NV partial sums (and NM partial maxima) to
// partials[linear block id * 16 + k], then the last block to arrive sums all blocks in
// block order and leaves the totals in tot[] (shared).  Returns true in the
// last block only.  Deterministic: the summation order is fixed.
template <int NV, int NM = 0>
__device__ inline bool grid_reduce(double (&v)[NV], double (&vm)[NM > 0 ? NM : 1], double* partials,
                                   unsigned* counter, double (&tot)[NV + (NM > 0 ? NM : 0)]) {
  __shared__ double bsum[NV + (NM > 0 ? NM : 0)];
  __shared__ double wtmp[16][NV + (NM > 0 ? NM : 0)];
  __shared__ int am_last;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int nw = blockDim.x >> 6;
  constexpr int NT = NV + (NM > 0 ? NM : 0);
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    double s = wave_sum(v[k]);
    if (lane == 0) wtmp[wid][k] = s;
  }
#pragma unroll
  for (int k = 0; k < NM; ++k) {
    double s = wave_max(vm[k]);
    if (lane == 0) wtmp[wid][NV + k] = s;
  }
  __syncthreads();
  if (threadIdx.x < NT) {
    const int k = threadIdx.x;
    double s = (k < NV) ? 0.0 : -1.0;
    for (int w = 0; w < nw; ++w) s = (k < NV) ? s + wtmp[w][k] : fmax(s, wtmp[w][k]);
    bsum[k] = s;
    const size_t bid = blockIdx.x + (size_t)gridDim.x * (blockIdx.y + (size_t)gridDim.y * blockIdx.z);
    partials[bid * 16 + k] = s;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    __threadfence();
    unsigned nb = gridDim.x * gridDim.y * gridDim.z;
    unsigned prev = __hip_atomic_fetch_add(counter, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
    am_last = (prev == nb - 1);
  }
  __syncthreads();
  if (!am_last) return false;
  __threadfence();
  const unsigned nb = gridDim.x * gridDim.y * gridDim.z;
  // per-thread strided partial sums in block order, then fixed-tree combine
  double acc[NT];
#pragma unroll
  for (int k = 0; k < NT; ++k) acc[k] = (k < NV) ? 0.0 : -1.0;
  for (unsigned b = threadIdx.x; b < nb; b += blockDim.x) {
#pragma unroll
    for (int k = 0; k < NT; ++k) {
      double x = __builtin_nontemporal_load(&partials[(size_t)b * 16 + k]);
      acc[k] = (k < NV) ? acc[k] + x : fmax(acc[k], x);
    }
  }
#pragma unroll
  for (int k = 0; k < NT; ++k) {
    double s = (k < NV) ? wave_sum(acc[k]) : wave_max(acc[k]);
    if (lane == 0) wtmp[wid][k] = s;
  }
  __syncthreads();
  if (threadIdx.x < NT) {
    const int k = threadIdx.x;
    double s = (k < NV) ? 0.0 : -1.0;
    for (int w = 0; w < nw; ++w) s = (k < NV) ? s + wtmp[w][k] : fmax(s, wtmp[w][k]);
    tot[k] = s;
  }
  if (threadIdx.x == 0) *counter = 0u;
  __syncthreads();
  return true;
}

}  // namespace topo
