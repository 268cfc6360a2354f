// Device helpers shared by the kernels: deterministic two-stage reductions
// and the BF16 storage of moduli.
//
// Stage 1 (inside a wide kernel): every block reduces its values in a fixed
// order and writes them to partials[linear block id * 16 + k].
// Stage 2 (a one-block "finalise" kernel launched right after): the block
// sums the partials in block order and applies the scalar update.  Kernel
// boundaries make the partials visible across XCDs, so no device-scope
// fence is needed inside the wide kernel.
#pragma once

#include <hip/hip_runtime.h>

namespace topo {

constexpr int kPartStride = 16;

// A modulus stored in BF16: the upper 16 bits of an IEEE single.
struct bf16m {
  uint16_t bits;
  __device__ __forceinline__ explicit operator float() const {
    return __uint_as_float((uint32_t)bits << 16);
  }
  __device__ __forceinline__ explicit operator double() const { return (double)float(*this); }
};

// Nearest BF16 of an FP64 value, ties to even, rounded once from the FP64
// bits (no intermediate FP32 rounding).  Values below the smallest normal
// BF16 give a signed zero, values above the largest finite BF16 a signed
// infinity; NaN is not expected (moduli are finite and non-negative).
__device__ inline uint16_t bf16_from_f64(double v) {
  const uint64_t u = (uint64_t)__double_as_longlong(v);
  const uint64_t sign = (u >> 63) << 15;
  const uint64_t mag = u & 0x7fffffffffffffffull;
  // keep 7 of the 52 fraction bits: add half an ulp minus one, plus the kept
  // lowest bit (ties to even), and drop the 45 low bits
  const uint64_t r = (mag + 0xfffffffffffull + ((mag >> 45) & 1)) >> 45;
  const int64_t e = (int64_t)(r >> 7) - 1023 + 127;   // BF16 biased exponent
  if (e <= 0) return (uint16_t)sign;
  if (e >= 255) return (uint16_t)(sign | 0x7f80);
  return (uint16_t)(sign | (uint64_t)(r - ((uint64_t)(1023 - 127) << 7)));
}

// Work-group barrier that orders LDS only.  __syncthreads() also waits for
// every outstanding global load and store of the wave, which would drain
// prefetches issued before the barrier; kernels whose barriers only hand LDS
// data between waves use this one.
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

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

__device__ inline size_t linear_block_id() {
  return blockIdx.x + (size_t)gridDim.x * (blockIdx.y + (size_t)gridDim.y * blockIdx.z);
}

// Stage 1: NV sums followed by NM maxima (maxima of non-negative values).
// blockDim.x must be a multiple of 64 and at most 1024.
template <int NV, int NM = 0>
__device__ inline void block_partials(const double (&v)[NV], const double (&vm)[NM > 0 ? NM : 1],
                                      double* partials) {
  constexpr int NT = NV + NM;
  __shared__ double wtmp[16][NT];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int nw = blockDim.x >> 6;
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    const double s = wave_sum(v[k]);
    if (lane == 0) wtmp[wid][k] = s;
  }
#pragma unroll
  for (int k = 0; k < NM; ++k) {
    const double s = wave_max(vm[k]);
    if (lane == 0) wtmp[wid][NV + k] = s;
  }
  __syncthreads();
  if (threadIdx.x < NT) {
    const int k = threadIdx.x;
    double s = 0.0;
    for (int w = 0; w < nw; ++w) s = (k < NV) ? s + wtmp[w][k] : fmax(s, wtmp[w][k]);
    partials[linear_block_id() * kPartStride + k] = s;
  }
}

// Stage 2, called by every thread of a single block: totals of the partials
// of blocks [b0, b1) in a fixed order (thread-strided over blocks, then a
// fixed tree).
template <int NV, int NM = 0>
__device__ inline void reduce_partials_range(const double* partials, long b0, long b1,
                                             double (&tot)[NV + NM]) {
  constexpr int NT = NV + NM;
  __shared__ double wtmp[16][NT];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int nw = blockDim.x >> 6;
  double acc[NT];
#pragma unroll
  for (int k = 0; k < NT; ++k) acc[k] = 0.0;
  // eight blocks' partials are loaded before any is added (independent
  // loads in flight); the additions keep the block order
  constexpr int U = 8;
  const long step = blockDim.x;
  long b = b0 + threadIdx.x;
  for (; b + (U - 1) * step < b1; b += U * step) {
    double xv[U][NT];
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int k = 0; k < NT; ++k) xv[u][k] = partials[(b + u * step) * kPartStride + k];
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int k = 0; k < NT; ++k) acc[k] = (k < NV) ? acc[k] + xv[u][k] : fmax(acc[k], xv[u][k]);
  }
  // the thread's last (at most U - 1) blocks: their loads issued together
  // too, then added in the same order as above
  if (b < b1) {
    double xv[U - 1][NT];
#pragma unroll
    for (int u = 0; u < U - 1; ++u)
#pragma unroll
      for (int k = 0; k < NT; ++k)
        xv[u][k] = b + u * step < b1 ? partials[(b + u * step) * kPartStride + k] : 0.0;
#pragma unroll
    for (int u = 0; u < U - 1; ++u) {
      if (b + u * step < b1) {
#pragma unroll
        for (int k = 0; k < NT; ++k) acc[k] = (k < NV) ? acc[k] + xv[u][k] : fmax(acc[k], xv[u][k]);
      }
    }
  }
#pragma unroll
  for (int k = 0; k < NT; ++k) {
    const double s = (k < NV) ? wave_sum(acc[k]) : wave_max(acc[k]);
    if (lane == 0) wtmp[wid][k] = s;
  }
  __syncthreads();
  if (threadIdx.x < NT) {
    const int k = threadIdx.x;
    double s = 0.0;
    for (int w = 0; w < nw; ++w) s = (k < NV) ? s + wtmp[w][k] : fmax(s, wtmp[w][k]);
    tot[k] = s;
  }
  __syncthreads();
}

template <int NV, int NM = 0>
__device__ inline void reduce_partials(const double* partials, long nb, double (&tot)[NV + NM]) {
  reduce_partials_range<NV, NM>(partials, 0, nb, tot);
}

}  // namespace topo
