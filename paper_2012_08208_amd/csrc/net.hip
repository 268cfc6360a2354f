// The convolutional preconditioner network on gfx950: forward, backward,
// K-norm training loss and Adam (the network is this library's addition to
// the method; the paper has no learned component).
//
// Convolutions are implicit GEMMs on MFMA 16x16x32 BF16 tiles with FP32
// accumulation.  For the forward (and the input gradient, which is again a
// convolution) the GEMM rows are output voxels, the columns output channels
// and the reduction runs over (tap, input channel): a lane's eight K values
// are eight consecutive channels of one tap of one voxel, a 16-byte load
// from the channels-last activation.  The weight gradient reduces over
// voxels instead; its two operands are staged through LDS transposed so
// that the voxel run of a channel is contiguous.
#include <limits.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include <new>

#include "common.h"
#include "net.h"
#include "topo_internal.h"

namespace topo {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }
__device__ __forceinline__ uint16_t f2bf(float f) {  // nearest, ties to even
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

static inline unsigned cdiv(long a, long b) { return (unsigned)((a + b - 1) / b); }

// layer table: level of the input, stride, cin, cout, leaky ReLU
static const int kSpec[kNetLayers][5] = {
    {0, 1, 8, 16, 1},   {0, 1, 16, 16, 1},  {0, 2, 16, 32, 1}, {1, 1, 32, 32, 1},
    {1, 2, 32, 64, 1},  {2, 1, 64, 64, 1},  {2, 2, 64, 64, 1}, {3, 1, 64, 64, 1},
    {2, 1, 128, 64, 1}, {1, 1, 96, 32, 1},  {0, 1, 48, 16, 1}, {0, 1, 16, 3, 0}};

static long round_up(long x, long m) { return (x + m - 1) / m * m; }

// ------------------------------------------------------------------ weights
// BF16 copies of one layer's FP32 weights W[co][t][ci]:
//   wf[co][k], k = t*cin + ci                       (rows padded to coutp)
//   wb[ci][k], k = t'*coutp + co, with W[co][26-t'][ci] for stride 1 (the
//   input gradient of a stride-1 convolution is the convolution with the
//   flipped kernel) and W[co][t'][ci] for stride 2 (used by the transposed
//   gather, which flips through its index map).
__global__ void weights_bf16_kernel(const float* __restrict__ w, uint16_t* wf, uint16_t* wb, int cin,
                                    int cout, int coutp, int kf, int kb, int stride, int cinp) {
  const long nf = (long)coutp * kf, nb = (long)cinp * kb;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < nf + nb;
       i += (long)gridDim.x * blockDim.x) {
    if (i < nf) {
      const int co = (int)(i / kf), k = (int)(i % kf);
      float v = 0.f;
      if (co < cout && k < 27 * cin) {
        const int t = k / cin, ci = k % cin;
        v = w[((long)co * 27 + t) * cin + ci];
      }
      wf[i] = f2bf(v);
    } else {
      const long j = i - nf;
      const int ci = (int)(j / kb), k = (int)(j % kb);
      float v = 0.f;
      if (ci < cin && k < 27 * coutp) {
        const int t = k / coutp, co = k % coutp;
        const int ts = stride == 1 ? 26 - t : t;
        if (co < cout) v = w[((long)co * 27 + ts) * cin + ci];
      }
      wb[j] = f2bf(v);
    }
  }
}

// -------------------------------------------------------------- convolution
struct ConvArgs {
  const uint16_t* x;
  int xpitch, xoff, cin;
  int inx, iny, inz;
  int onx, ony, onz;
  long nout;
  const uint16_t* w;
  int kpad, ktot;
  uint16_t* y;
  int ypitch, yoff, cout;
  float* ysoa;               // output layer: FP32 [cout][nout] instead of y
  const uint16_t* gate;      // multiply by the leaky-ReLU slope where gate <= 0
  int gpitch, goff;
  int act, accum;
  const int* stop;
};

// MODE 0: stride 1; MODE 1: stride 2 (output grid = ceil(input/2));
// MODE 2: transposed stride 2 (input = coarse grid, output = fine grid):
//   out[i] = sum_t W'[t] in[(i + 1 - d_t)/2] over taps where that is an
//   integer inside the coarse grid.
// A wave computes 32 output voxels x NCT*16 output channels.
template <int MODE, int NCT>
__global__ __launch_bounds__(256) void conv_kernel(ConvArgs a) {
  if (a.stop && *a.stop) return;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int row = lane & 15, kg = lane >> 4;
  const long base = ((long)blockIdx.x * 4 + wave) * 32;
  if (base >= a.nout) return;
  int ox[2], oy[2], oz[2];
#pragma unroll
  for (int mt = 0; mt < 2; ++mt) {
    long m = base + mt * 16 + row;
    if (m >= a.nout) m = a.nout - 1;  // clamped: computed, never stored
    ox[mt] = (int)(m % a.onx);
    const long t = m / a.onx;
    oy[mt] = (int)(t % a.ony);
    oz[mt] = (int)(t / a.ony);
  }
  f32x4 acc[2][NCT];
#pragma unroll
  for (int mt = 0; mt < 2; ++mt)
#pragma unroll
    for (int ct = 0; ct < NCT; ++ct) acc[mt][ct] = f32x4{0.f, 0.f, 0.f, 0.f};
  const int nks = a.kpad >> 5;
  for (int ks = 0; ks < nks; ++ks) {
    const int k0 = ks * 32 + kg * 8;
    uint4 av[2];
#pragma unroll
    for (int mt = 0; mt < 2; ++mt) av[mt] = make_uint4(0, 0, 0, 0);
    if (k0 < a.ktot) {
      const int tap = k0 / a.cin, ci = k0 - tap * a.cin;
      const int dz = tap / 9, dy = (tap / 3) % 3, dx = tap % 3;
#pragma unroll
      for (int mt = 0; mt < 2; ++mt) {
        int sx, sy, sz;
        bool ok;
        if (MODE == 0) {
          sx = ox[mt] + dx - 1; sy = oy[mt] + dy - 1; sz = oz[mt] + dz - 1;
          ok = sx >= 0 && sx < a.inx && sy >= 0 && sy < a.iny && sz >= 0 && sz < a.inz;
        } else if (MODE == 1) {
          sx = 2 * ox[mt] + dx - 1; sy = 2 * oy[mt] + dy - 1; sz = 2 * oz[mt] + dz - 1;
          ok = sx >= 0 && sx < a.inx && sy >= 0 && sy < a.iny && sz >= 0 && sz < a.inz;
        } else {
          const int tx = ox[mt] + 1 - dx, ty = oy[mt] + 1 - dy, tz = oz[mt] + 1 - dz;
          ok = tx >= 0 && ty >= 0 && tz >= 0 && !(tx & 1) && !(ty & 1) && !(tz & 1);
          sx = tx >> 1; sy = ty >> 1; sz = tz >> 1;
          ok = ok && sx < a.inx && sy < a.iny && sz < a.inz;
        }
        if (ok) {
          const long src = ((long)sz * a.iny + sy) * a.inx + sx;
          av[mt] = *reinterpret_cast<const uint4*>(a.x + src * a.xpitch + a.xoff + ci);
        }
      }
    }
#pragma unroll
    for (int ct = 0; ct < NCT; ++ct) {
      const uint4 wv = *reinterpret_cast<const uint4*>(a.w + (long)(ct * 16 + row) * a.kpad + k0);
      const bf16x8 bv = __builtin_bit_cast(bf16x8, wv);
#pragma unroll
      for (int mt = 0; mt < 2; ++mt)
        acc[mt][ct] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, av[mt]), bv,
                                                              acc[mt][ct], 0, 0, 0);
    }
  }
  // C tile: lane holds column (channel) row, rows (voxels) 4*kg + i
#pragma unroll
  for (int mt = 0; mt < 2; ++mt) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const long m = base + mt * 16 + kg * 4 + i;
      if (m >= a.nout) continue;
#pragma unroll
      for (int ct = 0; ct < NCT; ++ct) {
        const int co = ct * 16 + row;
        if (co >= a.cout) continue;
        float v = acc[mt][ct][i];
        if (a.ysoa) {
          a.ysoa[(long)co * a.nout + m] = v;
          continue;
        }
        uint16_t* yp = a.y + m * a.ypitch + a.yoff + co;
        if (a.accum) v += bf2f(*yp);
        if (a.gate && !(bf2f(a.gate[m * a.gpitch + a.goff + co]) > 0.f)) v *= kSlope;
        if (a.act && !(v > 0.f)) v *= kSlope;
        *yp = f2bf(v);
      }
    }
  }
}

template <int MODE>
static void conv_dispatch(int nct, dim3 g, hipStream_t s, const ConvArgs& a) {
  switch (nct) {
    case 1: conv_kernel<MODE, 1><<<g, 256, 0, s>>>(a); break;
    case 2: conv_kernel<MODE, 2><<<g, 256, 0, s>>>(a); break;
    case 3: conv_kernel<MODE, 3><<<g, 256, 0, s>>>(a); break;
    case 4: conv_kernel<MODE, 4><<<g, 256, 0, s>>>(a); break;
    case 6: conv_kernel<MODE, 6><<<g, 256, 0, s>>>(a); break;
    default: conv_kernel<MODE, 8><<<g, 256, 0, s>>>(a); break;
  }
}

// ------------------------------------------------ tiled forward convolution
// The forward layers run as implicit GEMMs over LDS-staged input tiles: a
// block owns a TX x TY x TZ box of output voxels and stages the input voxels
// it reads (its box plus the one-voxel halo; for stride 2 the box at twice
// the spacing), 32 channels at a time, zero outside the grid.  Every tap
// then reads its MFMA operand from LDS at a fixed offset from the lane's
// voxel, so each input voxel comes from L2 once per block and channel chunk
// instead of once per tap.  The K loop runs over the chunk's taps, unrolled
// at compile time (LDS and weight offsets are instruction immediates): with
// 32 staged channels one MFMA step is one tap; with 16 (8) channels one step
// covers 2 (4) consecutive taps, the lanes of K group kg taking tap
// t0 + kg*8/CC.  On large grids a block computes all output channels of an
// 8x8x4 box, one wave per 64 voxels.  On small grids (few boxes) a block
// computes 16 output channels of a 4x4x4 box and its 4 waves take every
// fourth K step; their FP32 sums are added through LDS in wave order.  The
// epilogue transposes each wave's C tile through LDS so that a lane stores
// 8 channels of a voxel at once.  The weights keep the wf layout
// [co][tap*cin + ci].

template <int V>
struct IC {
  static constexpr int value = V;
};

// lane offset (staged voxels) of tap t inside the input box
template <int MODE, int IX, int IY>
__host__ __device__ constexpr int tap_off(int t) {
  return ((t / 9) * IY + (t / 3) % 3) * IX + t % 3;
}

template <int MODE, int CIN, int NCT, int TX, int TY, int TZ, int WK>
__global__ __launch_bounds__(256) void convt_kernel(ConvArgs a) {
  constexpr int S = MODE == 1 ? 2 : 1;
  constexpr int IX = MODE == 1 ? 2 * TX + 1 : TX + 2;
  constexpr int IY = MODE == 1 ? 2 * TY + 1 : TY + 2;
  constexpr int IZ = MODE == 1 ? 2 * TZ + 1 : TZ + 2;
  constexpr int VI = IX * IY * IZ;
  constexpr int MTILES = TX * TY * TZ / 16;
  constexpr int WM = 4 / WK;
  constexpr int MT = MTILES / WM;
  constexpr int NCH = (CIN + 31) / 32;
  constexpr int CC0 = CIN < 32 ? CIN : 32;   // channels of the first (widest) chunk
  constexpr int PC = CC0 / 8;                 // staged 16-byte pieces per voxel
  constexpr int kLP = CC0 + 8;                // LDS pitch (bf16) of a staged voxel
  constexpr int VB = kLP * 2;                 // ... in bytes
  constexpr int NQ = (VI * PC + 255) / 256;   // staged pieces per thread
  constexpr int KPAD = (27 * CIN + 31) / 32 * 32;
  constexpr int NSPLIT = WK;
  constexpr int RED = WK > 1 ? (WK - 1) * MT * NCT * 4 * 64 : 0;   // floats
  constexpr int EPI = (WK > 1 ? 1 : WM) * MT * 16 * (NCT * 16 + 4);  // floats
  constexpr int LDS1 = VI * VB > RED * 4 ? VI * VB : RED * 4;
  constexpr int LDSB = LDS1 > EPI * 4 ? LDS1 : EPI * 4;
  static_assert(MTILES % WM == 0, "tile does not split over the waves");
  static_assert(CIN % 8 == 0, "channels must be a multiple of 8");
  static_assert(NCH <= 4 && NSPLIT <= 4, "unsupported layer shape");
  __shared__ __attribute__((aligned(16))) char smem[LDSB];
  const int stopped = a.stop ? *a.stop : 0;   // checked once the first tile loads are in flight
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wm = wave / WK, wk = wave % WK;
  const int row = lane & 15, kg = lane >> 4;
  const int gx = (a.onx + TX - 1) / TX, gy = (a.ony + TY - 1) / TY;
  const int tile = blockIdx.x;
  const int X0 = (tile % gx) * TX, Y0 = ((tile / gx) % gy) * TY, Z0 = (tile / (gx * gy)) * TZ;
  const int cb = blockIdx.y;   // output channels cb*NCT*16 .. +NCT*16
  const int q = wk;            // this wave's share of the K steps (uniform)

  // staging: thread tid moves pieces tid + 256 j (voxel, 16-byte piece);
  // offsets past the buffer (outside the grid) load zeros
  const int ix0 = S * X0 - 1, iy0 = S * Y0 - 1, iz0 = S * Z0 - 1;
  const unsigned nbytes = (unsigned)((long)a.inx * a.iny * a.inz * a.xpitch * 2);
  const __amdgpu_buffer_rsrc_t xr =
      __builtin_amdgcn_make_buffer_rsrc(const_cast<uint16_t*>(a.x), 0, (int)nbytes, 0x00020000);
  int voff[NQ];
#pragma unroll
  for (int j = 0; j < NQ; ++j) {
    const int it = tid + 256 * j;
    const int v = it / PC, pc = it % PC;
    const int vx = v % IX, vy = (v / IX) % IY, vz = v / (IX * IY);
    const int sx = ix0 + vx, sy = iy0 + vy, sz = iz0 + vz;
    const bool ok = it < VI * PC && sx >= 0 && sx < a.inx && sy >= 0 && sy < a.iny && sz >= 0 &&
                    sz < a.inz;
    voff[j] = ok ? (((sz * a.iny + sy) * a.inx + sx) * a.xpitch + a.xoff + 8 * pc) * 2
                 : (int)0x80000000;
  }
  const int ldsw = (tid / PC) * VB + (tid % PC) * 16;

  int la[MT];   // LDS byte address of the lane's output voxel at tap (0,0,0), per M tile
#pragma unroll
  for (int mt = 0; mt < MT; ++mt) {
    const int ml = (wm * MT + mt) * 16 + row;
    const int x = ml % TX, y = (ml / TX) % TY, z = ml / (TX * TY);
    la[mt] = (((S * z) * IY + S * y) * IX + S * x) * VB;
  }
  f32x4 acc[MT][NCT];
#pragma unroll
  for (int mt = 0; mt < MT; ++mt)
#pragma unroll
    for (int ct = 0; ct < NCT; ++ct) acc[mt][ct] = f32x4{0.f, 0.f, 0.f, 0.f};

  auto chunk = [&](auto cc) {
    constexpr int C = decltype(cc)::value;
    constexpr int CC = (CIN - 32 * C) >= 32 ? 32 : (CIN - 32 * C);
    constexpr int TPS = 32 / CC;                  // taps per K step
    constexpr int NS = (27 + TPS - 1) / TPS;      // K steps of this chunk
    if (C > 0) __syncthreads();
#pragma unroll
    for (int j = 0; j < NQ; ++j) {
      if (j < NQ - 1 || tid + 256 * j < VI * PC) {
        const uint4 h = __builtin_bit_cast(
            uint4, __builtin_amdgcn_raw_buffer_load_b128(xr, voff[j] + 64 * C, 0, 0));
        *reinterpret_cast<uint4*>(smem + ldsw + j * (256 / PC) * VB) = h;
      }
    }
    if (C == 0 && stopped) return;   // uniform over the block
    __syncthreads();
    const int jl = (kg * 8) / CC;   // the lane's tap within a step
    const int cl = (kg * 8) % CC;   // the lane's channel offset within the chunk
    int lac[MT];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) lac[mt] = la[mt] + cl * 2;
    const unsigned wl = (unsigned)((row * KPAD + jl * CIN + 32 * C + cl) * 2);
    auto steps = [&](auto qq) {
      constexpr int Q = decltype(qq)::value;
#pragma unroll
      for (int s = Q; s < NS; s += NSPLIT) {
        const int t0 = s * TPS;
        const bool last = t0 + TPS > 27;          // some lanes' tap is past the end
        const bool tok = !last || jl < 27 - t0;
        // B: weights of the lane's tap
        bf16x8 bv[NCT];
#pragma unroll
        for (int ct = 0; ct < NCT; ++ct) {
          const char* wb =
              reinterpret_cast<const char*>(a.w) + ((cb * NCT + ct) * 16 * KPAD + t0 * CIN) * 2;
          const unsigned o = tok ? wl : 0u;
          bv[ct] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(wb + o));
        }
        // A: the lane's staged voxel at that tap
        int toff = tap_off<MODE, IX, IY>(t0 < 27 ? t0 : 26);
        if (TPS >= 2) toff = jl >= 1 ? tap_off<MODE, IX, IY>(t0 + 1 < 27 ? t0 + 1 : 26) : toff;
        if (TPS >= 4) {
          toff = jl >= 2 ? tap_off<MODE, IX, IY>(t0 + 2 < 27 ? t0 + 2 : 26) : toff;
          toff = jl >= 3 ? tap_off<MODE, IX, IY>(t0 + 3 < 27 ? t0 + 3 : 26) : toff;
        }
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
          uint4 av = *reinterpret_cast<const uint4*>(smem + lac[mt] + toff * VB);
          if (last && !tok) av = make_uint4(0, 0, 0, 0);
          const bf16x8 ab = __builtin_bit_cast(bf16x8, av);
#pragma unroll
          for (int ct = 0; ct < NCT; ++ct)
            acc[mt][ct] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ab, bv[ct], acc[mt][ct], 0, 0, 0);
        }
      }
    };
    switch (q) {
#define TOPO_Q(QV) \
  case QV:         \
    if constexpr (QV < NSPLIT) steps(IC<QV>{}); \
    break;
      TOPO_Q(0) TOPO_Q(1) TOPO_Q(2) TOPO_Q(3) TOPO_Q(4) TOPO_Q(5) TOPO_Q(6) TOPO_Q(7)
      TOPO_Q(8) TOPO_Q(9) TOPO_Q(10) TOPO_Q(11) TOPO_Q(12) TOPO_Q(13) TOPO_Q(14) TOPO_Q(15)
#undef TOPO_Q
      default: break;
    }
  };
  chunk(IC<0>{});
  if (stopped) return;
  if constexpr (NCH > 1) chunk(IC<1>{});
  if constexpr (NCH > 2) chunk(IC<2>{});
  if constexpr (NCH > 3) chunk(IC<3>{});

  // sums of the WK waves that share these voxels, in wave order
  __syncthreads();   // the staged tile is dead from here on
  if (WK > 1) {
    float* red = reinterpret_cast<float*>(smem);
    if (wk > 0) {
#pragma unroll
      for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int ct = 0; ct < NCT; ++ct)
#pragma unroll
          for (int i = 0; i < 4; ++i)
            red[((((wk - 1) * MT + mt) * NCT + ct) * 4 + i) * 64 + lane] = acc[mt][ct][i];
    }
    __syncthreads();
    if (wk > 0) return;
#pragma unroll 1
    for (int w = 0; w < WK - 1; ++w)
#pragma unroll
      for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int ct = 0; ct < NCT; ++ct)
#pragma unroll
          for (int i = 0; i < 4; ++i)
            acc[mt][ct][i] += red[(((w * MT + mt) * NCT + ct) * 4 + i) * 64 + lane];
    __builtin_amdgcn_wave_barrier();
  }

  // Epilogue: the wave turns its C tile (lane = channel, rows = voxels)
  // into [voxel][channel] rows in LDS, then each lane handles whole groups
  // of 8 channels of a voxel: 16-byte loads of the gate and accumulated
  // values, 16-byte stores.
  constexpr int CP = NCT * 16 + 4;            // floats per voxel row (16-byte aligned)
  constexpr int GPV = NCT * 2;                // 8-channel groups per voxel
  constexpr int ITEMS = MT * 16 * GPV;        // per wave
  float* eo = reinterpret_cast<float*>(smem) + (WK > 1 ? 0 : wm * (MT * 16 * CP));
#pragma unroll
  for (int mt = 0; mt < MT; ++mt)
#pragma unroll
    for (int ct = 0; ct < NCT; ++ct)
#pragma unroll
      for (int i = 0; i < 4; ++i) eo[(mt * 16 + 4 * kg + i) * CP + ct * 16 + row] = acc[mt][ct][i];
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
  for (int it0 = 0; it0 < ITEMS; it0 += 64) {
    const int it = it0 + lane;
    const int vl = it / GPV, gc = it % GPV;
    const int ml = wm * MT * 16 + vl;
    const int x = X0 + ml % TX, y = Y0 + (ml / TX) % TY, z = Z0 + ml / (TX * TY);
    if (x >= a.onx || y >= a.ony || z >= a.onz) continue;
    const int m = (z * a.ony + y) * a.onx + x;
    const float4 v0 = *reinterpret_cast<const float4*>(eo + vl * CP + gc * 8);
    const float4 v1 = *reinterpret_cast<const float4*>(eo + vl * CP + gc * 8 + 4);
    float v[8] = {v0.x, v0.y, v0.z, v0.w, v1.x, v1.y, v1.z, v1.w};
    const int c0 = cb * NCT * 16 + gc * 8;   // first of the item's 8 output channels
    if (a.ysoa) {
#pragma unroll
      for (int k = 0; k < 8; ++k)
        if (c0 + k < a.cout) a.ysoa[(long)(c0 + k) * a.nout + m] = v[k];
      continue;
    }
    // channels c0 .. +8 < C of the output and gate views (C is a multiple of 16)
    uint16_t* yp = a.y + (long)m * a.ypitch + a.yoff + c0;
    if (a.accum) {
      const uint4 h = *reinterpret_cast<const uint4*>(yp);
      const uint16_t* hs = reinterpret_cast<const uint16_t*>(&h);
#pragma unroll
      for (int k = 0; k < 8; ++k) v[k] += bf2f(hs[k]);
    }
    if (a.gate) {
      const uint4 h = *reinterpret_cast<const uint4*>(a.gate + (long)m * a.gpitch + a.goff + c0);
      const uint16_t* hs = reinterpret_cast<const uint16_t*>(&h);
#pragma unroll
      for (int k = 0; k < 8; ++k)
        if (!(bf2f(hs[k]) > 0.f)) v[k] *= kSlope;
    }
    if (a.act) {
#pragma unroll
      for (int k = 0; k < 8; ++k)
        if (!(v[k] > 0.f)) v[k] *= kSlope;
    }
    uint4 o;
    uint32_t* ow = reinterpret_cast<uint32_t*>(&o);
#pragma unroll
    for (int k = 0; k < 4; ++k)
      ow[k] = (uint32_t)__builtin_bit_cast(uint16_t, (__bf16)v[2 * k]) |
              ((uint32_t)__builtin_bit_cast(uint16_t, (__bf16)v[2 * k + 1]) << 16);
    *reinterpret_cast<uint4*>(yp) = o;
  }
}

// tile shape of a forward layer with output grid od: 8x8x4 boxes with all
// output channels per block (one wave per 64 voxels), or 4x4x4 boxes with
// one block per 16 output channels and the K steps dealt over 4 waves
struct ConvPlan {
  bool big;
  int tiles;
};

// big_min: output voxels from which stride-1 layers use the 8x8x4 boxes
static ConvPlan conv_plan(int mode, const int* od, long big_min) {
  ConvPlan p;
  const long nout = (long)od[0] * od[1] * od[2];
  p.big = mode == 0 && nout >= big_min;
  const int T[3] = {p.big ? 8 : 4, p.big ? 8 : 4, 4};
  p.tiles = (int)(((od[0] + T[0] - 1) / T[0]) * (long)((od[1] + T[1] - 1) / T[1]) *
                  ((od[2] + T[2] - 1) / T[2]));
  return p;
}

template <int MODE, int CIN, int NCT>
static void convt_go(const ConvPlan& p, hipStream_t s, const ConvArgs& a) {
  if constexpr (MODE == 0) {
    if (p.big) {
      convt_kernel<MODE, CIN, NCT, 8, 8, 4, 1><<<dim3((unsigned)p.tiles, 1), 256, 0, s>>>(a);
      return;
    }
  }
  convt_kernel<MODE, CIN, 1, 4, 4, 4, 4><<<dim3((unsigned)p.tiles, NCT), 256, 0, s>>>(a);
}

// forward layers by (mode, cin, output channel tiles); false if not covered
static bool convt_dispatch(int mode, int cin, int nct, const ConvPlan& p, hipStream_t s,
                           const ConvArgs& a) {
#define TOPO_CONVT(M, C, N)                                  \
  if (mode == M && cin == C && nct == N) {                   \
    convt_go<M, C, N>(p, s, a);                              \
    return true;                                             \
  }
  TOPO_CONVT(0, 8, 1)
  TOPO_CONVT(0, 16, 1)
  TOPO_CONVT(0, 48, 1)
  TOPO_CONVT(0, 32, 2)
  TOPO_CONVT(0, 96, 2)
  TOPO_CONVT(0, 64, 4)
  TOPO_CONVT(0, 128, 4)
  TOPO_CONVT(1, 16, 2)
  TOPO_CONVT(1, 32, 4)
  TOPO_CONVT(1, 64, 4)
#undef TOPO_CONVT
  return false;
}

// ----------------------------------------------------------- weight gradient
struct DwArgs {
  const uint16_t* x;
  int xpitch, xoff, cin;
  int inx, iny, inz;
  const uint16_t* dy;
  int dpitch, doff, cout, coutp;
  int onx, ony, onz;
  long nout;
  int stride, ncols;
  long chunk;
  float* part;   // [chunk][cout][ncols]
};

constexpr int kDwVox = 64;         // voxels per LDS stage
constexpr int kDwCols = 64;        // GEMM columns (tap, ci) per block
constexpr int kDwPad = kDwVox + 8; // LDS row pitch (elements)

// dW[co][j] = sum_m dy[m][co] * x[src(m, tap_j)][ci_j]: rows co, columns
// j = tap*cin + ci, reduction over the voxels of one chunk.  blockIdx.x picks
// 64 columns, blockIdx.y the chunk; wave w owns column tile w.
__global__ __launch_bounds__(256) void dw_kernel(DwArgs a) {
  __shared__ __attribute__((aligned(16))) uint16_t sdy[64 * kDwPad];
  __shared__ __attribute__((aligned(16))) uint16_t sx[kDwCols * kDwPad];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int row = lane & 15, kg = lane >> 4;
  const int j0 = blockIdx.x * kDwCols;
  const long m0 = (long)blockIdx.y * a.chunk;
  long m1 = m0 + a.chunk;
  if (m1 > a.nout) m1 = a.nout;
  const int nct = a.coutp >> 4;
  const int cg8 = a.coutp >> 3;
  f32x4 acc[4];
#pragma unroll
  for (int ct = 0; ct < 4; ++ct) acc[ct] = f32x4{0.f, 0.f, 0.f, 0.f};
  for (long v0 = m0; v0 < m1; v0 += kDwVox) {
    // stage dy^T: sdy[co][v]
    for (int idx = tid; idx < kDwVox * cg8; idx += 256) {
      const int v = idx / cg8, g = idx % cg8;
      const long m = v0 + v;
      uint4 h = make_uint4(0, 0, 0, 0);
      if (m < m1) h = *reinterpret_cast<const uint4*>(a.dy + m * a.dpitch + a.doff + g * 8);
      const uint16_t* hs = reinterpret_cast<const uint16_t*>(&h);
#pragma unroll
      for (int q = 0; q < 8; ++q) sdy[(g * 8 + q) * kDwPad + v] = hs[q];
    }
    // stage the im2col tile transposed: sx[j][v]
    for (int idx = tid; idx < kDwVox * (kDwCols / 8); idx += 256) {
      const int v = idx >> 3, g = idx & 7;
      const int j = j0 + g * 8;
      const long m = v0 + v;
      uint4 h = make_uint4(0, 0, 0, 0);
      if (m < m1 && j < a.ncols) {
        const int tap = j / a.cin, ci = j - tap * a.cin;
        const int dz = tap / 9, dyy = (tap / 3) % 3, dx = tap % 3;
        const int ox = (int)(m % a.onx);
        const long t = m / a.onx;
        const int oy = (int)(t % a.ony), oz = (int)(t / a.ony);
        const int sx0 = a.stride * ox + dx - 1, sy0 = a.stride * oy + dyy - 1,
                  sz0 = a.stride * oz + dz - 1;
        if (sx0 >= 0 && sx0 < a.inx && sy0 >= 0 && sy0 < a.iny && sz0 >= 0 && sz0 < a.inz) {
          const long src = ((long)sz0 * a.iny + sy0) * a.inx + sx0;
          h = *reinterpret_cast<const uint4*>(a.x + src * a.xpitch + a.xoff + ci);
        }
      }
      const uint16_t* hs = reinterpret_cast<const uint16_t*>(&h);
#pragma unroll
      for (int q = 0; q < 8; ++q) sx[(g * 8 + q) * kDwPad + v] = hs[q];
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < kDwVox / 32; ++kk) {
      const uint4 bw = *reinterpret_cast<const uint4*>(&sx[(wave * 16 + row) * kDwPad + kk * 32 + kg * 8]);
      const bf16x8 bv = __builtin_bit_cast(bf16x8, bw);
#pragma unroll
      for (int ct = 0; ct < 4; ++ct) {
        if (ct < nct) {
          const uint4 aw = *reinterpret_cast<const uint4*>(&sdy[(ct * 16 + row) * kDwPad + kk * 32 + kg * 8]);
          acc[ct] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, aw), bv,
                                                            acc[ct], 0, 0, 0);
        }
      }
    }
    __syncthreads();
  }
  const int j = j0 + wave * 16 + row;
  if (j >= a.ncols) return;
  float* out = a.part + (long)blockIdx.y * a.cout * a.ncols;
#pragma unroll
  for (int ct = 0; ct < 4; ++ct) {
    if (ct >= nct) break;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int co = ct * 16 + kg * 4 + i;
      if (co < a.cout) out[(long)co * a.ncols + j] = acc[ct][i];
    }
  }
}

// grad[off + i] = sum over chunks (fixed order) of part[chunk][i]
__global__ void dw_reduce_kernel(const float* __restrict__ part, float* grad, long len, int nchunks) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < len; i += (long)gridDim.x * blockDim.x) {
    float s = 0.f;
    for (int c = 0; c < nchunks; ++c) s += part[(long)c * len + i];
    grad[i] = s;
  }
}

// ------------------------------------------------- upsampling and transpose
// fine[i] = mean of coarse[lo], coarse[hi] per axis, lo = i>>1,
// hi = (i+1)>>1 (hi = lo past the coarse edge); 8 channels per thread.
__global__ void upsample_kernel(const uint16_t* __restrict__ c, int cpitch, uint16_t* f, int fpitch,
                                int foff, int C, int cnx, int cny, int cnz, int fnx, int fny, int fnz,
                                const int* stop) {
  if (stop && *stop) return;
  const int cg = C >> 3;
  const long n = (long)fnx * fny * fnz * cg;
  for (long idx = (long)blockIdx.x * blockDim.x + threadIdx.x; idx < n;
       idx += (long)gridDim.x * blockDim.x) {
    const int g = (int)(idx % cg);
    const long v = idx / cg;
    const int i = (int)(v % fnx);
    const long t = v / fnx;
    const int j = (int)(t % fny), k = (int)(t / fny);
    int xs[2] = {i >> 1, (i + 1) >> 1}, ys[2] = {j >> 1, (j + 1) >> 1}, zs[2] = {k >> 1, (k + 1) >> 1};
    if (xs[1] >= cnx) xs[1] = xs[0];
    if (ys[1] >= cny) ys[1] = ys[0];
    if (zs[1] >= cnz) zs[1] = zs[0];
    float s[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int e = 0; e < 2; ++e) {
          const long src = ((long)zs[a] * cny + ys[b]) * cnx + xs[e];
          const uint4 h = *reinterpret_cast<const uint4*>(c + src * cpitch + g * 8);
          const uint16_t* hs = reinterpret_cast<const uint16_t*>(&h);
#pragma unroll
          for (int q = 0; q < 8; ++q) s[q] += bf2f(hs[q]);
        }
    uint16_t o[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) o[q] = f2bf(0.125f * s[q]);
    *reinterpret_cast<uint4*>(f + v * fpitch + foff + g * 8) = *reinterpret_cast<const uint4*>(o);
  }
}

// per-axis weights of the fine points that interpolate from coarse point J
__device__ inline int up_weights(int J, int nf, int nc, int* idx, float* w) {
  int n = 0;
  for (int i = 2 * J - 1; i <= 2 * J + 1; ++i) {
    if (i < 0 || i >= nf) continue;
    const int lo = i >> 1;
    int hi = (i + 1) >> 1;
    if (hi >= nc) hi = lo;
    const float ww = 0.5f * (lo == J) + 0.5f * (hi == J);
    if (ww != 0.f) { idx[n] = i; w[n] = ww; ++n; }
  }
  return n;
}

// coarse gradient = P^T (fine gradient, channels [0, C) of the fine view),
// times the leaky-ReLU slope where the coarse activation is <= 0
__global__ void restrict_kernel(const uint16_t* __restrict__ f, int fpitch, uint16_t* c, int cpitch,
                                const uint16_t* __restrict__ gate, int C, int cnx, int cny, int cnz,
                                int fnx, int fny, int fnz) {
  const int cg = C >> 3;
  const long n = (long)cnx * cny * cnz * cg;
  for (long idx = (long)blockIdx.x * blockDim.x + threadIdx.x; idx < n;
       idx += (long)gridDim.x * blockDim.x) {
    const int g = (int)(idx % cg);
    const long v = idx / cg;
    const int I = (int)(v % cnx);
    const long t = v / cnx;
    const int J = (int)(t % cny), K = (int)(t / cny);
    int xi[3], yi[3], zi[3];
    float xw[3], yw[3], zw[3];
    const int nxw = up_weights(I, fnx, cnx, xi, xw);
    const int nyw = up_weights(J, fny, cny, yi, yw);
    const int nzw = up_weights(K, fnz, cnz, zi, zw);
    float s[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    for (int a = 0; a < nzw; ++a)
      for (int b = 0; b < nyw; ++b)
        for (int e = 0; e < nxw; ++e) {
          const float w = zw[a] * yw[b] * xw[e];
          const long src = ((long)zi[a] * fny + yi[b]) * fnx + xi[e];
          const uint4 h = *reinterpret_cast<const uint4*>(f + src * fpitch + g * 8);
          const uint16_t* hs = reinterpret_cast<const uint16_t*>(&h);
#pragma unroll
          for (int q = 0; q < 8; ++q) s[q] += w * bf2f(hs[q]);
        }
    const uint4 gh = *reinterpret_cast<const uint4*>(gate + v * cpitch + g * 8);
    const uint16_t* gs = reinterpret_cast<const uint16_t*>(&gh);
    uint16_t o[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) o[q] = f2bf(bf2f(gs[q]) > 0.f ? s[q] : kSlope * s[q]);
    *reinterpret_cast<uint4*>(c + v * cpitch + g * 8) = *reinterpret_cast<const uint4*>(o);
  }
}

// -------------------------------------------------------- FE-side plumbing
// partial sums of r.r (one load case, [3][nn])
__global__ __launch_bounds__(256) void rr_kernel(const double* __restrict__ r, long n, double* partials,
                                                 const int* stop) {
  if (stop && *stop) return;
  double acc[1] = {0.0};
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    acc[0] += r[i] * r[i];
  const double none[1] = {0.0};
  block_partials<1, 0>(acc, none, partials);
}

__global__ void rms_fin(const double* partials, long nb, long n, double* scal, const int* stop) {
  if (stop && *stop) return;
  __shared__ double tot[1];
  reduce_partials<1, 0>(partials, nb, tot);
  if (threadIdx.x == 0) scal[0] = sqrt(tot[0] / (double)n);
}

// gate input: [0] mean density of the incident tetrahedra, [4] 1 if any
// component of the node is fixed, other channels 0
__global__ void prep_gate_kernel(const double* __restrict__ rho, const uint8_t* __restrict__ mask,
                                 uint16_t* X0, int nx, int ny, int nz, const int* stop) {
  if (stop && *stop) return;
  const int nx1 = nx + 1, ny1 = ny + 1, nz1 = nz + 1;
  const long nn = (long)nx1 * ny1 * nz1;
  // permutation t (lexicographic) -> first axis, second axis
  const int p0[6] = {0, 0, 1, 1, 2, 2};
  const int p1[6] = {1, 2, 0, 2, 0, 1};
  for (long n = (long)blockIdx.x * blockDim.x + threadIdx.x; n < nn; n += (long)gridDim.x * blockDim.x) {
    const int i = (int)(n % nx1);
    const long t = n / nx1;
    const int j = (int)(t % ny1), k = (int)(t / ny1);
    double s = 0.0;
    int cnt = 0;
    for (int oz = 0; oz < 2; ++oz)
      for (int oy = 0; oy < 2; ++oy)
        for (int ox = 0; ox < 2; ++ox) {
          // the node is corner (ox, oy, oz) of cube (i - ox, j - oy, k - oz)
          const int hi = i - ox, hj = j - oy, hk = k - oz;
          if (hi < 0 || hj < 0 || hk < 0 || hi >= nx || hj >= ny || hk >= nz) continue;
          const int o = ox | (oy << 1) | (oz << 2);
          const long h = ((long)hk * ny + hj) * nx + hi;
          for (int tt = 0; tt < 6; ++tt) {
            const int e0 = 1 << p0[tt], e1 = e0 | (1 << p1[tt]);
            if (o == 0 || o == 7 || o == e0 || o == e1) { s += rho[6 * h + tt]; ++cnt; }
          }
        }
    uint16_t o8[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    o8[0] = f2bf((float)(s / cnt));
    o8[4] = f2bf(mask[n] ? 1.f : 0.f);
    *reinterpret_cast<uint4*>(X0 + n * kNetIn) = *reinterpret_cast<const uint4*>(o8);
  }
}

// signal input: [1..3] r_c / rms, other channels 0
__global__ void prep_signal_kernel(const double* __restrict__ r, const double* scal, uint16_t* X0,
                                   long nn, const int* stop) {
  if (stop && *stop) return;
  const double rms = scal[0];
  const double inv = rms > 0.0 ? 1.0 / rms : 0.0;
  for (long n = (long)blockIdx.x * blockDim.x + threadIdx.x; n < nn; n += (long)gridDim.x * blockDim.x) {
    uint16_t o8[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int c = 0; c < 3; ++c) o8[1 + c] = f2bf((float)(r[(long)c * nn + n] * inv));
    *reinterpret_cast<uint4*>(X0 + n * kNetIn) = *reinterpret_cast<const uint4*>(o8);
  }
}

// z[c][n] = gamma * rms * free(c, n) * nout[c][n]
__global__ void out_kernel(const float* __restrict__ nout, const uint8_t* __restrict__ mask,
                           const double* scal, double gamma, double* z, long nn, const int* stop) {
  if (stop && *stop) return;
  const double s = gamma * scal[0];
  for (long d = (long)blockIdx.x * blockDim.x + threadIdx.x; d < 3 * nn; d += (long)gridDim.x * blockDim.x) {
    const long n = d % nn;
    const int c = (int)(d / nn);
    z[d] = ((mask[n] >> c) & 1) ? 0.0 : s * (double)nout[d];
  }
}

// gradient at the raw output, BF16 channels last [nn][16]: g = scale * free * gs
__global__ void grad_out_kernel(const double* __restrict__ gs, const uint8_t* __restrict__ mask,
                                const double* scal, int mode, double gamma, uint16_t* gz, long nn) {
  // mode 0: scale = gamma * rms (gradient of sum(gs * z)); mode 1: the loss,
  // scale = 2 gamma / den with gs = K d
  const double scale = mode == 0 ? gamma * scal[0] : 2.0 * gamma / scal[1];
  for (long n = (long)blockIdx.x * blockDim.x + threadIdx.x; n < nn; n += (long)gridDim.x * blockDim.x) {
    uint16_t o[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) o[q] = 0;
    for (int c = 0; c < 3; ++c)
      o[c] = ((mask[n] >> c) & 1) ? 0 : f2bf((float)(scale * gs[(long)c * nn + n]));
    uint4* dst = reinterpret_cast<uint4*>(gz + n * 16);
    dst[0] = reinterpret_cast<const uint4*>(o)[0];
    dst[1] = reinterpret_cast<const uint4*>(o)[1];
  }
}

// loss: d = gamma * free * nout - e / rms; partial (e/rms).(r/rms)
__global__ __launch_bounds__(256) void loss_prep_kernel(const float* __restrict__ nout,
                                                        const double* __restrict__ e,
                                                        const double* __restrict__ r,
                                                        const uint8_t* __restrict__ mask,
                                                        const double* scal, double gamma, double* d,
                                                        long nn, double* partials) {
  const double rms = scal[0];
  const double inv = rms > 0.0 ? 1.0 / rms : 0.0;
  double acc[1] = {0.0};
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < 3 * nn; i += (long)gridDim.x * blockDim.x) {
    const long n = i % nn;
    const int c = (int)(i / nn);
    const bool fixed = (mask[n] >> c) & 1;
    const double eh = fixed ? 0.0 : e[i] * inv;
    d[i] = fixed ? 0.0 : gamma * (double)nout[i] - eh;
    acc[0] += eh * (fixed ? 0.0 : r[i] * inv);
  }
  const double none[1] = {0.0};
  block_partials<1, 0>(acc, none, partials);
}

__global__ void scal_fin(const double* partials, long nb, double* scal, int slot) {
  __shared__ double tot[1];
  reduce_partials<1, 0>(partials, nb, tot);
  if (threadIdx.x == 0) scal[slot] = tot[0];
}

// partial d.Kd over free DOFs
__global__ __launch_bounds__(256) void dkd_kernel(const double* __restrict__ d,
                                                  const double* __restrict__ Kd,
                                                  const uint8_t* __restrict__ mask, long nn,
                                                  double* partials) {
  double acc[1] = {0.0};
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < 3 * nn; i += (long)gridDim.x * blockDim.x) {
    const long n = i % nn;
    const int c = (int)(i / nn);
    if (!((mask[n] >> c) & 1)) acc[0] += d[i] * Kd[i];
  }
  const double none[1] = {0.0};
  block_partials<1, 0>(acc, none, partials);
}

__global__ void loss_fin(const double* partials, long nb, double* scal, double* loss_out) {
  __shared__ double tot[1];
  reduce_partials<1, 0>(partials, nb, tot);
  if (threadIdx.x == 0) {
    scal[3] = tot[0];
    scal[2] = tot[0] / scal[1];
    if (loss_out) *loss_out = scal[2];
  }
}

// Adam with bias correction (Kingma and Ba), FP32 master weights
__global__ void adam_kernel(float* w, float* m, float* v, const float* __restrict__ g, long n, float lr,
                            float b1, float b2, float c1, float c2, float eps) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    w[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  }
}

__global__ void zero_f32_kernel(float* p, long n) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    p[i] = 0.f;
}

// ------------------------------------------------------------------- host
static void level_dims(int nx, int ny, int nz, int dims[4][3], long V[4]) {
  dims[0][0] = nx + 1;
  dims[0][1] = ny + 1;
  dims[0][2] = nz + 1;
  for (int l = 1; l < 4; ++l)
    for (int a = 0; a < 3; ++a) dims[l][a] = (dims[l - 1][a] + 1) / 2;
  for (int l = 0; l < 4; ++l) V[l] = (long)dims[l][0] * dims[l][1] * dims[l][2];
}

static void fill_layers(NetLayer* L) {
  long ow = 0, of = 0, ob = 0;
  for (int i = 0; i < kNetLayers; ++i) {
    NetLayer& y = L[i];
    y.lin = kSpec[i][0];
    y.stride = kSpec[i][1];
    y.lout = y.lin + (y.stride == 2 ? 1 : 0);
    y.cin = kSpec[i][2];
    y.cout = kSpec[i][3];
    y.coutp = (int)round_up(y.cout, 16);
    y.kf = (int)round_up(27L * y.cin, 32);
    y.kb = (int)round_up(27L * y.coutp, 32);
    y.off_w = ow;
    y.off_wf = of;
    y.off_wb = ob;
    ow += (long)y.cout * 27 * y.cin;
    of += (long)y.coutp * y.kf;
    ob += round_up(y.cin, 16) * y.kb;
  }
}

static long total_params(const NetLayer* L) {
  return L[kNetLayers - 1].off_w + (long)L[kNetLayers - 1].cout * 27 * L[kNetLayers - 1].cin;
}

// chunking of the weight-gradient reduction for a layer with nout voxels
static void dw_plan(const NetLayer& y, long nout, int* ncb, int* nchunks, long* chunk) {
  const int cb = (int)((27L * y.cin + kDwCols - 1) / kDwCols);
  long nc = (2048 + cb - 1) / cb;
  const long maxc = (nout + kDwVox - 1) / kDwVox;
  if (nc > maxc) nc = maxc;
  if (nc < 1) nc = 1;
  long ch = round_up((nout + nc - 1) / nc, kDwVox);
  nc = (nout + ch - 1) / ch;
  *ncb = cb;
  *nchunks = (int)nc;
  *chunk = ch;
}

struct NetLayout {
  size_t w, m, v, grad, wf, wb, dwp, scal, nout, gz, gC0, gCAT0, gC1, gCAT1, gC2, gCAT2, gB3, gA3, gA2,
      gA1, gA0a, d, Kd, rc, xc, qc, total;
  size_t f[2][12];   // forward buffers of the gate and signal passes
  long dwp_len;
};

static NetLayout net_layout(int nx, int ny, int nz) {
  NetLayer L[kNetLayers];
  fill_layers(L);
  int dims[4][3];
  long V[4];
  level_dims(nx, ny, nz, dims, V);
  NetLayout o;
  size_t at = 0;
  auto take = [&](size_t bytes) {
    size_t p = at;
    at = (at + bytes + 255) & ~(size_t)255;
    return p;
  };
  const long P = total_params(L);
  const long nwf = L[kNetLayers - 1].off_wf + (long)L[kNetLayers - 1].coutp * L[kNetLayers - 1].kf;
  const long nwb = L[kNetLayers - 1].off_wb + round_up(L[kNetLayers - 1].cin, 16) * L[kNetLayers - 1].kb;
  long dwp = 0;
  for (int i = 0; i < kNetLayers; ++i) {
    int cb, nch;
    long ch;
    dw_plan(L[i], V[L[i].lout], &cb, &nch, &ch);
    const long len = (long)nch * L[i].cout * 27 * L[i].cin;
    if (len > dwp) dwp = len;
  }
  o.dwp_len = dwp;
  o.w = take(P * 4);
  o.m = take(P * 4);
  o.v = take(P * 4);
  o.grad = take(P * 4);
  o.wf = take(nwf * 2);
  o.wb = take(nwb * 2);
  o.dwp = take(dwp * 4);
  o.scal = take(8 * 8);
  const size_t b = 2;
  // X0 A0a CAT0 A1 CAT1 A2 CAT2 A3 B3 C2 C1 C0
  const long fl[12] = {V[0] * 8,  V[0] * 16, V[0] * 48, V[1] * 32, V[1] * 96, V[2] * 64,
                       V[2] * 128, V[3] * 64, V[3] * 64, V[2] * 64, V[1] * 32, V[0] * 16};
  for (int ps = 0; ps < 2; ++ps)
    for (int i = 0; i < 12; ++i) o.f[ps][i] = take(fl[i] * b);
  o.nout = take(V[0] * 3 * 4);
  o.gz = take(V[0] * 16 * b);
  o.gC0 = take(V[0] * 16 * b);
  o.gCAT0 = take(V[0] * 48 * b);
  o.gC1 = take(V[1] * 32 * b);
  o.gCAT1 = take(V[1] * 96 * b);
  o.gC2 = take(V[2] * 64 * b);
  o.gCAT2 = take(V[2] * 128 * b);
  o.gB3 = take(V[3] * 64 * b);
  o.gA3 = take(V[3] * 64 * b);
  o.gA2 = take(V[2] * 64 * b);
  o.gA1 = take(V[1] * 32 * b);
  o.gA0a = take(V[0] * 16 * b);
  o.d = take(V[0] * 3 * 8);
  o.Kd = take(V[0] * 3 * 8);
  o.rc = take(V[0] * 3 * 8 * kMaxRhs);
  o.xc = take(V[0] * 3 * 8 * kMaxRhs);
  o.qc = take(V[0] * 3 * 8 * kMaxRhs);
  o.total = at;
  return o;
}

size_t net_workspace_bytes(int nx, int ny, int nz) { return net_layout(nx, ny, nz).total; }

int net_attach(Ctx* c, void* ws, size_t bytes) {
  const NetLayout o = net_layout(c->g.nx, c->g.ny, c->g.nz);
  if (bytes < o.total) return TOPO_E_WORKSPACE;
  if (((uintptr_t)ws & 255) != 0) return TOPO_E_SHAPE;
  NetState* n = c->net;
  if (!n) {
    n = new (std::nothrow) NetState();
    if (!n) return TOPO_E_INVALID;
    c->net = n;
  }
  memset(n, 0, sizeof(*n));
  fill_layers(n->layer);
  level_dims(c->g.nx, c->g.ny, c->g.nz, n->dims, n->V);
  n->nparams = total_params(n->layer);
  char* w = (char*)ws;
  n->ws = w;
  n->ws_bytes = bytes;
  n->w = (float*)(w + o.w);
  n->m = (float*)(w + o.m);
  n->v = (float*)(w + o.v);
  n->grad = (float*)(w + o.grad);
  n->wf = (uint16_t*)(w + o.wf);
  n->wb = (uint16_t*)(w + o.wb);
  n->dw_part = (float*)(w + o.dwp);
  n->dw_part_len = o.dwp_len;
  {
    // TOPO_CONV_BIG_MIN: output voxels from which stride-1 layers use 8x8x4 boxes
    const char* b = getenv("TOPO_CONV_BIG_MIN");
    n->conv_big_min = b && atol(b) > 0 ? atol(b) : 131072;
  }
  n->scal = (double*)(w + o.scal);
  for (int ps = 0; ps < 2; ++ps) {
    FwdBufs& f = ps == 0 ? n->fg : n->fs;
    uint16_t** dst[12] = {&f.X0, &f.A0a, &f.CAT0, &f.A1, &f.CAT1, &f.A2,
                          &f.CAT2, &f.A3, &f.B3, &f.C2, &f.C1, &f.C0};
    for (int i = 0; i < 12; ++i) *dst[i] = (uint16_t*)(w + o.f[ps][i]);
  }
  n->nout = (float*)(w + o.nout);
  n->gz = (uint16_t*)(w + o.gz);
  n->gC0 = (uint16_t*)(w + o.gC0);
  n->gCAT0 = (uint16_t*)(w + o.gCAT0);
  n->gC1 = (uint16_t*)(w + o.gC1);
  n->gCAT1 = (uint16_t*)(w + o.gCAT1);
  n->gC2 = (uint16_t*)(w + o.gC2);
  n->gCAT2 = (uint16_t*)(w + o.gCAT2);
  n->gB3 = (uint16_t*)(w + o.gB3);
  n->gA3 = (uint16_t*)(w + o.gA3);
  n->gA2 = (uint16_t*)(w + o.gA2);
  n->gA1 = (uint16_t*)(w + o.gA1);
  n->gA0a = (uint16_t*)(w + o.gA0a);
  n->d = (double*)(w + o.d);
  n->Kd = (double*)(w + o.Kd);
  n->rc = (double*)(w + o.rc);
  n->xc = (double*)(w + o.xc);
  n->qc = (double*)(w + o.qc);
  n->gamma = 1.0;
  n->fcg_maxit = 500;
  n->smooth = 1;
  n->attached = true;
  // zero everything the network reads before it is written: weights,
  // moments, and the activation buffers (padding channels stay zero)
  hipStream_t s = c->stream;
  zero_f32_kernel<<<1024, 256, 0, s>>>((float*)w, (long)(o.total / 4));
  return hipGetLastError() == hipSuccess ? TOPO_OK : TOPO_E_HIP;
}

static void convert_weights(Ctx* c) {
  NetState* n = c->net;
  for (int i = 0; i < kNetLayers; ++i) {
    const NetLayer& y = n->layer[i];
    const int cinp = (int)round_up(y.cin, 16);
    const long tot = (long)y.coutp * y.kf + (long)cinp * y.kb;
    weights_bf16_kernel<<<cdiv(tot, 256) < 2048 ? cdiv(tot, 256) : 2048, 256, 0, c->stream>>>(
        n->w + y.off_w, n->wf + y.off_wf, n->wb + y.off_wb, y.cin, y.cout, y.coutp, y.kf, y.kb,
        y.stride, cinp);
  }
}

void net_set_weights(Ctx* c, const float* w) {
  NetState* n = c->net;
  (void)hipMemcpyAsync(n->w, w, (size_t)n->nparams * 4, hipMemcpyDeviceToDevice, c->stream);
  zero_f32_kernel<<<1024, 256, 0, c->stream>>>(n->m, n->nparams);
  zero_f32_kernel<<<1024, 256, 0, c->stream>>>(n->v, n->nparams);
  n->step = 0;
  convert_weights(c);
}

static Act act(uint16_t* p, int pitch, int off, int C, int level) { return Act{p, pitch, off, C, level}; }

// one convolution launch; MODE from the layer's stride and direction
static void conv_launch(Ctx* c, int mode, const Act& in, const Act& out, const uint16_t* w, int kpad,
                        int ktot, int act_on, int accum, const Act* gate, float* ysoa, int ysoa_cout,
                        const int* stop) {
  NetState* n = c->net;
  ConvArgs a;
  memset(&a, 0, sizeof(a));
  a.x = in.p;
  a.xpitch = in.pitch;
  a.xoff = in.off;
  a.cin = in.C;
  a.inx = n->dims[in.level][0];
  a.iny = n->dims[in.level][1];
  a.inz = n->dims[in.level][2];
  a.onx = n->dims[out.level][0];
  a.ony = n->dims[out.level][1];
  a.onz = n->dims[out.level][2];
  a.nout = n->V[out.level];
  a.w = w;
  a.kpad = kpad;
  a.ktot = ktot;
  a.y = out.p;
  a.ypitch = out.pitch;
  a.yoff = out.off;
  a.cout = ysoa ? ysoa_cout : out.C;
  a.ysoa = ysoa;
  a.gate = gate ? gate->p : nullptr;
  a.gpitch = gate ? gate->pitch : 0;
  a.goff = gate ? gate->off : 0;
  a.act = act_on;
  a.accum = accum;
  a.stop = stop;
  const int nct = (int)(round_up(ysoa ? 16 : out.C, 16) / 16);
  if (mode != 2) {
    const ConvPlan p = conv_plan(mode, n->dims[out.level], n->conv_big_min);
    // the tiled kernel assumes weight rows of round_up(27 cin, 32)
    if (kpad != (int)round_up(27L * in.C, 32)) abort();
    if (convt_dispatch(mode, in.C, nct, p, c->stream, a)) return;
  }
  const dim3 g(cdiv(a.nout, 128));
  if (mode == 0) conv_dispatch<0>(nct, g, c->stream, a);
  else if (mode == 1) conv_dispatch<1>(nct, g, c->stream, a);
  else conv_dispatch<2>(nct, g, c->stream, a);
}

static void fwd_layer(Ctx* c, int li, const Act& in, const Act& out, float* ysoa, const int* stop) {
  NetState* n = c->net;
  const NetLayer& y = n->layer[li];
  conv_launch(c, y.stride == 2 ? 1 : 0, in, out, n->wf + y.off_wf, y.kf, 27 * y.cin, kSpec[li][4], 0,
              nullptr, ysoa, y.cout, stop);
}

// input gradient of layer li: from dy (at the layer output) to dx (at its input)
static void bwd_layer(Ctx* c, int li, const Act& dy, const Act& dx, int accum, const Act* gate) {
  NetState* n = c->net;
  const NetLayer& y = n->layer[li];
  conv_launch(c, y.stride == 2 ? 2 : 0, dy, dx, n->wb + y.off_wb, y.kb, 27 * y.coutp, 0, accum, gate,
              nullptr, 0, nullptr);
}

static void dw_layer(Ctx* c, int li, const Act& x, const Act& dy) {
  NetState* n = c->net;
  const NetLayer& y = n->layer[li];
  DwArgs a;
  a.x = x.p;
  a.xpitch = x.pitch;
  a.xoff = x.off;
  a.cin = y.cin;
  a.inx = n->dims[y.lin][0];
  a.iny = n->dims[y.lin][1];
  a.inz = n->dims[y.lin][2];
  a.dy = dy.p;
  a.dpitch = dy.pitch;
  a.doff = dy.off;
  a.cout = y.cout;
  a.coutp = y.coutp;
  a.onx = n->dims[y.lout][0];
  a.ony = n->dims[y.lout][1];
  a.onz = n->dims[y.lout][2];
  a.nout = n->V[y.lout];
  a.stride = y.stride;
  a.ncols = 27 * y.cin;
  int ncb, nch;
  long ch;
  dw_plan(y, a.nout, &ncb, &nch, &ch);
  a.chunk = ch;
  a.part = n->dw_part;
  dw_kernel<<<dim3(ncb, nch), 256, 0, c->stream>>>(a);
  const long len = (long)y.cout * 27 * y.cin;
  dw_reduce_kernel<<<cdiv(len, 256) < 1024 ? cdiv(len, 256) : 1024, 256, 0, c->stream>>>(
      n->dw_part, n->grad + y.off_w, len, nch);
}

static void up_launch(Ctx* c, const Act& coarse, const Act& fine, const int* stop) {
  NetState* n = c->net;
  const int* cd = n->dims[coarse.level];
  const int* fd = n->dims[fine.level];
  const long work = n->V[fine.level] * (coarse.C / 8);
  upsample_kernel<<<cdiv(work, 256) < 8192 ? cdiv(work, 256) : 8192, 256, 0, c->stream>>>(
      coarse.p, coarse.pitch, fine.p, fine.pitch, fine.off, coarse.C, cd[0], cd[1], cd[2], fd[0], fd[1],
      fd[2], stop);
}

static void restrict_launch(Ctx* c, const Act& fine, const Act& coarse, const Act& gate) {
  NetState* n = c->net;
  const int* cd = n->dims[coarse.level];
  const int* fd = n->dims[fine.level];
  const long work = n->V[coarse.level] * (coarse.C / 8);
  restrict_kernel<<<cdiv(work, 256) < 8192 ? cdiv(work, 256) : 8192, 256, 0, c->stream>>>(
      fine.p, fine.pitch, coarse.p, coarse.pitch, gate.p, coarse.C, cd[0], cd[1], cd[2], fd[0], fd[1],
      fd[2]);
}

static const int* net_stop(Ctx* c) { return c->net_stop; }

// One pass of the encoder-decoder into b.  Gate pass (gate == nullptr):
// leaky ReLU, stops at c0.  Signal pass: every activation replaced by the
// gate pass's slope at the same unit, then the linear output layer.
static void net_pass(Ctx* c, const FwdBufs& b, const FwdBufs* gate) {
  NetState* n = c->net;
  const int* stop = net_stop(c);
  const FwdBufs& g = gate ? *gate : b;
  auto L = [&](int li, const Act& in, const Act& out, const Act& gt) {
    const NetLayer& y = n->layer[li];
    conv_launch(c, y.stride == 2 ? 1 : 0, in, out, n->wf + y.off_wf, y.kf, 27 * y.cin,
                gate ? 0 : kSpec[li][4], 0, gate ? &gt : nullptr, nullptr, 0, stop);
  };
  L(0, act(b.X0, 8, 0, 8, 0), act(b.A0a, 16, 0, 16, 0), act(g.A0a, 16, 0, 16, 0));
  L(1, act(b.A0a, 16, 0, 16, 0), act(b.CAT0, 48, 32, 16, 0), act(g.CAT0, 48, 32, 16, 0));
  L(2, act(b.CAT0, 48, 32, 16, 0), act(b.A1, 32, 0, 32, 1), act(g.A1, 32, 0, 32, 1));
  L(3, act(b.A1, 32, 0, 32, 1), act(b.CAT1, 96, 64, 32, 1), act(g.CAT1, 96, 64, 32, 1));
  L(4, act(b.CAT1, 96, 64, 32, 1), act(b.A2, 64, 0, 64, 2), act(g.A2, 64, 0, 64, 2));
  L(5, act(b.A2, 64, 0, 64, 2), act(b.CAT2, 128, 64, 64, 2), act(g.CAT2, 128, 64, 64, 2));
  L(6, act(b.CAT2, 128, 64, 64, 2), act(b.A3, 64, 0, 64, 3), act(g.A3, 64, 0, 64, 3));
  L(7, act(b.A3, 64, 0, 64, 3), act(b.B3, 64, 0, 64, 3), act(g.B3, 64, 0, 64, 3));
  up_launch(c, act(b.B3, 64, 0, 64, 3), act(b.CAT2, 128, 0, 64, 2), stop);
  L(8, act(b.CAT2, 128, 0, 128, 2), act(b.C2, 64, 0, 64, 2), act(g.C2, 64, 0, 64, 2));
  up_launch(c, act(b.C2, 64, 0, 64, 2), act(b.CAT1, 96, 0, 64, 1), stop);
  L(9, act(b.CAT1, 96, 0, 96, 1), act(b.C1, 32, 0, 32, 1), act(g.C1, 32, 0, 32, 1));
  up_launch(c, act(b.C1, 32, 0, 32, 1), act(b.CAT0, 48, 0, 32, 0), stop);
  L(10, act(b.CAT0, 48, 0, 48, 0), act(b.C0, 16, 0, 16, 0), act(g.C0, 16, 0, 16, 0));
  if (gate) fwd_layer(c, 11, act(b.C0, 16, 0, 16, 0), act(nullptr, 0, 0, 3, 0), n->nout, stop);
}

// Weight gradient through the signal pass: GEMM operands from the signal
// activations (fs), slopes from the gate activations (fg).
void net_backward(Ctx* c) {
  NetState* n = c->net;
  const FwdBufs& S = n->fs;
  const FwdBufs& G = n->fg;
  const Act gz = act(n->gz, 16, 0, 16, 0);
  const Act gC0 = act(n->gC0, 16, 0, 16, 0), gCAT0 = act(n->gCAT0, 48, 0, 48, 0);
  const Act gC1 = act(n->gC1, 32, 0, 32, 1), gCAT1 = act(n->gCAT1, 96, 0, 96, 1);
  const Act gC2 = act(n->gC2, 64, 0, 64, 2), gCAT2 = act(n->gCAT2, 128, 0, 128, 2);
  const Act gB3 = act(n->gB3, 64, 0, 64, 3), gA3 = act(n->gA3, 64, 0, 64, 3);
  const Act gA2 = act(n->gA2, 64, 0, 64, 2), gA1 = act(n->gA1, 32, 0, 32, 1);
  const Act gA0a = act(n->gA0a, 16, 0, 16, 0);
  // signal-pass operands
  const Act C0 = act(S.C0, 16, 0, 16, 0), CAT0 = act(S.CAT0, 48, 0, 48, 0);
  const Act CAT1 = act(S.CAT1, 96, 0, 96, 1), CAT2 = act(S.CAT2, 128, 0, 128, 2);
  const Act A3 = act(S.A3, 64, 0, 64, 3), A2 = act(S.A2, 64, 0, 64, 2);
  const Act A1 = act(S.A1, 32, 0, 32, 1), A0a = act(S.A0a, 16, 0, 16, 0);
  const Act X0 = act(S.X0, 8, 0, 8, 0);
  const Act skip0 = act(S.CAT0, 48, 32, 16, 0), skip1 = act(S.CAT1, 96, 64, 32, 1),
            skip2 = act(S.CAT2, 128, 64, 64, 2);
  // gate-pass slopes
  const Act qC0 = act(G.C0, 16, 0, 16, 0), qC1 = act(G.C1, 32, 0, 32, 1);
  const Act qC2 = act(G.C2, 64, 0, 64, 2), qB3 = act(G.B3, 64, 0, 64, 3);
  const Act qA3 = act(G.A3, 64, 0, 64, 3), qA2 = act(G.A2, 64, 0, 64, 2);
  const Act qA1 = act(G.A1, 32, 0, 32, 1), qA0a = act(G.A0a, 16, 0, 16, 0);
  const Act qskip0 = act(G.CAT0, 48, 32, 16, 0), qskip1 = act(G.CAT1, 96, 64, 32, 1),
            qskip2 = act(G.CAT2, 128, 64, 64, 2);
  // gradient slices of the concatenations
  const Act gskip0 = act(n->gCAT0, 48, 32, 16, 0), gskip1 = act(n->gCAT1, 96, 64, 32, 1),
            gskip2 = act(n->gCAT2, 128, 64, 64, 2);
  const Act gup0 = act(n->gCAT0, 48, 0, 32, 0), gup1 = act(n->gCAT1, 96, 0, 64, 1),
            gup2 = act(n->gCAT2, 128, 0, 64, 2);

  dw_layer(c, 11, C0, gz);
  bwd_layer(c, 11, gz, gC0, 0, &qC0);
  dw_layer(c, 10, CAT0, gC0);
  bwd_layer(c, 10, gC0, gCAT0, 0, nullptr);
  restrict_launch(c, gup0, gC1, qC1);
  dw_layer(c, 9, CAT1, gC1);
  bwd_layer(c, 9, gC1, gCAT1, 0, nullptr);
  restrict_launch(c, gup1, gC2, qC2);
  dw_layer(c, 8, CAT2, gC2);
  bwd_layer(c, 8, gC2, gCAT2, 0, nullptr);
  restrict_launch(c, gup2, gB3, qB3);
  dw_layer(c, 7, A3, gB3);
  bwd_layer(c, 7, gB3, gA3, 0, &qA3);
  dw_layer(c, 6, skip2, gA3);
  bwd_layer(c, 6, gA3, gskip2, 1, &qskip2);
  dw_layer(c, 5, A2, gskip2);
  bwd_layer(c, 5, gskip2, gA2, 0, &qA2);
  dw_layer(c, 4, skip1, gA2);
  bwd_layer(c, 4, gA2, gskip1, 1, &qskip1);
  dw_layer(c, 3, A1, gskip1);
  bwd_layer(c, 3, gskip1, gA1, 0, &qA1);
  dw_layer(c, 2, skip0, gA1);
  bwd_layer(c, 2, gA1, gskip0, 1, &qskip0);
  dw_layer(c, 1, A0a, gskip0);
  bwd_layer(c, 1, gskip0, gA0a, 0, &qA0a);
  dw_layer(c, 0, X0, gA0a);
}

void net_gates(Ctx* c, const double* rho) {
  NetState* n = c->net;
  const long nn = c->g.nn;
  prep_gate_kernel<<<cdiv(nn, 256) < 8192 ? cdiv(nn, 256) : 8192, 256, 0, c->stream>>>(
      rho, c->mask, n->fg.X0, c->g.nx, c->g.ny, c->g.nz, net_stop(c));
  net_pass(c, n->fg, nullptr);
  n->gates_ready = true;
}

void net_signal(Ctx* c, const double* r) {
  NetState* n = c->net;
  const long nn = c->g.nn;
  const unsigned gb = red_grid(3 * nn);
  const int* stop = net_stop(c);
  rr_kernel<<<gb, 256, 0, c->stream>>>(r, 3 * nn, c->partials, stop);
  rms_fin<<<1, 256, 0, c->stream>>>(c->partials, gb, 3 * nn, n->scal, stop);
  prep_signal_kernel<<<cdiv(nn, 256) < 8192 ? cdiv(nn, 256) : 8192, 256, 0, c->stream>>>(
      r, n->scal, n->fs.X0, nn, stop);
  const int slot = c->timing ? timing_begin(c, 1) : -1;
  net_pass(c, n->fs, &n->fg);
  if (slot >= 0) timing_end(c, 1, slot);
}

void net_precondition(Ctx* c, const double* rho, const double* r, double* z, bool reuse_gates) {
  NetState* n = c->net;
  if (!reuse_gates || !n->gates_ready) net_gates(c, rho);
  net_signal(c, r);
  const long nn = c->g.nn;
  out_kernel<<<red_grid(3 * nn), 256, 0, c->stream>>>(n->nout, c->mask, n->scal, n->gamma, z, nn,
                                                      net_stop(c));
}

void net_backward_from_z(Ctx* c, const double* gz, float* grad) {
  NetState* n = c->net;
  const long nn = c->g.nn;
  grad_out_kernel<<<cdiv(nn, 256) < 8192 ? cdiv(nn, 256) : 8192, 256, 0, c->stream>>>(
      gz, c->mask, n->scal, 0, n->gamma, n->gz, nn);
  net_backward(c);
  if (grad && grad != n->grad)
    (void)hipMemcpyAsync(grad, n->grad, (size_t)n->nparams * 4, hipMemcpyDeviceToDevice, c->stream);
}

void net_adam(Ctx* c, float lr) {
  NetState* n = c->net;
  n->step += 1;
  const double b1 = 0.9, b2 = 0.999;
  const float c1 = (float)(1.0 - pow(b1, n->step));
  const float c2 = (float)(1.0 - pow(b2, n->step));
  adam_kernel<<<cdiv(n->nparams, 256) < 4096 ? cdiv(n->nparams, 256) : 4096, 256, 0, c->stream>>>(
      n->w, n->m, n->v, n->grad, n->nparams, lr, (float)b1, (float)b2, c1, c2, 1e-8f);
  convert_weights(c);
}

void net_train_step(Ctx* c, const double* rho, const double* r, const double* e, float lr,
                    double* loss_out) {
  NetState* n = c->net;
  const long nn = c->g.nn;
  hipStream_t s = c->stream;
  launch_simp_modulus(c, rho);
  net_gates(c, rho);
  net_signal(c, r);
  const unsigned gb = red_grid(3 * nn);
  loss_prep_kernel<<<gb, 256, 0, s>>>(n->nout, e, r, c->mask, n->scal, n->gamma, n->d, nn, c->partials);
  scal_fin<<<1, 256, 0, s>>>(c->partials, gb, n->scal, 1);
  launch_apply_op(c, fine_op(c), c->E, n->d, n->Kd, 1, false, false, nullptr);
  dkd_kernel<<<gb, 256, 0, s>>>(n->d, n->Kd, c->mask, nn, c->partials);
  loss_fin<<<1, 256, 0, s>>>(c->partials, gb, n->scal, loss_out);
  grad_out_kernel<<<cdiv(nn, 256) < 8192 ? cdiv(nn, 256) : 8192, 256, 0, s>>>(
      n->Kd, c->mask, n->scal, 1, n->gamma, n->gz, nn);
  net_backward(c);
  if (lr > 0.f) net_adam(c, lr);
}

// rc = b - rc on free DOFs, 0 on fixed ones
__global__ void resid_kernel(double* rc, const double* __restrict__ b, const uint8_t* __restrict__ mask,
                             long nn, int nr, const int* stop) {
  if (stop && *stop) return;
  const long nd = 3 * nn;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < nr * nd; i += (long)gridDim.x * blockDim.x) {
    const long d = i % nd;
    const long n = d % nn;
    const int cc = (int)(d / nn);
    rc[i] = ((mask[n] >> cc) & 1) ? 0.0 : b[i] - rc[i];
  }
}

__global__ void axpy_kernel(double* x, const double* __restrict__ y, long n, const int* stop) {
  if (stop && *stop) return;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    x[i] += y[i];
}

// partial (xc, r1) and (xc, K xc) per load case
__global__ __launch_bounds__(256) void corr_dots_kernel(const double* __restrict__ xc,
                                                        const double* __restrict__ r1,
                                                        const double* __restrict__ q, long nd, int nr,
                                                        double* partials, const int* stop) {
  if (stop && *stop) return;
  double acc[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < nd; i += (long)gridDim.x * blockDim.x) {
    for (int k = 0; k < nr; ++k) {
      const double v = xc[(long)k * nd + i];
      acc[2 * k] += v * r1[(long)k * nd + i];
      acc[2 * k + 1] += v * q[(long)k * nd + i];
    }
  }
  const double none[1] = {0.0};
  block_partials<8, 0>(acc, none, partials);
}

// alpha_k = (xc, r1) / (xc, K xc): the step along the network correction
// that minimises the K-norm error (0 if the correction is null)
__global__ void corr_alpha_fin(const double* partials, long nb, int nr, double* alpha, const int* stop) {
  if (stop && *stop) return;
  __shared__ double tot[8];
  reduce_partials<8, 0>(partials, nb, tot);
  if (threadIdx.x == 0)
    for (int k = 0; k < kMaxRhs; ++k)
      alpha[k] = (k < nr && tot[2 * k + 1] > 0.0) ? tot[2 * k] / tot[2 * k + 1] : 0.0;
}

__global__ void axpy_alpha_kernel(double* x, const double* __restrict__ y, const double* alpha, long nd,
                                  int nr, const int* stop) {
  if (stop && *stop) return;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < nr * nd; i += (long)gridDim.x * blockDim.x)
    x[i] += alpha[i / nd] * y[i];
}

// The learned preconditioner z = M(r): with smoothing, a two-level cycle
// whose coarse correction is the network,
//   x = S r;  r1 = r - K x;  c = N(r1);  x += alpha c;  x = x + S (r - K x)
// with S the fine-level Chebyshev-Jacobi smoother and alpha the K-norm
// optimal step along c, so a poor network output can never raise the error
// of the cycle above that of the smoothing alone; without smoothing,
// z = N(r).
void learned_precondition(Ctx* c, const double* b, double* x, int nr) {
  NetState* n = c->net;
  const long nd = c->g.nd, nn = c->g.nn;
  const int* stop = &c->scal->pcg.done;
  hipStream_t s = c->stream;
  c->net_stop = stop;
  if (n->smooth) {
    const unsigned gb = red_grid(nd);
    gmg_fine_smooth(c, b, x, nr, true);
    launch_apply_op(c, fine_op(c), c->E, x, n->rc, nr, false, false, stop);
    resid_kernel<<<red_grid(nr * nd), 256, 0, s>>>(n->rc, b, c->mask, nn, nr, stop);
    for (int k = 0; k < nr; ++k)
      net_precondition(c, c->cur_rho, n->rc + (long)k * nd, n->xc + (long)k * nd, true);
    launch_apply_op(c, fine_op(c), c->E, n->xc, n->qc, nr, false, false, stop);
    corr_dots_kernel<<<gb, 256, 0, s>>>(n->xc, n->rc, n->qc, nd, nr, c->partials, stop);
    corr_alpha_fin<<<1, 256, 0, s>>>(c->partials, gb, nr, n->scal + 4, stop);
    axpy_alpha_kernel<<<red_grid(nr * nd), 256, 0, s>>>(x, n->xc, n->scal + 4, nd, nr, stop);
    gmg_fine_smooth(c, b, x, nr, false);
  } else {
    for (int k = 0; k < nr; ++k)
      net_precondition(c, c->cur_rho, b + (long)k * nd, x + (long)k * nd, true);
  }
  c->net_stop = nullptr;
}

}  // namespace topo
