// Optimality-criteria update (Sec. 3.2, eq. kkt and eq. update; Sec. 3.2.1):
//   rho_new_e(lambda) = clamp(rho_e (-dcf_e / lambda)^eta, lo_e, hi_e),
//   lo_e = max(rho_min, rho_e - m),  hi_e = min(1, rho_e + m),
// with lambda such that sum_e rho_new_e = volfrac * N.
//
// The paper finds lambda by bisection.  Writing mu = lambda^(-eta) and
// a_e = rho_e (-dcf_e)^eta, every cell is clamp(a_e mu, lo_e, hi_e), so the
// volume V(mu) is piecewise linear and non-decreasing in mu, and its root
// gives the same (unique) design.  This kernel set finds that root with
// Newton steps on V(mu) - target safeguarded by a bisection bracket: a pass
// reduces V and its slope S = sum over unclamped cells of a_e; once the
// clamped set is right, one Newton step lands on the root to rounding.
// Each pass is one kernel with a fused single-pass reduction.  A fixed
// budget of passes is queued without any host wait (the call is
// stream-asynchronous); passes after the root return at once.
//
// Passive cells (Sec. 5.4: zones of fixed density) take lo_e = hi_e = their
// fixed value (rho_min for a void, 1 for solid material) in every
// evaluation, so the volume at each multiplier counts them; they contribute
// nothing to the slope, the first multiplier or the bracket.
//
// With the density filter (x~ = W x / R) the volume is that of the filtered
// design, sum_e x~_e = sum_e dv_e x_e with dv = W (1 / R) (the filter is
// linear), and the OC ratio uses the volume sensitivity:
// rho_new_e = clamp(rho_e (-dc_e / (lambda dv_e))^eta, lo_e, hi_e).  The
// kernels take dv as per-cell volume weights (null: all ones), so each
// evaluation is the same single pass.
#include <math.h>

#include <mutex>

#include "common.h"
#include "shared_dev.h"
#include "topo_internal.h"

namespace topo {

// move-limit bounds of cell e, pinned to the fixed value on passive cells
__device__ __forceinline__ void oc_bounds(long e, double r, double move, double rho_min,
                                          const uint8_t* __restrict__ passive, double& lo,
                                          double& hi) {
  lo = fmax(rho_min, r - move);
  hi = fmin(1.0, r + move);
  if (passive) {
    const int pv = passive[e];
    if (pv == TOPO_PASSIVE_VOID) lo = hi = rho_min;
    if (pv == TOPO_PASSIVE_SOLID) lo = hi = 1.0;
  }
}

// a_e = rho_e (-dcf_e / dv_e)^eta, zero on passive cells: stored by the
// first pass, or formed again in every pass when no per-cell array is given
// (the allocation-free entry point); both give the same bits.
__device__ __forceinline__ double oc_coef(long e, double r, const double* __restrict__ dcf,
                                          double eta, const uint8_t* __restrict__ passive,
                                          const double* __restrict__ vw) {
  if (passive && passive[e]) return 0.0;
  return oc_a(r, vw ? dcf[e] / vw[e] : dcf[e], eta);
}

__global__ __launch_bounds__(256) void oc_init_kernel(const double* __restrict__ rho,
                                                      const double* __restrict__ dcf, double* a_out,
                                                      long nc, double move, double eta,
                                                      double rho_min,
                                                      const uint8_t* __restrict__ passive,
                                                      const double* __restrict__ vw,
                                                      double* partials) {
  double acc[3] = {0.0, 0.0, 0.0};
  double mx[1] = {0.0};
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < nc; e += (long)gridDim.x * blockDim.x) {
    const double r = rho[e];
    double lo, hi;
    oc_bounds(e, r, move, rho_min, passive, lo, hi);
    const double w = vw ? vw[e] : 1.0;
    const double a = oc_coef(e, r, dcf, eta, passive, vw);
    if (a_out) a_out[e] = a;
    acc[0] += w * lo;
    acc[1] += w * ((a > 0.0) ? hi : lo);  // volume once mu is large
    acc[2] += w * a;
    if (a > 0.0) mx[0] = fmax(mx[0], hi / a);
  }
  block_partials<3, 1>(acc, mx, partials);
}

__global__ void oc_init_fin(const double* partials, long nb, long nc, double volfrac, OcState* st,
                            int* status) {
  __shared__ double tot[4];
  reduce_partials<3, 1>(partials, nb, tot);
  if (threadIdx.x == 0) oc_init_finish(tot, nc, volfrac, st, status);
}

__global__ __launch_bounds__(256) void oc_pass_kernel(const double* __restrict__ rho,
                                                      const double* __restrict__ a_in,
                                                      const double* __restrict__ dcf, double eta,
                                                      long nc, double move, double rho_min,
                                                      const uint8_t* __restrict__ passive,
                                                      const double* __restrict__ vw,
                                                      double* partials, const OcState* st) {
  if (st->done) return;
  const double mu = st->mu;
  double acc[2] = {0.0, 0.0};
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < nc; e += (long)gridDim.x * blockDim.x) {
    const double r = rho[e];
    const double a = a_in ? a_in[e] : oc_coef(e, r, dcf, eta, passive, vw);
    double lo, hi;
    oc_bounds(e, r, move, rho_min, passive, lo, hi);
    const double w = vw ? vw[e] : 1.0;
    const double v = a * mu;
    acc[0] += w * fmax(lo, fmin(hi, v));
    acc[1] += (v > lo && v < hi) ? w * a : 0.0;
  }
  const double none[1] = {0.0};
  block_partials<2, 0>(acc, none, partials);
}

__global__ void oc_pass_fin(const double* partials, long nb, long nc, OcState* st) {
  if (st->done) return;
  __shared__ double tot[2];
  reduce_partials<2, 0>(partials, nb, tot);
  if (threadIdx.x == 0) oc_pass_finish(tot, nc, st);
}

__global__ __launch_bounds__(256) void oc_final_kernel(const double* __restrict__ rho,
                                                       const double* __restrict__ a_in,
                                                       const double* __restrict__ dcf, double eta,
                                                       double* rho_new, long nc, double move,
                                                       double rho_min,
                                                       const uint8_t* __restrict__ passive,
                                                       const double* __restrict__ vw,
                                                       double* partials, const OcState* st) {
  const double mu = st->mu;
  double acc[1] = {0.0};
  double mx[1] = {0.0};
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < nc; e += (long)gridDim.x * blockDim.x) {
    const double r = rho[e];
    double lo, hi;
    oc_bounds(e, r, move, rho_min, passive, lo, hi);
    const double a = a_in ? a_in[e] : oc_coef(e, r, dcf, eta, passive, vw);
    const double v = fmax(lo, fmin(hi, a * mu));
    rho_new[e] = v;
    acc[0] += (vw ? vw[e] : 1.0) * v;
    mx[0] = fmax(mx[0], fabs(v - r));
  }
  block_partials<1, 1>(acc, mx, partials);
}

__global__ void oc_final_fin(const double* partials, long nb, long nc, double eta, OcState* st,
                             double* scalars, int* status) {
  __shared__ double tot[2];
  reduce_partials<1, 1>(partials, nb, tot);
  if (threadIdx.x == 0) oc_final_finish(tot, eta, nc, st, scalars, status);
}

void oc_update(Ctx* c, const double* rho, const double* dcf, double* rho_new, double* scalars) {
  const long nc = c->g.nc;
  const unsigned nb = red_grid(nc);
  const topo_problem& p = c->prob;
  OcState* st = &c->scal->oc;
  double* a = c->qsoa;
  const uint8_t* pas = c->has_passive ? c->passive : nullptr;
  const double* vw = p.filter == TOPO_FILTER_DENSITY ? c->dv : nullptr;
  hipStream_t s = c->stream;
  oc_init_kernel<<<nb, 256, 0, s>>>(rho, dcf, a, nc, p.move, p.eta, p.rho_min, pas, vw, c->partials);
  oc_init_fin<<<1, 256, 0, s>>>(c->partials, nb, nc, p.volfrac, st, &c->scal->status);
  // a fixed budget of passes, queued without waiting: the passes after the
  // root return at once on the device's done flag
  for (int k = 0; k < kOcPasses; ++k) {
    oc_pass_kernel<<<nb, 256, 0, s>>>(rho, a, dcf, p.eta, nc, p.move, p.rho_min, pas, vw,
                                      c->partials, st);
    oc_pass_fin<<<1, 256, 0, s>>>(c->partials, nb, nc, st);
  }
  oc_final_kernel<<<nb, 256, 0, s>>>(rho, a, dcf, p.eta, rho_new, nc, p.move, p.rho_min, pas, vw,
                                     c->partials, st);
  oc_final_fin<<<1, 256, 0, s>>>(c->partials, nb, nc, p.eta, st, scalars, &c->scal->status);
}

// The update for a plain design: no passive cells, every cell of volume
// weight 1, a_e formed again in every pass (no per-cell scratch).  Used by
// the allocation-free entry point and by the unstructured-mesh loop, whose
// volume constraint counts cells.
void oc_update_plain(hipStream_t s, long nc, const double* rho, const double* dcf,
                     double* rho_new, double volfrac, double move, double eta, double rho_min,
                     double* partials, OcState* st, int* status, double* scalars) {
  const unsigned nb = red_grid(nc);
  oc_init_kernel<<<nb, 256, 0, s>>>(rho, dcf, nullptr, nc, move, eta, rho_min, nullptr, nullptr,
                                    partials);
  oc_init_fin<<<1, 256, 0, s>>>(partials, nb, nc, volfrac, st, status);
  for (int k = 0; k < kOcPasses; ++k) {
    oc_pass_kernel<<<nb, 256, 0, s>>>(rho, nullptr, dcf, eta, nc, move, rho_min, nullptr, nullptr,
                                      partials, st);
    oc_pass_fin<<<1, 256, 0, s>>>(partials, nb, nc, st);
  }
  oc_final_kernel<<<nb, 256, 0, s>>>(rho, nullptr, dcf, eta, rho_new, nc, move, rho_min, nullptr,
                                     nullptr, partials, st);
  oc_final_fin<<<1, 256, 0, s>>>(partials, nb, nc, eta, st, scalars, status);
}

// ---------------------------------------------- allocation-free OC update
// The update above for a plain design of n cells (no passive cells, unit
// cell volumes), for callers that cannot allocate device memory.  Its
// scratch (the per-block partial sums, the multiplier state and a status
// word) is one file-scope device array, so each GPU holds one copy for the
// life of the process; calls that overlap on one GPU share it and race.
// Host code never passes the array's name to a kernel: its device address
// is looked up once per device (hipGetSymbolAddress) and kept.
namespace {
constexpr size_t kNaPartBytes = (size_t)kRedBlocks * kPartStride * sizeof(double);
constexpr size_t kNaStateOff = kNaPartBytes;
constexpr size_t kNaStatusOff = kNaStateOff + ((sizeof(OcState) + 255) / 256) * 256;
constexpr size_t kNaBytes = kNaStatusOff + 256;
constexpr int kNaMaxDevices = 64;

std::mutex na_mu;
char* na_ptr[kNaMaxDevices];
}  // namespace

static __device__ __align__(256) char scratch[kNaBytes];

__global__ void oc_na_reset(int* status) { *status = 0; }

__global__ void oc_na_status(const int* status, double* out) { out[3] = (double)*status; }

// device address of this GPU's scratch array (looked up on first use)
static char* na_scratch(int dev) {
  std::lock_guard<std::mutex> lk(na_mu);
  if (!na_ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess) return nullptr;
    na_ptr[dev] = static_cast<char*>(p);
  }
  return na_ptr[dev];
}

}  // namespace topo

using namespace topo;

extern "C" int topo_oc_update_noalloc(int64_t n, const double* rho, const double* dcf,
                                      double* rho_new, double volfrac, double move, double eta,
                                      double rho_min, double* out, void* stream) {
  if (!rho || !dcf || !rho_new || !out || rho == rho_new || dcf == rho_new) return TOPO_E_INVALID;
  if (!(volfrac > 0.0 && volfrac <= 1.0) || !(move > 0.0) || !(eta > 0.0) ||
      !(rho_min > 0.0 && rho_min < 1.0))
    return TOPO_E_INVALID;
  if (n < 1 || n > TOPO_OC_NOALLOC_MAX_CELLS) return TOPO_E_SHAPE;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kNaMaxDevices) return TOPO_E_HIP;
  char* base = na_scratch(dev);
  if (!base) return TOPO_E_HIP;
  double* partials = reinterpret_cast<double*>(base);
  OcState* st = reinterpret_cast<OcState*>(base + kNaStateOff);
  int* status = reinterpret_cast<int*>(base + kNaStatusOff);
  hipStream_t s = static_cast<hipStream_t>(stream);
  oc_na_reset<<<1, 1, 0, s>>>(status);
  oc_update_plain(s, (long)n, rho, dcf, rho_new, volfrac, move, eta, rho_min, partials, st, status,
                  out);
  oc_na_status<<<1, 1, 0, s>>>(status, out);
  return hipGetLastError() == hipSuccess ? TOPO_OK : TOPO_E_HIP;
}
