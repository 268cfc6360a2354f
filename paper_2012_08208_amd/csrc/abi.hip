// C ABI entry points: argument checks, workspace carving and the host-side
// drivers of the SIMP loop (Sec. 4.3-4.5 and the Appendix code: solve ->
// sensitivity -> filter -> OC -> change).
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include <new>

#include "common.h"
#include "net.h"
#include "topo_internal.h"

using namespace topo;

namespace topo {

static size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

static bool valid_problem(const topo_problem* p) {
  if (!p) return false;
  if (p->dim != 2 && p->dim != 3) return false;
  for (int a = 0; a < p->dim; ++a)
    if (p->nel[a] < 1 || p->nel[a] > (1 << 20)) return false;
  if (p->nrhs < 1 || p->nrhs > kMaxRhs) return false;
  if (!(p->volfrac > 0.0 && p->volfrac <= 1.0)) return false;
  if (!(p->rmin > 0.0 && p->rmin <= 16.0)) return false;
  if (!(p->penal >= 1.0 && p->penal <= 10.0)) return false;
  if (!(p->nu > -1.0 && p->nu < 0.5)) return false;
  if (!(p->E0 > 0.0) || !(p->Emin >= 0.0) || !(p->Emin < p->E0)) return false;
  if (!(p->move > 0.0) || !(p->eta > 0.0) || !(p->rho_min > 0.0 && p->rho_min < 1.0)) return false;
  if (!(p->rtol > 0.0) || p->maxit < 1) return false;
  if (p->precision != TOPO_FP64 && p->precision != TOPO_MIXED_FP32 &&
      p->precision != TOPO_MIXED_IR && p->precision != TOPO_MIXED_BF16 &&
      p->precision != TOPO_MIXED_RU)
    return false;
  if (p->precond != TOPO_PC_JACOBI && p->precond != TOPO_PC_GMG && p->precond != TOPO_PC_LEARNED)
    return false;
  if (p->precond == TOPO_PC_LEARNED && (p->dim != 3 || p->precision != TOPO_FP64)) return false;
  if (p->dim == 2 && p->split2d != TOPO_SPLIT_ALT_ROWS && p->split2d != TOPO_SPLIT_UNIFORM)
    return false;
  if (p->filter != TOPO_FILTER_DISTANCE && p->filter != TOPO_FILTER_HELMHOLTZ &&
      p->filter != TOPO_FILTER_DENSITY)
    return false;
  if (p->sync_mode != TOPO_SYNC_POLL && p->sync_mode != TOPO_SYNC_NONE) return false;
  if (p->gmg_dense != 0 && (p->gmg_dense < 128 || p->gmg_dense > kDense3)) return false;
  // the no-wait mode has no host-driven refinement loop and no learned cycle
  if (p->sync_mode == TOPO_SYNC_NONE &&
      (p->precision == TOPO_MIXED_IR || p->precond == TOPO_PC_LEARNED))
    return false;
  return true;
}

static Grid make_grid(const topo_problem* p) {
  Grid g;
  g.dim = p->dim;
  g.nx = p->nel[0];
  g.ny = p->nel[1];
  g.nz = p->dim == 3 ? p->nel[2] : 1;
  g.nn = (int64_t)(g.nx + 1) * (g.ny + 1) * (p->dim == 3 ? (g.nz + 1) : 1);
  g.nc = (int64_t)g.nx * g.ny * (p->dim == 3 ? g.nz : 1) * (p->dim == 3 ? 6 : 2);
  g.nd = g.nn * g.dim;
  g.split = p->dim == 2 ? p->split2d : TOPO_SPLIT_UNIFORM;
  return g;
}

int pick_kz(int dim, int nx, int ny, int nz) {
  const char* env = getenv("TOPO_APPLY_KZ");
  if (env) {
    int v = atoi(env);
    if (v >= 1 && v <= 1024) return v;
  }
  if (dim == 2) return 1;
  const long cols = (long)((nx + 15) / 15) * ((ny + 15) / 15);
  long kz = (long)(nz + 1) * cols / 1024;
  if (kz < 4) kz = 4;
  if (kz > 16) kz = 16;
  return (int)kz;
}

static int pick_kz(const Grid& g) { return pick_kz(g.dim, g.nx, g.ny, g.nz); }

// z-chunk of a coarse multigrid level
static int pick_kz_coarse(int dim, int nx, int ny, int nz) {
  if (dim == 2) return 1;
  int lo = 2;   // short sweeps: the small levels are latency-bound
  if (const char* e = getenv("TOPO_COARSE_KZMIN")) {
    const int v = atoi(e);
    if (v >= 1 && v <= 16) lo = v;
  }
  const long cols = (long)((nx + 15) / 15) * ((ny + 15) / 15);
  long kz = (long)(nz + 1) * cols / 1024;
  if (kz < lo) kz = lo;
  if (kz > 16) kz = 16;
  return (int)kz;
}

// Multigrid levels: halve (rounding up) every axis until the level has at
// most 128 DOFs, the size the dense coarsest solve handles.
int gmg_dense_max(const topo_problem* p) {
  if (p->gmg_dense > 0) return p->gmg_dense;
  int v = kDense3;
  if (const char* e = getenv("TOPO_GMG_DENSE")) v = atoi(e);
  return v < 128 ? 128 : (v > kDense3 ? kDense3 : v);
}

std::vector<LevelDims> gmg_plan_dims(int dim, int nx, int ny, int nz, int dense_max) {
  std::vector<LevelDims> out;
  LevelDims d{nx, ny, dim == 3 ? nz : 1};
  out.push_back(d);
  for (int l = 0; l < 24; ++l) {
    const long nn = (long)(d.nx + 1) * (d.ny + 1) * (dim == 3 ? (d.nz + 1) : 1);
    if (nn * dim <= dense_max) break;
    LevelDims e{(d.nx + 1) / 2, (d.ny + 1) / 2, dim == 3 ? (d.nz + 1) / 2 : 1};
    if (e.nx == d.nx && e.ny == d.ny && e.nz == d.nz) break;
    d = e;
    out.push_back(d);
  }
  return out;
}

static std::vector<LevelDims> gmg_plan(const topo_problem* p, const Grid& g) {
  return gmg_plan_dims(g.dim, g.nx, g.ny, g.nz, gmg_dense_max(p));
}

// Coarse node mask: a component is fixed when any fine node of the support
// of the coarse basis function has it fixed.
std::vector<uint8_t> coarse_mask_host(const std::vector<uint8_t>& fm, const LevelDims& f,
                                      const LevelDims& d, int dim) {
  std::vector<uint8_t> cm((size_t)(d.nx + 1) * (d.ny + 1) * (dim == 3 ? (d.nz + 1) : 1), 0);
  const int nzf = dim == 3 ? f.nz : 0, nzc = dim == 3 ? d.nz : 0;
  for (int K = 0; K <= nzc; ++K)
    for (int J = 0; J <= d.ny; ++J)
      for (int I = 0; I <= d.nx; ++I) {
        uint8_t m = 0;
        for (int dz = -1; dz <= 1; ++dz)
          for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx) {
              if (dim == 2 && dz != 0) continue;
              // only the 2C +- d offsets with d in {0,1}^dim
              const bool pos = dx >= 0 && dy >= 0 && dz >= 0;
              const bool neg = dx <= 0 && dy <= 0 && dz <= 0;
              if (!pos && !neg) continue;
              const int fi = 2 * I + dx, fj = 2 * J + dy, fk = 2 * K + dz;
              if (fi < 0 || fj < 0 || fk < 0 || fi > f.nx || fj > f.ny || fk > nzf) continue;
              m |= fm[((size_t)fk * (f.ny + 1) + fj) * (f.nx + 1) + fi];
            }
        cm[((size_t)K * (d.ny + 1) + J) * (d.nx + 1) + I] = m;
      }
  return cm;
}

static long apply_blocks(const Grid& g, int kz, int nrhs) {
  long tiles = (long)((g.nx + 15) / 15) * ((g.ny + 15) / 15);
  if (g.dim == 3) tiles *= (g.nz + 1 + kz - 1) / kz;
  return 8L * ((tiles + 7) / 8) * nrhs;
}

static WsLayout make_layout(const topo_problem* p, const Grid& g, int kz) {
  WsLayout L;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t at = o;
    o = align_up(o + bytes);
    return at;
  };
  const size_t nr = (size_t)p->nrhs;
  const bool mixed = p->precision != TOPO_FP64;
  long nblk = apply_blocks(g, kz, p->nrhs);
  if (nblk < kRedBlocks) nblk = kRedBlocks;
  L.mask = take((size_t)g.nn);
  L.f = take(nr * g.nd * 8);
  L.E = take((size_t)g.nc * 8);
  L.E32 = mixed ? take((size_t)g.nc * 4) : 0;
  L.E16 = p->precision == TOPO_MIXED_BF16 ? take((size_t)g.nc * 2) : 0;
  L.invd = take((size_t)g.nd * 8);
  L.invd32 = mixed ? take((size_t)g.nd * 4) : 0;
  L.r = take(nr * g.nd * 8);
  L.p = take(nr * g.nd * 8);
  L.q = take(nr * g.nd * 8);
  L.z = 0;
  L.wv = 0;
  L.partials = take((size_t)nblk * 16 * 8);
  L.scal = take(sizeof(DevScalars));
  L.R = take((size_t)g.nc * 8);
  // tap lists of every class, as long as the longest (filter_taps_host)
  const size_t tst = (size_t)filter_tap_stride(g.dim, g.split, p->rmin);
  L.taps = take((size_t)8 * tst * sizeof(FilterTap) + 64);
  L.ttaps = g.dim == 3 ? take((size_t)6 * tst * sizeof(TiledTap)) : 0;
  L.qsoa = take((size_t)g.nc * 8);
  L.dc = take((size_t)g.nc * 8);
  L.dcf = take((size_t)g.nc * 8);
  L.rho_new = take((size_t)g.nc * 8);
  L.rho_tmp = take((size_t)g.nc * 8);
  L.passive = take((size_t)g.nc);
  L.helm = p->filter == TOPO_FILTER_HELMHOLTZ ? take((size_t)5 * g.nn * 8) : 0;
  L.rho_phys = p->filter == TOPO_FILTER_DENSITY ? take((size_t)g.nc * 8) : 0;
  L.dv = p->filter == TOPO_FILTER_DENSITY ? take((size_t)g.nc * 8) : 0;
  L.r32 = L.p32 = L.q32 = L.z32 = L.z32b = L.x32 = 0;
  if (mixed) {
    L.r32 = take(nr * g.nd * 4);
    L.p32 = take(nr * g.nd * 4);
    L.q32 = take(nr * g.nd * 4);
    L.z32 = take(nr * g.nd * 4);
    L.z32b = take(nr * g.nd * 4);
    L.x32 = take(nr * g.nd * 4);
  }
  L.gmg_scal = 0;
  L.pring = L.qring = 0;
  if (p->precond == TOPO_PC_LEARNED) {
    L.pring = take((size_t)kFcgRing * nr * g.nd * 8);
    L.qring = take((size_t)kFcgRing * nr * g.nd * 8);
  }
  L.levels.clear();
  if (p->precond != TOPO_PC_JACOBI) {
    L.z = take(nr * g.nd * 8);
    const bool flex = flex_mixed(*p) || p->precond == TOPO_PC_LEARNED;
    L.wv = flex ? take(nr * g.nd * 8) : 0;
    const std::vector<LevelDims> plan = gmg_plan(p, g);
    L.gmg_scal = take(8 * 2 * (plan.size() + 1));
    for (size_t l = 0; l < plan.size(); ++l) {
      GmgLevel lv;
      memset(&lv, 0, sizeof(lv));
      const LevelDims& d = plan[l];
      const long nn = (long)(d.nx + 1) * (d.ny + 1) * (g.dim == 3 ? (d.nz + 1) : 1);
      const long nc = (long)d.nx * d.ny * (g.dim == 3 ? d.nz * 6 : 2);
      const long nd = nn * g.dim;
      const bool last = l + 1 == plan.size();
      if (l > 0) {
        lv.off_E = take((size_t)nc * 8);
        lv.off_invd = take((size_t)nd * 8);
        if (mixed) {
          lv.off_E32 = take((size_t)nc * 4);
          lv.off_invd32 = take((size_t)nd * 4);
        }
        lv.off_b = take(nr * nd * 8);
        lv.off_x = take(nr * nd * 8);
        lv.off_mask = take((size_t)nn);
      }
      if (!last) {
        lv.off_r = take(nr * nd * 8);
        lv.off_d = take(nr * nd * 8);
        lv.off_q = take(nr * nd * 8);
        lv.off_pv = take((size_t)nd * 8);
        lv.off_pw = take((size_t)nd * 8);
      } else if (nd <= 128) {
        lv.off_A = take((size_t)nd * nd * 8);
      } else {
        // blocked elimination: the matrix padded to whole blocks (identity
        // rows and columns), its FP32 copy, the pivot block and column panel
        const size_t np = (size_t)((nd + kGjBlock - 1) / kGjBlock * kGjBlock);
        lv.np = (int)np;
        lv.off_A = take(np * np * 8);
        lv.off_A32 = mixed ? take(np * np * 4) : 0;
        lv.off_gj = take((2 * (size_t)kGjBlock * kGjBlock + 2 * np * kGjBlock) * 8);
      }
      L.levels.push_back(lv);
    }
  }
  L.total = o;
  return L;
}

int timing_begin(Ctx* c, int chan) {
  auto& tv = c->tev[chan];
  if (c->tev_used[chan] >= tv.size()) {
    hipEvent_t a, b;
    if (hipEventCreate(&a) != hipSuccess) return -1;
    if (hipEventCreate(&b) != hipSuccess) return -1;
    tv.push_back({a, b});
  }
  const int slot = (int)c->tev_used[chan]++;
  (void)hipEventRecord(tv[slot].first, c->stream);
  return slot;
}

void timing_end(Ctx* c, int chan, int slot) {
  (void)hipEventRecord(c->tev[chan][slot].second, c->stream);
}

static int timing_read_chan(Ctx* c, int chan, int64_t* launches, double* total_ms) {
  TOPO_HIP(hipStreamSynchronize(c->stream));
  double tot = 0.0;
  for (size_t i = 0; i < c->tev_used[chan]; ++i) {
    float ms = 0.f;
    TOPO_HIP(hipEventElapsedTime(&ms, c->tev[chan][i].first, c->tev[chan][i].second));
    tot += ms;
  }
  if (launches) *launches = (int64_t)c->tev_used[chan];
  if (total_ms) *total_ms = tot;
  c->tev_used[chan] = 0;
  return TOPO_OK;
}

__global__ void log_record_kernel(const DevScalars* sc, double* rec, long nc, int nr) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double mx = 0.0;
  for (int k = 0; k < nr; ++k)
    if (sc->pcg.ff[k] > 0.0) mx = fmax(mx, sqrt(sc->pcg.rr[k] / sc->pcg.ff[k]));
  rec[0] = sc->compliance;
  rec[1] = sc->c_paper;
  rec[2] = sc->oc.vol / (double)nc;
  rec[3] = sc->oc.change;
  rec[4] = sc->oc.lam;
  rec[5] = sc->pcg.iters;
  rec[6] = mx;
  rec[7] = (sc->pcg.done && !sc->pcg.breakdown) ? 1.0 : 0.0;
}

// mixed precision: the iteration count is the total over refinement steps
// (plus a closing FP64 solve if refinement stagnated), and the residual is
// the FP64 true residual of the refinement
__global__ void log_record_mixed_kernel(const DevScalars* sc, double* rec, long nc, int nr) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double mx = 0.0;
  for (int k = 0; k < nr; ++k)
    if (sc->ir.ff[k] > 0.0) mx = fmax(mx, sqrt(sc->ir.rr[k] / sc->ir.ff[k]));
  rec[0] = sc->compliance;
  rec[1] = sc->c_paper;
  rec[2] = sc->oc.vol / (double)nc;
  rec[3] = sc->oc.change;
  rec[4] = sc->oc.lam;
  rec[5] = sc->ir.inner_total + (sc->ir.stagnated ? sc->pcg.iters : 0);
  rec[6] = sc->ir.stagnated ? 0.0 : mx;
  rec[7] = sc->ir.done ? 1.0 : ((sc->pcg.done && !sc->pcg.breakdown) ? 1.0 : 0.0);
}

}  // namespace topo

struct topo_ctx : public Ctx {};

extern "C" {

int topo_workspace_size(const topo_problem* prob, size_t* bytes) {
  if (!valid_problem(prob) || !bytes) return TOPO_E_INVALID;
  Grid g = make_grid(prob);
  *bytes = make_layout(prob, g, pick_kz(g)).total;
  return TOPO_OK;
}

int topo_create(const topo_problem* prob, const uint8_t* fixed_mask, void* workspace,
                size_t ws_bytes, void* stream, topo_ctx** out) {
  if (!out) return TOPO_E_INVALID;
  *out = nullptr;
  if (!valid_problem(prob) || !fixed_mask || !workspace) return TOPO_E_INVALID;
  if (((uintptr_t)workspace & 255) != 0) return TOPO_E_SHAPE;
  topo_ctx* c = new (std::nothrow) topo_ctx();
  if (!c) return TOPO_E_INVALID;
  c->prob = *prob;
  c->g = make_grid(prob);
  c->apply_kz = pick_kz(c->g);
  c->gp = gmg_params_env();
  c->env_nrb = 0;
  c->env_g = 1;
  if (const char* e = getenv("TOPO_APPLY_NRB")) c->env_nrb = atoi(e);
  if (const char* e = getenv("TOPO_APPLY_G")) c->env_g = atoi(e);
  c->L = make_layout(prob, c->g, c->apply_kz);
  if (ws_bytes < c->L.total) {
    delete c;
    return TOPO_E_WORKSPACE;
  }
  c->stream = (hipStream_t)stream;
  c->ws = (char*)workspace;
  c->ws_bytes = ws_bytes;
  const WsLayout& L = c->L;
  char* w = c->ws;
  c->mask = (uint8_t*)(w + L.mask);
  c->f = (double*)(w + L.f);
  c->E = (double*)(w + L.E);
  c->E32 = L.E32 ? (float*)(w + L.E32) : nullptr;
  c->E16 = L.E16 ? (uint16_t*)(w + L.E16) : nullptr;
  c->invd = (double*)(w + L.invd);
  c->invd32 = L.invd32 ? (float*)(w + L.invd32) : nullptr;
  c->r = (double*)(w + L.r);
  c->p = (double*)(w + L.p);
  c->q = (double*)(w + L.q);
  c->wv = L.wv ? (double*)(w + L.wv) : nullptr;
  c->partials = (double*)(w + L.partials);
  c->scal = (DevScalars*)(w + L.scal);
  c->R = (double*)(w + L.R);
  c->taps = (FilterTap*)(w + L.taps);
  c->ttaps = L.ttaps ? (TiledTap*)(w + L.ttaps) : nullptr;
  c->qsoa = (double*)(w + L.qsoa);
  c->dc = (double*)(w + L.dc);
  c->dcf = (double*)(w + L.dcf);
  c->rho_new = (double*)(w + L.rho_new);
  c->rho_tmp = (double*)(w + L.rho_tmp);
  c->passive = (uint8_t*)(w + L.passive);
  c->has_passive = false;
  c->hx = c->hr = c->hp = c->hq = c->hinvd = nullptr;
  c->rho_phys = L.rho_phys ? (double*)(w + L.rho_phys) : nullptr;
  c->dv = L.dv ? (double*)(w + L.dv) : nullptr;
  if (L.helm) {
    double* hb = (double*)(w + L.helm);
    c->hx = hb;
    c->hr = hb + c->g.nn;
    c->hp = hb + 2 * c->g.nn;
    c->hq = hb + 3 * c->g.nn;
    c->hinvd = hb + 4 * c->g.nn;
  }
  c->z = L.z ? (double*)(w + L.z) : nullptr;
  c->r32 = L.r32 ? (float*)(w + L.r32) : nullptr;
  c->p32 = L.p32 ? (float*)(w + L.p32) : nullptr;
  c->q32 = L.q32 ? (float*)(w + L.q32) : nullptr;
  c->z32 = L.z32 ? (float*)(w + L.z32) : nullptr;
  c->z32b = L.z32b ? (float*)(w + L.z32b) : nullptr;
  c->x32 = L.x32 ? (float*)(w + L.x32) : nullptr;
  c->pring = L.pring ? (double*)(w + L.pring) : nullptr;
  c->qring = L.qring ? (double*)(w + L.qring) : nullptr;
  // material of the unit-modulus element law
  Material& m = c->m;
  const double nu = prob->nu;
  if (prob->paper_mode) {
    m.lam0 = 0.6;
    m.mu0 = 0.4;
  } else if (prob->dim == 2) {
    m.lam0 = nu / (1.0 - nu * nu);  // plane stress
    m.mu0 = 1.0 / (2.0 * (1.0 + nu));
  } else {
    m.lam0 = nu / ((1.0 + nu) * (1.0 - 2.0 * nu));
    m.mu0 = 1.0 / (2.0 * (1.0 + nu));
  }
  m.vol = prob->dim == 2 ? 0.5 : 1.0 / 6.0;
  m.E0 = prob->E0;
  m.Emin = prob->Emin;
  m.penal = prob->penal;
  m.paper = prob->paper_mode ? 1 : 0;
  // node mask: bit c set when component c is fixed
  std::vector<uint8_t> bits((size_t)c->g.nn, 0);
  for (int comp = 0; comp < prob->dim; ++comp)
    for (int64_t n = 0; n < c->g.nn; ++n)
      if (fixed_mask[(size_t)comp * c->g.nn + n]) bits[n] |= (uint8_t)(1u << comp);
  bool mask_ok = true;
  std::vector<std::vector<uint8_t>> lmasks;
  if (prob->precond != TOPO_PC_JACOBI) {
    const std::vector<LevelDims> plan = gmg_plan(&c->prob, c->g);
    lmasks.push_back(bits);
    for (size_t l = 0; l < plan.size(); ++l) {
      GmgLevel lv = L.levels[l];
      const LevelDims& d = plan[l];
      lv.op.dim = c->g.dim;
      lv.op.nx = d.nx;
      lv.op.ny = d.ny;
      lv.op.nz = d.nz;
      lv.op.nn = (int64_t)(d.nx + 1) * (d.ny + 1) * (c->g.dim == 3 ? (d.nz + 1) : 1);
      lv.op.split_uniform = l == 0 ? (c->g.split == TOPO_SPLIT_UNIFORM) : 1;
      lv.op.kz = l == 0 ? c->apply_kz : pick_kz_coarse(c->g.dim, d.nx, d.ny, d.nz);
      lv.nc = (int64_t)d.nx * d.ny * (c->g.dim == 3 ? d.nz * 6 : 2);
      double* gs = (double*)(w + L.gmg_scal);
      lv.lmax = gs + 2 * l;
      lv.pscale = gs + 2 * l + 1;
      if (l == 0) {
        lv.E = c->E;
        lv.invd = c->invd;
        lv.E32 = c->E32;
        lv.E16 = c->E16;
        lv.invd32 = c->invd32;
        lv.mask = c->mask;
        lv.b = lv.x = nullptr;
      } else {
        lv.E = (double*)(w + lv.off_E);
        lv.invd = (double*)(w + lv.off_invd);
        lv.E32 = lv.off_E32 ? (float*)(w + lv.off_E32) : nullptr;
        lv.E16 = nullptr;
        lv.invd32 = lv.off_invd32 ? (float*)(w + lv.off_invd32) : nullptr;
        lv.b = (double*)(w + lv.off_b);
        lv.x = (double*)(w + lv.off_x);
        lv.mask = (uint8_t*)(w + lv.off_mask);
        // coarse mask: fixed when any fine node of the basis support is fixed
        std::vector<uint8_t> cm = coarse_mask_host(lmasks[l - 1], plan[l - 1], d, c->g.dim);
        lmasks.push_back(cm);
        mask_ok = mask_ok && hipMemcpy(lv.mask, cm.data(), cm.size(), hipMemcpyHostToDevice) == hipSuccess;
      }
      lv.op.mask = lv.mask;
      lv.r = lv.off_r ? (double*)(w + lv.off_r) : nullptr;
      lv.d = lv.off_d ? (double*)(w + lv.off_d) : nullptr;
      lv.q = lv.off_q ? (double*)(w + lv.off_q) : nullptr;
      lv.pv = lv.off_pv ? (double*)(w + lv.off_pv) : nullptr;
      lv.pw = lv.off_pw ? (double*)(w + lv.off_pw) : nullptr;
      lv.Ainv = lv.off_A ? (double*)(w + lv.off_A) : nullptr;
      lv.Ainv32 = lv.off_A32 ? (float*)(w + lv.off_A32) : nullptr;
      lv.gj = lv.off_gj ? (double*)(w + lv.off_gj) : nullptr;
      c->lv.push_back(lv);
    }
  }
  void* pin = nullptr;
  if (!mask_ok || hipHostMalloc(&pin, 64, hipHostMallocDefault) != hipSuccess) {
    delete c;
    return TOPO_E_HIP;
  }
  c->pinned = (volatile int*)pin;
  memset(pin, 0, 64);
  if (hipEventCreateWithFlags(&c->ev_poll[0], hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&c->ev_poll[1], hipEventDisableTiming) != hipSuccess) {
    (void)hipHostFree(pin);
    delete c;
    return TOPO_E_HIP;
  }
  bool ok = hipMemcpy(c->mask, bits.data(), bits.size(), hipMemcpyHostToDevice) == hipSuccess;
  DevScalars zero;
  memset(&zero, 0, sizeof(zero));
  ok = ok && hipMemcpy(c->scal, &zero, sizeof(zero), hipMemcpyHostToDevice) == hipSuccess;
  if (ok) {
    build_filter_taps(c);
    launch_filter_rowsums(c);
    if (c->hinvd) {
      build_helm_coef(c);
      launch_helm_diag(c);
    }
    if (c->dv) launch_density_volume_weights(c, c->dv);
    ok = hipStreamSynchronize(c->stream) == hipSuccess && hipGetLastError() == hipSuccess;
  }
  if (!ok) {
    (void)hipEventDestroy(c->ev_poll[0]);
    (void)hipEventDestroy(c->ev_poll[1]);
    (void)hipHostFree(pin);
    delete c;
    return TOPO_E_HIP;
  }
  c->loads_set = false;
  c->timing = false;
  c->tev_used[0] = c->tev_used[1] = 0;
  c->t_launches = 0;
  c->t_ms = 0.0;
  *out = c;
  return TOPO_OK;
}

int topo_destroy(topo_ctx* c) {
  if (!c) return TOPO_E_INVALID;
  (void)hipStreamSynchronize(c->stream);
  for (auto& tv : c->tev)
    for (auto& e : tv) {
      (void)hipEventDestroy(e.first);
      (void)hipEventDestroy(e.second);
    }
  (void)hipEventDestroy(c->ev_poll[0]);
  (void)hipEventDestroy(c->ev_poll[1]);
  (void)hipHostFree((void*)c->pinned);
  delete c->net;
  delete c;
  return TOPO_OK;
}

int topo_set_loads(topo_ctx* c, const double* f, int nrhs) {
  if (!c || !f) return TOPO_E_INVALID;
  if (nrhs != c->prob.nrhs) return TOPO_E_SHAPE;
  TOPO_HIP(hipMemcpyAsync(c->f, f, (size_t)nrhs * c->g.nd * 8, hipMemcpyDeviceToDevice, c->stream));
  c->loads_set = true;
  return TOPO_OK;
}

static int solve_impl(topo_ctx* c, const double* rho, double* u, double* info, bool warm) {
  if (c->prob.precond == TOPO_PC_LEARNED && !(c->net && c->net->attached && c->net->weights_set))
    return TOPO_E_STATE;
  launch_simp_modulus(c, rho);
  launch_diagonal(c, c->invd, true);
  topo_problem saved = c->prob;
  c->prob.warm_start = warm ? 1 : 0;
  c->cur_rho = rho;
  if (c->net) c->net->gates_ready = false;   // the gate pass follows the design
  pcg_solve(c, u, info);
  c->cur_rho = nullptr;
  c->prob = saved;
  return hipGetLastError() == hipSuccess ? TOPO_OK : TOPO_E_HIP;
}

int topo_solve(topo_ctx* c, const double* rho, double* u, double* info) {
  if (!c || !rho || !u) return TOPO_E_INVALID;
  if (!c->loads_set) return TOPO_E_STATE;
  return solve_impl(c, rho, u, info, c->prob.warm_start != 0);
}

int topo_sensitivity(topo_ctx* c, const double* rho, const double* u, double* dc,
                     double* compliance) {
  if (!c || !rho || !u || !dc) return TOPO_E_INVALID;
  if (!c->loads_set) return TOPO_E_STATE;
  launch_sensitivity(c, rho, u, dc, compliance);
  return hipGetLastError() == hipSuccess ? TOPO_OK : TOPO_E_HIP;
}

int topo_filter(topo_ctx* c, const double* rho, const double* dc, double* dcf) {
  if (!c || !rho || !dc || !dcf || dc == dcf) return TOPO_E_INVALID;
  launch_filter(c, rho, dc, dcf);
  return hipGetLastError() == hipSuccess ? TOPO_OK : TOPO_E_HIP;
}

int topo_oc_update(topo_ctx* c, const double* rho, const double* dcf, double* rho_new,
                   double* scalars) {
  if (!c || !rho || !dcf || !rho_new || rho == rho_new) return TOPO_E_INVALID;
  oc_update(c, rho, dcf, rho_new, scalars);
  return hipGetLastError() == hipSuccess ? TOPO_OK : TOPO_E_HIP;
}

int topo_iterate(topo_ctx* c, double* rho, double* u, int max_iter, double change_tol,
                 double* log, int* n_done) {
  if (!c || !rho || !u || max_iter < 0) return TOPO_E_INVALID;
  if (change_tol > 0.0 && c->prob.sync_mode == TOPO_SYNC_NONE) return TOPO_E_INVALID;
  if (!c->loads_set) return TOPO_E_STATE;
  int done = 0;
  const bool dens = c->prob.filter == TOPO_FILTER_DENSITY;
  for (int it = 0; it < max_iter; ++it) {
    const bool warm = it > 0 || c->prob.warm_start != 0;
    // density filter: the physics sees x~ = W x / R, the design is x
    const double* phys = rho;
    if (dens) {
      launch_density_filter(c, rho, c->rho_phys);
      phys = c->rho_phys;
    }
    int rc = solve_impl(c, phys, u, nullptr, warm);
    if (rc != TOPO_OK) return rc;
    launch_sensitivity(c, phys, u, c->dc, nullptr);
    launch_filter(c, rho, c->dc, c->dcf);
    oc_update(c, rho, c->dcf, c->rho_new, nullptr);
    if (log) {
      double* rec = log + (size_t)it * TOPO_LOG_LEN;
      if (c->prob.precision == TOPO_MIXED_IR)
        log_record_mixed_kernel<<<1, 64, 0, c->stream>>>(c->scal, rec, c->g.nc, c->prob.nrhs);
      else
        log_record_kernel<<<1, 64, 0, c->stream>>>(c->scal, rec, c->g.nc, c->prob.nrhs);
    }
    TOPO_HIP(hipMemcpyAsync(rho, c->rho_new, (size_t)c->g.nc * 8, hipMemcpyDeviceToDevice,
                            c->stream));
    ++done;
    if (change_tol > 0.0) {
      double ch = 0.0;
      TOPO_HIP(hipMemcpyAsync((void*)&c->pinned[4], &c->scal->oc.change, sizeof(double),
                              hipMemcpyDeviceToHost, c->stream));
      TOPO_HIP(hipStreamSynchronize(c->stream));
      memcpy(&ch, (const void*)&c->pinned[4], sizeof(double));
      if (ch < change_tol) break;
    }
  }
  if (n_done) *n_done = done;
  return hipGetLastError() == hipSuccess ? TOPO_OK : TOPO_E_HIP;
}

int topo_apply(topo_ctx* c, const double* rho, const double* x, double* y) {
  if (!c || !rho || !x || !y || x == y) return TOPO_E_INVALID;
  launch_simp_modulus(c, rho);
  launch_mask_copy(c, x, c->q, c->prob.nrhs);
  launch_apply(c, c->q, y, c->prob.nrhs, false);
  return hipGetLastError() == hipSuccess ? TOPO_OK : TOPO_E_HIP;
}

int topo_apply_f32(topo_ctx* c, const double* rho, const float* x, float* y) {
  if (!c || !rho || !x || !y || (const void*)x == (const void*)y) return TOPO_E_INVALID;
  if (c->prob.precision == TOPO_FP64 || !c->E32 || !c->p32) return TOPO_E_STATE;
  launch_simp_modulus(c, rho);
  launch_mask_copy_f32(c, x, c->p32, c->prob.nrhs);
  if (c->E16)
    launch_apply_op_bf16(c, fine_op(c), c->E16, c->p32, y, c->prob.nrhs, true, nullptr);
  else
    launch_apply_op_f32(c, fine_op(c), c->E32, c->p32, y, c->prob.nrhs, true, nullptr);
  return hipGetLastError() == hipSuccess ? TOPO_OK : TOPO_E_HIP;
}

int topo_diagonal(topo_ctx* c, const double* rho, double* d) {
  if (!c || !rho || !d) return TOPO_E_INVALID;
  launch_simp_modulus(c, rho);
  launch_diagonal(c, d, false);
  return hipGetLastError() == hipSuccess ? TOPO_OK : TOPO_E_HIP;
}

int topo_density_filter(topo_ctx* c, const double* x, double* x_phys) {
  if (!c || !x || !x_phys || x == x_phys) return TOPO_E_INVALID;
  launch_density_filter(c, x, x_phys);
  return hipGetLastError() == hipSuccess ? TOPO_OK : TOPO_E_HIP;
}

int topo_filter_rowsums(topo_ctx* c, double* R) {
  if (!c || !R) return TOPO_E_INVALID;
  TOPO_HIP(hipMemcpyAsync(R, c->R, (size_t)c->g.nc * 8, hipMemcpyDeviceToDevice, c->stream));
  return TOPO_OK;
}

int topo_set_passive(topo_ctx* c, const uint8_t* passive) {
  if (!c) return TOPO_E_INVALID;
  if (!passive) {
    c->has_passive = false;
    return TOPO_OK;
  }
  const long nc = (long)c->g.nc;
  long marked = 0;
  for (long e = 0; e < nc; ++e) {
    if (passive[e] > TOPO_PASSIVE_SOLID) return TOPO_E_INVALID;
    marked += passive[e] != TOPO_PASSIVE_FREE;
  }
  TOPO_HIP(hipMemcpyAsync(c->passive, passive, (size_t)nc, hipMemcpyHostToDevice, c->stream));
  TOPO_HIP(hipStreamSynchronize(c->stream));
  c->has_passive = marked > 0;
  return TOPO_OK;
}

int topo_timing_enable(topo_ctx* c, int enable) {
  if (!c) return TOPO_E_INVALID;
  c->timing = enable != 0;
  return TOPO_OK;
}

int topo_timing_read(topo_ctx* c, int64_t* launches, double* total_ms) {
  if (!c) return TOPO_E_INVALID;
  return timing_read_chan(c, 0, launches, total_ms);
}

int topo_timing_read_net(topo_ctx* c, int64_t* passes, double* total_ms) {
  if (!c) return TOPO_E_INVALID;
  return timing_read_chan(c, 1, passes, total_ms);
}

int topo_sync(topo_ctx* c, int* device_status) {
  if (!c) return TOPO_E_INVALID;
  TOPO_HIP(hipStreamSynchronize(c->stream));
  int st = 0;
  TOPO_HIP(hipMemcpy(&st, &c->scal->status, sizeof(int), hipMemcpyDeviceToHost));
  int zero = 0;
  TOPO_HIP(hipMemcpy(&c->scal->status, &zero, sizeof(int), hipMemcpyHostToDevice));
  if (device_status) *device_status = st;
  return TOPO_OK;
}

int topo_filter_taps(int32_t dim, int32_t split, double rmin, int32_t* ntaps, int32_t* nclasses) {
  if ((dim != 2 && dim != 3) || !(rmin > 0.0 && rmin <= 16.0) || !ntaps || !nclasses)
    return TOPO_E_INVALID;
  if (dim == 2 && split != TOPO_SPLIT_ALT_ROWS && split != TOPO_SPLIT_UNIFORM) return TOPO_E_INVALID;
  std::vector<FilterTap> tab;
  int nt[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  int st = 0;
  const int ncls = filter_taps_host(dim, dim == 2 ? split : TOPO_SPLIT_UNIFORM, rmin, tab, nt, &st);
  for (int k = 0; k < 8; ++k) ntaps[k] = k < ncls ? nt[k] : 0;
  *nclasses = ncls;
  return TOPO_OK;
}

const char* topo_status_string(int code) {
  switch (code) {
    case TOPO_OK: return "ok";
    case TOPO_E_INVALID: return "invalid argument";
    case TOPO_E_SHAPE: return "shape or alignment mismatch";
    case TOPO_E_STATE: return "call out of order (loads not set?)";
    case TOPO_E_HIP: return "HIP runtime error";
    case TOPO_E_WORKSPACE: return "workspace too small";
    case TOPO_S_NOT_CONVERGED: return "solve not converged within maxit";
    case TOPO_S_LEARNED_FALLBACK: return "learned-preconditioner CG fell back to multigrid PCG";
    case TOPO_S_NUMERIC: return "non-finite value or CG breakdown";
    case TOPO_S_OC_INFEASIBLE: return "OC volume target infeasible";
    case TOPO_S_OC_INEXACT: return "OC multiplier search stopped before the volume constraint was met";
    default: return "unknown status";
  }
}

// ------------------------------------------------- learned preconditioner
static bool net_ready(topo_ctx* c) { return c && c->g.dim == 3 && c->net && c->net->attached; }

int topo_precond_num_params(int64_t* n) {
  if (!n) return TOPO_E_INVALID;
  *n = 0;
  const int spec[kNetLayers][2] = {{8, 16},  {16, 16}, {16, 32}, {32, 32}, {32, 64},  {64, 64},
                                   {64, 64}, {64, 64}, {128, 64}, {96, 32}, {48, 16}, {16, 3}};
  for (int i = 0; i < kNetLayers; ++i) *n += (int64_t)spec[i][0] * 27 * spec[i][1];
  return TOPO_OK;
}

int topo_precond_workspace_size(const topo_problem* prob, size_t* bytes) {
  if (!valid_problem(prob) || !bytes || prob->dim != 3) return TOPO_E_INVALID;
  *bytes = net_workspace_bytes(prob->nel[0], prob->nel[1], prob->nel[2]);
  return TOPO_OK;
}

int topo_precond_attach(topo_ctx* c, void* ws, size_t bytes) {
  if (!c || !ws || c->g.dim != 3) return TOPO_E_INVALID;
  return net_attach(c, ws, bytes);
}

int topo_precond_set_weights(topo_ctx* c, const float* w) {
  if (!net_ready(c) || !w) return TOPO_E_INVALID;
  net_set_weights(c, w);
  c->net->weights_set = true;
  return hipGetLastError() == hipSuccess ? TOPO_OK : TOPO_E_HIP;
}

int topo_precond_get_weights(topo_ctx* c, float* w) {
  if (!net_ready(c) || !w) return TOPO_E_INVALID;
  TOPO_HIP(hipMemcpyAsync(w, c->net->w, (size_t)c->net->nparams * 4, hipMemcpyDeviceToDevice,
                          c->stream));
  return TOPO_OK;
}

int topo_precond_config(topo_ctx* c, double gamma, int fcg_maxit, int smooth) {
  if (!net_ready(c) || !(gamma > 0.0) || fcg_maxit < 1 || (smooth != 0 && smooth != 1))
    return TOPO_E_INVALID;
  if (smooth && c->lv.empty()) return TOPO_E_STATE;  // smoothing needs the multigrid level 0
  c->net->gamma = gamma;
  c->net->fcg_maxit = fcg_maxit;
  c->net->smooth = smooth;
  return TOPO_OK;
}

int topo_precond_apply(topo_ctx* c, const double* rho, const double* r, double* z) {
  if (!net_ready(c) || !rho || !r || !z || r == z) return TOPO_E_INVALID;
  if (!c->net->weights_set) return TOPO_E_STATE;
  net_precondition(c, rho, r, z, false);
  return hipGetLastError() == hipSuccess ? TOPO_OK : TOPO_E_HIP;
}

int topo_precond_backward(topo_ctx* c, const double* gz, float* grad) {
  if (!net_ready(c) || !gz || !grad) return TOPO_E_INVALID;
  if (!c->net->weights_set) return TOPO_E_STATE;
  net_backward_from_z(c, gz, grad);
  return hipGetLastError() == hipSuccess ? TOPO_OK : TOPO_E_HIP;
}

int topo_precond_train_step(topo_ctx* c, const double* rho, const double* r, const double* e,
                            float lr, double* loss) {
  if (!net_ready(c) || !rho || !r || !e || !(lr >= 0.f)) return TOPO_E_INVALID;
  if (!c->net->weights_set) return TOPO_E_STATE;
  net_train_step(c, rho, r, e, lr, loss);
  return hipGetLastError() == hipSuccess ? TOPO_OK : TOPO_E_HIP;
}

int topo_precond_get_grad(topo_ctx* c, float* grad) {
  if (!net_ready(c) || !grad) return TOPO_E_INVALID;
  TOPO_HIP(hipMemcpyAsync(grad, c->net->grad, (size_t)c->net->nparams * 4, hipMemcpyDeviceToDevice,
                          c->stream));
  return TOPO_OK;
}

int topo_precond_harvest(topo_ctx* c, const double* rho, const int* iters, int n, double* r_out,
                         double* e_out, int presmooth, int* final_iters) {
  if (!c || !rho || !iters || n < 1 || !r_out || !e_out) return TOPO_E_INVALID;
  if (c->prob.nrhs != 1 || c->lv.empty()) return TOPO_E_INVALID;
  if (!c->loads_set) return TOPO_E_STATE;
  for (int i = 0; i < n; ++i)
    if (iters[i] < 0 || (i > 0 && iters[i] <= iters[i - 1])) return TOPO_E_INVALID;
  if (presmooth != 0 && presmooth != 1) return TOPO_E_INVALID;
  return pcg_harvest(c, rho, iters, n, r_out, e_out, presmooth, final_iters);
}

int topo_precond_stats(topo_ctx* c, int* fcg_iters, int* fallback) {
  if (!net_ready(c)) return TOPO_E_INVALID;
  if (fcg_iters) *fcg_iters = c->net->last_iters;
  if (fallback) *fallback = c->net->last_fallback;
  return TOPO_OK;
}

}  // extern "C"
