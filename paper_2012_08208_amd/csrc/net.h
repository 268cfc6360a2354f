// The convolutional preconditioner network (not part of the paper): state
// and launchers.  The network maps (node density, residual) on the FE node
// grid to an approximation of the error K^{-1} r:
//   level 0 = the node grid (nx+1, ny+1, nz+1), level l+1 = ceil(n/2) per axis;
//   3x3x3 convolutions, zero padding 1, no bias, leaky ReLU (slope 1/8);
//   encoder e0a e0b | d1 e1 | d2 e2 | d3 e3 (d = stride 2), decoder with
//   nested-linear upsampling and channel concatenation of the encoder
//   outputs: c2 [up(e3), e2], c1 [up(c2), e1], c0 [up(c1), e0b], out (3 ch).
// Activations are BF16, channels last ([voxel][channel], x fastest);
// convolutions run on MFMA 16x16x32 BF16 tiles with FP32 accumulation.
// Master weights, gradients and Adam moments are FP32; the flat parameter
// vector holds W[co][tap][ci] per layer, tap = (dz*3 + dy)*3 + dx.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace topo {

struct Ctx;

constexpr int kNetLayers = 12;
constexpr int kNetIn = 8;          // input channels (5 used)
constexpr float kSlope = 0.125f;   // leaky ReLU negative slope

struct NetLayer {
  int lin, lout;     // grid level of input and output
  int stride;        // 1 or 2
  int cin, cout;     // channels (cout = 3 for the output layer)
  int coutp;         // cout rounded up to 16
  int kf, kb;        // padded K of the forward / input-gradient GEMMs
  long off_w;        // offset in the flat FP32 parameter vector
  long off_wf, off_wb;  // offsets (elements) of the BF16 weight copies
};

// A channels-last BF16 activation view: element (v, c) at p[v*pitch + off + c].
struct Act {
  uint16_t* p;
  int pitch, off, C, level;
};

// Forward activations of one pass (gate pass or signal pass).
struct FwdBufs {
  uint16_t *X0, *A0a, *CAT0, *A1, *CAT1, *A2, *CAT2, *A3, *B3, *C2, *C1, *C0;
};

struct NetState {
  bool attached;
  bool weights_set;
  char* ws;
  size_t ws_bytes;
  int dims[4][3];    // (nx, ny, nz) of each level
  long V[4];         // voxels per level
  NetLayer layer[kNetLayers];
  long nparams;
  // weights
  float *w, *m, *v, *grad;  // [nparams]
  uint16_t *wf, *wb;        // BF16 forward / input-gradient weight copies
  float* dw_part;           // [chunks][cout*27*cin] weight-gradient partials
  long dw_part_len;
  long conv_big_min;        // output voxels from which stride-1 layers use 8x8x4 tiles
  // activations (BF16, channels last): gate pass and signal pass
  FwdBufs fg, fs;
  bool gates_ready;         // fg holds the gate pass of the current design
  float* nout;              // [3][V0] raw network output
  // activation gradients
  uint16_t *gz, *gC0, *gCAT0, *gC1, *gCAT1, *gC2, *gCAT2, *gB3, *gA3, *gA2, *gA1, *gA0a;
  // FE-side vectors [3][nn] FP64
  double *d, *Kd, *rc, *xc, *qc;
  double* scal;             // [0] rms, [1] den, [2] loss, [3] dKd, [4..7] correction steps
  double gamma;
  int step;                 // Adam step counter
  int fcg_maxit;            // FCG iterations before the multigrid fallback
  int smooth;               // 1: Chebyshev pre/post smoothing around the network
  int last_iters;           // FCG iterations of the last learned solve (host copy)
  int last_fallback;
};

size_t net_workspace_bytes(int nx, int ny, int nz);
int net_attach(Ctx* c, void* ws, size_t bytes);
void net_set_weights(Ctx* c, const float* w);
// z = gamma * rms(r) * mask * N(rho, r) for one load case (r, z: [3][nn]);
// reuse_gates keeps the gate pass of an earlier call with the same rho
void net_precondition(Ctx* c, const double* rho, const double* r, double* z, bool reuse_gates);
// weight gradient of sum(gz * z) after net_precondition (FP32 [nparams])
void net_backward_from_z(Ctx* c, const double* gz, float* grad);
// one training step on (rho, r, e); loss to loss_out (device double)
void net_train_step(Ctx* c, const double* rho, const double* r, const double* e, float lr,
                    double* loss_out);
// gate pass (density and fixed-node channels) into fg
void net_gates(Ctx* c, const double* rho);
// signal pass of r (gated by fg) into fs and nout
void net_signal(Ctx* c, const double* r);
// backward from gz (BF16 channels last) to c->net->grad
void net_backward(Ctx* c);
void net_adam(Ctx* c, float lr);

}  // namespace topo
