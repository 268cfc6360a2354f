"""The convolutional preconditioner network, forward and backward (test oracle).

The paper has no learned component.  This library adds one: a small
encoder-decoder network on the FE node grid that maps (density, residual) to
an approximation of the error K^{-1} r, used as the coarse correction of a
preconditioner inside flexible CG.  Its definition is this library's own.
This module writes that definition out in FP64 NumPy, one plain loop over
the 27 taps per convolution, so the HIP kernels can be checked against it.

Definition
----------
Grids.  Level 0 is the FE node grid (nx+1, ny+1, nz+1), x fastest.  Level
l+1 has ceil(n/2) points per axis.  Tensors are (nz, ny, nx, C), channels
last.

Convolution.  Every convolution is 3x3x3 with zero padding 1 and no bias:
    y[m, co] = sum_t sum_ci W[co, t, ci] * x[s*m + d_t - 1, ci]
with stride s (1 or 2), tap t = (dz*3 + dy)*3 + dx and d_t = (dx, dy, dz)
in {0,1,2}^3 (index order (z, y, x) in the arrays).  Entries outside the
grid are zero.

Activation.  Leaky ReLU with slope 1/8 on the negative side.

Two passes.  The weights are applied twice.  The gate pass feeds the
density and fixed-node channels (residual channels zeroed) through the
leaky-ReLU network.  The signal pass feeds the residual channels (density
and fixed channels zeroed) through the same layers, but each activation is
replaced by multiplication with the slope the gate pass chose at the same
unit: 1 where the gate activation is positive, 1/8 elsewhere.  With no
biases the output is then exactly linear in the residual for a fixed
design, N(r) = A(rho) r, so inside a solve the preconditioner is one fixed
linear operator; the density enters through the gates only.

Upsampling.  Nested linear interpolation, per axis:
    fine[i] = (coarse[floor(i/2)] + coarse[ceil(i/2)]) / 2;
if ceil(i/2) falls off the coarse grid, fine[i] = coarse[floor(i/2)].

Layers, in the order of the flat parameter vector (W[co, t, ci] each):
    e0a  L0 s1   8 -> 16   lrelu   input: 8 channels (5 used)
    e0b  L0 s1  16 -> 16   lrelu   -> skip0
    d1   L0->L1 s2 16 -> 32 lrelu
    e1   L1 s1  32 -> 32   lrelu   -> skip1
    d2   L1->L2 s2 32 -> 64 lrelu
    e2   L2 s1  64 -> 64   lrelu   -> skip2
    d3   L2->L3 s2 64 -> 64 lrelu
    e3   L3 s1  64 -> 64   lrelu
    c2   L2 s1 128 -> 64   lrelu   input [up(e3), skip2]
    c1   L1 s1  96 -> 32   lrelu   input [up(c2), skip1]
    c0   L0 s1  48 -> 16   lrelu   input [up(c1), skip0]
    out  L0 s1  16 -> 3    linear

Input channels (per node): 0 the mean density of the cells incident to the
node; 1..3 the residual components divided by rms(r) = ||r|| / sqrt(n_dof);
4 one where any component of the node is fixed; 5..7 zero.

Preconditioner output: z = gamma * rms(r) * mask * N(input), with N's three
output channels as the displacement components and mask zero on fixed DOFs.

Rounding.  The GPU computes in BF16 storage with FP32 accumulation.  With
``bf16=True`` the oracle rounds (to nearest even) at the same points the
kernels store: the input tensor, the weights, every stored activation, and
every stored activation gradient.  Everything else is FP64.

Training loss (per sample with residual r and error e = K^{-1} r, both
scaled by 1/rms(r)): the K-norm error of the masked prediction,
    L = (g N - e)^T K (g N - e) / (e^T K e),
whose gradient with respect to N is 2 g (g K N - r) / (e^T r), using r = K e.
Optimizer: Adam (Kingma and Ba, 2015) with bias correction, FP32 master
weights.

This module is test infrastructure: only tests, the smoke check and the
benchmark's CPU-baseline leg may import it.  It shares no code with the HIP
path.
"""

from __future__ import annotations

import numpy as np

SLOPE = 0.125
N_IN = 8

# name, level_in, stride, cin, cout, activation
LAYERS = [
    ("e0a", 0, 1, 8, 16, True),
    ("e0b", 0, 1, 16, 16, True),
    ("d1", 0, 2, 16, 32, True),
    ("e1", 1, 1, 32, 32, True),
    ("d2", 1, 2, 32, 64, True),
    ("e2", 2, 1, 64, 64, True),
    ("d3", 2, 2, 64, 64, True),
    ("e3", 3, 1, 64, 64, True),
    ("c2", 2, 1, 128, 64, True),
    ("c1", 1, 1, 96, 32, True),
    ("c0", 0, 1, 48, 16, True),
    ("out", 0, 1, 16, 3, False),
]


def n_params() -> int:
    return sum(co * 27 * ci for (_, _, _, ci, co, _) in LAYERS)


def split_params(flat):
    """Flat vector -> list of W[co, 27, ci] arrays (views)."""
    out, o = [], 0
    for (_, _, _, ci, co, _) in LAYERS:
        n = co * 27 * ci
        out.append(np.asarray(flat[o:o + n], dtype=np.float64).reshape(co, 27, ci))
        o += n
    return out


def init_params(seed: int = 0) -> np.ndarray:
    """He-style normal initialisation (variance 2 / fan_in), FP32 values."""
    rng = np.random.default_rng(seed)
    parts = []
    for (_, _, _, ci, co, act) in LAYERS:
        std = np.sqrt((2.0 if act else 1.0) / (27 * ci))
        parts.append(rng.standard_normal(co * 27 * ci) * std)
    return np.concatenate(parts).astype(np.float32)


def bf16(x):
    """Round FP64/FP32 values to the nearest BF16 (ties to even), as FP64."""
    a = np.asarray(x, dtype=np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def level_shape(shape0, level):
    s = tuple(shape0)
    for _ in range(level):
        s = tuple((n + 1) // 2 for n in s)
    return s


def _taps():
    return [(dz, dy, dx) for dz in range(3) for dy in range(3) for dx in range(3)]


def _src_index(m, stride, d, n_in):
    """Input index s*m + d - 1 along one axis, with a validity mask."""
    i = stride * m + d - 1
    ok = (i >= 0) & (i < n_in)
    return np.where(ok, i, 0), ok


def conv(x, W, stride, out_shape):
    """y[m, co] = sum_t sum_ci W[co, t, ci] x[s m + d_t - 1, ci]."""
    nz, ny, nx = out_shape
    y = np.zeros((nz, ny, nx, W.shape[0]))
    Z, Y, X = x.shape[:3]
    mz, my, mx = np.arange(nz), np.arange(ny), np.arange(nx)
    for t, (dz, dy, dx) in enumerate(_taps()):
        iz, okz = _src_index(mz, stride, dz, Z)
        iy, oky = _src_index(my, stride, dy, Y)
        ix, okx = _src_index(mx, stride, dx, X)
        xs = x[iz][:, iy][:, :, ix]
        ok = okz[:, None, None] & oky[None, :, None] & okx[None, None, :]
        xs = xs * ok[..., None]
        y += xs @ W[:, t, :].T
    return y


def conv_grad_input(gy, W, stride, in_shape):
    """Transpose of conv with respect to x: scatter each tap back."""
    gx = np.zeros(tuple(in_shape) + (W.shape[2],))
    nz, ny, nx = gy.shape[:3]
    Z, Y, X = in_shape
    mz, my, mx = np.arange(nz), np.arange(ny), np.arange(nx)
    for t, (dz, dy, dx) in enumerate(_taps()):
        iz, okz = _src_index(mz, stride, dz, Z)
        iy, oky = _src_index(my, stride, dy, Y)
        ix, okx = _src_index(mx, stride, dx, X)
        contrib = gy @ W[:, t, :]  # [nz, ny, nx, ci]
        ok = okz[:, None, None] & oky[None, :, None] & okx[None, None, :]
        contrib = contrib * ok[..., None]
        zz, yy, xx = np.meshgrid(iz, iy, ix, indexing="ij")
        np.add.at(gx, (zz, yy, xx), contrib)
    return gx


def conv_grad_weight(x, gy, stride):
    """dW[co, t, ci] = sum_m gy[m, co] x[s m + d_t - 1, ci]."""
    nz, ny, nx, co = gy.shape
    ci = x.shape[3]
    Z, Y, X = x.shape[:3]
    gW = np.zeros((co, 27, ci))
    mz, my, mx = np.arange(nz), np.arange(ny), np.arange(nx)
    g2 = gy.reshape(-1, co)
    for t, (dz, dy, dx) in enumerate(_taps()):
        iz, okz = _src_index(mz, stride, dz, Z)
        iy, oky = _src_index(my, stride, dy, Y)
        ix, okx = _src_index(mx, stride, dx, X)
        xs = x[iz][:, iy][:, :, ix]
        ok = okz[:, None, None] & oky[None, :, None] & okx[None, None, :]
        xs = (xs * ok[..., None]).reshape(-1, ci)
        gW[:, t, :] = g2.T @ xs
    return gW


def lrelu(y):
    return np.where(y > 0, y, SLOPE * y)


def lrelu_grad(a, g):
    """Gradient through the activation, from the activation output a (the
    sign of a equals the sign of its input because the slope is positive)."""
    return np.where(a > 0, g, SLOPE * g)


def _interp_matrix(n_f, n_c):
    """Dense 1D nested interpolation matrix P[n_f, n_c]."""
    P = np.zeros((n_f, n_c))
    for i in range(n_f):
        lo, hi = i // 2, (i + 1) // 2
        if hi >= n_c:
            P[i, lo] = 1.0
        else:
            P[i, lo] += 0.5
            P[i, hi] += 0.5
    return P


def upsample(c, fine_shape):
    """Tensor-product nested interpolation of a coarse (nz,ny,nx,C) field."""
    Pz = _interp_matrix(fine_shape[0], c.shape[0])
    Py = _interp_matrix(fine_shape[1], c.shape[1])
    Px = _interp_matrix(fine_shape[2], c.shape[2])
    return np.einsum("ai,bj,ck,ijkq->abcq", Pz, Py, Px, c)


def upsample_transpose(f, coarse_shape):
    Pz = _interp_matrix(f.shape[0], coarse_shape[0])
    Py = _interp_matrix(f.shape[1], coarse_shape[1])
    Px = _interp_matrix(f.shape[2], coarse_shape[2])
    return np.einsum("ai,bj,ck,abcq->ijkq", Pz, Py, Px, f)


def jittered_bf16(rng, eps=1e-7):
    """BF16 rounding after a random relative perturbation of size eps.  Two
    evaluations that differ only in FP32-level summation order round a few
    values the other way; running the oracle with this rounding instead of
    ``bf16`` measures how far such flips carry (the noise floor of a
    BF16-storage comparison)."""
    return lambda a: bf16(np.asarray(a, dtype=np.float64) * (1.0 + eps * rng.standard_normal(np.shape(a))))


def _encdec(W, x, S, R, gates):
    """Encoder-decoder body up to c0.  gates=None: leaky ReLU (the gate
    pass); otherwise every activation is replaced by the slope the gate
    pass chose at the same unit (1 where the gate activation is positive,
    1/8 elsewhere), which keeps the body linear in x."""
    def act(name, y):
        if gates is None:
            return R(lrelu(y))
        return R(lrelu_grad(gates[name], y))

    a = {"in": x}
    a["e0a"] = act("e0a", conv(a["in"], W[0], 1, S[0]))
    a["e0b"] = act("e0b", conv(a["e0a"], W[1], 1, S[0]))
    a["d1"] = act("d1", conv(a["e0b"], W[2], 2, S[1]))
    a["e1"] = act("e1", conv(a["d1"], W[3], 1, S[1]))
    a["d2"] = act("d2", conv(a["e1"], W[4], 2, S[2]))
    a["e2"] = act("e2", conv(a["d2"], W[5], 1, S[2]))
    a["d3"] = act("d3", conv(a["e2"], W[6], 2, S[3]))
    a["e3"] = act("e3", conv(a["d3"], W[7], 1, S[3]))
    a["cat2"] = np.concatenate([R(upsample(a["e3"], S[2])), a["e2"]], axis=3)
    a["c2"] = act("c2", conv(a["cat2"], W[8], 1, S[2]))
    a["cat1"] = np.concatenate([R(upsample(a["c2"], S[1])), a["e1"]], axis=3)
    a["c1"] = act("c1", conv(a["cat1"], W[9], 1, S[1]))
    a["cat0"] = np.concatenate([R(upsample(a["c1"], S[0])), a["e0b"]], axis=3)
    a["c0"] = act("c0", conv(a["cat0"], W[10], 1, S[0]))
    return a


def split_input(x_in):
    """Gate input (density and fixed-node channels) and signal input
    (residual channels) of an (nz, ny, nx, 8) input tensor."""
    xg = np.array(x_in, dtype=np.float64, copy=True)
    xg[..., 1:4] = 0.0
    xs = np.zeros_like(xg)
    xs[..., 1:4] = x_in[..., 1:4]
    return xg, xs


def forward(params, x_in, bf16_round: bool = True, rounder=None):
    """Network forward.  ``params`` is the flat FP32 vector; ``x_in`` is the
    (nz, ny, nx, 8) input.  Two passes share the weights: the gate pass runs
    the leaky-ReLU network on the density/fixed channels; the signal pass
    runs it on the residual channels with each activation replaced by the
    slope the gate pass chose, so the output is linear in the residual.
    Returns (out[..., 3], cache).  ``rounder`` replaces the BF16 rounding of
    activations and gradients (weights are always rounded plainly)."""
    R = bf16 if bf16_round else (lambda a: np.asarray(a, dtype=np.float64))
    if rounder is not None:
        R = rounder
    W = [(bf16(w) if bf16_round else w) for w in split_params(params)]
    s0 = x_in.shape[:3]
    S = [level_shape(s0, l) for l in range(4)]
    xg, xs = split_input(x_in)
    g = _encdec(W, R(xg), S, R, None)
    a = _encdec(W, R(xs), S, R, g)
    out = conv(a["c0"], W[11], 1, S[0])
    return out, {"W": W, "a": a, "g": g, "S": S, "R": R}


def backward(cache, g_out):
    """Weight gradient of sum(g_out * out) through the signal pass (the
    gates are piecewise constant in the weights).  Returns the flat FP64
    gradient.  Activation gradients are rounded where the GPU stores them."""
    W, a, G, S, R = cache["W"], cache["a"], cache["g"], cache["S"], cache["R"]
    gW = [None] * len(LAYERS)
    g = np.asarray(g_out, dtype=np.float64)
    gW[11] = conv_grad_weight(a["c0"], g, 1)
    g = R(lrelu_grad(G["c0"], conv_grad_input(g, W[11], 1, S[0])))      # at c0
    gW[10] = conv_grad_weight(a["cat0"], g, 1)
    gcat0 = R(conv_grad_input(g, W[10], 1, S[0]))
    g = R(lrelu_grad(G["c1"], upsample_transpose(gcat0[..., :32], S[1])))  # at c1
    gskip0 = gcat0[..., 32:]
    gW[9] = conv_grad_weight(a["cat1"], g, 1)
    gcat1 = R(conv_grad_input(g, W[9], 1, S[1]))
    g = R(lrelu_grad(G["c2"], upsample_transpose(gcat1[..., :64], S[2])))  # at c2
    gskip1 = gcat1[..., 64:]
    gW[8] = conv_grad_weight(a["cat2"], g, 1)
    gcat2 = R(conv_grad_input(g, W[8], 1, S[2]))
    g = R(lrelu_grad(G["e3"], upsample_transpose(gcat2[..., :64], S[3])))  # at e3
    gskip2 = gcat2[..., 64:]
    gW[7] = conv_grad_weight(a["d3"], g, 1)
    g = R(lrelu_grad(G["d3"], conv_grad_input(g, W[7], 1, S[3])))        # at d3
    gW[6] = conv_grad_weight(a["e2"], g, 2)
    g = R(lrelu_grad(G["e2"], gskip2 + conv_grad_input(g, W[6], 2, S[2])))  # at e2
    gW[5] = conv_grad_weight(a["d2"], g, 1)
    g = R(lrelu_grad(G["d2"], conv_grad_input(g, W[5], 1, S[2])))        # at d2
    gW[4] = conv_grad_weight(a["e1"], g, 2)
    g = R(lrelu_grad(G["e1"], gskip1 + conv_grad_input(g, W[4], 2, S[1])))  # at e1
    gW[3] = conv_grad_weight(a["d1"], g, 1)
    g = R(lrelu_grad(G["d1"], conv_grad_input(g, W[3], 1, S[1])))        # at d1
    gW[2] = conv_grad_weight(a["e0b"], g, 2)
    g = R(lrelu_grad(G["e0b"], gskip0 + conv_grad_input(g, W[2], 2, S[0])))  # at e0b
    gW[1] = conv_grad_weight(a["e0a"], g, 1)
    g = R(lrelu_grad(G["e0a"], conv_grad_input(g, W[1], 1, S[0])))      # at e0a
    gW[0] = conv_grad_weight(a["in"], g, 1)
    return np.concatenate([w.ravel() for w in gW])


# ---------------------------------------------------------------------------
# FE-side plumbing: network input from (rho, r), output to a DOF vector.


def node_density(mesh, rho):
    """Mean density of the cells incident to each node."""
    acc = np.zeros(mesh.n_nodes)
    cnt = np.zeros(mesh.n_nodes)
    for v in range(mesh.cells.shape[1]):
        np.add.at(acc, mesh.cells[:, v], rho)
        np.add.at(cnt, mesh.cells[:, v], 1.0)
    return acc / cnt


def net_input(mesh, rho, r, fixed):
    """Build the (nz, ny, nx, 8) input tensor and rms(r).

    ``r`` is the SoA residual [3][N_n]; ``fixed`` is the [3][N_n] Dirichlet
    mask (nonzero = fixed)."""
    nx, ny, nz = (n + 1 for n in mesh.nel)
    r = np.asarray(r, dtype=np.float64).reshape(3, -1)
    rms = np.sqrt(np.sum(r * r) / r.size)
    x = np.zeros((nz, ny, nx, N_IN))
    x[..., 0] = node_density(mesh, rho).reshape(nz, ny, nx)
    for c in range(3):
        x[..., 1 + c] = (r[c] / rms).reshape(nz, ny, nx)
    x[..., 4] = (np.asarray(fixed).reshape(3, -1).any(axis=0)).reshape(nz, ny, nx)
    return x, rms


def precondition(mesh, params, gamma, rho, r, fixed, bf16_round=True, rounder=None):
    """z = gamma * rms(r) * mask * N(input), as a [3][N_n] SoA vector."""
    x, rms = net_input(mesh, rho, r, fixed)
    out, cache = forward(params, x, bf16_round, rounder)
    z = np.stack([out[..., c].ravel() for c in range(3)])
    free = 1.0 - (np.asarray(fixed).reshape(3, -1) != 0)
    return gamma * rms * free * z, (x, rms, cache)


def loss_and_grad_out(K, free, gamma, n_out, r_hat, e_hat):
    """K-norm loss of the masked, scaled prediction and its gradient with
    respect to the raw network output (flattened SoA [3*N_n]).

    ``K`` is the assembled operator on all DOFs with fixed rows/columns set
    to identity; ``free`` is 1 on free DOFs."""
    n = free * n_out
    d = gamma * n - e_hat
    Kd = K @ d
    den = float(e_hat @ r_hat)
    L = float(d @ Kd) / den
    g = 2.0 * gamma * free * Kd / den
    return L, g


def adam_step(w, g, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step with bias correction (t counts from 1)."""
    m = beta1 * m + (1 - beta1) * g
    v = beta2 * v + (1 - beta2) * g * g
    mh = m / (1 - beta1 ** t)
    vh = v / (1 - beta2 ** t)
    return w - lr * mh / (np.sqrt(vh) + eps), m, v
