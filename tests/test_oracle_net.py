"""Pins for the preconditioner network oracle (oracle/net.py).

Each check ties the oracle to something other than itself: a library
correlation, an adjoint identity between independently written forward and
transpose code, exact interpolation of affine fields, finite differences,
and the closed form of a first Adam step.
"""

import numpy as np
import pytest
import scipy.ndimage as ndi
import torch

import synth
from oracle import mesh as omesh
from oracle import net


def _rand(shape, seed):
    return np.random.default_rng(seed).standard_normal(shape)


def test_param_count_and_split():
    n = net.n_params()
    assert n == sum(co * 27 * ci for (_, _, _, ci, co, _) in net.LAYERS)
    flat = np.arange(n, dtype=np.float64)
    parts = net.split_params(flat)
    assert parts[0].shape == (16, 27, 8)
    assert parts[-1].shape == (3, 27, 16)
    assert parts[0][0, 0, 1] == 1.0 and parts[1][0, 0, 0] == 16 * 27 * 8


def test_bf16_rounding_matches_torch():
    vals = np.array([1.0, 1 + 2.0 ** -8, 1 + 3 * 2.0 ** -8, -2.5e-3, 3.14159, 1e30, 6e-39, 0.0])
    ref = torch.tensor(vals, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(net.bf16(vals), ref)
    assert net.bf16(1 + 2.0 ** -8) == 1.0                    # tie to even
    assert net.bf16(1 + 3 * 2.0 ** -8) == 1 + 2.0 ** -6      # tie to even (up)
    x = _rand(10000, 1)
    np.testing.assert_array_equal(
        net.bf16(x), torch.tensor(x, dtype=torch.float32).to(torch.bfloat16).double().numpy())


def test_conv_stride1_equals_library_correlation():
    x = _rand((5, 6, 7, 3), 2)
    W = _rand((2, 27, 3), 3)
    y = net.conv(x, W, 1, (5, 6, 7))
    ref = np.zeros_like(y)
    for co in range(2):
        for ci in range(3):
            k = W[co, :, ci].reshape(3, 3, 3)  # (dz, dy, dx)
            ref[..., co] += ndi.correlate(x[..., ci], k, mode="constant", cval=0.0)
    np.testing.assert_allclose(y, ref, rtol=1e-13, atol=1e-12)


@pytest.mark.parametrize("shape", [(9, 5, 7), (8, 6, 4)])
def test_conv_stride2_is_subsampled_stride1(shape):
    x = _rand(shape + (4,), 4)
    W = _rand((3, 27, 4), 5)
    y1 = net.conv(x, W, 1, shape)
    out_shape = tuple((n + 1) // 2 for n in shape)
    y2 = net.conv(x, W, 2, out_shape)
    np.testing.assert_allclose(y2, y1[::2, ::2, ::2], rtol=1e-13, atol=1e-12)


@pytest.mark.parametrize("stride", [1, 2])
def test_conv_adjoints(stride):
    shape = (7, 5, 6)
    out_shape = shape if stride == 1 else tuple((n + 1) // 2 for n in shape)
    x = _rand(shape + (3,), 6)
    W = _rand((4, 27, 3), 7)
    g = _rand(out_shape + (4,), 8)
    y = net.conv(x, W, stride, out_shape)
    gx = net.conv_grad_input(g, W, stride, shape)
    gW = net.conv_grad_weight(x, g, stride)
    np.testing.assert_allclose(np.sum(y * g), np.sum(x * gx), rtol=1e-12)
    np.testing.assert_allclose(np.sum(y * g), np.sum(W * gW), rtol=1e-12)


def test_upsample_exact_on_affine_fields_and_adjoint():
    cs = (5, 4, 6)
    fs = (9, 7, 11)  # odd fine sizes: 2*(n_c - 1) + 1
    zc, yc, xc = np.meshgrid(*(np.arange(n) for n in cs), indexing="ij")
    c = np.stack([1.0 + 2 * xc - 3 * yc + 0.5 * zc, np.ones_like(xc, dtype=float)], axis=-1)
    f = net.upsample(c, fs)
    zf, yf, xf = np.meshgrid(*(np.arange(n) for n in fs), indexing="ij")
    np.testing.assert_allclose(f[..., 0], 1.0 + xf - 1.5 * yf + 0.25 * zf, rtol=1e-14, atol=1e-13)
    np.testing.assert_allclose(f[..., 1], 1.0)
    # even fine size: the last point copies the last coarse value; constants kept
    fe = net.upsample(np.ones((3, 3, 3, 1)), (6, 6, 6))
    np.testing.assert_allclose(fe, 1.0)
    a = _rand(cs + (2,), 9)
    b = _rand((10, 8, 11, 2), 10)
    up = net.upsample(a, (10, 8, 11))
    dn = net.upsample_transpose(b, cs)
    np.testing.assert_allclose(np.sum(up * b), np.sum(a * dn), rtol=1e-12)


def test_backward_matches_finite_differences():
    shape = (5, 5, 9)  # levels 5x5x9, 3x3x5, 2x2x3, 1x1x2
    params = net.init_params(11).astype(np.float64)
    x = _rand(shape + (8,), 12)
    g = _rand(shape + (3,), 13)

    def L(p):
        out, _ = net.forward(p, x, bf16_round=False)
        return np.sum(out * g)

    out, cache = net.forward(params, x, bf16_round=False)
    grad = net.backward(cache, g)
    rng = np.random.default_rng(14)
    # probe entries of every layer
    offs = np.cumsum([0] + [co * 27 * ci for (_, _, _, ci, co, _) in net.LAYERS])
    for li in range(len(net.LAYERS)):
        for idx in rng.integers(offs[li], offs[li + 1], size=3):
            h = 1e-6
            pp = params.copy(); pp[idx] += h
            pm = params.copy(); pm[idx] -= h
            fd = (L(pp) - L(pm)) / (2 * h)
            assert abs(fd - grad[idx]) <= 1e-6 * max(1.0, abs(fd)), (li, idx, fd, grad[idx])


def test_node_density_and_input():
    p = synth.cantilever3d(4, 2, 2, nrhs=1)
    m = omesh.build(3, p.nel)
    rho = np.full(m.n_cells, 0.37)
    np.testing.assert_allclose(net.node_density(m, rho), 0.37, rtol=1e-15)
    cnt = np.zeros(m.n_nodes)
    np.add.at(cnt, m.cells.ravel(), 1.0)
    assert cnt.sum() == 4 * m.n_cells
    interior = int(synth.node_id(p.nel, 2, 1, 1))
    assert cnt[interior] == 24  # Kuhn triangulation: 24 tetrahedra meet at an interior vertex
    r = _rand((3, m.n_nodes), 15)
    x, rms = net.net_input(m, rho, r, p.fixed)
    assert x.shape == (3, 3, 5, 8)
    np.testing.assert_allclose(np.mean(x[..., 1:4] ** 2), 1.0, rtol=1e-12)
    assert np.all(x[:, :, 0, 4] == 1) and np.all(x[:, :, 1:, 4] == 0)
    assert np.all(x[..., 5:] == 0)


def test_loss_gradient_and_minimum():
    from oracle import fem
    p = synth.cantilever3d(4, 2, 2, nrhs=1)
    m = omesh.build(3, p.nel)
    E = fem.simp_modulus(np.random.default_rng(16).uniform(0.1, 1, m.n_cells))
    K = fem.assemble(m, E, p.nu)
    fixed = np.asarray(p.fixed).reshape(-1) != 0
    free = (~fixed).astype(float)
    Kr = K.tolil()
    for i in np.nonzero(fixed)[0]:
        Kr[i, :] = 0; Kr[:, i] = 0; Kr[i, i] = 1.0
    Kr = Kr.tocsr()
    e = _rand(free.size, 17) * free
    r = Kr @ e
    gamma = 2.0
    n = _rand(free.size, 18)
    L, g = net.loss_and_grad_out(Kr, free, gamma, n, r, e)
    assert L > 0
    L0, _ = net.loss_and_grad_out(Kr, free, gamma, e / gamma, r, e)
    assert abs(L0) < 1e-24
    d = _rand(free.size, 19)
    h = 1e-6
    Lp, _ = net.loss_and_grad_out(Kr, free, gamma, n + h * d, r, e)
    Lm, _ = net.loss_and_grad_out(Kr, free, gamma, n - h * d, r, e)
    np.testing.assert_allclose((Lp - Lm) / (2 * h), g @ d, rtol=1e-6)


def test_adam_first_step_closed_form():
    w = np.array([1.0, -2.0, 0.5])
    g = np.array([0.3, -4.0, 1e-3])
    w1, m, v = net.adam_step(w, g, np.zeros(3), np.zeros(3), 1, lr=0.01, eps=0.0)
    np.testing.assert_allclose(w1, w - 0.01 * np.sign(g), rtol=1e-14)
    np.testing.assert_allclose(m, 0.1 * g)
    np.testing.assert_allclose(v, 0.001 * g * g)


def test_output_is_linear_in_the_residual():
    """The signal pass is gated by the density-only pass, so for a fixed
    design the network is a linear map of the residual channels."""
    shape = (5, 5, 9)
    params = net.init_params(21).astype(np.float64)
    base = _rand(shape + (8,), 22)
    x1, x2 = base.copy(), base.copy()
    x2[..., 1:4] = _rand(shape + (3,), 23)
    a, b = 0.7, -2.3
    x3 = base.copy()
    x3[..., 1:4] = a * x1[..., 1:4] + b * x2[..., 1:4]
    o1, _ = net.forward(params, x1, bf16_round=False)
    o2, _ = net.forward(params, x2, bf16_round=False)
    o3, _ = net.forward(params, x3, bf16_round=False)
    np.testing.assert_allclose(o3, a * o1 + b * o2, rtol=1e-11, atol=1e-12 * np.abs(o3).max())
    # the density channel changes the gates (and so the map), not an offset
    x4 = x1.copy()
    x4[..., 1:4] = 0.0
    o4, _ = net.forward(params, x4, bf16_round=False)
    assert np.all(o4 == 0.0)
