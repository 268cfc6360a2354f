"""GPU parity of the learned preconditioner against the FP64 oracle
(oracle/net.py), called through the C ABI.

The oracle rounds to BF16 where the kernels store (input, weights, every
activation and activation gradient), so the remaining differences are FP32
accumulation order against FP64 and the BF16 rounding flips it causes.  The
bar for each compared quantity is derived from that mechanism: the oracle
is run twice more with an FP32-level (1e-7 relative) jitter before every
BF16 rounding, the spread of those runs from the clean one is the noise
floor, and the GPU must stay within 2.5x the floor (never looser than 5e-2
for the output, 2e-2 for the loss, 1.5e-1 per layer gradient; the gate
pass makes some slope choices on near-zero activations, so single flips move
the linear map).  A wrong index or a dropped term gives errors of order
one.  Adam is checked to FP32 rounding; harvested
pairs satisfy r = K e to 1e-11 relative.  Solves with the learned
preconditioner are judged by the FP64 true residual and the direct
solution.
"""

import numpy as np
import pytest

import synth
from oracle import fem, mesh as M, net

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda:0"
CASES = [("odd", (16, 8, 8)), ("ragged", (15, 7, 9)), ("tiny", (3, 2, 2))]


def _t(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device=DEV)


def _ctx(p, **kw):
    from paper_2012_08208_amd import learned
    return learned.gmg_context(p, device=DEV, **kw)


def _rel(a, b):
    return float(np.linalg.norm(np.ravel(a) - np.ravel(b)) / max(np.linalg.norm(np.ravel(b)), 1e-300))


def _layer_slices():
    offs = np.cumsum([0] + [co * 27 * ci for (_, _, _, ci, co, _) in net.LAYERS])
    return [(net.LAYERS[i][0], offs[i], offs[i + 1]) for i in range(len(net.LAYERS))]


def _setup(nel, seed):
    p = synth.cantilever3d(*nel, nrhs=1)
    m = M.build(3, p.nel)
    rho = synth.rho_random(seed, m.n_cells, 0.05, 1.0)
    r = synth.vec_random(seed + 1, (3, m.n_nodes), p.fixed)
    w = net.init_params(seed + 2)
    return p, m, rho, r, w


def _to_grid(soa, m):
    nx, ny, nz = (n + 1 for n in m.nel)
    return np.stack([soa[c].reshape(nz, ny, nx) for c in range(3)], axis=-1)


def _bar(err, floor, cap):
    """GPU error against the oracle must stay within 2.5x the rounding-flip
    noise floor (and below ``cap``)."""
    return err <= min(max(2.5 * floor, 1e-4), cap)


@pytest.mark.parametrize("tiles", ["auto", "big"])
@pytest.mark.parametrize("name,nel", CASES)
def test_forward_and_backward_match_oracle(name, nel, tiles, monkeypatch):
    """``big``: every stride-1 layer on the 8x8x4 output boxes the library
    uses on large grids (at these sizes it would pick 4x4x4 boxes with split
    K sums)."""
    print(f"[net fwd/bwd] {name} nel={nel} tiles={tiles}", flush=True)
    if tiles == "big":
        monkeypatch.setenv("TOPO_CONV_BIG_MIN", "1")
    p, m, rho, r, w = _setup(nel, 10)
    gamma = 1.7
    t = _ctx(p)
    t.precond_set_weights(_t(w, torch.float32))
    t.precond_config(gamma, 10, 1)
    z = torch.zeros(p.n_dofs, dtype=torch.float64, device=DEV)
    t.precond_apply(_t(rho), _t(r), z)
    gz = np.random.default_rng(11).standard_normal((3, m.n_nodes))
    grad = torch.zeros(net.n_params(), dtype=torch.float32, device=DEV)
    t.precond_backward(_t(gz), grad)
    assert t.sync() == 0
    free = (p.fixed == 0)

    def oracle(rounder):
        z_ref, (x, rms, cache) = net.precondition(m, w, gamma, rho, r, p.fixed, True, rounder)
        g_out = net.bf16(gamma * rms * free * gz)
        return z_ref.ravel(), net.backward(cache, _to_grid(g_out, m))

    z_ref, gref = oracle(None)
    noisy = [oracle(net.jittered_bf16(np.random.default_rng(s))) for s in (1, 2)]
    e = _rel(z.cpu().numpy(), z_ref)
    fl = max(_rel(zn, z_ref) for zn, _ in noisy)
    print(f"  forward rel L2 {e:.2e} (floor {fl:.2e})", flush=True)
    assert _bar(e, fl, 5e-2)
    g = grad.cpu().numpy().astype(np.float64)
    for lname, a, b in _layer_slices():
        el = _rel(g[a:b], gref[a:b])
        fl = max(_rel(gn[a:b], gref[a:b]) for _, gn in noisy)
        print(f"  grad {lname}: {el:.2e} (floor {fl:.2e})", flush=True)
        assert _bar(el, fl, 1.5e-1), (lname, el, fl)


def _free_operator(m, p, rho):
    E = fem.simp_modulus(rho, p.E0, p.Emin, p.penal)
    K = fem.assemble(m, E, p.nu).tolil()
    fixed = p.fixed.reshape(-1) != 0
    for i in np.nonzero(fixed)[0]:
        K[i, :] = 0
        K[:, i] = 0
        K[i, i] = 1.0
    return K.tocsr(), (~fixed).astype(float)


@pytest.mark.parametrize("name,nel", CASES[:2])
def test_loss_gradient_and_adam_match_oracle(name, nel):
    print(f"[net loss] {name} nel={nel}", flush=True)
    p, m, rho, _, w = _setup(nel, 20)
    K, free = _free_operator(m, p, rho)
    e = synth.vec_random(23, (3, m.n_nodes), p.fixed).ravel()
    r = K @ e
    gamma = 3.0
    t = _ctx(p)
    t.precond_set_weights(_t(w, torch.float32))
    t.precond_config(gamma, 10, 1)
    loss = torch.zeros(1, dtype=torch.float64, device=DEV)
    t.precond_train_step(_t(rho), _t(r), _t(e), 0.0, loss)
    grad = torch.zeros(net.n_params(), dtype=torch.float32, device=DEV)
    t.precond_get_grad(grad)
    assert t.sync() == 0
    rms = np.sqrt(np.mean(r * r))
    x, _ = net.net_input(m, rho, r.reshape(3, -1), p.fixed)

    def oracle(rounder):
        out, cache = net.forward(w, x, True, rounder)
        n_out = np.stack([out[..., c].ravel() for c in range(3)]).ravel()
        L, gsoa = net.loss_and_grad_out(K, free, gamma, n_out, r / rms, e / rms)
        return L, net.backward(cache, _to_grid(net.bf16(gsoa.reshape(3, -1)), m)), n_out

    L, gref, n_ref = oracle(None)
    noisy = [oracle(net.jittered_bf16(np.random.default_rng(s))) for s in (1, 2, 3)]
    # the loss is one scalar: its floor is taken from the spread of the loss
    # and of the network output it is computed from
    fl = max(max(abs(Ln - L) / abs(L) for Ln, _, _ in noisy),
             0.5 * max(_rel(nn_, n_ref) for _, _, nn_ in noisy))
    el = abs(loss.item() - L) / abs(L)
    print(f"  loss gpu {loss.item():.6e} oracle {L:.6e} rel {el:.1e} (floor {fl:.1e})", flush=True)
    assert _bar(el, fl, 2e-2)
    g = grad.cpu().numpy().astype(np.float64)
    for lname, a, b in _layer_slices():
        el = _rel(g[a:b], gref[a:b])
        fl = max(_rel(gn[a:b], gref[a:b]) for _, gn, _ in noisy)
        assert _bar(el, fl, 1.5e-1), (lname, el, fl)
    # one Adam step from fresh moments, checked with the GPU's own gradient
    lr = 1e-3
    t.precond_set_weights(_t(w, torch.float32))
    t.precond_train_step(_t(rho), _t(r), _t(e), lr, loss)
    t.precond_get_grad(grad)
    w1 = torch.zeros_like(grad)
    t.precond_get_weights(w1)
    assert t.sync() == 0
    g = grad.cpu().numpy().astype(np.float64)
    w_ref, _, _ = net.adam_step(w.astype(np.float64), g, np.zeros_like(g), np.zeros_like(g), 1, lr)
    np.testing.assert_allclose(w1.cpu().numpy(), w_ref, rtol=1e-5, atol=1e-7)


def test_harvest_pairs_are_exact():
    p = synth.cantilever3d(12, 6, 6, nrhs=1)
    m = M.build(3, p.nel)
    rho = synth.rho_random(30, m.n_cells, 0.05, 1.0)
    K, free = _free_operator(m, p, rho)
    f = p.loads.reshape(-1) * free
    u_ref = fem.solve(fem.assemble(m, fem.simp_modulus(rho), p.nu), p.loads.reshape(1, -1),
                      p.fixed.ravel())[0]
    t = _ctx(p, rtol=1e-12)
    its = [0, 1, 2, 4, 8]
    R = torch.zeros(len(its) * p.n_dofs, dtype=torch.float64, device=DEV)
    E = torch.zeros_like(R)
    n, fin = t.precond_harvest(_t(rho), its, R, E)
    assert t.sync() == 0
    assert n == len(its) and fin > 8
    R = R.cpu().numpy().reshape(n, -1)
    E = E.cpu().numpy().reshape(n, -1)
    np.testing.assert_allclose(E[0], u_ref, rtol=0, atol=1e-9 * np.abs(u_ref).max())
    np.testing.assert_allclose(R[0], f, rtol=0, atol=1e-9 * np.abs(f).max())
    energy = []
    for k in range(n):
        Ke = K @ E[k]
        assert _rel(R[k], Ke) <= 1e-11
        assert np.all(E[k][free == 0] == 0)
        energy.append(E[k] @ Ke)
    assert all(energy[i + 1] < energy[i] for i in range(n - 1))  # CG decreases the K-norm error
    # pre-smoothed pairs (x = S r): still exact, and smoothing lowers the K-norm error
    R2 = torch.zeros(len(its) * p.n_dofs, dtype=torch.float64, device=DEV)
    E2 = torch.zeros_like(R2)
    n2, _ = t.precond_harvest(_t(rho), its, R2, E2, True)
    assert t.sync() == 0 and n2 == n
    R2 = R2.cpu().numpy().reshape(n, -1)
    E2 = E2.cpu().numpy().reshape(n, -1)
    for k in range(n):
        Ke = K @ E2[k]
        assert _rel(R2[k], Ke) <= 1e-11
        assert E2[k] @ Ke < energy[k]


def _solve(t, p, rho):
    u = torch.zeros(p.n_dofs * p.nrhs, dtype=torch.float64, device=DEV)
    info = torch.zeros(6, dtype=torch.float64, device=DEV)
    t.solve(_t(rho), u, info)
    st = t.sync()
    return u.cpu().numpy().reshape(p.nrhs, -1), info.cpu().numpy(), st


@pytest.mark.parametrize("nrhs", [2, 4])
@pytest.mark.parametrize("weights", ["zero", "random"])
def test_learned_fcg_solves_to_direct(weights, nrhs):
    """nrhs 4: the 8-direction window needs two dot-product launches."""
    from paper_2012_08208_amd import TOPO_S_LEARNED_FALLBACK, learned
    p = synth.cantilever3d(16, 8, 8, nrhs=nrhs)
    m = M.build(3, p.nel)
    rho = synth.rho_random(40, m.n_cells, 0.05, 1.0)
    u_ref = fem.solve(fem.assemble(m, fem.simp_modulus(rho), p.nu), p.loads.reshape(nrhs, -1),
                      p.fixed.ravel())
    w = np.zeros(net.n_params(), np.float32) if weights == "zero" else net.init_params(41)
    t = learned.learned_context(p, _t(w, torch.float32), 1.0, 400, 1, rtol=1e-10, device=DEV)
    u, info, st = _solve(t, p, rho)
    fcg, fb = t.precond_stats()
    print(f"[learned fcg] {weights} nrhs {nrhs}: iters {info[0]:.0f} fcg {fcg} fallback {fb} "
          f"status {st}", flush=True)
    assert st in (0, TOPO_S_LEARNED_FALLBACK)
    if weights == "zero":
        assert st == 0 and fb == 0
    assert info[1] == 1.0 and max(info[2:4]) <= 1e-10
    for k in range(nrhs):
        assert _rel(u[k], u_ref[k]) <= 1e-7


def test_learned_fallback_to_multigrid():
    from paper_2012_08208_amd import TOPO_S_LEARNED_FALLBACK, learned
    p = synth.cantilever3d(16, 8, 8, nrhs=1)
    m = M.build(3, p.nel)
    rho = synth.rho_random(50, m.n_cells, 0.05, 1.0)
    u_ref = fem.solve(fem.assemble(m, fem.simp_modulus(rho), p.nu), p.loads.reshape(1, -1),
                      p.fixed.ravel())
    t = learned.learned_context(p, _t(np.zeros(net.n_params(), np.float32), torch.float32), 1.0,
                                2, 1, rtol=1e-10, device=DEV)
    u, info, st = _solve(t, p, rho)
    fcg, fb = t.precond_stats()
    assert st == TOPO_S_LEARNED_FALLBACK and fb == 1
    assert info[1] == 1.0 and info[0] > 2 and info[2] <= 1e-10
    assert _rel(u[0], u_ref[0]) <= 1e-7


def test_training_on_gpu_cuts_fcg_iterations():
    """The network trained on the GPU by the library's kernels, on pairs
    harvested from multigrid PCG along a SIMP history, against the same
    two-level cycle without the network (zero weights) on a held-out later
    design of the history."""
    from paper_2012_08208_amd import learned
    p = synth.cantilever3d(24, 12, 12, nrhs=1, volfrac=0.3, rmin=1.5)
    t = _ctx(p, rtol=1e-10)
    ps = learned.harvest_history(t, n_designs=6, simp_steps=3,
                                 harvest_iters=[1, 2, 3, 5, 8, 12, 16])
    gamma = learned.choose_gamma(ps)
    rho_test = ps.rhos[-1].clone()
    u = torch.zeros(p.n_dofs, dtype=torch.float64, device=DEV)
    t.iterate(rho_test, u, 3)   # a later design than any used for training
    w0 = learned.init_weights(60, DEV)
    t.precond_set_weights(w0)
    t.precond_config(gamma, 500, 1)
    losses = learned.train(t, ps, steps=3000, lr=3e-4, seed=61, lr_final=3e-5)
    w = torch.zeros_like(w0)
    t.precond_get_weights(w)
    assert t.sync() == 0
    L = losses.cpu().numpy()
    print(f"[train] gamma {gamma:.3e} pairs {ps.R.shape[0]} loss first50 {L[:50].mean():.3e} "
          f"last100 {L[-100:].mean():.3e}", flush=True)
    assert np.all(np.isfinite(L)) and L[-100:].mean() < 0.5 * L[:50].mean()
    rho_np = rho_test.cpu().numpy()
    its = {}
    for name, ww in (("trained", w), ("none", torch.zeros_like(w))):
        tl = learned.learned_context(p, ww, gamma, 500, 1, rtol=1e-8, device=DEV)
        _, info, st = _solve(tl, p, rho_np)
        assert st == 0 and info[1] == 1.0
        its[name] = info[0]
    print(f"[gain] FCG iterations trained {its['trained']:.0f} vs without network "
          f"{its['none']:.0f}", flush=True)
    assert its["trained"] <= 0.8 * its["none"]


def test_streaming_replay_training_cuts_fcg_iterations():
    """Pairs streamed through a replay buffer smaller than the pairs seen
    (the buffer wraps several times, over seeded random SIMP histories of
    varying volume fraction and radius) train the network by the library's
    kernels; only pairs whose design is still held are drawn; the trained
    network beats the cycle without it on a held-out design."""
    from paper_2012_08208_amd import learned
    p = synth.cantilever3d(24, 12, 12, nrhs=1, volfrac=0.3, rmin=1.5)
    t = _ctx(p, rtol=1e-10)
    rng = np.random.default_rng(7)
    hist = [dict(volfrac=float(rng.uniform(0.3, 0.5)), rmin=float(rng.uniform(1.5, 3.0)))
            for _ in range(64)]

    def histories(h):
        return synth.cantilever3d(24, 12, 12, nrhs=1, rtol=1e-10, **hist[h])

    w0 = learned.init_weights(60, DEV)
    t.precond_set_weights(w0)
    # output gain from a first small harvest, as the fixed-set recipe does
    ps = learned.harvest_history(t, n_designs=2, simp_steps=3, harvest_iters=[1, 2, 4, 8])
    gamma = learned.choose_gamma(ps)
    t.precond_config(gamma, 500, 1)
    res = learned.stream_train(t, histories, n_pairs=600, harvest_iters=[1, 2, 3, 5, 8, 12, 16],
                               capacity=96, steps_per_pair=4.0, lr=3e-4, lr_final=3e-5, seed=5,
                               simp_steps=2, designs_per_history=12)
    L = res["losses"].cpu().numpy()
    print(f"[stream] pairs {res['pairs']} designs {res['designs']} histories {res['histories']} "
          f"steps {res['steps']} loss first50 {L[:50].mean():.3e} last100 {L[-100:].mean():.3e}",
          flush=True)
    assert res["pairs"] >= 600 and res["pairs"] > 5 * res["capacity"] and res["histories"] >= 2
    assert res["steps"] >= 0.9 * 4 * 600
    # the streamed loss is measured on pairs of ever new designs, so it falls
    # less than the loss of a fixed set that the network can memorise
    assert np.all(np.isfinite(L)) and L[-100:].mean() < 0.7 * L[:50].mean()
    w = torch.zeros_like(w0)
    t.precond_get_weights(w)
    assert t.sync() == 0
    rho_test = ps.rhos[-1].clone()
    u = torch.zeros(p.n_dofs, dtype=torch.float64, device=DEV)
    t.iterate(rho_test, u, 6)   # a later design of the canonical history
    rho_np = rho_test.cpu().numpy()
    its = {}
    for name, ww in (("trained", w), ("none", torch.zeros_like(w))):
        tl = learned.learned_context(p, ww, gamma, 500, 1, rtol=1e-8, device=DEV)
        _, info, st = _solve(tl, p, rho_np)
        assert st == 0 and info[1] == 1.0
        its[name] = info[0]
    print(f"[stream gain] FCG iterations trained {its['trained']:.0f} vs without network "
          f"{its['none']:.0f}", flush=True)
    assert its["trained"] <= 0.8 * its["none"]


def test_network_full_size_properties():
    """The 128 x 64 x 64 learned-preconditioner grid (129 x 65 x 65 nodes, the
    configuration the learned bench times), where the oracle's full forward
    would take minutes: properties that hold exactly at any size.  The pass
    is deterministic (two calls agree bit for bit); scaling r by 2 scales z
    by exactly 2 (the input is r / rms(r), and power-of-two scaling is exact
    through the sum of squares and the square root); z is exactly zero on
    fixed DOFs; a zero residual gives a zero output."""
    p = synth.learned3d()
    assert p.nel == (128, 64, 64)
    print("[net] full-size properties 128x64x64", flush=True)
    m_nodes = p.n_nodes
    rho = synth.rho_random(21, p.n_cells, 0.05, 1.0)
    r = synth.vec_random(22, (3, m_nodes), p.fixed)
    w = net.init_params(23)
    t = _ctx(p)
    t.precond_set_weights(_t(w, torch.float32))
    t.precond_config(1.3, 10, 1)
    z1 = torch.zeros(p.n_dofs, dtype=torch.float64, device=DEV)
    z2 = torch.zeros_like(z1)
    z3 = torch.zeros_like(z1)
    t.precond_apply(_t(rho), _t(r), z1)
    t.precond_apply(_t(rho), _t(r), z2)
    t.precond_apply(_t(rho), _t(2.0 * r), z3)
    assert t.sync() == 0
    a, b, c = (v.cpu().numpy() for v in (z1, z2, z3))
    assert np.array_equal(a, b)
    assert np.array_equal(c, 2.0 * a)
    fixed = p.fixed.reshape(-1) != 0
    assert np.all(a[fixed] == 0.0) and np.count_nonzero(a[~fixed]) > 0.9 * np.count_nonzero(~fixed)
    t.precond_apply(_t(rho), torch.zeros(p.n_dofs, dtype=torch.float64, device=DEV), z1)
    assert t.sync() == 0
    assert torch.count_nonzero(z1).item() == 0
    t.close()
