"""The learned warm start on the GPU against the CPU reference network (oracle/unet.py):
forward pass, loss gradient, Adam, input packing, and what the trained network gains
over a zero initial guess."""
import math

import numpy as np
import pytest
import torch

from gpu_util import dev, host, rel, say
from oracle import unet as ref
from oracle import operator as op
from synth import random_field_object, plane_wave

pytestmark = pytest.mark.gpu

api = pytest.importorskip("paper_1104_4263_amd.api")
from paper_1104_4263_amd._lib import DieTeError  # noqa: E402

CONFIGS = [(1, 8, 8, 8, 2), (2, 8, 16, 16, 2), (3, 16, 32, 32, 1), (2, 16, 16, 48, 3)]
# base 32 on 64 x 64: every 3x3 layer but the first and its adjoints take the LDS-staged convolution
# (widths multiples of 32, both output-tile widths)
LDS_CONV = (2, 32, 64, 64, 1)


def rand_inputs(rng, B, H, W):
    return rng.standard_normal((B, H, W, 8)).astype(np.float32)


def params_of(net):
    return net.get_params().numpy().astype(np.float64)


@pytest.mark.parametrize("levels,base,H,W,B", CONFIGS + [LDS_CONV])
def test_forward_matches_oracle(levels, base, H, W, B):
    say(f"unet forward L={levels} C={base} {H}x{W} B={B}")
    rng = np.random.default_rng(levels * 100 + base)
    net = api.UNet(levels, base, H, W, max_batch=B, seed=11)
    assert net.n_params == ref.n_params(levels, base)
    x = rand_inputs(rng, B, H, W)
    y = net.forward(torch.from_numpy(x).cuda()).cpu().numpy().astype(np.float64)
    yr = ref.forward(params_of(net), x, levels, base, bf16=True).detach().numpy()
    err = rel(y, yr)
    say(f"  rel err {err:.2e}")
    assert err < 1e-2
    assert np.max(np.abs(y - yr)) < 3e-2 * np.max(np.abs(yr))


# the last two shapes have W % 32 == 0 at every level: all their weight and bias gradients come
# from the LDS-staged gradient kernel (the first three mix both gradient kernels)
@pytest.mark.parametrize("levels,base,H,W,B", CONFIGS[:3] + [(2, 8, 64, 64, 1), (1, 16, 32, 64, 2), LDS_CONV])
def test_gradient_matches_oracle(levels, base, H, W, B):
    say(f"unet gradient L={levels} C={base} {H}x{W} B={B}")
    rng = np.random.default_rng(7 + levels)
    net = api.UNet(levels, base, H, W, max_batch=B, seed=5)
    x = rand_inputs(rng, B, H, W)
    t = rng.standard_normal((B, H, W, 4)).astype(np.float32)
    loss = net.loss_grad(torch.from_numpy(x).cuda(), torch.from_numpy(t).cuda())
    g = net.get_grads().numpy().astype(np.float64)
    lr_, gr = ref.loss_and_grad(params_of(net), x, t, levels, base, bf16=True)
    say(f"  loss {loss:.6f} vs {lr_:.6f}; grad rel err {rel(g, gr):.2e}")
    assert abs(loss - lr_) <= 1e-3 * lr_
    assert rel(g, gr) < 2e-2
    off = 0
    for name, ci, co, taps in ref.layer_specs(levels, base):
        n = co * taps * ci + co
        e = rel(g[off:off + n], gr[off:off + n])
        assert e < 5e-2, (name, e)
        off += n


def test_adam_matches_oracle():
    rng = np.random.default_rng(3)
    levels, base, H, W, B = 2, 8, 16, 16, 2
    net = api.UNet(levels, base, H, W, max_batch=B, seed=2)
    p = params_of(net)
    m = np.zeros_like(p)
    v = np.zeros_like(p)
    for step in (1, 2):
        x = rand_inputs(rng, B, H, W)
        t = rng.standard_normal((B, H, W, 4)).astype(np.float32)
        net.loss_grad(torch.from_numpy(x).cuda(), torch.from_numpy(t).cuda())
        g = net.get_grads().numpy().astype(np.float64)
        net.adam(1e-3)
        p_new = params_of(net)
        p_ref, m, v = ref.adam_step(p, g, m, v, step, 1e-3)
        err = np.max(np.abs(p_new - p_ref) / (np.abs(p_ref) + 1e-3))
        say(f"  adam step {step}: max rel err {err:.2e}")
        assert err < 1e-5
        p = p_new


def test_set_params_round_trip_and_reset():
    net = api.UNet(2, 8, 16, 16, max_batch=1, seed=1)
    p = np.random.default_rng(0).standard_normal(net.n_params).astype(np.float32) * 0.1
    net.set_params(p)
    assert np.array_equal(net.get_params().numpy(), p)
    with pytest.raises(DieTeError):
        bad = p.copy()
        bad[3] = np.nan
        net.set_params(bad)


def test_pack_inputs_and_targets_match_oracle():
    rng = np.random.default_rng(9)
    nobj, per, ny, nx = 2, 3, 8, 16
    eps = 1 + rng.random((nobj, ny, nx)) * 5 + 0.3j * rng.random((nobj, ny, nx))
    e_in = rng.standard_normal((nobj * per, 2, ny, nx)) + 1j * rng.standard_normal((nobj * per, 2, ny, nx))
    e_tot = e_in + 0.1 * (rng.standard_normal(e_in.shape) + 1j * rng.standard_normal(e_in.shape))
    x = api.UNet.pack_inputs(dev(eps), dev(e_in)).cpu().numpy()
    chi = np.repeat(eps - 1.0, per, axis=0)
    assert np.array_equal(x, ref.pack_inputs(chi, e_in).astype(np.float32))
    t = api.UNet.pack_targets(dev(e_tot), dev(e_in)).cpu().numpy()
    assert np.array_equal(t, ref.pack_targets(e_tot, e_in).astype(np.float32))


def test_invalid_shapes_are_rejected():
    with pytest.raises(DieTeError):
        api.UNet(3, 8, 16, 16, max_batch=1)  # the coarsest level would be 4 wide
    net = api.UNet(1, 8, 8, 8, max_batch=2)
    with pytest.raises(DieTeError):
        net.forward(torch.zeros(3, 8, 8, 8, device="cuda"))  # batch above max_batch


def test_training_fits_a_fixed_batch():
    rng = np.random.default_rng(4)
    net = api.UNet(2, 16, 16, 16, max_batch=4, seed=3)
    x = torch.from_numpy(rand_inputs(rng, 4, 16, 16)).cuda()
    t = torch.from_numpy((0.5 * rng.standard_normal((4, 16, 16, 4))).astype(np.float32)).cuda()
    first = net.train_step(x, t, 3e-3)
    for _ in range(150):
        last = net.train_step(x, t, 3e-3)
    say(f"  loss {first:.4f} -> {last:.4f}")
    assert last < 0.2 * first


def _solve_pairs(objs, psis, x0=None, **kw):
    """Object o lit by the angle psis[o], all in one batched solve."""
    g = objs[0][0]
    eps = np.stack([e for _, e in objs])
    b = np.stack([plane_wave(g, p) for p in psis])
    s = api.Solver.from_grid(g, eps)
    B = dev(b)
    u, rc, info = s.solve(B, x0=x0, **kw)
    return s, B, u, rc, info, eps


def test_warm_start_gains_over_zero_guess():
    """Train on solver-generated solutions of small random-field objects (one random
    angle each), then compare GMRES iterations from the network's guess and from zero
    on held-out objects and angles."""
    n, levels, base, ntrain, ntest = 32, 2, 16, 1024, 64
    rng = np.random.default_rng(12)
    train = [random_field_object(n, seed=50_000 + i) for i in range(ntrain)]
    psis = list(2 * math.pi * rng.random(ntrain))
    s, B, U, rc, info, eps = _solve_pairs(train, psis, restart=30, max_iters=5000, tol=1e-8, mixed=True)
    assert rc == 0
    X = api.UNet.pack_inputs(dev(eps), B)
    T = api.UNet.pack_targets(U, B)
    del s
    net = api.UNet(levels, base, n, n, max_batch=32, seed=7)
    order = np.arange(ntrain)
    losses = []
    for epoch in range(60):
        rng.shuffle(order)
        for k in range(0, ntrain, 32):
            idx = torch.from_numpy(order[k:k + 32]).cuda()
            losses.append(net.train_step(X[idx], T[idx], 1e-3))
    say(f"  training loss {losses[0]:.4f} -> {np.mean(losses[-32:]):.4f}")
    assert np.mean(losses[-32:]) < 0.5 * losses[0]
    test = [random_field_object(n, seed=90_000 + i) for i in range(ntest)]
    tpsi = list(2 * math.pi * rng.random(ntest))
    s0, Bt, U0, rc0, info0, eps_t = _solve_pairs(test, tpsi, restart=30, max_iters=5000, tol=1e-8)
    x0 = net.warm_start(s0, Bt)
    # the ABI path equals pack + forward + e_in
    y = net.forward(api.UNet.pack_inputs(dev(eps_t), Bt)[:32])
    ynp = y.cpu().numpy()
    x0_ref = host(Bt)[:32].copy()
    x0_ref[:, 0] += ynp[..., 0] + 1j * ynp[..., 1]
    x0_ref[:, 1] += ynp[..., 2] + 1j * ynp[..., 3]
    assert rel(host(x0)[:32], x0_ref) < 1e-12
    u1, rc1, info1 = s0.solve(Bt, x0=x0, restart=30, max_iters=5000, tol=1e-8)
    assert rc0 == 0 and rc1 == 0
    it0 = np.array([i["iters"] for i in info0])
    it1 = np.array([i["iters"] for i in info1])
    uh, bh, xh = host(U0), host(Bt), host(x0)
    e_net = np.array([rel(xh[r], uh[r]) for r in range(ntest)])
    e_inc = np.array([rel(bh[r], uh[r]) for r in range(ntest)])
    say(f"  held-out guess error median: network {np.median(e_net):.3f}, incident field {np.median(e_inc):.3f}; "
        f"iterations zero guess {it0.mean():.1f}, warm start {it1.mean():.1f}")
    for r in range(ntest):
        assert info1[r]["rel_res_true"] <= 1e-8
    assert rel(host(u1), uh) < 1e-6
    assert np.median(e_net) < np.median(e_inc)
    assert it1.mean() < it0.mean()


@pytest.mark.slow
def test_configured_network_forward_at_256():
    """The configured network (4 levels, 32 base channels) at 256 x 256, one sample."""
    rng = np.random.default_rng(21)
    net = api.UNet(4, 32, 256, 256, max_batch=1, seed=13)
    x = rand_inputs(rng, 1, 256, 256)
    y = net.forward(torch.from_numpy(x).cuda()).cpu().numpy().astype(np.float64)
    yr = ref.forward(params_of(net), x, 4, 32, bf16=True).detach().numpy()
    err = rel(y, yr)
    say(f"  256^2 forward rel err {err:.2e}")
    assert err < 1e-2
