"""Pins of the CPU reference U-Net (oracle/unet.py) against things other than itself."""
import numpy as np
import pytest
import torch

from oracle import unet


def test_bf16_round_bit_level():
    # 1 + 2^-8 is halfway between 1 and 1 + 2^-7: ties go to the even mantissa (1)
    vals = np.array([1.0, 1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -9, 1.0 + 2.0 ** -7 + 2.0 ** -8, -2.5, 3.0e-3])
    got = unet.bf16_round(vals)
    want = []
    for v in vals:
        u = np.array([v], np.float32).view(np.uint32)[0]
        u = (int(u) + 0x7FFF + ((int(u) >> 16) & 1)) & 0xFFFF0000
        want.append(np.array([u], np.uint32).view(np.float32)[0])
    assert np.array_equal(got, np.array(want, np.float64))
    assert got[1] == 1.0 and got[2] == 1.0 + 2.0 ** -7 and got[3] == 1.0 + 2.0 ** -6
    x = np.random.default_rng(0).standard_normal(1000)
    r = unet.bf16_round(x)
    assert np.all(np.abs(r - x) <= 2.0 ** -8 * np.abs(x) * (1 + 1e-6))  # unit roundoff 2^-8
    assert np.array_equal(unet.bf16_round(r), r)


def test_param_count_of_the_configured_network():
    # 4 levels, 32 base channels, written out layer by layer: 9 ci co + co per 3x3 layer
    layers = [(8, 32), (32, 32), (32, 64), (64, 64), (64, 128), (128, 128), (128, 256), (256, 256),
              (384, 128), (128, 128), (192, 64), (64, 64), (96, 32), (32, 32)]
    count = sum(9 * ci * co + co for ci, co in layers) + 32 * 4 + 4
    assert count == 1_948_420
    assert unet.n_params(4, 32) == count
    assert [s[1:3] for s in unet.layer_specs(4, 32)[:-1]] == layers


def test_one_convolution_against_loops():
    rng = np.random.default_rng(1)
    B, H, W, ci, co = 2, 5, 6, 8, 3
    x = rng.standard_normal((B, H, W, ci))
    w = rng.standard_normal((co, 9, ci))
    b = rng.standard_normal(co)
    # the tap convention W[co][3 (dy + 1) + (dx + 1)][ci] through the same reshape the oracle uses
    wt = torch.tensor(w).reshape(co, 3, 3, ci).permute(0, 3, 1, 2)
    got = torch.nn.functional.conv2d(torch.tensor(x).permute(0, 3, 1, 2), wt, torch.tensor(b), padding=1)
    got = got.permute(0, 2, 3, 1).numpy()
    ref = np.zeros((B, H, W, co))
    for n in range(B):
        for y in range(H):
            for xx in range(W):
                for o in range(co):
                    s = b[o]
                    for dy in (-1, 0, 1):
                        for dx in (-1, 0, 1):
                            yy, xq = y + dy, xx + dx
                            if 0 <= yy < H and 0 <= xq < W:
                                s += w[o, 3 * (dy + 1) + (dx + 1)] @ x[n, yy, xq]
                    ref[n, y, xx, o] = s
    assert np.allclose(got, ref, rtol=1e-12, atol=1e-12)


def _tiny(levels=2, base=2, B=2, H=8, W=8, seed=3):
    rng = np.random.default_rng(seed)
    p = rng.standard_normal(unet.n_params(levels, base)) * 0.3
    x = rng.standard_normal((B, H, W, unet.IN_CH))
    t = rng.standard_normal((B, H, W, unet.OUT_CH))
    return p, x, t


@pytest.mark.parametrize("levels", [1, 2, 3])
def test_gradient_against_finite_differences(levels):
    p, x, t = _tiny(levels=levels)
    loss, g = unet.loss_and_grad(p, x, t, levels, 2, bf16=False)
    rng = np.random.default_rng(4)
    idx = rng.choice(p.size, 25, replace=False)
    h = 1e-6
    for i in idx:
        pp, pm = p.copy(), p.copy()
        pp[i] += h
        pm[i] -= h
        lp = float(((unet.forward(pp, x, levels, 2, bf16=False).numpy() - t) ** 2).mean())
        lm = float(((unet.forward(pm, x, levels, 2, bf16=False).numpy() - t) ** 2).mean())
        fd = (lp - lm) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)), (i, fd, g[i])


def test_bf16_forward_stays_close_to_exact():
    p, x, t = _tiny(levels=3, base=4, H=16, W=16)
    a = unet.forward(p, x, 3, 4, bf16=True).numpy()
    b = unet.forward(p, x, 3, 4, bf16=False).numpy()
    assert np.linalg.norm(a - b) / np.linalg.norm(b) < 3e-2


def test_adam_closed_form_for_constant_gradient():
    # with a constant gradient g the bias-corrected moments are g and g^2 at every step,
    # so each step moves w by lr * g / (|g| + eps)
    w = np.array([1.0, -2.0, 0.5])
    g = np.array([0.3, -4.0, 1e-3])
    m = np.zeros(3)
    v = np.zeros(3)
    lr = 1e-2
    for step in range(1, 6):
        w_new, m, v = unet.adam_step(w, g, m, v, step, lr)
        assert np.allclose(w - w_new, lr * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=1e-15)
        w = w_new


def test_pool_and_upsample_are_adjoint_up_to_four():
    rng = np.random.default_rng(5)
    a = torch.tensor(rng.standard_normal((2, 3, 4, 6)))
    b = torch.tensor(rng.standard_normal((2, 3, 8, 12)))
    up = torch.nn.functional.interpolate(a, scale_factor=2, mode="nearest")
    pool = torch.nn.functional.avg_pool2d(b, 2)
    assert abs(float((up * b).sum()) - 4.0 * float((a * pool).sum())) < 1e-9


def test_pack_inputs_and_targets():
    rng = np.random.default_rng(6)
    chi = rng.standard_normal((2, 4, 5)) + 1j * rng.standard_normal((2, 4, 5))
    e = rng.standard_normal((2, 2, 4, 5)) + 1j * rng.standard_normal((2, 2, 4, 5))
    u = e + 0.5
    x = unet.pack_inputs(chi, e)
    assert x.shape == (2, 4, 5, 8) and np.all(x[..., 6:] == 0)
    assert np.array_equal(x[..., 0], chi.real) and np.array_equal(x[..., 5], e[:, 1].imag)
    tg = unet.pack_targets(u, e)
    assert np.allclose(tg[..., 0], 0.5) and np.allclose(tg[..., 1], 0.0)
