"""Learned warm start: plain CPU reference of the U-Net the library trains.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Not part of the paper.  The GMRES initial guess x0 of Section 4 is free; this
network proposes one, and restarted GMRES on the FP64 true residual still
decides every solution, so a poor guess costs iterations, never accuracy.

Network (levels L, base width C; input 8 channels, output 4):
  encoder level l = 0..L-1: two 3x3 convolutions (zero padding 1) with ReLU,
    widths C 2^l; after levels 0..L-2 a 2x2 average pool;
  decoder level l = L-2..0: nearest-neighbour 2x upsampling of the level below,
    channel concatenation [upsampled, encoder output of level l], two 3x3
    convolutions with ReLU, widths C 2^l;
  head: a 1x1 convolution to 4 channels, no activation.
Input channels: Re chi, Im chi, Re E1_in, Im E1_in, Re E2_in, Im E2_in, 0, 0.
Output channels: Re, Im of E1 - E1_in and E2 - E2_in (the scattered part).

Parameter vector (float32 in the library): layer by layer in the order above,
the weights W[co][t][ci] (t = 3 (dy + 1) + (dx + 1) for the tap that multiplies
the input at (y + dy, x + dx); a 1x1 layer has the single tap t = 0), then the
bias[co].

Numerics mirrored from the library: convolution operands are bfloat16 (the
weights and every stored activation are rounded to bfloat16, round to nearest
even from float32), sums are exact here (float64) and float32 there; the
gradient entering each convolution's backward pass is rounded to bfloat16;
the loss, its gradient, the bias gradients and the optimiser run in float32
there and float64 here.  The rounding points are identity maps for the
gradient (straight-through) except where stated.

Pinned by tests/test_oracle_unet.py: bfloat16 rounding against its bit-level
definition, one convolution against explicit loops, whole-network gradients
against central finite differences (rounding off), Adam against its closed
form for a constant gradient, and the pool/upsample pair against adjointness.
"""

from __future__ import annotations

import math

import numpy as np
import torch
import torch.nn.functional as F

IN_CH = 8
OUT_CH = 4


def layer_specs(levels: int, base: int) -> list[tuple[str, int, int, int]]:
    """(name, c_in, c_out, taps) of every convolution in parameter order."""
    if levels < 1 or base < 1:
        raise ValueError("levels and base must be >= 1")
    width = [base * 2 ** l for l in range(levels)]
    specs = []
    for l in range(levels):
        cin = IN_CH if l == 0 else width[l - 1]
        specs.append((f"enc{l}a", cin, width[l], 9))
        specs.append((f"enc{l}b", width[l], width[l], 9))
    for l in range(levels - 2, -1, -1):
        specs.append((f"dec{l}a", width[l + 1] + width[l], width[l], 9))
        specs.append((f"dec{l}b", width[l], width[l], 9))
    specs.append(("head", width[0], OUT_CH, 1))
    return specs


def n_params(levels: int, base: int) -> int:
    return sum(co * t * ci + co for _, ci, co, t in layer_specs(levels, base))


def bf16_round(a) -> np.ndarray:
    """Round to the nearest bfloat16 (ties to even) through float32, as float64 values."""
    t = torch.as_tensor(np.asarray(a, dtype=np.float64)).to(torch.float32)
    return t.to(torch.bfloat16).to(torch.float64).numpy()


def _bf16(t: torch.Tensor) -> torch.Tensor:
    return t.to(torch.float32).to(torch.bfloat16).to(t.dtype)


class _StoreRound(torch.autograd.Function):
    """Forward: round to bfloat16 (a stored operand); backward: identity."""

    @staticmethod
    def forward(ctx, x):
        return _bf16(x)

    @staticmethod
    def backward(ctx, g):
        return g


class _GradRound(torch.autograd.Function):
    """Forward: identity; backward: round the incoming gradient to bfloat16."""

    @staticmethod
    def forward(ctx, x):
        return x.clone()

    @staticmethod
    def backward(ctx, g):
        return _bf16(g)


def _unpack(flat: torch.Tensor, levels: int, base: int):
    layers, off = [], 0
    for name, ci, co, t in layer_specs(levels, base):
        w = flat[off:off + co * t * ci].reshape(co, t, ci)
        off += co * t * ci
        b = flat[off:off + co]
        off += co
        k = 3 if t == 9 else 1
        layers.append((name, w.reshape(co, k, k, ci).permute(0, 3, 1, 2), b))
    if off != flat.numel():
        raise ValueError(f"parameter vector has {flat.numel()} entries, the network {off}")
    return layers


def forward(params, x, levels: int, base: int, bf16: bool = True) -> torch.Tensor:
    """Network output [B, H, W, 4] (float64 torch tensor, differentiable in params when
    params is a tensor that requires grad).  x: [B, H, W, 8]."""
    flat = params if isinstance(params, torch.Tensor) else torch.as_tensor(np.asarray(params, np.float64))
    flat = flat.to(torch.float64)
    xs = torch.as_tensor(np.asarray(x, np.float64)) if not isinstance(x, torch.Tensor) else x.to(torch.float64)
    if xs.shape[-1] != IN_CH:
        raise ValueError("x must be [B, H, W, 8]")
    div = 2 ** (levels - 1)
    if xs.shape[1] % div or xs.shape[2] % div:
        raise ValueError(f"H and W must be multiples of {div}")
    store = _StoreRound.apply if bf16 else (lambda v: v)
    gradr = _GradRound.apply if bf16 else (lambda v: v)
    layers = iter(_unpack(flat, levels, base))

    def conv(h, relu):
        _, w, b = next(layers)
        pad = 1 if w.shape[-1] == 3 else 0
        z = F.conv2d(h, store(w), bias=b, padding=pad)
        z = gradr(z)
        return store(torch.relu(z)) if relu else z

    h = store(xs.permute(0, 3, 1, 2))
    skips = []
    for l in range(levels):
        h = conv(h, True)
        h = conv(h, True)
        if l < levels - 1:
            skips.append(h)
            h = store(F.avg_pool2d(h, 2))
    for l in range(levels - 2, -1, -1):
        u = F.interpolate(h, scale_factor=2, mode="nearest")
        h = torch.cat([u, skips[l]], dim=1)
        h = conv(h, True)
        h = conv(h, True)
    out = conv(h, False)
    return out.permute(0, 2, 3, 1)


def loss_and_grad(params, x, target, levels: int, base: int, bf16: bool = True):
    """Mean-square loss over all outputs and its gradient in the parameter layout."""
    flat = torch.tensor(np.asarray(params, np.float64), requires_grad=True)
    out = forward(flat, x, levels, base, bf16)
    tgt = torch.as_tensor(np.asarray(target, np.float64))
    loss = ((out - tgt) ** 2).mean()
    loss.backward()
    return float(loss.detach()), flat.grad.numpy().copy()


def adam_step(w, g, m, v, step: int, lr: float, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8):
    """One Adam update (Kingma & Ba 2015, Algorithm 1) with bias correction.
    Returns (w, m, v); step counts from 1."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mh = m / (1.0 - beta1 ** step)
    vh = v / (1.0 - beta2 ** step)
    return w - lr * mh / (np.sqrt(vh) + eps), m, v


def pack_inputs(chi: np.ndarray, e_in: np.ndarray) -> np.ndarray:
    """Network input [B, H, W, 8] from chi [B, ny, nx] and E_in [B, 2, ny, nx] (complex)."""
    chi = np.asarray(chi, np.complex128)
    e = np.asarray(e_in, np.complex128)
    z = np.zeros(chi.shape, np.float64)
    ch = [chi.real, chi.imag, e[:, 0].real, e[:, 0].imag, e[:, 1].real, e[:, 1].imag, z, z]
    return np.stack(ch, axis=-1)


def pack_targets(e_tot: np.ndarray, e_in: np.ndarray) -> np.ndarray:
    """Training target [B, H, W, 4]: the scattered field E - E_in, real and imaginary parts."""
    d = np.asarray(e_tot, np.complex128) - np.asarray(e_in, np.complex128)
    return np.stack([d[:, 0].real, d[:, 0].imag, d[:, 1].real, d[:, 1].imag], axis=-1)


def he_scale(fan_in: int) -> float:
    return math.sqrt(2.0 / fan_in)
