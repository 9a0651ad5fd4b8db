"""FP64 reference of the refinement network's BF16 form (TEST INFRASTRUCTURE
ONLY: the test-suite and the benchmark's CPU-baseline leg call it; the product
path never does).

The network is the one of ora_unet.c (the configured 3-level U-Net of Section
3.4: eleven 3x3 convs with zero same-padding, ReLU, 2x2 average pooling,
nearest x2 upsampling, skip concatenation, input-skip head on the crop and
the residual onto the linear reconstruction), evaluated here in FP64 with
PyTorch CPU convolutions, plus explicit round-to-nearest-even to BF16 at the
points where the BF16 form stores or feeds BF16 values:

  forward   weights; the network input where a conv reads it; every hidden
            activation after bias and ReLU; every pooled activation.  The
            head output, bias additions and the residual stay unrounded.
  backward  the gradient at every conv output after the ReLU mask (the
            operand of both the input-gradient and the weight-gradient
            products); gradients between convs stay unrounded.

With rounding switched off this is the plain FP64 network and backward, which
the tests pin against the C oracle.  The BF16 form takes its ReLU masks from
rounded activations, so its gradient differs from the exact one wherever a
pre-activation lies within a rounding step of zero; this reference takes the
same decisions.
"""
from __future__ import annotations

import numpy as np
import torch
import torch.nn.functional as F

# (cin, cout) per layer: enc1a enc1b enc2a enc2b bot_a bot_b dec2a dec2b dec1a dec1b head
LAYERS = [(8, 16), (16, 16), (16, 32), (32, 32), (32, 64), (64, 64), (96, 32), (32, 32), (48, 16), (16, 16),
          (24, 4)]


def bf16_round(t: torch.Tensor) -> torch.Tensor:
    """Round to BF16 through FP32 (round to nearest even); same dtype back."""
    return t.to(torch.float32).to(torch.bfloat16).to(t.dtype)


class _RoundValue(torch.autograd.Function):
    """Value rounded to BF16; gradient passed unchanged."""

    @staticmethod
    def forward(ctx, t):
        return bf16_round(t)

    @staticmethod
    def backward(ctx, g):
        return g


class _RoundGrad(torch.autograd.Function):
    """Value passed unchanged; gradient rounded to BF16."""

    @staticmethod
    def forward(ctx, t):
        return t.clone()

    @staticmethod
    def backward(ctx, g):
        return bf16_round(g)


def _params(w: np.ndarray, rounding: bool, dtype=torch.float64):
    """Flat layout per layer: W[cout][3][3][cin] then b[cout]."""
    out, off = [], 0
    for ci, co in LAYERS:
        W = torch.from_numpy(np.asarray(w[off:off + co * 9 * ci], np.float64).reshape(co, 3, 3, ci).copy())
        off += co * 9 * ci
        b = torch.from_numpy(np.asarray(w[off:off + co], np.float64).copy())
        off += co
        W = W.permute(0, 3, 1, 2).contiguous()  # [cout][cin][ky][kx]
        if rounding:
            W = bf16_round(W)
        out.append((W.to(dtype).requires_grad_(True), b.to(dtype).requires_grad_(True)))
    return out


def _network(params, x, res: int, pad: int, rounding: bool):
    """x: [n][8][R][R] (requires grad) -> y [n][4][res][res]."""
    rv = _RoundValue.apply if rounding else (lambda t: t)
    rg = _RoundGrad.apply if rounding else (lambda t: t)

    def conv(inp, l, relu=True):
        W, b = params[l]
        z = rg(F.conv2d(inp, W, b, padding=1))
        return rv(F.relu(z)) if relu else z

    def pool(t):
        return rv(F.avg_pool2d(t, 2))

    def up(t):
        return F.interpolate(t, scale_factor=2, mode="nearest")

    xin = rv(x)
    a1 = conv(xin, 0)
    a2 = conv(a1, 1)
    a3 = conv(pool(a2), 2)
    a4 = conv(a3, 3)
    a5 = conv(pool(a4), 4)
    a6 = conv(a5, 5)
    a7 = conv(torch.cat([up(a6), a4], 1), 6)
    a8 = conv(a7, 7)
    a9 = conv(torch.cat([up(a8), a2], 1), 8)
    a10 = conv(a9, 9)
    head = conv(torch.cat([a10, xin], 1), 10, relu=False)[:, :, pad:pad + res, pad:pad + res]
    lin = x[:, [0, 2, 3, 4], pad:pad + res, pad:pad + res]
    return lin + head


# `accum` is the arithmetic between rounding points: FP64 (the reference) or
# FP32 (another valid accumulation order, as on the matrix cores).  Rounding
# ties decided differently by the two propagate through the layers; their
# distance measures how far two correct evaluations of the BF16 form can be.
def forward(w, x, res: int, pad: int, rounding: bool = True, accum=torch.float64) -> np.ndarray:
    """x [n][R][R][8] -> y [n][res][res][4] (FP64 array)."""
    params = _params(w, rounding, accum)
    xt = torch.from_numpy(np.asarray(x, np.float64)).to(accum).permute(0, 3, 1, 2).contiguous()
    with torch.no_grad():
        y = _network(params, xt, res, pad, rounding)
    return y.permute(0, 2, 3, 1).double().numpy().copy()


def backward(w, x, dy, res: int, pad: int, rounding: bool = True, accum=torch.float64):
    """Gradient of sum(dy * y): returns (gw [P] in the flat layout, gx [n][R][R][8])."""
    params = _params(w, rounding, accum)
    xt = torch.from_numpy(np.asarray(x, np.float64)).to(accum).permute(0, 3, 1, 2).contiguous().requires_grad_(True)
    y = _network(params, xt, res, pad, rounding)
    g = torch.from_numpy(np.asarray(dy, np.float64)).to(accum).permute(0, 3, 1, 2)
    (y * g).sum().backward()
    parts = []
    for W, b in params:
        parts.append(W.grad.permute(0, 2, 3, 1).reshape(-1))
        parts.append(b.grad.reshape(-1))
    gw = torch.cat(parts).double().numpy().copy()
    return gw, xt.grad.permute(0, 2, 3, 1).double().numpy().copy()


def all_active_weights(w: np.ndarray, bias: float = 0.05) -> np.ndarray:
    """Non-negative weights scaled to keep activations of order one, and
    positive biases: from the second conv on every unit is active, so no
    rounding difference can flip a ReLU mask (a test configuration)."""
    w = np.array(w, np.float64)
    off = 0
    for ci, co in LAYERS:
        n = co * 9 * ci
        W = np.abs(w[off:off + n])
        w[off:off + n] = W / max(W.reshape(co, -1).sum(1).mean(), 1e-30)
        off += n
        w[off:off + co] = bias
        off += co
    return w
