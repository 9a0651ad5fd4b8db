"""Pins for the oracle's refinement network (Section 3.4) forward and
backward: torch.nn.functional in float64 on the CPU (a library), the zero-head
special case (the Linear baseline of Section 4.2), and FP64 central
differences of the oracle itself."""
import numpy as np
import pytest
import torch
import torch.nn.functional as F

import synth


def _layers(w):
    out = {}
    off = 0
    for name, ci, co in synth.UNET_SHAPES:
        W = torch.from_numpy(w[off:off + co * 9 * ci].reshape(co, 3, 3, ci)).permute(0, 3, 1, 2).contiguous()
        off += co * 9 * ci
        b = torch.from_numpy(w[off:off + co].copy())
        off += co
        out[name] = (W, b)
    return out


def torch_unet(w, x, res, pad):
    """Independent float64 forward with library convolutions (NCHW)."""
    L = _layers(w)
    X = x.permute(0, 3, 1, 2)

    def conv(t, n, relu=True):
        W, b = L[n]
        y = F.conv2d(t, W, b, padding=1)
        return F.relu(y) if relu else y
    a1 = conv(X, "enc1a")
    a2 = conv(a1, "enc1b")
    a3 = conv(F.avg_pool2d(a2, 2), "enc2a")
    a4 = conv(a3, "enc2b")
    a5 = conv(F.avg_pool2d(a4, 2), "bot_a")
    a6 = conv(a5, "bot_b")
    a7 = conv(torch.cat([F.interpolate(a6, scale_factor=2, mode="nearest"), a4], 1), "dec2a")
    a8 = conv(a7, "dec2b")
    a9 = conv(torch.cat([F.interpolate(a8, scale_factor=2, mode="nearest"), a2], 1), "dec1a")
    a10 = conv(a9, "dec1b")
    head = conv(torch.cat([a10, X], 1), "head", relu=False)[:, :, pad:pad + res, pad:pad + res]
    y = X[:, [0, 2, 3, 4], pad:pad + res, pad:pad + res] + head
    return y.permute(0, 2, 3, 1)


def _inputs(n, R, seed):
    rng = np.random.default_rng(seed)
    x = rng.standard_normal((n, R, R, 8)) * 0.1
    x[..., 2:] = rng.random((n, R, R, 6))
    return x


@pytest.mark.parametrize("res,pad,n", [(64, 16, 2), (8, 4, 3), (16, 0, 2)])
def test_forward_matches_torch(oracle_lib, res, pad, n):
    w = synth.unet_weights(1, head_std=0.05, bias_std=0.1)
    x = _inputs(n, res + 2 * pad, 3)
    y = oracle_lib.unet_forward(w, x, res, pad)
    ref = torch_unet(w, torch.from_numpy(x), res, pad).numpy()
    np.testing.assert_allclose(y, ref, rtol=1e-11, atol=1e-12)


def test_zero_head_is_linear_baseline(oracle_lib):
    w = synth.unet_weights(2, bias_std=0.1)
    off = sum(co * 9 * ci + co for _, ci, co in synth.UNET_SHAPES[:-1])
    w[off:] = 0.0
    x = _inputs(2, 96, 4)
    y = oracle_lib.unet_forward(w, x, 64, 16)
    assert np.array_equal(y, x[:, 16:80, 16:80][..., [0, 2, 3, 4]])


def test_backward_matches_autograd(oracle_lib):
    res, pad, n = 16, 8, 2
    w = synth.unet_weights(3, head_std=0.1, bias_std=0.1)
    x = _inputs(n, res + 2 * pad, 5)
    rng = np.random.default_rng(6)
    G = rng.standard_normal((n, res, res, 4))
    gw, gx = oracle_lib.unet_backward(w, x, G, res, pad, want_gx=True)
    wt = torch.from_numpy(w.copy()).requires_grad_(True)
    xt = torch.from_numpy(x.copy()).requires_grad_(True)
    # rebuild the torch graph from the flat weight tensor so autograd reaches it
    L = {}
    off = 0
    for name, ci, co in synth.UNET_SHAPES:
        L[name] = (wt[off:off + co * 9 * ci].view(co, 3, 3, ci).permute(0, 3, 1, 2),
                   wt[off + co * 9 * ci:off + co * 9 * ci + co])
        off += co * 9 * ci + co
    X = xt.permute(0, 3, 1, 2)

    def conv(t, nme, relu=True):
        W, b = L[nme]
        y = F.conv2d(t, W, b, padding=1)
        return F.relu(y) if relu else y
    a2 = conv(conv(X, "enc1a"), "enc1b")
    a4 = conv(conv(F.avg_pool2d(a2, 2), "enc2a"), "enc2b")
    a6 = conv(conv(F.avg_pool2d(a4, 2), "bot_a"), "bot_b")
    a8 = conv(conv(torch.cat([F.interpolate(a6, scale_factor=2), a4], 1), "dec2a"), "dec2b")
    a10 = conv(conv(torch.cat([F.interpolate(a8, scale_factor=2), a2], 1), "dec1a"), "dec1b")
    head = conv(torch.cat([a10, X], 1), "head", relu=False)[:, :, pad:pad + res, pad:pad + res]
    y = (X[:, [0, 2, 3, 4], pad:pad + res, pad:pad + res] + head).permute(0, 2, 3, 1)
    (y * torch.from_numpy(G)).sum().backward()
    np.testing.assert_allclose(gw, wt.grad.numpy(), rtol=1e-9, atol=1e-10)
    np.testing.assert_allclose(gx, xt.grad.numpy(), rtol=1e-9, atol=1e-10)


def test_backward_finite_differences(oracle_lib):
    """Central differences (h = 1e-6) of the probe loss <G, y> at random
    coordinates of every layer and in random directions."""
    res, pad, n = 8, 4, 2
    w = synth.unet_weights(4, head_std=0.1, bias_std=0.1)
    x = _inputs(n, res + 2 * pad, 7)
    rng = np.random.default_rng(8)
    G = rng.standard_normal((n, res, res, 4))
    gw, _ = oracle_lib.unet_backward(w, x, G, res, pad)

    def loss(wv):
        return float((oracle_lib.unet_forward(wv, x, res, pad) * G).sum())
    h = 1e-6
    off = 0
    checked = 0
    for name, ci, co in synth.UNET_SHAPES:
        size = co * 9 * ci + co
        for k in rng.choice(size, 6, replace=False):
            e = np.zeros_like(w)
            e[off + k] = h
            fd = (loss(w + e) - loss(w - e)) / (2 * h)
            assert abs(fd - gw[off + k]) <= 1e-6 * max(1.0, abs(gw[off + k])), (name, k, fd, gw[off + k])
            checked += 1
        off += size
    for _ in range(4):
        d = rng.standard_normal(w.size)
        d /= np.linalg.norm(d)
        fd = (loss(w + h * d) - loss(w - h * d)) / (2 * h)
        assert abs(fd - gw @ d) <= 1e-6 * max(1.0, abs(gw @ d))
    assert checked == 66
