"""Pins for the oracle's version of the paper's refinement network (Section
3.4, architecture paragraph): an independent float64 forward built from
torch.nn.functional layers (conv2d, avg_pool2d, interpolate, linear) on the
CPU, the zero final layer giving the Linear baseline exactly, the flatten
order of the fully connected layers, and the parameter count (about 2.5 M,
as the paper states)."""
import numpy as np
import pytest
import torch
import torch.nn.functional as F

import synth


def torch_pnet(w, x, res, pad):
    R = res + 2 * pad
    layers = synth.pnet_layers(R)
    P, off = {}, 0
    for name, kind, ci, co in layers:
        if kind == "conv":
            W = torch.from_numpy(w[off:off + co * 9 * ci].reshape(co, 3, 3, ci)).permute(0, 3, 1, 2).contiguous()
            off += co * 9 * ci
        else:
            W = torch.from_numpy(w[off:off + co * ci].reshape(co, ci).copy())
            off += co * ci
        P[name] = (W, torch.from_numpy(w[off:off + co].copy()))
        off += co
    X = torch.from_numpy(x).permute(0, 3, 1, 2)  # NCHW

    def conv(t, n, relu=True):
        y = F.conv2d(t, *P[n], padding=1)
        return F.relu(y) if relu else y

    feats = []
    for nm, chans in (("hlin", [0]), ("hnn", [1]), ("rgblin", [2, 3, 4]), ("rgbnn", [5, 6, 7])):
        e = X[:, chans]
        for k in range(4):
            e = F.avg_pool2d(conv(e, f"enc_{nm}{k + 1}"), 2)
        feats.append(e.permute(0, 2, 3, 1).reshape(e.shape[0], -1))  # (row, column, channel) order
    zh = F.relu(F.linear(torch.cat([feats[0], feats[1]], 1), *P["fc1_h"]))
    zc = F.relu(F.linear(torch.cat([feats[2], feats[3]], 1), *P["fc1_c"]))
    z = torch.cat([zh, zc], 1)
    dec = []
    for k in ("h", "t"):
        d = F.relu(F.linear(z, *P[f"fc2_{k}"])).reshape(-1, R // 16, R // 16, 32).permute(0, 3, 1, 2)
        for j in range(4):
            d = conv(F.interpolate(d, scale_factor=2, mode="nearest"), f"dec_{k}{j + 1}")
        dec.append(d)
    S = torch.cat(dec + [X], 1)
    f = conv(conv(S, "fin1"), "fin2")
    f3 = conv(f, "fin3", relu=False)[:, :, pad:pad + res, pad:pad + res]
    y = X[:, [0, 2, 3, 4], pad:pad + res, pad:pad + res] + f3
    return y.permute(0, 2, 3, 1).numpy()


def _inputs(n, R, seed):
    rng = np.random.default_rng(seed)
    x = rng.standard_normal((n, R, R, 8)) * 0.1
    x[..., 2:] = rng.random((n, R, R, 6))
    return x


def test_parameter_count():
    assert synth.pnet_weights(0).size == 2_528_708
    # "in total 2.5 M learnable parameters"
    assert abs(2_528_708 - 2.5e6) / 2.5e6 < 0.02


@pytest.mark.parametrize("res,pad,n", [(64, 16, 2), (64, 0, 1), (16, 8, 3)])
def test_forward_matches_torch(oracle_lib, res, pad, n):
    R = res + 2 * pad
    w = synth.pnet_weights(1, R=R, final_std=0.05, bias_std=0.05)
    assert w.size == oracle_lib.pnet_num_params(R)
    x = _inputs(n, R, 3)
    y = oracle_lib.pnet_forward(w, x, res, pad)
    ref = torch_pnet(w, x, res, pad)
    np.testing.assert_allclose(y, ref, rtol=1e-10, atol=1e-12)
    # the network is not trivially the residual
    assert np.abs(y - x[:, pad:pad + res, pad:pad + res][..., [0, 2, 3, 4]]).max() > 1e-3


def test_zero_final_layer_is_linear_baseline(oracle_lib):
    w = synth.pnet_weights(2, bias_std=0.1)
    n_final = 4 * 9 * 32 + 4
    w[-n_final:] = 0.0
    x = _inputs(2, 96, 4)
    y = oracle_lib.pnet_forward(w, x, 64, 16)
    assert np.array_equal(y, x[:, 16:80, 16:80][..., [0, 2, 3, 4]])


def test_inputs_reach_through_their_own_encoders(oracle_lib):
    """Changing only the NN height input changes the output only through the
    h_nn encoder and the skip: with that encoder's weights zero and the
    skip's weights on channel 1 zero, the output ignores channel 1."""
    R = 32
    w = synth.pnet_weights(3, R=R, final_std=0.05, bias_std=0.05)
    layers = synth.pnet_layers(R)
    off = 0
    for name, kind, ci, co in layers:
        size = synth.pnet_layer_size(kind, ci, co)
        if name.startswith("enc_hnn"):
            w[off:off + size] = 0.0
        if name == "fin1":
            W = w[off:off + co * 9 * ci].reshape(co, 3, 3, ci)
            W[..., 32 + 1] = 0.0  # skip channel 1 = x channel 1 (h_nn)
        off += size
    x = _inputs(1, R, 5)
    y0 = oracle_lib.pnet_forward(w, x, 16, 8)
    x2 = x.copy()
    x2[..., 1] += np.random.default_rng(6).standard_normal((1, R, R))
    y1 = oracle_lib.pnet_forward(w, x2, 16, 8)
    assert np.array_equal(y0, y1)
