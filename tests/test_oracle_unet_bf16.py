"""Pins of the FP64 reference of the BF16 network form: with rounding off it
is the C oracle's network and backward; its rounding is round-to-nearest-even
on hand-picked ties; a zero head reproduces the residual exactly."""
import numpy as np

import oracle
from oracle import unet_bf16 as U
import synth
import torch


def _case(n=2, seed=3):
    rng = np.random.default_rng(seed)
    x = rng.standard_normal((n, 32, 32, 8)) * 0.1
    w = synth.unet_weights(1, head_std=0.05, bias_std=0.05)
    return w, x


def test_unrounded_forward_equals_c_oracle():
    w, x = _case()
    y = U.forward(w, x, 24, 4, rounding=False)
    y_ref = oracle.unet_forward(w, x, 24, 4)
    assert np.abs(y - y_ref).max() <= 1e-12 * max(1.0, np.abs(y_ref).max())


def test_unrounded_backward_equals_c_oracle():
    w, x = _case()
    dy = np.random.default_rng(5).standard_normal((2, 24, 24, 4))
    gw, gx = U.backward(w, x, dy, 24, 4, rounding=False)
    gw_ref, gx_ref = oracle.unet_backward(w, x, dy, 24, 4, want_gx=True)
    assert np.linalg.norm(gw - gw_ref) <= 1e-10 * np.linalg.norm(gw_ref)
    assert np.linalg.norm(gx - gx_ref) <= 1e-10 * np.linalg.norm(gx_ref)


def test_bf16_round_nearest_even_ties():
    one = 1.0
    v = torch.tensor([one + 2.0 ** -8, one + 3 * 2.0 ** -8, one + 2.0 ** -8 + 2.0 ** -20, -(one + 2.0 ** -8),
                      3.0e-39, 65504.0 + 16.0], dtype=torch.float64)
    r = U.bf16_round(v).numpy()
    # halfway cases go to the even mantissa; just above halfway goes up
    assert r[0] == 1.0 and r[1] == one + 2.0 ** -6 and r[2] == one + 2.0 ** -7 and r[3] == -1.0
    assert r[4] > 0  # BF16 keeps FP32's exponent range (subnormals included)
    assert r[5] == 65536.0


def test_zero_head_gives_the_residual_exactly():
    w, x = _case()
    off = sum(co * 9 * ci + co for ci, co in U.LAYERS[:-1])
    w = w.copy()
    w[off:] = 0
    y = U.forward(w, x, 24, 4, rounding=True)
    assert np.array_equal(y, x[:, 4:28, 4:28][..., [0, 2, 3, 4]])


def test_rounding_changes_the_result_by_bf16_amounts():
    w, x = _case()
    y0 = U.forward(w, x, 24, 4, rounding=False)
    y1 = U.forward(w, x, 24, 4, rounding=True)
    d = np.abs(y1 - y0).max() / np.abs(y0).max()
    assert 1e-5 < d < 5e-2


def test_fp32_accumulation_unrounded_close_to_c_oracle():
    w, x = _case()
    y = U.forward(w, x, 24, 4, rounding=False, accum=torch.float32)
    y_ref = oracle.unet_forward(w, x, 24, 4)
    assert np.abs(y - y_ref).max() <= 1e-5 * max(1.0, np.abs(y_ref).max())


def test_all_active_weights_keep_every_deep_unit_active():
    w, x = _case()
    wa = U.all_active_weights(w)
    params = U._params(wa, False)
    assert all(bool((W >= 0).all()) and bool((b > 0).all()) for W, b in params)
    y = U.forward(wa, x, 24, 4, rounding=True)
    assert np.isfinite(y).all() and np.abs(y).max() < 1e3
