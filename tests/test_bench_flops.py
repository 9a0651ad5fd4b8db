"""The training FLOP count the benchmark reports as unavoidable
(`bench.train_flops`), pinned to a brute-force propagation of where each
gradient of the U-Net can be nonzero: boolean planes dilated by every 3x3
conv, split and summed at the concatenations, upsampled and pooled like
the network's data, starting from the res x res crop of the output."""
import importlib.util
import os

import numpy as np
import pytest

import synth

_spec = importlib.util.spec_from_file_location(
    "bench_module", os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "bench.py"))
bench = importlib.util.module_from_spec(_spec)
_spec.loader.exec_module(bench)


def _dilate(m):
    out = m.copy()
    out[1:, :] |= m[:-1, :]
    out[:-1, :] |= m[1:, :]
    m2 = out.copy()
    out[:, 1:] |= m2[:, :-1]
    out[:, :-1] |= m2[:, 1:]
    return out


def _down(m):  # a low-resolution pixel touches any of its 2 x 2 block
    h = m.shape[0] // 2
    return m[:2 * h, :2 * h].reshape(h, 2, h, 2).any(axis=(1, 3))


def _up(m):
    return np.repeat(np.repeat(m, 2, axis=0), 2, axis=1)


def _brute(res, pad, grad_x):
    R = res + 2 * pad
    S = synth.UNET_SHAPES
    flops = bench.unet_flops(res, pad, inference=True)

    def layer(l, out_mask, in_channels=None):
        nonlocal flops
        _, ci, co = S[l]
        flops += 2 * int(out_mask.sum()) * co * 9 * ci
        in_mask = _dilate(out_mask)
        if in_channels is not None:
            flops += 2 * int(in_mask.sum()) * in_channels * 9 * co
        return in_mask

    crop = np.zeros((R, R), bool)
    crop[pad:pad + res, pad:pad + res] = True
    d10 = layer(10, crop, 24 if grad_x else 16)   # head: input = (A10, x)
    d9 = layer(9, d10, 16)                        # dec1b
    du1 = layer(8, d9, 48)                        # dec1a: input = (up(A8), A2)
    d8 = _down(du1)
    d7 = layer(7, d8, 32)                         # dec2b
    du2 = layer(6, d7, 96)                        # dec2a: input = (up(A6), A4)
    d6 = _down(du2)
    d5 = layer(5, d6, 64)                         # bot_b
    dp2 = layer(4, d5, 32)                        # bot_a, input = pool(A4)
    d4 = du2 | _up(dp2)                           # skip + pool adjoint
    d3 = layer(3, d4, 32)                         # enc2b
    dp1 = layer(2, d3, 16)                        # enc2a, input = pool(A2)
    d2 = du1 | _up(dp1)
    d1 = layer(1, d2, 16)                         # enc1b
    layer(0, d1, 8 if grad_x else None)           # enc1a: input x
    return flops


@pytest.mark.parametrize("res,pad", [(64, 16), (64, 4), (64, 0), (32, 16), (48, 8)])
@pytest.mark.parametrize("grad_x", [False, True])
def test_train_flops_matches_brute_force(res, pad, grad_x):
    assert bench.train_flops(res, pad, grad_x) == pytest.approx(_brute(res, pad, grad_x), rel=0, abs=0.5)


def test_train_flops_below_whole_planes():
    whole = 3 * bench.unet_flops(64, 16, inference=False)
    assert bench.train_flops(64, 16) < whole
    # with no padding nothing is saved except the network input's gradient
    # and the head input skip's 8 channels
    R = 64
    skip = 2 * R * R * 16 * 9 * 8 + 2 * R * R * 8 * 9 * 4
    assert bench.train_flops(64, 0, grad_x=False) == pytest.approx(3 * bench.unet_flops(64, 0, inference=False) - skip)


def test_binning_memberships_match_the_oracle_binning():
    """The binning figure's window-membership count (8 B read per point, 4 B
    written per membership) equals what the oracle's binning produces."""
    import oracle

    w = synth.batch_tiles(seed=2, tiles_x=6, tiles_y=5)
    x, y, _, _ = w.points.numpy()
    tiles = np.arange(w.region.tiles_x * w.region.tiles_y, dtype=np.int32)
    _, idx = oracle.bin_points(w.region, x, y, tiles)
    r = bench.binning_rate(w.region, w.points.x, w.points.y, {"bin_count": 0.01, "bin_scan": 0.01, "bin_scatter": 0.01})
    assert r["memberships"] == len(idx)
    assert r["points"] == len(x)
