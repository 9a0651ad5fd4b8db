"""Pins for the oracle's ground-truth targets and training losses (Section
3.4, training data and training): hand-derived fixtures, np.add.at /
bincount for the sums, permutation invariance, accumulation across calls,
and finite differences of the losses."""
import math
import os

import numpy as np
import pytest

import synth

HERE = os.path.dirname(os.path.abspath(__file__))


def _rows(name):
    out = []
    with open(os.path.join(HERE, "golden", name)) as f:
        for line in f:
            line = line.split("#")[0].strip()
            if line:
                out.append(line.split())
    return out


def _region2(res=2, tile=2000, tiles_x=1, tiles_y=1, pad=0, ox=0, oy=0):
    return synth.Region(origin_x=ox, origin_y=oy, tile_size=tile, res=res, pad=pad, tiles_x=tiles_x, tiles_y=tiles_y)


def test_golden_mean_target(oracle_lib):
    rows = _rows("mean_target_2x2.txt")
    pts = np.array([[int(v) for v in r[1:]] for r in rows if r[0] == "point"], np.int64)
    x, y, z, rgb = pts[:, 0], pts[:, 1], pts[:, 2], pts[:, 3:6].astype(np.uint16)
    reg = _region2()
    acc, dropped = oracle_lib.splat_mean(reg, x, y, z, rgb, np.zeros(1, np.int32), 1)
    assert dropped == int([r for r in rows if r[0] == "dropped"][0][1])
    for r in rows:
        if r[0] == "sum":
            i, j = int(r[1]), int(r[2])
            assert acc[0, i, j].tolist() == [int(v) for v in r[3:8]], r
    tex = oracle_lib.resolve_mean(acc, 0.01, 0.0)
    for r in rows:
        if r[0] == "tex":
            i, j = int(r[1]), int(r[2])
            want = np.array([float(v) for v in r[3:7]], np.float64).astype(np.float32)
            got = tex[0, i, j]
            if np.isnan(want).all():
                assert np.isnan(got).all()
            else:
                assert np.array_equal(got, want), (r, got)


def _dense(seed, region, n, slots):
    rng = np.random.default_rng(seed)
    W = region.tiles_x * region.tile_size
    Hh = region.tiles_y * region.tile_size
    # a margin outside the region on every side, so some points drop
    x = rng.integers(region.origin_x - 3000, region.origin_x + W + 3000, n)
    y = rng.integers(region.origin_y - 3000, region.origin_y + Hh + 3000, n)
    z = rng.integers(-2_000_000_000, 2_000_000_000, n)
    rgb = rng.integers(0, 65536, (n, 3)).astype(np.uint16)
    return x, y, z, rgb


def test_sums_equal_add_at_and_bincount(oracle_lib):
    reg = _region2(res=8, tile=8000, tiles_x=3, tiles_y=2, ox=-5000, oy=12000)
    slots = np.array([0, -1, 1, 2, 3, -1], np.int32)  # two unmapped tiles
    x, y, z, rgb = _dense(1, reg, 20000, slots)
    acc, dropped = oracle_lib.splat_mean(reg, x, y, z, rgb, slots, 4)
    C = reg.tile_size // reg.res
    gx = np.floor_divide(x - reg.origin_x, C)
    gy = np.floor_divide(y - reg.origin_y, C)
    inside = (gx >= 0) & (gy >= 0) & (gx < reg.tiles_x * reg.res) & (gy < reg.tiles_y * reg.res)
    s = np.full(x.shape, -1)
    s[inside] = slots[(gy[inside] // reg.res) * reg.tiles_x + gx[inside] // reg.res]
    keep = s >= 0
    assert dropped == int((~keep).sum())
    cell = (s[keep] * reg.res + gy[keep] % reg.res) * reg.res + gx[keep] % reg.res
    want = np.zeros((4 * reg.res * reg.res, 5), np.int64)
    np.add.at(want[:, 0], cell, z[keep])
    for c in range(3):
        np.add.at(want[:, 1 + c], cell, rgb[keep, c].astype(np.int64))
    want[:, 4] = np.bincount(cell, minlength=want.shape[0])
    assert np.array_equal(acc.reshape(-1, 5), want)


def test_sums_permutation_invariant_and_accumulate(oracle_lib):
    reg = _region2(res=4, tile=4000, tiles_x=2, tiles_y=2)
    slots = np.arange(4, dtype=np.int32)
    x, y, z, rgb = _dense(2, reg, 5000, slots)
    a, _ = oracle_lib.splat_mean(reg, x, y, z, rgb, slots, 4)
    p = np.random.default_rng(3).permutation(x.size)
    b, _ = oracle_lib.splat_mean(reg, x[p], y[p], z[p], rgb[p], slots, 4)
    assert np.array_equal(a, b)
    h = x.size // 2
    c1, d1 = oracle_lib.splat_mean(reg, x[:h], y[:h], z[:h], rgb[:h], slots, 4)
    c2, d2 = oracle_lib.splat_mean(reg, x[h:], y[h:], z[h:], rgb[h:], slots, 4, acc=c1)
    assert np.array_equal(c2, a)


def test_resolve_mean_of_constant_texel_is_the_value(oracle_lib):
    """k copies of one point average to exactly that point (the division of
    k*z by k is exact in double), so the texture equals the point's own
    height and colour; gaps are NaN in every channel."""
    rng = np.random.default_rng(4)
    acc = np.zeros((50, 5), np.int64)
    zs = rng.integers(-2**31, 2**31, 49)
    cs = rng.integers(0, 65536, (49, 3))
    ks = rng.integers(1, 100000, 49)
    acc[:49, 0] = zs * ks
    acc[:49, 1:4] = cs * ks[:, None]
    acc[:49, 4] = ks
    tex = oracle_lib.resolve_mean(acc, 0.01, 123.0)
    assert np.array_equal(tex[:49, 0], (zs * 0.01 + 123.0).astype(np.float32))
    assert np.array_equal(tex[:49, 1:], (cs / 65535.0).astype(np.float32))
    assert np.isnan(tex[49]).all()


def _golden_loss(oracle_lib, kind):
    rows = _rows("target_loss_2x2.txt")
    y = np.zeros((1, 2, 2, 4), np.float32)
    t = np.zeros((1, 2, 2, 4), np.float32)
    for r in rows:
        if r[0] == "texel":
            i, j = int(r[1]), int(r[2])
            y[0, i, j] = [float(v) for v in r[3:7]]
            t[0, i, j] = [float(v) for v in r[7:11]]
    reg = _region2()
    assert (reg.tile_size // 2 + reg.pad * reg.cell) * reg.scale_xy == 10.0
    (L, Lh, Lc), g = oracle_lib.target_loss(y, t, np.zeros(1), reg, kind)
    name = "mse" if kind == oracle_lib.LOSS_CLIPPED_MSE else "l1"
    want = [float(v) for v in [r for r in rows if r[0] == name][0][1:4]]
    np.testing.assert_allclose([L, Lh, Lc], want, rtol=1e-15, atol=0)
    for r in rows:
        if r[0] == name + "_grad":
            i, j = int(r[1]), int(r[2])
            np.testing.assert_allclose(g[0, i, j], [float(v) for v in r[3:7]], rtol=1e-15, atol=0)


def test_golden_clipped_mse(oracle_lib):
    _golden_loss(oracle_lib, oracle_lib.LOSS_CLIPPED_MSE)


def test_golden_l1(oracle_lib):
    _golden_loss(oracle_lib, oracle_lib.LOSS_L1)


def _random_loss_case(seed, n=3, res=8, gap_frac=0.2):
    rng = np.random.default_rng(seed)
    y = (rng.standard_normal((n, res, res, 4)) * 0.6).astype(np.float32)
    t = (rng.standard_normal((n, res, res, 4)) * 0.5).astype(np.float32)
    cz = rng.standard_normal(n) * 20.0
    reg = _region2(res=res, tile=res * 1000, pad=2)
    r_m = (reg.tile_size // 2 + reg.pad * reg.cell) * reg.scale_xy
    t[..., 0] = (cz[:, None, None] + r_m * t[..., 0]).astype(np.float32)  # target heights in metres
    gaps = rng.random((n, res, res)) < gap_frac
    t[gaps] = np.nan
    return y, t, cz, reg


@pytest.mark.parametrize("kind", [0, 1])
def test_loss_gradient_finite_differences(oracle_lib, kind):
    """Central differences of L in float64 at every element of a small case
    (y perturbed in float64 through the loss's own evaluation is not possible
    with a float32 interface, so the perturbation is a power of two that keeps
    y exact in float32 and away from the clip and sign kinks)."""
    y, t, cz, reg = _random_loss_case(5, n=1, res=4)
    (L, _, _), g = oracle_lib.target_loss(y, t, cz, reg, kind)
    h = 2.0 ** -12
    r_m = (reg.tile_size // 2 + reg.pad * reg.cell) * reg.scale_xy
    tn = t.astype(np.float64)
    tn[..., 0] = (tn[..., 0] - cz[:, None, None]) / r_m
    d = y.astype(np.float64) - tn
    checked = 0
    for idx in np.ndindex(y.shape):
        if np.isnan(tn[idx]):
            assert g[idx] == 0.0
            continue
        dv = d[idx]
        if kind == 0 and abs(abs(dv) - 1.0) < 2 * h:
            continue
        if kind == 1 and abs(dv) < 2 * h:
            continue
        yp, ym = y.copy(), y.copy()
        yp[idx] += np.float32(h)
        ym[idx] -= np.float32(h)
        (Lp, _, _), _ = oracle_lib.target_loss(yp, t, cz, reg, kind)
        (Lm, _, _), _ = oracle_lib.target_loss(ym, t, cz, reg, kind)
        fd = (Lp - Lm) / (float(yp[idx]) - float(ym[idx]))
        assert abs(fd - g[idx]) <= 1e-9 * max(1.0, abs(g[idx])) + 1e-12, (idx, fd, g[idx])
        checked += 1
    assert checked > 40


def test_loss_special_cases(oracle_lib):
    y, t, cz, reg = _random_loss_case(6)
    # every target a gap: zero loss and gradient
    (L, Lh, Lc), g = oracle_lib.target_loss(y, np.full_like(t, np.nan), cz, reg, 0)
    assert L == Lh == Lc == 0.0 and not g.any()
    # the output equal to the normalised target: zero loss for both kinds
    # (dyadic outputs and c_z = 0, so the target's normalisation is exact)
    r_m = (reg.tile_size // 2 + reg.pad * reg.cell) * reg.scale_xy
    y3 = (np.round(y * 64) / 64).astype(np.float32)
    t3 = y3.copy()
    t3[..., 0] = (r_m * y3[..., 0].astype(np.float64)).astype(np.float32)
    for kind in (0, 1):
        (L, _, _), g = oracle_lib.target_loss(y3, t3, np.zeros(y.shape[0]), reg, kind)
        assert L == 0.0 and not g.any()
    # errors all beyond 1 in magnitude: the clipped MSE is exactly 1 per
    # non-gap element, with zero gradient
    big = y.copy()
    big[..., 0] = np.float32(1e3)
    big[..., 1:] = np.float32(-1e3)
    (L, Lh, Lc), g = oracle_lib.target_loss(big, t, cz, reg, 0)
    valid = ~np.isnan(t)
    assert math.isclose(Lh, valid[..., 0].mean(), rel_tol=1e-15)
    assert math.isclose(Lc, valid[..., 1:].mean(), rel_tol=1e-15)
    assert not g.any()
    # gap elements count in the denominators: halving the valid elements of a
    # case with every error the same halves the loss
    y4 = np.zeros((1, 4, 4, 4), np.float32)
    t4 = np.full((1, 4, 4, 4), 0.5, np.float32)
    r4 = _region2(res=4, tile=4000)
    t4[..., 0] = np.float32(-0.5 * (r4.tile_size // 2) * r4.scale_xy)
    (La, _, _), _ = oracle_lib.target_loss(y4, t4, np.zeros(1), r4, 0)
    t4[0, :2] = np.nan
    (Lb, _, _), _ = oracle_lib.target_loss(y4, t4, np.zeros(1), r4, 0)
    assert La == 0.25 and Lb == 0.125
