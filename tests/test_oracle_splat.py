"""Pins for the oracle's full-resolution splat and resolve (Sections 3.5-3.6):
an independent NumPy per-cell maximum (np.maximum.at), permutation
invariance, accumulation across calls, and a direct decode of the keys."""
import numpy as np

import synth


def _numpy_keys(region, x, y, z, rgb, tile_slot, n_slots):
    C = region.cell
    res = region.res
    gx = np.floor_divide(x.astype(np.int64) - region.origin_x, C)
    gy = np.floor_divide(y.astype(np.int64) - region.origin_y, C)
    ok = (gx >= 0) & (gy >= 0) & (gx < region.tiles_x * res) & (gy < region.tiles_y * res)
    slot = np.full(x.shape, -1, np.int64)
    slot[ok] = tile_slot[(gy[ok] // res) * region.tiles_x + gx[ok] // res]
    ok &= slot >= 0
    hi = (z.astype(np.int64) & 0xFFFFFFFF) ^ 0x80000000
    rgb = rgb.astype(np.uint64)
    key = (hi.astype(np.uint64) << np.uint64(32)) | ((rgb[:, 0] >> np.uint64(8)) << np.uint64(24)) | \
        ((rgb[:, 1] >> np.uint64(8)) << np.uint64(16)) | ((rgb[:, 2] >> np.uint64(8)) << np.uint64(8)) | np.uint64(0xFF)
    keys = np.zeros(n_slots * res * res, np.uint64)
    cell = (slot * res + gy % res) * res + gx % res
    np.maximum.at(keys, cell[ok], key[ok])
    return keys.reshape(n_slots, res, res), int((~ok).sum())


def _points(seed, region, n):
    rng = np.random.default_rng(seed)
    W = region.tiles_x * region.tile_size
    H = region.tiles_y * region.tile_size
    x = rng.integers(region.origin_x - 5000, region.origin_x + W + 5000, n).astype(np.int32)
    y = rng.integers(region.origin_y - 5000, region.origin_y + H + 5000, n).astype(np.int32)
    z = rng.integers(-2 ** 31, 2 ** 31, n, dtype=np.int64).astype(np.int32)
    z[: n // 2] = rng.integers(-3, 3, n // 2)  # many equal heights -> colour ties
    rgb = rng.integers(0, 65536, (n, 3)).astype(np.uint16)
    return x, y, z, rgb


def test_splat_matches_numpy_max(oracle_lib):
    region = synth.Region(origin_x=-3000, origin_y=1000, tiles_x=3, tiles_y=2, res=8)
    x, y, z, rgb = _points(0, region, 20000)
    tile_slot = np.array([2, -1, 0, 1, 4, 3], np.int32)
    keys, dropped = oracle_lib.splat(region, x, y, z, rgb, tile_slot, 5)
    want, wd = _numpy_keys(region, x, y, z, rgb, tile_slot, 5)
    assert np.array_equal(keys, want)
    assert dropped == wd
    assert dropped > 0


def test_splat_permutation_invariant_and_accumulates(oracle_lib):
    region = synth.Region(tiles_x=2, tiles_y=2, res=16)
    x, y, z, rgb = _points(1, region, 30000)
    ts = np.arange(4, dtype=np.int32)
    k1, _ = oracle_lib.splat(region, x, y, z, rgb, ts, 4)
    p = np.random.default_rng(2).permutation(len(x))
    k2, _ = oracle_lib.splat(region, x[p], y[p], z[p], rgb[p], ts, 4)
    assert np.array_equal(k1, k2)
    h = len(x) // 3
    ka, _ = oracle_lib.splat(region, x[:h], y[:h], z[:h], rgb[:h], ts, 4)
    kb, _ = oracle_lib.splat(region, x[h:], y[h:], z[h:], rgb[h:], ts, 4, keys=ka)
    assert np.array_equal(kb, k1)


def test_resolve_decodes(oracle_lib):
    region = synth.Region(tiles_x=1, tiles_y=1, res=8)
    x, y, z, rgb = _points(3, region, 500)
    ts = np.zeros(1, np.int32)
    keys, _ = oracle_lib.splat(region, x, y, z, rgb, ts, 1)
    tex0 = np.full((1, 8, 8, 4), -7.0, np.float32)
    tex = oracle_lib.resolve(keys, tex0, 0.01, 100.0)
    kf = keys.ravel()
    for c in range(64):
        t = tex.reshape(-1, 4)[c]
        if kf[c] == 0:
            assert np.all(t == -7.0)
            continue
        zr = np.int64(((int(kf[c]) >> 32) ^ 0x80000000)).astype(np.int64)
        zr = zr - (1 << 32) if zr >= (1 << 31) else zr
        assert t[0] == np.float32(np.float64(zr) * 0.01 + 100.0)
        for k, sh in enumerate((24, 16, 8)):
            assert t[1 + k] == np.float32((int(kf[c]) >> sh) & 0xFF) / np.float32(255.0)
    # the winning key belongs to the highest point of its texel
    gx = (x.astype(np.int64)) // 8000
    gy = (y.astype(np.int64)) // 8000
    ok = (gx >= 0) & (gx < 8) & (gy >= 0) & (gy < 8)
    for c in range(64):
        sel = ok & (gy * 8 + gx == c)
        if sel.any():
            zr = ((int(kf[c]) >> 32) ^ 0x80000000)
            zr = zr - (1 << 32) if zr >= (1 << 31) else zr
            assert zr == z[sel].max()
