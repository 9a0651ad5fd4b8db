"""Pins for the oracle's point rasteriser (Section 3.6, points): a
hand-derived fixture, an exact pixel mapping checked by integer brute force,
rays through the camera (the nearest point wins), permutation invariance,
accumulation across calls and culling."""
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
EMPTY = np.iinfo(np.uint64).max
PINHOLE = np.array([[1, 0, 0, 0], [0, 1, 0, 0], [0, 0, 0, 0], [0, 0, 1, 0]], np.float64)
S = 1.0 / 128.0  # a power of two: positions are exact in double


def _rows(name):
    out = []
    with open(os.path.join(HERE, "golden", name)) as f:
        for line in f:
            line = line.split("#")[0].strip()
            if line:
                out.append(line.split())
    return out


def test_golden_raster(oracle_lib):
    rows = _rows("raster_points.txt")
    pts = np.array([[int(v) for v in r[1:]] for r in rows if r[0] == "point"], np.int64)
    fb, drawn = oracle_lib.raster(PINHOLE, (0, 0), S, S, 0.0, 4, 4, pts[:, 0], pts[:, 1], pts[:, 2],
                                  pts[:, 3:6].astype(np.uint16))
    assert drawn == int([r for r in rows if r[0] == "drawn"][0][1])
    want = np.full((4, 4), EMPTY, np.uint64)
    for r in rows:
        if r[0] == "key":
            want[int(r[1]), int(r[2])] = np.uint64(int(r[3], 16))
    assert np.array_equal(fb, want)
    rgba = oracle_lib.raster_resolve(fb)
    want_rgba = np.zeros((4, 4), np.uint32)
    for r in rows:
        if r[0] == "rgba":
            want_rgba[int(r[1]), int(r[2])] = int(r[3], 16)
    assert np.array_equal(rgba, want_rgba)


def test_exact_pixel_mapping_brute_force(oracle_lib):
    """w = 1 everywhere and power-of-two scales: pixel = (x >> 5, y >> 5)
    exactly; every pixel keeps its smallest colour word."""
    a, m = 3, 6  # ndc = X / 8 - 1, 64 x 64 pixels
    M = np.array([[2.0 ** -a, 0, 0, -1], [0, 2.0 ** -a, 0, -1], [0, 0, 0, 0], [0, 0, 0, 1]])
    rng = np.random.default_rng(1)
    n = 30000
    x = rng.integers(-300, 2048 + 300, n)
    y = rng.integers(-300, 2048 + 300, n)
    z = rng.integers(-10**6, 10**6, n)
    rgb = rng.integers(0, 65536, (n, 3)).astype(np.uint16)
    fb, drawn = oracle_lib.raster(M, (0, 0), S, 0.01, 0.0, 64, 64, x, y, z, rgb)
    inside = (x >= 0) & (x < 2048) & (y >= 0) & (y < 2048)
    assert drawn == int(inside.sum())
    col = (0xFF << 24) | ((rgb[:, 2] >> 8).astype(np.int64) << 16) | ((rgb[:, 1] >> 8).astype(np.int64) << 8) | \
        (rgb[:, 0] >> 8).astype(np.int64)
    want = np.full(64 * 64, EMPTY, np.uint64)
    pix = (y[inside] >> 5) * 64 + (x[inside] >> 5)
    key = (np.uint64(0x3F800000) << np.uint64(32)) | col[inside].astype(np.uint64)
    np.minimum.at(want, pix, key)
    assert np.array_equal(fb.reshape(-1), want)


def test_nearest_point_on_each_ray_wins(oracle_lib):
    """Points scaled by powers of two along rays through the camera centre
    land on one pixel (numerator and denominator scale alike); the nearest
    of each ray is the one kept, whatever the order."""
    rng = np.random.default_rng(2)
    base = np.stack([rng.integers(-100, 100, 200), rng.integers(-100, 100, 200), rng.integers(100, 200, 200)], 1)
    reps = []
    for j in range(4):
        reps.append(base * (2 ** j))
    pts = np.concatenate(reps)
    rgb = rng.integers(0, 65536, (len(pts), 3)).astype(np.uint16)
    perm = rng.permutation(len(pts))
    fb, drawn = oracle_lib.raster(PINHOLE, (0, 0), S, S, 0.0, 256, 256, pts[perm, 0], pts[perm, 1], pts[perm, 2],
                                  rgb[perm])
    fb0, _ = oracle_lib.raster(PINHOLE, (0, 0), S, S, 0.0, 256, 256, base[:, 0], base[:, 1], base[:, 2], rgb[:200])
    # every drawn pixel of the far copies is also a pixel of the base set,
    # and where the base point is the unique nearest there, its key stays
    assert drawn == 4 * _drawn(oracle_lib, base)
    assert np.array_equal(fb != EMPTY, fb0 != EMPTY)
    hi = (fb >> np.uint64(32)).astype(np.uint32).view(np.float32)
    hi0 = (fb0 >> np.uint64(32)).astype(np.uint32).view(np.float32)
    assert np.array_equal(hi[fb != EMPTY], hi0[fb0 != EMPTY])


def _drawn(oracle_lib, pts):
    _, d = oracle_lib.raster(PINHOLE, (0, 0), S, S, 0.0, 256, 256, pts[:, 0], pts[:, 1], pts[:, 2],
                             np.zeros((len(pts), 3), np.uint16))
    return d


def test_permutation_invariance_and_accumulation(oracle_lib):
    rng = np.random.default_rng(3)
    n = 20000
    # a perspective camera looking down on a 64 m square from 100 m above its centre
    f = 1.5
    M = np.array([[f, 0, 0, -32 * f], [0, f, 0, -32 * f], [0, 0, 0, 0], [0, 0, -1, 100.0]])
    x = rng.integers(0, 6400, n)
    y = rng.integers(0, 6400, n)
    z = rng.integers(-2000, 2000, n)
    rgb = rng.integers(0, 65536, (n, 3)).astype(np.uint16)
    fb, d = oracle_lib.raster(M, (0, 0), 0.01, 0.01, 0.0, 128, 96, x, y, z, rgb)
    p = rng.permutation(n)
    fb2, d2 = oracle_lib.raster(M, (0, 0), 0.01, 0.01, 0.0, 128, 96, x[p], y[p], z[p], rgb[p])
    assert d == d2 and np.array_equal(fb, fb2)
    h = n // 2
    fa, da = oracle_lib.raster(M, (0, 0), 0.01, 0.01, 0.0, 128, 96, x[:h], y[:h], z[:h], rgb[:h])
    fc, dc = oracle_lib.raster(M, (0, 0), 0.01, 0.01, 0.0, 128, 96, x[h:], y[h:], z[h:], rgb[h:], fb=fa)
    assert da + dc == d and np.array_equal(fc, fb)
    assert 0 < d <= n and (fb != EMPTY).sum() > 1000


def test_behind_camera_never_drawn(oracle_lib):
    rng = np.random.default_rng(4)
    n = 5000
    pts = np.stack([rng.integers(-100, 100, n), rng.integers(-100, 100, n), rng.integers(-500, 1, n)], 1)
    fb, d = oracle_lib.raster(PINHOLE, (0, 0), S, S, 0.0, 64, 64, pts[:, 0], pts[:, 1], pts[:, 2],
                              np.zeros((n, 3), np.uint16))
    assert d == 0 and (fb == EMPTY).all()
