"""GPU parity: point rasteriser with packed 64-bit depth-and-colour keys and
its resolve (Section 3.6, points) against the oracle's sequential loop; the
frame buffer, the drawn count and the resolved colours are bit-exact."""
import numpy as np
import pytest
import torch

import oracle
import paper_2509_20198_amd as ls
import synth
from gpu_helpers import arrays_to_dev, points_to_dev

pytestmark = pytest.mark.gpu

EMPTY = np.iinfo(np.uint64).max


def _look_down(f=1.5, side_m=64.0, height_m=100.0):
    """Perspective camera above the centre of a side_m square, looking down."""
    c = side_m / 2
    return np.array([[f, 0, 0, -c * f], [0, f, 0, -c * f], [0, 0, 0, 0], [0, 0, -1, height_m]], np.float64)


def _oblique(seed):
    """A random perspective view: rotation, translation and a projection."""
    rng = np.random.default_rng(seed)
    a, b = rng.uniform(-0.6, 0.6, 2)
    Rz = np.array([[np.cos(a), -np.sin(a), 0], [np.sin(a), np.cos(a), 0], [0, 0, 1]])
    Rx = np.array([[1, 0, 0], [0, np.cos(b), -np.sin(b)], [0, np.sin(b), np.cos(b)]])
    V = np.eye(4)
    V[:3, :3] = Rx @ Rz
    V[:3, 3] = [-300.0, -250.0, -400.0]
    P = np.array([[1.2, 0, 0.1, 0], [0, 1.6, -0.05, 0], [0, 0, -1.0, -0.2], [0, 0, -1, 0]])
    return P @ V


def _run(M, origin, sxy, sz, oz, w, h, x, y, z, rgb, fb=None):
    view = ls.View(m=M, origin_x=origin[0], origin_y=origin[1], scale_xy=sxy, scale_z=sz, offset_z=oz, width=w,
                   height=h)
    xt, yt, zt, rt = arrays_to_dev(x, y, z, rgb)
    fbt, nd = ls.raster_points(view, xt, yt, zt, rt, fb=fb)
    torch.cuda.synchronize()
    return fbt, int(nd.item())


@pytest.mark.parametrize("n", [0, 1, 2047, 2048, 2049, 100_003])
def test_raster_look_down_bit_exact(n):
    rng = np.random.default_rng(n + 1)
    x = rng.integers(-500, 6900, n).astype(np.int32)
    y = rng.integers(-500, 6900, n).astype(np.int32)
    z = rng.integers(-2000, 2000, n).astype(np.int32)
    rgb = rng.integers(0, 65536, (n, 3)).astype(np.uint16)
    M = _look_down()
    want, wd = oracle.raster(M, (0, 0), 0.01, 0.01, 0.0, 160, 120, x, y, z, rgb)
    fb, d = _run(M, (0, 0), 0.01, 0.01, 0.0, 160, 120, x, y, z, rgb)
    got = fb.cpu().numpy().view(np.uint64)
    assert d == wd
    assert np.array_equal(got, want)
    rgba = ls.raster_resolve(fb)
    torch.cuda.synchronize()
    assert np.array_equal(rgba.cpu().numpy().view(np.uint32), oracle.raster_resolve(want))


@pytest.mark.parametrize("seed", [1, 2])
def test_raster_oblique_terrain_bit_exact(seed):
    """Morton-ordered terrain points seen obliquely, some behind the camera
    and some outside the view; a non-zero view origin and height offset."""
    region = synth.Region(origin_x=100_000, origin_y=-50_000, tiles_x=2, tiles_y=2)
    ps = synth.fullres_uniform(region, 300_000, seed=seed)
    x, y, z, rgb = ps.numpy()
    M = _oblique(seed)
    origin = (region.origin_x, region.origin_y)
    want, wd = oracle.raster(M, origin, 0.01, 0.01, 3.25, 320, 200, x, y, z, rgb)
    view = ls.View(m=M, origin_x=origin[0], origin_y=origin[1], scale_xy=0.01, scale_z=0.01, offset_z=3.25,
                   width=320, height=200)
    xt, yt, zt, rt = points_to_dev(ps)
    fb, nd = ls.raster_points(view, xt, yt, zt, rt)
    torch.cuda.synchronize()
    assert int(nd.item()) == wd
    assert np.array_equal(fb.cpu().numpy().view(np.uint64), want)
    assert 0 < wd < len(x) and (want != EMPTY).sum() > 1000


def test_raster_accumulates_and_permutation_invariant():
    rng = np.random.default_rng(7)
    n = 50_000
    x = rng.integers(0, 6400, n).astype(np.int32)
    y = rng.integers(0, 6400, n).astype(np.int32)
    z = rng.integers(-2000, 2000, n).astype(np.int32)
    rgb = rng.integers(0, 65536, (n, 3)).astype(np.uint16)
    M = _look_down()
    want, wd = oracle.raster(M, (0, 0), 0.01, 0.01, 0.0, 128, 96, x, y, z, rgb)
    h = 20_001
    fb, d1 = _run(M, (0, 0), 0.01, 0.01, 0.0, 128, 96, x[:h], y[:h], z[:h], rgb[:h])
    fb, d2 = _run(M, (0, 0), 0.01, 0.01, 0.0, 128, 96, x[h:], y[h:], z[h:], rgb[h:], fb=fb)
    assert d1 + d2 == wd
    assert np.array_equal(fb.cpu().numpy().view(np.uint64), want)
    p = rng.permutation(n)
    fb2, d3 = _run(M, (0, 0), 0.01, 0.01, 0.0, 128, 96, x[p], y[p], z[p], rgb[p])
    assert d3 == wd and np.array_equal(fb2.cpu().numpy().view(np.uint64), want)


def test_raster_behind_camera_never_drawn():
    rng = np.random.default_rng(4)
    n = 5000
    S = 1.0 / 128.0
    pinhole = np.array([[1, 0, 0, 0], [0, 1, 0, 0], [0, 0, 0, 0], [0, 0, 1, 0]], np.float64)
    x = rng.integers(-100, 100, n).astype(np.int32)
    y = rng.integers(-100, 100, n).astype(np.int32)
    z = rng.integers(-500, 1, n).astype(np.int32)
    rgb = np.zeros((n, 3), np.uint16)
    fb, d = _run(pinhole, (0, 0), S, S, 0.0, 64, 64, x, y, z, rgb)
    assert d == 0 and (fb.cpu().numpy().view(np.uint64) == EMPTY).all()
