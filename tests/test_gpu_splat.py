"""GPU parity: full-resolution splat and resolve (Sections 3.5-3.6) against
the oracle's sequential per-texel maximum; bit-exact."""
import numpy as np
import pytest
import torch

import oracle
import paper_2509_20198_amd as ls
import synth
from gpu_helpers import arrays_to_dev, points_to_dev

pytestmark = pytest.mark.gpu


def _rand(seed, region, n, spill=5000):
    rng = np.random.default_rng(seed)
    W = region.tiles_x * region.tile_size
    H = region.tiles_y * region.tile_size
    x = rng.integers(region.origin_x - spill, region.origin_x + W + spill, n).astype(np.int32)
    y = rng.integers(region.origin_y - spill, region.origin_y + H + spill, n).astype(np.int32)
    z = rng.integers(-2 ** 31, 2 ** 31, n, dtype=np.int64).astype(np.int32)
    z[: n // 2] = rng.integers(-3, 3, n // 2)
    rgb = rng.integers(0, 65536, (n, 3)).astype(np.uint16)
    return x, y, z, rgb


@pytest.mark.parametrize("n", [0, 1, 4095, 4096, 4097, 200001])
def test_splat_random_order_bit_exact(n):
    region = synth.Region(origin_x=-3000, origin_y=1000, tiles_x=3, tiles_y=2, res=64)
    x, y, z, rgb = _rand(n, region, n)
    ts = np.array([2, -1, 0, 1, 4, 3], np.int32)
    want, wd = oracle.splat(region, x, y, z, rgb, ts, 5)
    g = ls.Grid.of(region)
    xt, yt, zt, rt = arrays_to_dev(x, y, z, rgb)
    keys, nd = ls.splat_points(g, xt, yt, zt, rt, torch.from_numpy(ts).cuda(), 5)
    torch.cuda.synchronize()
    got = keys.cpu().numpy().view(np.uint64)
    assert np.array_equal(got, want)
    assert int(nd.item()) == wd


def test_splat_morton_chunks_accumulate_and_resolve():
    region = synth.Region(tiles_x=4, tiles_y=4)
    ps = synth.fullres_uniform(region, 300_000, seed=3)
    x, y, z, rgb = ps.numpy()
    ts = np.arange(16, dtype=np.int32)[::-1].copy()
    ts[5] = -1
    want, wd = oracle.splat(region, x, y, z, rgb, ts, 16)
    g = ls.Grid.of(region)
    xt, yt, zt, rt = points_to_dev(ps)
    tst = torch.from_numpy(ts).cuda()
    h = 123_457
    keys, nd = ls.splat_points(g, xt[:h], yt[:h], zt[:h], rt[:h], tst, 16)
    tex0 = torch.full((16, 64, 64, 4), -5.0, device="cuda")
    keys, nd = ls.splat_points(g, xt[h:], yt[h:], zt[h:], rt[h:], tst, 16, keys=keys, n_dropped=nd,
                               tex_inout=tex0)
    torch.cuda.synchronize()
    got = keys.cpu().numpy().view(np.uint64)
    assert np.array_equal(got, want)
    assert int(nd.item()) == wd
    tex_want = oracle.resolve(want, np.full((16, 64, 64, 4), -5.0, np.float32), 0.01, 0.0)
    assert np.array_equal(tex0.cpu().numpy().view(np.uint32), tex_want.view(np.uint32))


def test_splat_wide_grid_direct_atomics():
    """A texel grid wider than 65,536 columns (1,025 tiles of 64 texels):
    Morton codes no longer fit 16-bit halves and every key goes straight to
    the global array."""
    region = synth.Region(origin_x=-70000, origin_y=5000, tiles_x=1025, tiles_y=1, res=64)
    x, y, z, rgb = _rand(11, region, 60000)
    ts = np.full(1025, -1, np.int32)
    ts[[0, 1, 512, 1023, 1024]] = [4, 0, 2, 1, 3]
    want, wd = oracle.splat(region, x, y, z, rgb, ts, 5)
    g = ls.Grid.of(region)
    xt, yt, zt, rt = arrays_to_dev(x, y, z, rgb)
    keys, nd = ls.splat_points(g, xt, yt, zt, rt, torch.from_numpy(ts).cuda(), 5)
    torch.cuda.synchronize()
    assert np.array_equal(keys.cpu().numpy().view(np.uint64), want)
    assert int(nd.item()) == wd
    assert np.count_nonzero(want) > 0


def test_splat_permutation_invariant():
    region = synth.Region(tiles_x=2, tiles_y=2)
    ps = synth.fullres_uniform(region, 100_000, seed=4)
    g = ls.Grid.of(region)
    ts = torch.arange(4, dtype=torch.int32, device="cuda")
    xt, yt, zt, rt = points_to_dev(ps)
    k1, _ = ls.splat_points(g, xt, yt, zt, rt, ts, 4)
    perm = torch.randperm(ps.n, generator=torch.Generator().manual_seed(0)).cuda()
    k2, _ = ls.splat_points(g, xt[perm].contiguous(), yt[perm].contiguous(), zt[perm].contiguous(),
                            rt[perm].contiguous(), ts, 4)
    assert torch.equal(k1, k2)


def test_splat_resolve_offset_bit_exact():
    region = synth.Region(tiles_x=1, tiles_y=1, res=64, scale_z=0.001, offset_z=123.456)
    x, y, z, rgb = _rand(7, region, 20000, spill=0)
    ts = np.zeros(1, np.int32)
    want, _ = oracle.splat(region, x, y, z, rgb, ts, 1)
    tex_want = oracle.resolve(want, np.zeros((1, 64, 64, 4), np.float32), 0.001, 123.456)
    g = ls.Grid.of(region)
    xt, yt, zt, rt = arrays_to_dev(x, y, z, rgb)
    tex = torch.zeros((1, 64, 64, 4), device="cuda")
    ls.splat_points(g, xt, yt, zt, rt, torch.zeros(1, dtype=torch.int32, device="cuda"), 1, tex_inout=tex)
    torch.cuda.synchronize()
    assert np.array_equal(tex.cpu().numpy().view(np.uint32), tex_want.view(np.uint32))
