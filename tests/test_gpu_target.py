"""GPU parity: ground-truth mean splat, its resolve and the training losses
(Section 3.4, training data and training) against the oracle.  The sums are
integers, so they are compared bit for bit; the resolved means and the
per-element gradients are computed by the same IEEE double operations on
both sides and compared bit for bit too; the loss values are sums whose
order differs, compared to 1e-12 relative."""
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


def _same_tex(got, want):
    """Bit equality where the oracle has a value, NaN where it has a gap."""
    gap = np.isnan(want)
    assert np.array_equal(np.isnan(got), gap)
    assert np.array_equal(got[~gap].view(np.uint32), want[~gap].view(np.uint32))


@pytest.mark.parametrize("n", [0, 1, 4095, 2048, 2049, 200001])
def test_mean_splat_random_order_bit_exact(n):
    region = synth.Region(origin_x=-3000, origin_y=1000, tiles_x=3, tiles_y=2, res=64)
    x, y, z, rgb = _rand(n + 17, region, n)
    ts = np.array([2, -1, 0, 1, 4, 3], np.int32)
    want, wd = oracle.splat_mean(region, x, y, z, rgb, ts, 5)
    g = ls.Grid.of(region)
    xt, yt, zt, rt = arrays_to_dev(x, y, z, rgb)
    acc, nd = ls.splat_mean(g, xt, yt, zt, rt, torch.from_numpy(ts).cuda(), 5)
    torch.cuda.synchronize()
    assert np.array_equal(acc.cpu().numpy(), want)
    assert int(nd.item()) == wd
    tex = ls.resolve_mean(g, acc)
    torch.cuda.synchronize()
    _same_tex(tex.cpu().numpy(), oracle.resolve_mean(want, 0.01, 0.0))


def test_mean_splat_morton_chunks_accumulate():
    """Morton-ordered dense points (the LDS window path), split over two
    calls that accumulate, with an unmapped tile and a custom height scale."""
    region = synth.Region(tiles_x=4, tiles_y=4, scale_z=0.001, offset_z=-12.5)
    ps = synth.fullres_uniform(region, 400_000, seed=5)
    x, y, z, rgb = ps.numpy()
    ts = np.arange(16, dtype=np.int32)[::-1].copy()
    ts[6] = -1
    want, wd = oracle.splat_mean(region, x, y, z, rgb, ts, 16)
    g = ls.Grid.of(region)
    xt, yt, zt, rt = points_to_dev(ps)
    tst = torch.from_numpy(ts).cuda()
    h = 150_001
    acc, nd = ls.splat_mean(g, xt[:h], yt[:h], zt[:h], rt[:h], tst, 16)
    acc, nd = ls.splat_mean(g, xt[h:], yt[h:], zt[h:], rt[h:], tst, 16, acc=acc, n_dropped=nd)
    tex = ls.resolve_mean(g, acc)
    torch.cuda.synchronize()
    assert np.array_equal(acc.cpu().numpy(), want)
    assert int(nd.item()) == wd
    _same_tex(tex.cpu().numpy(), oracle.resolve_mean(want, 0.001, -12.5))
    # the unmapped tile's points are dropped, and every slot that has points has some
    assert wd > 0 and (want[..., 4] > 0).sum() > 10000


def test_mean_splat_wide_grid_direct_atomics():
    region = synth.Region(origin_x=-70000, origin_y=5000, tiles_x=1025, tiles_y=1, res=64)
    x, y, z, rgb = _rand(12, region, 60000)
    ts = np.full(1025, -1, np.int32)
    ts[[0, 1, 512, 1023, 1024]] = [4, 0, 2, 1, 3]
    want, wd = oracle.splat_mean(region, x, y, z, rgb, ts, 5)
    g = ls.Grid.of(region)
    xt, yt, zt, rt = arrays_to_dev(x, y, z, rgb)
    acc, nd = ls.splat_mean(g, xt, yt, zt, rt, torch.from_numpy(ts).cuda(), 5)
    torch.cuda.synchronize()
    assert np.array_equal(acc.cpu().numpy(), want)
    assert int(nd.item()) == wd
    assert want[..., 4].sum() > 0


def test_mean_splat_many_points_per_texel():
    """2,000,000 points on one tile (about 490 per texel, the training
    targets' density): per-batch LDS sums stay exact and the mean matches."""
    region = synth.Region(tiles_x=1, tiles_y=1)
    ps = synth.fullres_points(region, np.array([0]), 2_000_000, seed=9, noise_sigma_m=0.0, terrain_seed=4)
    x, y, z, rgb = ps.numpy()
    ts = np.zeros(1, np.int32)
    want, _ = oracle.splat_mean(region, x, y, z, rgb, ts, 1)
    g = ls.Grid.of(region)
    xt, yt, zt, rt = points_to_dev(ps)
    acc, _ = ls.splat_mean(g, xt, yt, zt, rt, torch.zeros(1, dtype=torch.int32, device="cuda"), 1)
    tex = ls.resolve_mean(g, acc)
    torch.cuda.synchronize()
    assert np.array_equal(acc.cpu().numpy(), want)
    _same_tex(tex.cpu().numpy(), oracle.resolve_mean(want, 0.01, 0.0))


@pytest.mark.parametrize("kind", [ls.LOSS_CLIPPED_MSE, ls.LOSS_L1])
@pytest.mark.parametrize("nt", [1, 5])
def test_target_loss_matches_oracle(kind, nt):
    """Random outputs against a target with gaps (NaN), large errors (the
    clip) and exact hits (sign(0) = 0); gradient bits equal the oracle's
    gradient rounded once to FP32."""
    region = synth.Region(tiles_x=nt, tiles_y=1)
    rng = np.random.default_rng(40 + nt + 10 * kind)
    y = rng.normal(0.0, 0.6, (nt, 64, 64, 4)).astype(np.float32)
    cz = rng.normal(10.0, 20.0, nt)
    t = np.empty_like(y)
    t[..., 0] = (cz[:, None, None] + 480.0 * rng.normal(0.0, 0.6, (nt, 64, 64))).astype(np.float32)
    t[..., 1:] = rng.uniform(0.0, 1.0, (nt, 64, 64, 3)).astype(np.float32)
    t[rng.random(t.shape) < 0.1] = np.nan
    # exact hits on colour channels
    hit = rng.random((nt, 64, 64)) < 0.05
    t[..., 2][hit] = y[..., 2][hit]
    (L, Lh, Lc), gref = oracle.target_loss(y, t, cz, region, kind=kind)
    g = ls.Grid.of(region)
    d = "cuda"
    loss, grad = ls.target_loss(torch.from_numpy(y).to(d), torch.from_numpy(t).to(d), torch.from_numpy(cz).to(d), g,
                                kind)
    torch.cuda.synchronize()
    got = loss.cpu().numpy()
    assert np.allclose(got, [L, Lh, Lc], rtol=1e-12, atol=0)
    assert np.array_equal(grad.cpu().numpy().view(np.uint32), gref.astype(np.float32).view(np.uint32))
    if kind == ls.LOSS_CLIPPED_MSE:
        # some elements are clipped (zero gradient with a finite target)
        clipped = (~np.isnan(t)) & (gref == 0.0)
        assert clipped.sum() > 100


def test_target_loss_all_gaps_zero():
    region = synth.Region(tiles_x=2, tiles_y=1)
    g = ls.Grid.of(region)
    y = torch.randn((2, 64, 64, 4), device="cuda")
    t = torch.full((2, 64, 64, 4), float("nan"), device="cuda")
    cz = torch.zeros(2, dtype=torch.float64, device="cuda")
    loss, grad = ls.target_loss(y, t, cz, g, ls.LOSS_CLIPPED_MSE)
    torch.cuda.synchronize()
    assert loss.cpu().tolist() == [0.0, 0.0, 0.0]
    assert torch.count_nonzero(grad).item() == 0


def test_training_targets_from_dense_points_end_to_end():
    """The paper's target pipeline on two tiles: mean splat of dense points,
    resolve with gaps, clipped MSE of the linear baseline (reconstruction
    input cropped) against it, all on the GPU and equal to the oracle's."""
    region = synth.Region(tiles_x=2, tiles_y=1)
    work = synth.sparse_workload("t", 2, 1, np.array([300, 500]), seed=3)
    dense = synth.fullres_points(region, np.array([0, 1]), 200_000, seed=8, noise_sigma_m=0.0, terrain_seed=3)
    x, y, z, rgb = dense.numpy()
    ts = np.empty(2, np.int32)
    ts[work.tile_list] = np.arange(2, dtype=np.int32)  # slot k holds tile_list[k], like the recon output
    acc_ref, _ = oracle.splat_mean(region, x, y, z, rgb, ts, 2)
    tex_ref = oracle.resolve_mean(acc_ref, 0.01, 0.0)
    sx, sy, sz, srgb = work.points.numpy()
    xo_ref, cz_ref, _ = oracle.recon_tiles(work.region, sx, sy, sz, srgb, work.tile_list)
    y_lin = np.ascontiguousarray(xo_ref[:, 16:80, 16:80][..., [0, 2, 3, 4]], dtype=np.float32)
    (L, _, _), gref = oracle.target_loss(y_lin, tex_ref, cz_ref, region)
    g = ls.Grid.of(region)
    xt, yt, zt, rt = points_to_dev(dense)
    acc, _ = ls.splat_mean(g, xt, yt, zt, rt, torch.from_numpy(ts).cuda(), 2)
    tex = ls.resolve_mean(g, acc)
    loss, grad = ls.target_loss(torch.from_numpy(y_lin).cuda(), tex, torch.from_numpy(cz_ref).cuda(), g)
    torch.cuda.synchronize()
    assert abs(float(loss[0].item()) - L) <= 1e-12 * abs(L)
    assert np.array_equal(grad.cpu().numpy().view(np.uint32), gref.astype(np.float32).view(np.uint32))
