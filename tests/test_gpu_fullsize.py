"""Parity at the workloads' full sizes, in the launch configurations the
benchmark uses, on outputs the oracle computes one by one:

* the 100 M-point Morton-ordered splat over 64 x 64 tiles (keys at sampled
  texels against the oracle's sequential maximum over every point near them);
* the 16,384-tile streaming workload (Pareto counts, viewpoint order): recon
  and BF16 refinement of sampled tiles, and the 500 M-point splat over the
  256 nearest tiles (sampled texels);
* the 256-tile refinement backward with the output gradient restricted to a
  few tiles (by linearity, their gradient alone) against the oracle.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_2509_20198_amd as ls
import synth
from gpu_helpers import R_M, rms_per_tile

pytestmark = pytest.mark.gpu


def _sampled_splat_check(region, ps, tile_slot, n_slots, keys, n_sample, seed):
    """Compare keys at sampled texels with the oracle run on every point
    whose texel lies within one texel of a sampled one (a superset)."""
    rng = np.random.default_rng(seed)
    res = region.res
    ts = np.asarray(tile_slot)
    mapped = np.nonzero(ts >= 0)[0]
    tiles = rng.choice(mapped, n_sample)
    rows, cols = rng.integers(0, res, n_sample), rng.integers(0, res, n_sample)
    gw, gh = region.tiles_x * res, region.tiles_y * res
    gx_s = (tiles % region.tiles_x) * res + cols
    gy_s = (tiles // region.tiles_x) * res + rows
    dev = ps.x.device
    near = torch.zeros((gh + 2, gw + 2), dtype=torch.bool, device=dev)
    for dy in (-1, 0, 1):
        for dx in (-1, 0, 1):
            near[torch.from_numpy(gy_s + 1 + dy).to(dev), torch.from_numpy(gx_s + 1 + dx).to(dev)] = True
    C = region.cell
    gx = torch.div(ps.x.long() - region.origin_x, C, rounding_mode="floor").clamp(-1, gw) + 1
    gy = torch.div(ps.y.long() - region.origin_y, C, rounding_mode="floor").clamp(-1, gh) + 1
    sel = near[gy, gx].nonzero().squeeze(1)
    sub = [t[sel].cpu().numpy() for t in (ps.x, ps.y, ps.z)] + [ps.rgb_u16()[sel].cpu().numpy()]
    want, _ = oracle.splat(region, *sub, ts.astype(np.int32), n_slots)
    got = keys.cpu().numpy().view(np.uint64)
    slots = ts[tiles]
    assert np.array_equal(got[slots, rows, cols], want[slots, rows, cols])
    return len(sel)


def test_splat_100m_points_sampled():
    dev = torch.device("cuda")
    region = synth.Region(tiles_x=64, tiles_y=64)
    ps = synth.fullres_uniform(region, 100_000_000, seed=3, device=dev)
    g = ls.Grid.of(region)
    ts = torch.arange(4096, dtype=torch.int32, device=dev)
    keys, nd = ls.splat_points(g, ps.x, ps.y, ps.z, ps.rgb_u16(), ts, 4096)
    torch.cuda.synchronize()
    assert int(nd.item()) == 0
    n = _sampled_splat_check(region, ps, np.arange(4096), 4096, keys, 3000, 1)
    print(f"checked 3000 texels with {n} nearby points")


def test_streaming_16k_tiles_sampled():
    dev = torch.device("cuda")
    work = synth.stream_tiles(seed=5, device=dev)
    region = work.region
    g = ls.Grid.of(region)
    ps = work.points
    nt = len(work.tile_list)
    tl = torch.from_numpy(work.tile_list).to(dev)
    x, cz, st = ls.recon_tiles(g, ps.x, ps.y, ps.z, ps.rgb_u16(), tl)
    wts = synth.unet_weights(0)
    w = torch.from_numpy(wts.astype(np.float32)).to(dev)
    wb = ls.pack_weights_bf16(w)
    _, tex = ls.refine_tiles(w, x, cz, g, ls.BF16, w_bf16=wb, want_y=False)
    torch.cuda.synchronize()
    rng = np.random.default_rng(2)
    ks = np.concatenate([[0, 1, nt - 1], rng.choice(nt, 5, replace=False)])
    pn = ps.numpy()
    xo, czo, sto = oracle.recon_tiles(region, *pn, work.tile_list[ks])
    xg = x[ks].cpu().numpy().astype(np.float64)
    assert np.abs(xg[..., 0] - xo[..., 0]).max() * R_M <= 1e-4
    assert np.abs(xg[..., 1] - xo[..., 1]).max() * R_M <= 1e-5
    assert np.array_equal(st[ks].cpu().numpy() & 3, sto)
    y_ref = oracle.unet_forward(wts, xo, region.res, region.pad)
    t_ref = oracle.texture(y_ref, czo, region)
    rms = rms_per_tile(tex[ks].cpu().numpy()[..., 0], t_ref[..., 0])
    print(f"streaming tiles: BF16 RMS max {rms.max():.4f} m, flags {np.bincount(st.cpu().numpy())}")
    assert rms.max() <= 0.05
    assert int((st.cpu().numpy() & ~3).sum()) == 0  # no CAP / DEGENERATE / BADID


def test_streaming_splat_500m_points_sampled():
    dev = torch.device("cuda")
    work = synth.stream_tiles(seed=5)
    region = work.region
    near = np.asarray(work.tile_list[:256], np.int64)
    n_per = 500_000_000 // 256
    ps = synth.fullres_points(region, near, n_per, seed=11, device=dev)
    slot = np.full(region.tiles_x * region.tiles_y, -1, np.int32)
    slot[near] = np.arange(256, dtype=np.int32)
    g = ls.Grid.of(region)
    keys, nd = ls.splat_points(g, ps.x, ps.y, ps.z, ps.rgb_u16(), torch.from_numpy(slot).to(dev), 256)
    torch.cuda.synchronize()
    assert int(nd.item()) == 0
    n = _sampled_splat_check(region, ps, slot, 256, keys, 2000, 3)
    print(f"checked 2000 texels with {n} nearby points of {ps.n}")


def test_backward_256_tiles_restricted_gradient():
    dev = torch.device("cuda")
    work = synth.train_tiles(seed=4)
    region = work.region
    pn = work.points.numpy()
    xo, cz, _ = oracle.recon_tiles(region, *pn, work.tile_list)
    x32 = xo.astype(np.float32)
    nt = x32.shape[0]
    wts = synth.unet_weights(1, head_std=0.05, bias_std=0.05)
    w32 = wts.astype(np.float32)
    rng = np.random.default_rng(6)
    ks = rng.choice(nt, 3, replace=False)
    G = np.zeros((nt, 64, 64, 4))
    G[ks] = rng.standard_normal((3, 64, 64, 4))
    g = ls.Grid.of(region)
    gw, _ = ls.refine_backward(torch.from_numpy(w32).to(dev), torch.from_numpy(x32).to(dev),
                               torch.from_numpy(G.astype(np.float32)).to(dev), g, ls.FP32)
    torch.cuda.synchronize()
    gw_ref, _ = oracle.unet_backward(w32.astype(np.float64), x32[ks].astype(np.float64), G[ks], 64, 16)
    gw = gw.cpu().numpy().astype(np.float64)
    rel = np.linalg.norm(gw - gw_ref) / np.linalg.norm(gw_ref)
    print(f"256-tile backward, gradient restricted to tiles {ks.tolist()}: rel {rel:.2e}")
    assert rel <= 1e-3
