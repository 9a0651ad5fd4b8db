"""Training the refinement network through RefineFn (Section 3.4): targets
are max-height splats of dense points of the same terrain; AdamW steps must
lower the L1 loss, and the BF16 and FP32 paths must agree on the first
gradient to BF16 accuracy."""
import numpy as np
import pytest
import torch

import paper_2509_20198_amd as ls
import synth
from paper_2509_20198_amd import train as T

pytestmark = pytest.mark.gpu


def _small_set(dense_per_tile=200_000):
    dev = torch.device("cuda")
    work = synth.train_tiles(seed=4, tiles_x=4, tiles_y=4, device=dev)
    region = work.region
    g = ls.Grid.of(region)
    ps = work.points
    tl = torch.from_numpy(work.tile_list).to(dev)
    x, cz, st = ls.recon_tiles(g, ps.x, ps.y, ps.z, ps.rgb_u16(), tl)
    nt = len(work.tile_list)
    ids = np.asarray(work.tile_list, np.int64)
    slot = torch.full((region.tiles_x * region.tiles_y,), -1, dtype=torch.int32, device=dev)
    slot[torch.from_numpy(ids).to(dev)] = torch.arange(nt, dtype=torch.int32, device=dev)
    d = synth.fullres_points(region, ids, dense_per_tile, seed=99, noise_sigma_m=0.0, device=dev, terrain_seed=4)
    keys, _ = ls.splat_points(g, d.x, d.y, d.z, d.rgb_u16(), slot, nt)
    tex = torch.zeros((nt, region.res, region.res, 4), dtype=torch.float32, device=dev)
    ls.resolve_keys(g, keys, tex)
    r_m = (region.tile_size / 2 + region.pad * region.cell) * region.scale_xy
    torch.cuda.synchronize()
    assert int((keys == 0).sum().item()) == 0  # every texel has a dense point
    return g, x, T.normalise_target(tex, cz, r_m)


def test_adamw_lowers_l1_loss():
    g, x, t = _small_set()
    w0 = torch.from_numpy(synth.unet_weights(1).astype(np.float32)).cuda()
    base = float(T.l1_loss(T.linear_baseline(x, g.pad, g.res), t))
    tr = T.Trainer(w0, g, ls.BF16, save_acts=False, total_steps=40, lr=1e-3)
    losses = [float(tr.step(x, t)) for _ in range(40)]
    print(f"linear baseline {base:.5f}; loss {losses[0]:.5f} -> {losses[-1]:.5f}")
    assert all(np.isfinite(losses))
    assert losses[-1] < losses[0]
    assert min(losses) < base


def test_first_gradient_bf16_close_to_fp32():
    g, x, t = _small_set()
    w0 = torch.from_numpy(synth.unet_weights(1).astype(np.float32)).cuda()
    grads = []
    for prec in (ls.FP32, ls.BF16):
        w = w0.clone().requires_grad_(True)
        T.l1_loss(ls.RefineFn.apply(x, w, g, prec, True), t).backward()
        grads.append(w.grad.double().cpu().numpy())
    rel = np.linalg.norm(grads[1] - grads[0]) / np.linalg.norm(grads[0])
    print(f"bf16 vs fp32 first gradient: rel {rel:.2e}")
    assert rel < 0.1
