"""Training the refinement network through RefineFn and the library's loss
(Section 3.4): targets built from dense points of the same terrain, either
the paper's per-texel mean (with gaps) and its NaN-masked clipped MSE, or the
configured max-height splat and L1; AdamW steps must lower the loss below
the linear baseline, the BF16 and FP32 paths must agree on the first
gradient to BF16 accuracy, and a checkpoint (weights, AdamW moments,
schedule) must resume a run bit for bit."""
import numpy as np
import pytest
import torch

import paper_2509_20198_amd as ls
import synth
from paper_2509_20198_amd import train as T

pytestmark = pytest.mark.gpu


def _small_set(dense_per_tile=200_000, mean=False):
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
    if mean:
        acc, _ = ls.splat_mean(g, d.x, d.y, d.z, d.rgb_u16(), slot, nt)
        tex = ls.resolve_mean(g, acc)
        empty = int((acc[..., 4] == 0).sum().item())
    else:
        keys, _ = ls.splat_points(g, d.x, d.y, d.z, d.rgb_u16(), slot, nt)
        tex = torch.zeros((nt, region.res, region.res, 4), dtype=torch.float32, device=dev)
        ls.resolve_keys(g, keys, tex)
        empty = int((keys == 0).sum().item())
    torch.cuda.synchronize()
    assert empty == 0  # every texel has a dense point
    return g, x, cz, tex


@pytest.mark.parametrize("kind", [ls.LOSS_L1, ls.LOSS_CLIPPED_MSE])
def test_adamw_lowers_loss(kind):
    g, x, cz, tex = _small_set(mean=kind == ls.LOSS_CLIPPED_MSE)
    w0 = torch.from_numpy(synth.unet_weights(1).astype(np.float32)).cuda()
    base = T.loss_value(T.linear_baseline(x, g.pad, g.res), tex, cz, g, kind)
    tr = T.Trainer(w0, g, ls.BF16, save_acts=False, total_steps=40, lr=1e-3, loss_kind=kind)
    losses = [float(tr.step(x, tex, cz)) for _ in range(40)]
    print(f"kind {kind}: linear baseline {base:.6g}; loss {losses[0]:.6g} -> {losses[-1]:.6g}")
    assert all(np.isfinite(losses))
    assert losses[-1] < losses[0]
    assert min(losses) < base


def test_mean_targets_with_gaps_are_masked():
    """Sparse dense points leave gaps (NaN) in the mean target; the loss and
    its gradient ignore them, so training still proceeds."""
    g, x, cz, _ = _small_set()
    dev = x.device
    work = synth.train_tiles(seed=4, tiles_x=4, tiles_y=4)
    nt = len(work.tile_list)
    ids = np.asarray(work.tile_list, np.int64)
    slot = torch.full((16,), -1, dtype=torch.int32, device=dev)
    slot[torch.from_numpy(ids).to(dev)] = torch.arange(nt, dtype=torch.int32, device=dev)
    d = synth.fullres_points(work.region, ids, 3000, seed=7, noise_sigma_m=0.0, device=dev, terrain_seed=4)
    acc, _ = ls.splat_mean(g, d.x, d.y, d.z, d.rgb_u16(), slot, nt)
    tex = ls.resolve_mean(g, acc)
    gaps = int(torch.isnan(tex[..., 0]).sum().item())
    assert gaps > 1000
    w0 = torch.from_numpy(synth.unet_weights(1).astype(np.float32)).cuda()
    w = w0.clone().requires_grad_(True)
    y = ls.RefineFn.apply(x, w, g, ls.BF16, True)
    loss = T.TargetLossFn.apply(y, tex, cz, g, ls.LOSS_CLIPPED_MSE)
    loss.backward()
    assert torch.isfinite(loss) and torch.isfinite(w.grad).all()
    assert float(w.grad.abs().sum()) > 0


def test_first_gradient_bf16_close_to_fp32():
    g, x, cz, tex = _small_set()
    w0 = torch.from_numpy(synth.unet_weights(1).astype(np.float32)).cuda()
    grads = []
    for prec in (ls.FP32, ls.BF16):
        w = w0.clone().requires_grad_(True)
        T.TargetLossFn.apply(ls.RefineFn.apply(x, w, g, prec, True), tex, cz, g, ls.LOSS_L1).backward()
        grads.append(w.grad.double().cpu().numpy())
    rel = np.linalg.norm(grads[1] - grads[0]) / np.linalg.norm(grads[0])
    print(f"bf16 vs fp32 first gradient: rel {rel:.2e}")
    assert rel < 0.1


def test_checkpoint_resumes_bit_for_bit(tmp_path):
    g, x, cz, tex = _small_set(mean=True)
    w0 = torch.from_numpy(synth.unet_weights(1).astype(np.float32)).cuda()
    a = T.Trainer(w0, g, ls.BF16, total_steps=6, lr=1e-3)
    for _ in range(6):
        a.step(x, tex, cz)
    b = T.Trainer(w0, g, ls.BF16, total_steps=6, lr=1e-3)
    for _ in range(3):
        b.step(x, tex, cz)
    path = str(tmp_path / "ckpt.pt")
    b.save(path)
    c = T.Trainer(torch.zeros_like(w0), g, ls.FP32, total_steps=6, lr=5.0, loss_kind=ls.LOSS_L1)
    c.load(path)
    for _ in range(3):
        c.step(x, tex, cz)
    torch.cuda.synchronize()
    assert torch.equal(c.w.detach(), a.w.detach())
