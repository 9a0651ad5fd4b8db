"""GPU parity: the paper's refinement network (Section 3.4, architecture
paragraph) against the FP64 oracle.  FP32: texture heights within 1e-4 m of
the oracle (and the normalised colours within 1e-5); BF16: per-tile RMS of
the texture height within 0.05 m, reported next to the RMS of the network's
own contribution so the gate is not vacuous; a zero final layer gives the
linear input exactly (the paper's Linear baseline)."""
import numpy as np
import pytest
import torch

import oracle
import paper_2509_20198_amd as ls
import synth

pytestmark = pytest.mark.gpu


def _inputs(tiles_x, tiles_y, seed, pad=16, res=64):
    """Network inputs from the GPU reconstruction of synthetic sparse tiles
    (the refinement parity is about the network: both sides get the same x)."""
    counts = synth.counts_loguniform(seed, tiles_x * tiles_y)
    work = synth.sparse_workload("lsnet", tiles_x, tiles_y, counts, seed, pad=pad, res=res)
    g = ls.Grid.of(work.region)
    d = "cuda"
    ps = work.points
    x, cz, st = ls.recon_tiles(g, ps.x.to(d), ps.y.to(d), ps.z.to(d), ps.rgb_u16().to(d),
                               torch.from_numpy(work.tile_list).to(d))
    torch.cuda.synchronize()
    assert int(st.max().item()) == 0
    return work.region, g, x, cz


def _oracle(w64, x, cz, region, idx=None):
    xs = x.cpu().numpy().astype(np.float64)
    czs = cz.cpu().numpy()
    if idx is not None:
        xs, czs = xs[idx], czs[idx]
    y = oracle.pnet_forward(w64, xs, region.res, region.pad)
    return y, oracle.texture(y, czs, region)


@pytest.mark.parametrize("pad", [16, 0])
def test_fp32_matches_oracle(pad):
    """Default initialisation (the final layer small, as for training from
    scratch) with non-zero biases: the 1e-4 m gate, absolute."""
    region, g, x, cz = _inputs(3, 2, 21 + pad, pad=pad)
    w64 = synth.pnet_weights(1, R=g.R, bias_std=0.02)
    w = torch.from_numpy(w64.astype(np.float32)).cuda()
    y, tex = ls.lsnet_refine_tiles(w, x, cz, g, ls.FP32)
    torch.cuda.synchronize()
    # the oracle on the FP32-rounded weights the GPU sees
    y_ref, tex_ref = _oracle(w64.astype(np.float32).astype(np.float64), x, cz, region)
    dh = np.abs(tex.cpu().numpy()[..., 0].astype(np.float64) - tex_ref[..., 0]).max()
    dc = np.abs(y.cpu().numpy()[..., 1:].astype(np.float64) - y_ref[..., 1:]).max()
    head = y_ref - x.cpu().numpy()[:, pad:pad + 64, pad:pad + 64][..., [0, 2, 3, 4]]
    head_rms = float(np.sqrt((head[..., 0] ** 2).mean())) * 480.0
    assert dh <= 1e-4, f"max |dh| {dh:.3e} m (head RMS {head_rms:.3f} m)"
    assert dc <= 1e-5, f"max |drgb| {dc:.3e}"
    assert head_rms > 0.2, f"head RMS {head_rms:.3f} m: the gate would be vacuous"


def test_fp32_large_head_relative():
    """A final layer 34 times the default (the network's own contribution
    up to about 80 m): FP32 rounding then scales with the output, so the
    gate is relative to the output scale, 1e-5 of the largest |y|, as for
    the U-Net's large-head test."""
    region, g, x, cz = _inputs(3, 2, 37)
    w64 = synth.pnet_weights(1, R=g.R, final_std=0.02, bias_std=0.02)
    w = torch.from_numpy(w64.astype(np.float32)).cuda()
    y, _ = ls.lsnet_refine_tiles(w, x, cz, g, ls.FP32, want_tex=False)
    torch.cuda.synchronize()
    y_ref, _ = _oracle(w64.astype(np.float32).astype(np.float64), x, cz, region)
    head = np.abs(y_ref[..., 0] - x.cpu().numpy()[:, 16:80, 16:80, 0]).max() * 480.0
    assert head > 50.0
    d = np.abs(y.cpu().numpy() - y_ref).max()
    assert d <= 1e-5 * np.abs(y_ref).max(), f"max |dy| {d:.3e}, max |y| {np.abs(y_ref).max():.3f}"


def test_bf16_within_rms_gate():
    region, g, x, cz = _inputs(3, 3, 31)
    w64 = synth.pnet_weights(2, R=g.R)
    w = torch.from_numpy(w64.astype(np.float32)).cuda()
    _, tex = ls.lsnet_refine_tiles(w, x, cz, g, ls.BF16, want_y=False)
    torch.cuda.synchronize()
    _, tex_ref = _oracle(w64, x, cz, region)
    d = tex.cpu().numpy()[..., 0].astype(np.float64) - tex_ref[..., 0]
    rms = np.sqrt((d ** 2).reshape(d.shape[0], -1).mean(1))
    base = oracle.texture(x.cpu().numpy()[:, 16:80, 16:80][..., [0, 2, 3, 4]].astype(np.float64), cz.cpu().numpy(),
                          region)
    head_rms = np.sqrt(((tex_ref[..., 0] - base[..., 0]) ** 2).reshape(d.shape[0], -1).mean(1))
    print(f"BF16 lsnet: RMS per tile max {rms.max():.4f} m mean {rms.mean():.4f} m; head RMS mean "
          f"{head_rms.mean():.3f} m")
    assert rms.max() <= 0.05
    assert head_rms.mean() > 0.2


@pytest.mark.parametrize("prec", [ls.FP32, ls.BF16])
def test_zero_final_layer_is_linear_baseline(prec):
    region, g, x, cz = _inputs(2, 1, 41)
    w64 = synth.pnet_weights(3, R=g.R, bias_std=0.1)
    w64[-(4 * 9 * 32 + 4):] = 0.0
    w = torch.from_numpy(w64.astype(np.float32)).cuda()
    y, _ = ls.lsnet_refine_tiles(w, x, cz, g, prec, want_tex=False)
    torch.cuda.synchronize()
    want = x[:, 16:80, 16:80][..., [0, 2, 3, 4]]
    assert torch.equal(y, want.contiguous())


@pytest.mark.parametrize("prec,nt", [(ls.FP32, 300), (ls.BF16, 1100)])
def test_chunked_batch_sampled(prec, nt):
    """More tiles than one chunk of the workspace (256 FP32, 1024 BF16):
    sampled tiles on both sides of every chunk boundary against the oracle,
    and the whole batch equal to per-chunk calls."""
    side = int(np.ceil(np.sqrt(nt)))
    region, g, x, cz = _inputs(side, side, 51)
    x, cz = x[:nt].contiguous(), cz[:nt].contiguous()
    w64 = synth.pnet_weights(4, R=g.R)
    w = torch.from_numpy(w64.astype(np.float32)).cuda()
    _, tex = ls.lsnet_refine_tiles(w, x, cz, g, prec, want_y=False)
    torch.cuda.synchronize()
    chunk = 256 if prec == ls.FP32 else 1024
    idx = np.array([0, chunk - 1, chunk, nt - 1])
    w_or = w64.astype(np.float32).astype(np.float64) if prec == ls.FP32 else w64
    _, tex_ref = _oracle(w_or, x, cz, region, idx)
    d = tex.cpu().numpy()[idx][..., 0].astype(np.float64) - tex_ref[..., 0]
    if prec == ls.FP32:
        assert np.abs(d).max() <= 1e-4
    else:
        assert np.sqrt((d ** 2).reshape(len(idx), -1).mean(1)).max() <= 0.05
    # a call on the second chunk alone gives the same bits
    _, tex2 = ls.lsnet_refine_tiles(w, x[chunk:].contiguous(), cz[chunk:].contiguous(), g, prec, want_y=False)
    torch.cuda.synchronize()
    assert torch.equal(tex2, tex[chunk:])
