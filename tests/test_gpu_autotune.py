"""Conv tilings and their autotuner: every tiling of a (layer, precision,
pass) computes the same result (bit-identical where the per-output
accumulation order is the same, close where the weight-gradient chunking
changes the summation), and the tuner applies and caches a valid choice."""
import json

import numpy as np
import pytest
import torch

import paper_2509_20198_amd as ls
import synth
from paper_2509_20198_amd import autotune as AT

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _reset_configs():
    yield
    for prec in (ls.FP32, ls.BF16):
        AT.reset(prec)


def _case(n=4):
    w = synth.batch_tiles(seed=3, tiles_x=2, tiles_y=2)
    g = ls.Grid.of(w.region)
    ps = w.points
    tl = torch.from_numpy(w.tile_list).cuda()
    x, cz, _ = ls.recon_tiles(g, ps.x.cuda(), ps.y.cuda(), ps.z.cuda(), ps.rgb_u16().cuda(), tl)
    wt = torch.from_numpy(synth.unet_weights(1, head_std=0.05, bias_std=0.05).astype(np.float32)).cuda()
    gy = torch.randn((x.shape[0], 64, 64, 4), device="cuda", generator=torch.Generator(device="cuda").manual_seed(1))
    return g, x, cz, wt, gy


def _run(g, x, wt, gy, prec):
    wb = ls.pack_weights_bf16(wt) if prec == ls.BF16 else None
    y, _ = ls.refine_tiles(wt, x, None, g, prec, w_bf16=wb, want_tex=False)
    gw, gx = ls.refine_backward(wt, x, gy, g, prec, w_bf16=wb, want_grad_x=True)
    torch.cuda.synchronize()
    return y.cpu().numpy(), gw.cpu().numpy(), gx.cpu().numpy()


@pytest.mark.parametrize("prec", [ls.FP32, ls.BF16])
def test_all_tilings_agree(prec):
    g, x, cz, wt, gy = _case()
    y0, gw0, gx0 = _run(g, x, wt, gy, prec)
    for p in (0, 1, 2):
        n = max(ls.conv_num_configs(l, prec, p) for l in range(11))
        for c in range(n):
            AT.reset(prec)
            for l in range(11):
                if c < ls.conv_num_configs(l, prec, p):
                    ls.set_conv_config(l, prec, p, c)
            y, gw, gx = _run(g, x, wt, gy, prec)
            assert np.array_equal(y, y0), (p, c)
            assert np.array_equal(gx, gx0), (p, c)
            # chunked weight-gradient sums: same terms, other grouping (the
            # input-gradient tiling of the head and dec1b also decides whether
            # decoder level 1 runs on windows, which regroups its sums)
            if p in (1, 2):
                assert np.linalg.norm(gw - gw0) <= 1e-5 * np.linalg.norm(gw0), (p, c)
            else:
                assert np.array_equal(gw, gw0), (p, c)


def test_autotune_applies_and_caches(tmp_path):
    g, x, cz, wt, gy = _case()
    path = str(tmp_path / "tune.json")
    r = AT.autotune(g, 16, ls.BF16, passes=(0, 1, 2), reps=2, cache_path=path)
    assert not r["cached"] and r["ms_tuned"] > 0
    for k, c in r["choice"].items():
        layer, p = (int(v) for v in k.split(","))
        assert -1 <= c < ls.conv_num_configs(layer, ls.BF16, p)
        assert ls.get_conv_config(layer, ls.BF16, p) == c
    # the defaults are kept unless the tuned set is faster
    if r["kept_default"]:
        assert r["ms_tuned"] == r["ms_default"] and all(c == -1 for c in r["choice"].values())
    else:
        assert r["ms_tuned"] < r["ms_default"]
    assert r["key"] in json.load(open(path))
    assert AT.library_hash() in r["key"]
    AT.reset(ls.BF16)
    r2 = AT.autotune(g, 16, ls.BF16, passes=(0, 1, 2), cache_path=path)
    assert r2["cached"] and r2["choice"] == r["choice"]
    for k, c in r2["choice"].items():
        layer, p = (int(v) for v in k.split(","))
        assert ls.get_conv_config(layer, ls.BF16, p) == c
