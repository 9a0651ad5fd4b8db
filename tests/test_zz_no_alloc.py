"""GPU: the allocation-free reconstruction entry point (fixed device scratch)
gives the same bits as ls_recon_tiles with a caller workspace, on two calls in
a row (the second smaller, so it runs over the first call's leftovers), in
both processing orders and with the CSR outputs; oversized inputs are refused
on the host."""
import ctypes

import numpy as np
import pytest
import torch

import paper_2509_20198_amd as ls
import synth
from gpu_helpers import points_to_dev

pytestmark = pytest.mark.gpu


def _both(w, order):
    g = ls.Grid.of(w.region)
    x, y, z, rgb = points_to_dev(w.points)
    tl = torch.from_numpy(w.tile_list).cuda()
    nt = tl.numel()
    cap = 4 * x.numel() + 1
    outs = []
    for fn in (ls.recon_tiles, ls.recon_tiles_noalloc):
        bo = torch.full((nt + 1,), -7, dtype=torch.int32, device="cuda")
        bi = torch.full((cap,), -7, dtype=torch.int32, device="cuda")
        xo, cz, st = fn(g, x, y, z, rgb, tl, order=order, bin_off=bo, bin_idx=bi, bin_cap=cap)
        torch.cuda.synchronize()
        m = int(bo[-1].item())
        outs.append((xo.cpu().numpy(), cz.cpu().numpy(), st.cpu().numpy(), bo.cpu().numpy(), bi[:m].cpu().numpy()))
    return outs


def _same(a, b):
    for u, v in zip(a, b):
        assert u.shape == v.shape
        assert np.array_equal(u.view(np.uint8), v.view(np.uint8))


@pytest.mark.parametrize("order", [ls.ORDER_LIST, ls.ORDER_LONGEST_FIRST])
def test_noalloc_equals_workspace_entry_two_calls(order):
    # 144 tiles, 78k points: more than the scratch holds with one workgroup per
    # tile slot, so the call runs on fewer workgroups; then two smaller inputs
    # over the leftovers of the previous call
    cases = [synth.batch_tiles(seed=23, tiles_x=12, tiles_y=12), synth.batch_tiles(seed=21, tiles_x=6, tiles_y=5),
             synth.batch_tiles(seed=22, tiles_x=2, tiles_y=3)]
    g0 = ls.Grid.of(cases[0].region)
    assert ls.workspace_bytes(ls.OP_RECON, g0, 144, cases[0].points.n) > ls.RECON_SCRATCH_BYTES
    assert cases[1].points.n < cases[0].points.n and cases[2].points.n < cases[1].points.n
    for w in cases:
        print(f"noalloc case: {w.tile_list.size} tiles, {w.points.n} points, order {order}", flush=True)
        ref, got = _both(w, order)
        _same(ref, got)
        assert (ref[2] & ~ls.TILE_NN_ONLY == 0).all()


def test_noalloc_refuses_oversized_input_on_the_host():
    g = ls.Grid(tiles_x=4, tiles_y=4)
    n = 200_000  # about 120 MB of workspace with one workgroup: beyond the 48 MiB scratch
    x = torch.zeros(n, dtype=torch.int32, device="cuda")
    rgb = torch.zeros((n, 3), dtype=torch.int16, device="cuda")
    tl = torch.arange(16, dtype=torch.int32, device="cuda")
    xo = torch.empty((16, 96, 96, 8), dtype=torch.float32, device="cuda")
    cz = torch.empty(16, dtype=torch.float64, device="cuda")
    st = torch.empty(16, dtype=torch.int32, device="cuda")
    lib = ls.load_library()
    gc = g.c()
    p = lambda t: ctypes.c_void_p(t.data_ptr())  # noqa: E731
    rc = lib.ls_recon_tiles_noalloc(ctypes.byref(gc), p(x), p(x), p(x), p(rgb), n, p(tl), 16, 0, p(xo), p(cz), None,
                                    None, 0, p(st), None)
    assert rc == ls.LS_ESCRATCH
    assert ls.workspace_bytes(ls.OP_RECON, g, 16, n) > ls.RECON_SCRATCH_BYTES
