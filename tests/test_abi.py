"""CPU checks of the C-ABI library: it loads, exports every function the
header declares, and its host-only queries answer (no GPU work here)."""
import ctypes
import os
import re

import pytest

import paper_2509_20198_amd as ls
import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lidarscout.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ls_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(ls.LIB_PATH):
        pytest.fail("liblidarscout.so is not built (run __graft_entry__.build())")
    return ls.load_library()


def test_every_declared_symbol_exported(lib):
    names = _declared()
    assert len(names) >= 14
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(ls.EXPORTS)


def test_host_queries(lib):
    assert ls.num_params() == synth.N_PARAMS == 119844
    assert "gfx950" in ls.version()
    for rc in (0, -1, -2, -3, -4, -5, -6, -7):
        assert lib.ls_status_string(rc)
    g = ls.Grid(tiles_x=32, tiles_y=32)
    a = ls.workspace_bytes(ls.OP_RECON, g, 1024, 541141)
    b = ls.workspace_bytes(ls.OP_RECON, g, 1024, 2 * 541141)
    assert 0 < a < b
    f32 = ls.act_bytes(g, 1024, ls.FP32)
    assert f32 == 2 * ls.act_bytes(g, 1024, ls.BF16)
    # 110 R^2 activation values per tile
    assert f32 == 1024 * 110 * 96 * 96 * 4
    assert ls.workspace_bytes(ls.OP_BACKWARD, g, 4, 0, ls.FP32) > ls.workspace_bytes(ls.OP_REFINE, g, 4, 0, ls.FP32)


def test_grid_validation(lib):
    bad = [ls.Grid(res=63), ls.Grid(pad=15, res=64), ls.Grid(tile_size=64001), ls.Grid(tiles_x=0),
           ls.Grid(tile_size=600000, pad=16)]
    for g in bad:
        assert ls.workspace_bytes(ls.OP_RECON, g, 1, 1) == 0
    # entry points reject invalid arguments on the host, before touching the GPU
    gc = ls.Grid(res=63).c()
    rc = lib.ls_recon_tiles(ctypes.byref(gc), None, None, None, None, 0, None, 0, 0, None, None, None, None, 0,
                            None, None, 0, None)
    assert rc == ls.LS_ERANGE
    gc = ls.Grid().c()
    rc = lib.ls_recon_tiles(ctypes.byref(gc), None, None, None, None, 10, None, 1, 0, None, None, None, None, 0,
                            None, None, 0, None)
    assert rc == ls.LS_EINVAL
    # an unknown processing order
    rc = lib.ls_recon_tiles(ctypes.byref(gc), None, None, None, None, 0, None, 0, 2, None, None, None, None, 0,
                            None, None, 0, None)
    assert rc == ls.LS_ERANGE
    rc = lib.ls_refine_tiles(None, None, 7, None, None, 1, ctypes.byref(gc), None, None, None, None, 0, None)
    assert rc == ls.LS_ERANGE
    rc = lib.ls_splat_points(ctypes.byref(gc), None, None, None, None, 5, None, 1, None, None, None, None)
    assert rc == ls.LS_EINVAL
    assert lib.ls_set_conv_config(99, 0, 0, 0) == ls.LS_ERANGE
    rc = lib.ls_splat_mean(ctypes.byref(gc), None, None, None, None, 5, None, 1, None, None, None)
    assert rc == ls.LS_EINVAL
    rc = lib.ls_resolve_mean(ctypes.byref(gc), None, 2, None, None)
    assert rc == ls.LS_EINVAL
    rc = lib.ls_target_loss(None, None, None, 1, ctypes.byref(gc), 2, None, None, None, 0, None)
    assert rc == ls.LS_ERANGE
    rc = lib.ls_target_loss(None, None, None, 1, ctypes.byref(gc), ls.LOSS_L1, None, None, None, 0, None)
    assert rc == ls.LS_EINVAL
    assert ls.workspace_bytes(ls.OP_LOSS, ls.Grid(), 4) > 0
    v = ls.View(m=[1.0] * 16, width=0, height=4).c()
    assert lib.ls_raster_points(ctypes.byref(v), None, None, None, None, 0, None, None, None) == ls.LS_ERANGE
    v = ls.View(m=[1.0] * 16, width=4, height=4).c()
    assert lib.ls_raster_points(ctypes.byref(v), None, None, None, None, 3, None, None, None) == ls.LS_EINVAL
    assert lib.ls_raster_points(None, None, None, None, None, 0, None, None, None) == ls.LS_EINVAL
    assert lib.ls_raster_resolve(None, 5, None, None) == ls.LS_EINVAL
    gc = ls.Grid(pad=2).c()  # R = 68, not a multiple of 16
    assert lib.ls_lsnet_num_params(ctypes.byref(gc)) == -1
    assert lib.ls_lsnet_refine_tiles(None, 0, 15, None, None, 0, ctypes.byref(gc), None, None, None, 0, None) == \
        ls.LS_ERANGE
    gc = ls.Grid().c()
    assert lib.ls_lsnet_refine_tiles(None, 0, 15, None, None, 2, ctypes.byref(gc), None, None, None, 0, None) == \
        ls.LS_EINVAL
    assert lib.ls_lsnet_refine_tiles(None, 3, 15, None, None, 0, ctypes.byref(gc), None, None, None, 0, None) == \
        ls.LS_ERANGE
    for bad in (0, 16, -1):
        assert lib.ls_lsnet_refine_tiles(None, 0, bad, None, None, 0, ctypes.byref(gc), None, None, None, 0,
                                         None) == ls.LS_ERANGE


def test_lsnet_parameter_count(lib):
    """The library's layer table of the paper's network agrees with the
    weight generator's (and so with the oracle's) at every padded side."""
    for res, pad in ((64, 16), (64, 0), (16, 8), (32, 16)):
        g = ls.Grid(res=res, pad=pad, tile_size=res * 1000)
        assert ls.lsnet_num_params(g) == synth.pnet_weights(0, R=res + 2 * pad).size
    assert ls.lsnet_num_params(ls.Grid()) == 2_528_708
    for prec in (ls.FP32, ls.BF16):
        a = ls.workspace_bytes(ls.OP_REFINE_LSNET, ls.Grid(), 8, 0, prec)
        b = ls.workspace_bytes(ls.OP_REFINE_LSNET, ls.Grid(), 4096, 0, prec)
        assert 0 < a < b
    # bounded: the batch is taken in chunks
    assert ls.workspace_bytes(ls.OP_REFINE_LSNET, ls.Grid(), 16384, 0, ls.BF16) == \
        ls.workspace_bytes(ls.OP_REFINE_LSNET, ls.Grid(), 4096, 0, ls.BF16)


def test_python_binding_rejects_cpu_tensors(lib):
    import torch
    g = ls.Grid()
    x = torch.zeros(4, dtype=torch.int32)
    with pytest.raises(ValueError):
        ls.recon_tiles(g, x, x, x, torch.zeros((4, 3), dtype=torch.int16), torch.zeros(1, dtype=torch.int32))
