"""MI355X (gfx950) per-tile heightmap library: Python binding.

Thin ctypes layer over liblidarscout.so (C-ABI in include/lidarscout.h).
Each function takes torch tensors that live on the current HIP device,
checks their dtypes and shapes on the host (so no kernel is launched on
inconsistent operands), allocates missing outputs with torch, and calls the
entry point of the same name on torch's current stream.  Every step of the
hot path runs in the library's HIP kernels; there is no fallback: if the
library is missing or no GPU is present, the calls raise.
"""
from __future__ import annotations

import ctypes
import os
import threading
from dataclasses import dataclass

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblidarscout.so")

LS_OK, LS_EINVAL, LS_ERANGE, LS_EHIP, LS_ENOTIMPL, LS_EWORKSPACE, LS_ECAP, LS_ESCRATCH = 0, -1, -2, -3, -4, -5, -6, -7
RECON_SCRATCH_BYTES = 48 << 20  # LS_RECON_SCRATCH_BYTES
TILE_EMPTY, TILE_NN_ONLY, TILE_CAP, TILE_DEGENERATE, TILE_BADID = 1, 2, 4, 8, 16
FP32, BF16 = 0, 1
OP_RECON, OP_REFINE, OP_BACKWARD, OP_SPLAT, OP_LOSS, OP_REFINE_LSNET = 0, 1, 2, 3, 4, 5
LOSS_CLIPPED_MSE, LOSS_L1 = 0, 1
IN_HLIN, IN_HNN, IN_RGBLIN, IN_RGBNN, IN_ALL = 1, 2, 4, 8, 15
IN_HM_ONLY, IN_NN_ONLY, IN_LIN_ONLY = IN_HLIN | IN_HNN, IN_HNN | IN_RGBNN, IN_HLIN | IN_RGBLIN
ORDER_LIST, ORDER_LONGEST_FIRST = 0, 1

EXPORTS = [
    "ls_num_params", "ls_workspace_bytes", "ls_act_bytes", "ls_recon_tiles", "ls_recon_tiles_noalloc",
    "ls_refine_tiles",
    "ls_refine_backward", "ls_splat_points", "ls_resolve_keys", "ls_pack_weights_bf16",
    "ls_conv_num_configs", "ls_set_conv_config", "ls_get_conv_config", "ls_status_string",
    "ls_last_error", "ls_version", "ls_trace_enable", "ls_trace_count", "ls_trace_record",
    "ls_splat_mean", "ls_resolve_mean", "ls_target_loss", "ls_raster_points", "ls_raster_resolve",
    "ls_lsnet_num_params", "ls_lsnet_refine_tiles",
]


class LsGrid(ctypes.Structure):
    _fields_ = [("origin_x", ctypes.c_int64), ("origin_y", ctypes.c_int64), ("tile_size", ctypes.c_int32),
                ("res", ctypes.c_int32), ("pad", ctypes.c_int32), ("tiles_x", ctypes.c_int32),
                ("tiles_y", ctypes.c_int32), ("scale_xy", ctypes.c_double), ("scale_z", ctypes.c_double),
                ("offset_z", ctypes.c_double)]


class LsView(ctypes.Structure):
    _fields_ = [("m", ctypes.c_double * 16), ("origin_x", ctypes.c_int64), ("origin_y", ctypes.c_int64),
                ("scale_xy", ctypes.c_double), ("scale_z", ctypes.c_double), ("offset_z", ctypes.c_double),
                ("width", ctypes.c_int32), ("height", ctypes.c_int32)]


@dataclass
class Grid:
    """Region and tiling (mirror of ls_grid)."""
    origin_x: int = 0
    origin_y: int = 0
    tile_size: int = 64000
    res: int = 64
    pad: int = 16
    tiles_x: int = 1
    tiles_y: int = 1
    scale_xy: float = 0.01
    scale_z: float = 0.01
    offset_z: float = 0.0

    @property
    def R(self) -> int:
        return self.res + 2 * self.pad

    @classmethod
    def of(cls, g) -> "Grid":
        return cls(**{k: getattr(g, k) for k in cls.__dataclass_fields__})

    def c(self) -> LsGrid:
        return LsGrid(self.origin_x, self.origin_y, self.tile_size, self.res, self.pad, self.tiles_x, self.tiles_y,
                      self.scale_xy, self.scale_z, self.offset_z)


_lock = threading.Lock()
_lib = None


class LidarScoutError(RuntimeError):
    pass


def load_library(path: str = LIB_PATH):
    """Load liblidarscout.so; raises if it is missing (there is no fallback)."""
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(path):
            raise LidarScoutError(f"{path} is not built; run __graft_entry__.build() or "
                                  "python paper_2509_20198_amd/build.py")
        lib = ctypes.CDLL(path)
        P, i32, i64, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
        G = ctypes.POINTER(LsGrid)
        lib.ls_num_params.restype = ctypes.c_int
        lib.ls_workspace_bytes.restype = sz
        lib.ls_workspace_bytes.argtypes = [ctypes.c_int, G, i32, i64, ctypes.c_int]
        lib.ls_act_bytes.restype = sz
        lib.ls_act_bytes.argtypes = [G, i32, ctypes.c_int]
        lib.ls_recon_tiles.restype = ctypes.c_int
        lib.ls_recon_tiles.argtypes = [G, P, P, P, P, i64, P, i32, i32, P, P, P, P, i64, P, P, sz, P]
        lib.ls_recon_tiles_noalloc.restype = ctypes.c_int
        lib.ls_recon_tiles_noalloc.argtypes = [G, P, P, P, P, i64, P, i32, i32, P, P, P, P, i64, P, P]
        lib.ls_refine_tiles.restype = ctypes.c_int
        lib.ls_refine_tiles.argtypes = [P, P, ctypes.c_int, P, P, i32, G, P, P, P, P, sz, P]
        lib.ls_refine_backward.restype = ctypes.c_int
        lib.ls_refine_backward.argtypes = [P, P, ctypes.c_int, P, P, P, i32, G, P, P, P, sz, P]
        lib.ls_splat_points.restype = ctypes.c_int
        lib.ls_splat_points.argtypes = [G, P, P, P, P, i64, P, i32, P, P, P, P]
        lib.ls_resolve_keys.restype = ctypes.c_int
        lib.ls_resolve_keys.argtypes = [G, P, i32, P, P]
        lib.ls_splat_mean.restype = ctypes.c_int
        lib.ls_splat_mean.argtypes = [G, P, P, P, P, i64, P, i32, P, P, P]
        lib.ls_resolve_mean.restype = ctypes.c_int
        lib.ls_resolve_mean.argtypes = [G, P, i32, P, P]
        lib.ls_target_loss.restype = ctypes.c_int
        lib.ls_target_loss.argtypes = [P, P, P, i32, G, ctypes.c_int, P, P, P, sz, P]
        lib.ls_raster_points.restype = ctypes.c_int
        lib.ls_raster_points.argtypes = [ctypes.POINTER(LsView), P, P, P, P, i64, P, P, P]
        lib.ls_raster_resolve.restype = ctypes.c_int
        lib.ls_raster_resolve.argtypes = [P, i64, P, P]
        lib.ls_lsnet_num_params.restype = i64
        lib.ls_lsnet_num_params.argtypes = [G]
        lib.ls_lsnet_refine_tiles.restype = ctypes.c_int
        lib.ls_lsnet_refine_tiles.argtypes = [P, ctypes.c_int, i32, P, P, i32, G, P, P, P, sz, P]
        lib.ls_pack_weights_bf16.restype = ctypes.c_int
        lib.ls_pack_weights_bf16.argtypes = [P, P, P]
        lib.ls_conv_num_configs.restype = ctypes.c_int
        lib.ls_conv_num_configs.argtypes = [ctypes.c_int] * 3
        lib.ls_set_conv_config.restype = ctypes.c_int
        lib.ls_set_conv_config.argtypes = [ctypes.c_int] * 4
        lib.ls_get_conv_config.restype = ctypes.c_int
        lib.ls_get_conv_config.argtypes = [ctypes.c_int] * 3
        lib.ls_status_string.restype = ctypes.c_char_p
        lib.ls_status_string.argtypes = [ctypes.c_int]
        lib.ls_last_error.restype = ctypes.c_char_p
        lib.ls_version.restype = ctypes.c_char_p
        lib.ls_trace_enable.restype = ctypes.c_int
        lib.ls_trace_enable.argtypes = [ctypes.c_int]
        lib.ls_trace_count.restype = ctypes.c_int
        lib.ls_trace_record.restype = ctypes.c_int
        lib.ls_trace_record.argtypes = [ctypes.c_int, ctypes.POINTER(ctypes.c_char_p), ctypes.POINTER(ctypes.c_float)]
        _lib = lib
        return lib


def _check(rc: int, what: str):
    if rc != LS_OK:
        lib = load_library()
        msg = lib.ls_status_string(rc).decode()
        if rc == LS_EHIP:
            msg += ": " + lib.ls_last_error().decode()
        raise LidarScoutError(f"{what} failed ({rc}): {msg}")


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _need(t: torch.Tensor, name: str, dtypes, numel=None, shape=None):
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must be on the GPU")
    if t.dtype not in dtypes:
        raise TypeError(f"{name}: dtype {t.dtype} not in {dtypes}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if numel is not None and t.numel() < numel:
        raise ValueError(f"{name} holds {t.numel()} elements, needs {numel}")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")


U16 = (torch.int16, torch.uint16)


def num_params() -> int:
    return load_library().ls_num_params()


def version() -> str:
    return load_library().ls_version().decode()


def workspace_bytes(op: int, grid: Grid, n_tiles: int, n_points: int = 0, precision: int = FP32) -> int:
    g = Grid.of(grid).c()
    return int(load_library().ls_workspace_bytes(op, ctypes.byref(g), n_tiles, n_points, precision))


def act_bytes(grid: Grid, n_tiles: int, precision: int = FP32) -> int:
    g = Grid.of(grid).c()
    return int(load_library().ls_act_bytes(ctypes.byref(g), n_tiles, precision))


def alloc_workspace(nbytes: int, device=None) -> torch.Tensor:
    return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device or "cuda")


def recon_tiles(grid, x, y, z, rgb, tile_list, *, order: int = ORDER_LIST, x_out=None, cz_out=None, bin_off=None,
                bin_idx=None, bin_cap: int = 0, status=None, ws=None, stream=None):
    """Binning + Algorithm 1 + normalisation -> (x_out [n,R,R,8] f32, cz [n] f64, status [n] i32).

    order: ORDER_LIST processes the tiles in tile_list order (viewpoint
    priority), ORDER_LONGEST_FIRST by descending window point count."""
    lib = load_library()
    g = Grid.of(grid)
    n = x.numel()
    nt = tile_list.numel()
    for name, t in (("x", x), ("y", y), ("z", z)):
        _need(t, name, (torch.int32,), shape=(n,))
    _need(rgb, "rgb", U16, shape=(n, 3))
    _need(tile_list, "tile_list", (torch.int32,))
    dev = x.device
    R = g.R
    if x_out is None:
        x_out = torch.empty((nt, R, R, 8), dtype=torch.float32, device=dev)
    if cz_out is None:
        cz_out = torch.empty(nt, dtype=torch.float64, device=dev)
    if status is None:
        status = torch.empty(nt, dtype=torch.int32, device=dev)
    _need(x_out, "x_out", (torch.float32,), shape=(nt, R, R, 8))
    _need(cz_out, "cz_out", (torch.float64,), shape=(nt,))
    _need(status, "status", (torch.int32,), shape=(nt,))
    if (bin_off is None) != (bin_idx is None):
        raise ValueError("bin_off and bin_idx go together")
    if bin_off is not None:
        _need(bin_off, "bin_off", (torch.int32,), shape=(nt + 1,))
        _need(bin_idx, "bin_idx", (torch.int32,))
        bin_cap = min(int(bin_cap) if bin_cap else bin_idx.numel(), bin_idx.numel())
    need = workspace_bytes(OP_RECON, g, nt, n)
    if ws is None:
        ws = alloc_workspace(need, dev)
    _need(ws, "ws", (torch.uint8,), numel=need)
    gc = g.c()
    rc = lib.ls_recon_tiles(ctypes.byref(gc), _ptr(x), _ptr(y), _ptr(z), _ptr(rgb), n, _ptr(tile_list), nt,
                            int(order), _ptr(x_out), _ptr(cz_out), _ptr(bin_off), _ptr(bin_idx), int(bin_cap), _ptr(status),
                            _ptr(ws), ws.numel(), _stream(stream))
    _check(rc, "ls_recon_tiles")
    return x_out, cz_out, status


def recon_tiles_noalloc(grid, x, y, z, rgb, tile_list, *, order: int = ORDER_LIST, x_out=None, cz_out=None,
                        bin_off=None, bin_idx=None, bin_cap: int = 0, status=None, stream=None):
    """recon_tiles through the allocation-free entry point (no workspace: the
    library's fixed device scratch).  Outputs the caller does not pass are
    allocated here with torch, before the call."""
    lib = load_library()
    g = Grid.of(grid)
    n = x.numel()
    nt = tile_list.numel()
    for name, t in (("x", x), ("y", y), ("z", z)):
        _need(t, name, (torch.int32,), shape=(n,))
    _need(rgb, "rgb", U16, shape=(n, 3))
    _need(tile_list, "tile_list", (torch.int32,))
    dev = x.device
    R = g.R
    if x_out is None:
        x_out = torch.empty((nt, R, R, 8), dtype=torch.float32, device=dev)
    if cz_out is None:
        cz_out = torch.empty(nt, dtype=torch.float64, device=dev)
    if status is None:
        status = torch.empty(nt, dtype=torch.int32, device=dev)
    _need(x_out, "x_out", (torch.float32,), shape=(nt, R, R, 8))
    _need(cz_out, "cz_out", (torch.float64,), shape=(nt,))
    _need(status, "status", (torch.int32,), shape=(nt,))
    if (bin_off is None) != (bin_idx is None):
        raise ValueError("bin_off and bin_idx go together")
    if bin_off is not None:
        _need(bin_off, "bin_off", (torch.int32,), shape=(nt + 1,))
        _need(bin_idx, "bin_idx", (torch.int32,))
        bin_cap = min(int(bin_cap) if bin_cap else bin_idx.numel(), bin_idx.numel())
    gc = g.c()
    rc = lib.ls_recon_tiles_noalloc(ctypes.byref(gc), _ptr(x), _ptr(y), _ptr(z), _ptr(rgb), n, _ptr(tile_list), nt,
                                    int(order), _ptr(x_out), _ptr(cz_out), _ptr(bin_off), _ptr(bin_idx),
                                    int(bin_cap), _ptr(status), _stream(stream))
    _check(rc, "ls_recon_tiles_noalloc")
    return x_out, cz_out, status


def pack_weights_bf16(w: torch.Tensor, out=None, stream=None) -> torch.Tensor:
    P = num_params()
    _need(w, "w", (torch.float32,), shape=(P,))
    if out is None:
        out = torch.empty(P, dtype=torch.int16, device=w.device)
    _need(out, "w_bf16", U16, shape=(P,))
    _check(load_library().ls_pack_weights_bf16(_ptr(w), _ptr(out), _stream(stream)), "ls_pack_weights_bf16")
    return out


def refine_tiles(w, x, cz, grid, precision: int = FP32, *, w_bf16=None, y_out=None, tex_out=None,
                 want_y: bool = True, want_tex: bool = True, act_save=None, ws=None, stream=None):
    """Refinement network forward -> (y [n,res,res,4], tex [n,res,res,4]) (either may be None)."""
    lib = load_library()
    g = Grid.of(grid)
    P = num_params()
    nt = x.shape[0]
    R, res = g.R, g.res
    _need(w, "w", (torch.float32,), shape=(P,))
    _need(x, "x", (torch.float32,), shape=(nt, R, R, 8))
    if precision == BF16:
        if w_bf16 is None:
            raise ValueError("BF16 needs w_bf16 (pack_weights_bf16)")
        _need(w_bf16, "w_bf16", U16, shape=(P,))
    dev = x.device
    if y_out is None and want_y:
        y_out = torch.empty((nt, res, res, 4), dtype=torch.float32, device=dev)
    if tex_out is None and want_tex:
        tex_out = torch.empty((nt, res, res, 4), dtype=torch.float32, device=dev)
    if y_out is not None:
        _need(y_out, "y_out", (torch.float32,), shape=(nt, res, res, 4))
    if tex_out is not None:
        _need(tex_out, "tex_out", (torch.float32,), shape=(nt, res, res, 4))
        _need(cz, "cz", (torch.float64,), shape=(nt,))
    if act_save is not None:
        _need(act_save, "act_save", (torch.uint8,), numel=act_bytes(g, nt, precision))
    need = workspace_bytes(OP_REFINE, g, nt, 0, precision)
    if ws is None:
        ws = alloc_workspace(need, dev)
    _need(ws, "ws", (torch.uint8,), numel=need)
    gc = g.c()
    rc = lib.ls_refine_tiles(_ptr(w), _ptr(w_bf16) if precision == BF16 else None, precision, _ptr(x),
                             _ptr(cz), nt, ctypes.byref(gc), _ptr(y_out), _ptr(tex_out), _ptr(act_save), _ptr(ws),
                             ws.numel(), _stream(stream))
    _check(rc, "ls_refine_tiles")
    return y_out, tex_out


def lsnet_num_params(grid) -> int:
    """Parameters of the paper's refinement network at the grid's padded side (2,528,708 at 96)."""
    g = Grid.of(grid).c()
    n = int(load_library().ls_lsnet_num_params(ctypes.byref(g)))
    if n < 0:
        raise LidarScoutError("the paper's network needs res + 2*pad divisible by 16")
    return n


def lsnet_refine_tiles(w, x, cz, grid, precision: int = FP32, *, inputs: int = IN_ALL, y_out=None, tex_out=None,
                       want_y: bool = True, want_tex: bool = True, ws=None, stream=None):
    """The paper's refinement network forward -> (y [n,res,res,4], tex [n,res,res,4]) (either may be None).

    inputs: IN_* bits of the maps the network sees (IN_HM_ONLY, IN_NN_ONLY, IN_LIN_ONLY for the
    ablation variants); absent inputs read as zero."""
    lib = load_library()
    g = Grid.of(grid)
    P = lsnet_num_params(g)
    nt = x.shape[0]
    R, res = g.R, g.res
    _need(w, "w", (torch.float32,), shape=(P,))
    _need(x, "x", (torch.float32,), shape=(nt, R, R, 8))
    dev = x.device
    if y_out is None and want_y:
        y_out = torch.empty((nt, res, res, 4), dtype=torch.float32, device=dev)
    if tex_out is None and want_tex:
        tex_out = torch.empty((nt, res, res, 4), dtype=torch.float32, device=dev)
    if y_out is not None:
        _need(y_out, "y_out", (torch.float32,), shape=(nt, res, res, 4))
    if tex_out is not None:
        _need(tex_out, "tex_out", (torch.float32,), shape=(nt, res, res, 4))
        _need(cz, "cz", (torch.float64,), shape=(nt,))
    need = workspace_bytes(OP_REFINE_LSNET, g, nt, 0, precision)
    if ws is None:
        ws = alloc_workspace(need, dev)
    _need(ws, "ws", (torch.uint8,), numel=need)
    gc = g.c()
    rc = lib.ls_lsnet_refine_tiles(_ptr(w), precision, int(inputs), _ptr(x), _ptr(cz), nt, ctypes.byref(gc), _ptr(y_out),
                                   _ptr(tex_out), _ptr(ws), ws.numel(), _stream(stream))
    _check(rc, "ls_lsnet_refine_tiles")
    return y_out, tex_out


def refine_backward(w, x, grad_y, grid, precision: int = FP32, *, w_bf16=None, act_save=None, grad_w=None,
                    want_grad_x: bool = False, grad_x=None, ws=None, stream=None):
    """Backward of refine_tiles -> (grad_w [P], grad_x [n,R,R,8] or None)."""
    lib = load_library()
    g = Grid.of(grid)
    P = num_params()
    nt = x.shape[0]
    R, res = g.R, g.res
    _need(w, "w", (torch.float32,), shape=(P,))
    _need(x, "x", (torch.float32,), shape=(nt, R, R, 8))
    _need(grad_y, "grad_y", (torch.float32,), shape=(nt, res, res, 4))
    if precision == BF16:
        if w_bf16 is None:
            raise ValueError("BF16 needs w_bf16")
        _need(w_bf16, "w_bf16", U16, shape=(P,))
    dev = x.device
    if grad_w is None:
        grad_w = torch.empty(P, dtype=torch.float32, device=dev)
    _need(grad_w, "grad_w", (torch.float32,), shape=(P,))
    if want_grad_x and grad_x is None:
        grad_x = torch.empty_like(x)
    if grad_x is not None:
        _need(grad_x, "grad_x", (torch.float32,), shape=(nt, R, R, 8))
    if act_save is not None:
        _need(act_save, "act_save", (torch.uint8,), numel=act_bytes(g, nt, precision))
    need = workspace_bytes(OP_BACKWARD, g, nt, 0, precision)
    if ws is None:
        ws = alloc_workspace(need, dev)
    _need(ws, "ws", (torch.uint8,), numel=need)
    gc = g.c()
    rc = lib.ls_refine_backward(_ptr(w), _ptr(w_bf16) if precision == BF16 else None, precision, _ptr(x),
                                _ptr(act_save), _ptr(grad_y), nt, ctypes.byref(gc), _ptr(grad_w), _ptr(grad_x),
                                _ptr(ws), ws.numel(), _stream(stream))
    _check(rc, "ls_refine_backward")
    return grad_w, grad_x


class RefineFn(torch.autograd.Function):
    """y = refine(x; w) as an autograd op over ls_refine_tiles / ls_refine_backward.

    RefineFn.apply(x, w, grid, precision, save_acts) -> y [n, res, res, 4]
    (normalised).  save_acts=False keeps no activations between forward and
    backward: the backward recomputes the forward (activation recomputation,
    for batches whose activations do not fit).  BF16 packs the weights on
    every forward, so optimiser updates of w are seen."""

    @staticmethod
    def forward(ctx, x, w, grid, precision=FP32, save_acts=True):
        g = Grid.of(grid)
        x = x.contiguous()
        wb = pack_weights_bf16(w) if precision == BF16 else None
        act = None
        if save_acts:
            act = torch.empty(act_bytes(g, x.shape[0], precision), dtype=torch.uint8, device=x.device)
        y, _ = refine_tiles(w, x, None, g, precision, w_bf16=wb, act_save=act, want_tex=False)
        ctx.save_for_backward(x, w)
        ctx.grid, ctx.precision, ctx.wb, ctx.act = g, precision, wb, act
        return y

    @staticmethod
    def backward(ctx, grad_y):
        x, w = ctx.saved_tensors
        gw, gx = refine_backward(w, x, grad_y.contiguous(), ctx.grid, ctx.precision, w_bf16=ctx.wb,
                                 act_save=ctx.act, want_grad_x=bool(ctx.needs_input_grad[0]))
        ctx.act = None
        return gx, gw, None, None, None


def splat_points(grid, x, y, z, rgb, tile_slot, n_slots: int, keys=None, tex_inout=None, n_dropped=None,
                 stream=None):
    """Max-key splat of full-resolution points -> (keys [n_slots,res,res] int64 bits, n_dropped [1])."""
    lib = load_library()
    g = Grid.of(grid)
    n = x.numel()
    for name, t in (("x", x), ("y", y), ("z", z)):
        _need(t, name, (torch.int32,), shape=(n,))
    _need(rgb, "rgb", U16, shape=(n, 3))
    _need(tile_slot, "tile_slot", (torch.int32,), shape=(g.tiles_x * g.tiles_y,))
    dev = x.device
    res = g.res
    if keys is None:
        keys = torch.zeros((n_slots, res, res), dtype=torch.int64, device=dev)
    _need(keys, "keys", (torch.int64, torch.uint64), shape=(n_slots, res, res))
    if n_dropped is None:
        n_dropped = torch.zeros(1, dtype=torch.int64, device=dev)
    _need(n_dropped, "n_dropped", (torch.int64, torch.uint64), shape=(1,))
    if tex_inout is not None:
        _need(tex_inout, "tex_inout", (torch.float32,), shape=(n_slots, res, res, 4))
    gc = g.c()
    rc = lib.ls_splat_points(ctypes.byref(gc), _ptr(x), _ptr(y), _ptr(z), _ptr(rgb), n, _ptr(tile_slot), n_slots,
                             _ptr(keys), _ptr(tex_inout), _ptr(n_dropped), _stream(stream))
    _check(rc, "ls_splat_points")
    return keys, n_dropped


def resolve_keys(grid, keys, tex_inout, stream=None):
    lib = load_library()
    g = Grid.of(grid)
    n_slots = keys.shape[0]
    _need(keys, "keys", (torch.int64, torch.uint64), shape=(n_slots, g.res, g.res))
    _need(tex_inout, "tex_inout", (torch.float32,), shape=(n_slots, g.res, g.res, 4))
    gc = g.c()
    _check(lib.ls_resolve_keys(ctypes.byref(gc), _ptr(keys), n_slots, _ptr(tex_inout), _stream(stream)),
           "ls_resolve_keys")
    return tex_inout


def splat_mean(grid, x, y, z, rgb, tile_slot, n_slots: int, acc=None, n_dropped=None, stream=None):
    """Ground-truth sums per texel -> (acc [n_slots,res,res,5] int64 = (sum z, sum R, sum G, sum B,
    count), n_dropped [1]); acc accumulates when given."""
    lib = load_library()
    g = Grid.of(grid)
    n = x.numel()
    for name, t in (("x", x), ("y", y), ("z", z)):
        _need(t, name, (torch.int32,), shape=(n,))
    _need(rgb, "rgb", U16, shape=(n, 3))
    _need(tile_slot, "tile_slot", (torch.int32,), shape=(g.tiles_x * g.tiles_y,))
    dev = x.device
    if acc is None:
        acc = torch.zeros((n_slots, g.res, g.res, 5), dtype=torch.int64, device=dev)
    _need(acc, "acc", (torch.int64,), shape=(n_slots, g.res, g.res, 5))
    if n_dropped is None:
        n_dropped = torch.zeros(1, dtype=torch.int64, device=dev)
    _need(n_dropped, "n_dropped", (torch.int64, torch.uint64), shape=(1,))
    gc = g.c()
    rc = lib.ls_splat_mean(ctypes.byref(gc), _ptr(x), _ptr(y), _ptr(z), _ptr(rgb), n, _ptr(tile_slot), n_slots,
                           _ptr(acc), _ptr(n_dropped), _stream(stream))
    _check(rc, "ls_splat_mean")
    return acc, n_dropped


def resolve_mean(grid, acc, tex=None, stream=None):
    """Mean texture [n_slots,res,res,4] (metres, [0, 1]; NaN where no point) from splat_mean sums."""
    lib = load_library()
    g = Grid.of(grid)
    n_slots = acc.shape[0]
    _need(acc, "acc", (torch.int64,), shape=(n_slots, g.res, g.res, 5))
    if tex is None:
        tex = torch.empty((n_slots, g.res, g.res, 4), dtype=torch.float32, device=acc.device)
    _need(tex, "tex", (torch.float32,), shape=(n_slots, g.res, g.res, 4))
    gc = g.c()
    _check(lib.ls_resolve_mean(ctypes.byref(gc), _ptr(acc), n_slots, _ptr(tex), _stream(stream)), "ls_resolve_mean")
    return tex


def target_loss(y, t, cz, grid, kind: int = LOSS_CLIPPED_MSE, *, want_grad: bool = True, loss_out=None, grad=None,
                ws=None, stream=None):
    """Training loss of the normalised output y against the target texture t (NaN = no target)
    -> (loss [3] float64 on the device = (L, L_h, L_rgb), dL/dy [n,res,res,4] or None)."""
    lib = load_library()
    g = Grid.of(grid)
    nt = y.shape[0]
    res = g.res
    _need(y, "y", (torch.float32,), shape=(nt, res, res, 4))
    _need(t, "t", (torch.float32,), shape=(nt, res, res, 4))
    _need(cz, "cz", (torch.float64,), shape=(nt,))
    dev = y.device
    if loss_out is None:
        loss_out = torch.empty(3, dtype=torch.float64, device=dev)
    _need(loss_out, "loss_out", (torch.float64,), shape=(3,))
    if grad is None and want_grad:
        grad = torch.empty_like(y)
    if grad is not None:
        _need(grad, "grad", (torch.float32,), shape=(nt, res, res, 4))
    need = workspace_bytes(OP_LOSS, g, nt)
    if ws is None:
        ws = alloc_workspace(need, dev)
    _need(ws, "ws", (torch.uint8,), numel=need)
    gc = g.c()
    rc = lib.ls_target_loss(_ptr(y), _ptr(t), _ptr(cz), nt, ctypes.byref(gc), int(kind), _ptr(loss_out), _ptr(grad),
                            _ptr(ws), ws.numel(), _stream(stream))
    _check(rc, "ls_target_loss")
    return loss_out, grad


@dataclass
class View:
    """Point-rasteriser view (mirror of ls_view): m is the 4 x 4 row-major view-projection on metres
    relative to (origin_x, origin_y)."""
    m: tuple
    origin_x: int = 0
    origin_y: int = 0
    scale_xy: float = 0.01
    scale_z: float = 0.01
    offset_z: float = 0.0
    width: int = 1024
    height: int = 1024

    def c(self) -> LsView:
        m = [float(v) for v in (self.m.reshape(-1) if hasattr(self.m, "reshape") else self.m)]
        if len(m) != 16:
            raise ValueError("view matrix must have 16 entries")
        return LsView((ctypes.c_double * 16)(*m), int(self.origin_x), int(self.origin_y), float(self.scale_xy),
                      float(self.scale_z), float(self.offset_z), int(self.width), int(self.height))


def raster_points(view: View, x, y, z, rgb, fb=None, n_drawn=None, stream=None):
    """Nearest point per pixel via packed 64-bit keys -> (fb [height,width] int64 bits, n_drawn [1]);
    a new fb starts all ones (empty), a given one accumulates."""
    lib = load_library()
    n = x.numel()
    for name, t in (("x", x), ("y", y), ("z", z)):
        _need(t, name, (torch.int32,), shape=(n,))
    _need(rgb, "rgb", U16, shape=(n, 3))
    dev = x.device
    if fb is None:
        fb = torch.full((view.height, view.width), -1, dtype=torch.int64, device=dev)
    _need(fb, "fb", (torch.int64, torch.uint64), shape=(view.height, view.width))
    if n_drawn is None:
        n_drawn = torch.zeros(1, dtype=torch.int64, device=dev)
    _need(n_drawn, "n_drawn", (torch.int64, torch.uint64), shape=(1,))
    vc = view.c()
    rc = lib.ls_raster_points(ctypes.byref(vc), _ptr(x), _ptr(y), _ptr(z), _ptr(rgb), n, _ptr(fb), _ptr(n_drawn),
                              _stream(stream))
    _check(rc, "ls_raster_points")
    return fb, n_drawn


def raster_resolve(fb, rgba=None, stream=None):
    """RGBA8 words [height,width] (int32 bits; 0 = empty pixel) of a raster_points frame buffer."""
    _need(fb, "fb", (torch.int64, torch.uint64))
    if rgba is None:
        rgba = torch.empty(fb.shape, dtype=torch.int32, device=fb.device)
    _need(rgba, "rgba", (torch.int32, torch.uint32), shape=tuple(fb.shape))
    _check(load_library().ls_raster_resolve(_ptr(fb), fb.numel(), _ptr(rgba), _stream(stream)), "ls_raster_resolve")
    return rgba


def set_conv_config(layer: int, precision: int, pass_: int, config: int):
    _check(load_library().ls_set_conv_config(layer, precision, pass_, config), "ls_set_conv_config")


def get_conv_config(layer: int, precision: int, pass_: int) -> int:
    return int(load_library().ls_get_conv_config(layer, precision, pass_))


def conv_num_configs(layer: int, precision: int, pass_: int) -> int:
    return int(load_library().ls_conv_num_configs(layer, precision, pass_))


def trace_enable(on: bool = True):
    """Bracket every kernel group the library enqueues with HIP events."""
    _check(load_library().ls_trace_enable(1 if on else 0), "ls_trace_enable")


def trace_records():
    """[(kernel group name, elapsed ms)] for the groups recorded since trace_enable."""
    lib = load_library()
    out = []
    for i in range(lib.ls_trace_count()):
        name = ctypes.c_char_p()
        ms = ctypes.c_float()
        _check(lib.ls_trace_record(i, ctypes.byref(name), ctypes.byref(ms)), "ls_trace_record")
        out.append((name.value.decode(), float(ms.value)))
    return out
