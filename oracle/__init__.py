"""FP64 CPU oracle for the LidarScout heightmap hot path (ctypes binding).

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the benchmark's
CPU-baseline leg are the only callers.  The product path never imports this
package.  The C sources beside this file are built with gcc (no HIP headers,
no shared code with the GPU library).

Functions mirror the C entry points; arrays are NumPy, sizes are derived
from them.  Each docstring names the part of the paper it follows.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# LS_ORACLE_LIB loads another, already built copy of the same sources (the
# sanitizer build that a test makes with build_sanitized); nothing rebuilds it
_LIB_ENV = os.environ.get("LS_ORACLE_LIB")
_LIB_PATH = _LIB_ENV or os.path.join(_HERE, "liboracle.so")
_SOURCES = ["ora_recon.c", "ora_unet.c", "ora_splat.c", "ora_target.c", "ora_raster.c", "ora_pnet.c"]
_lock = threading.Lock()
_lib = None

ORA_OK, ORA_EMPTY, ORA_NN_ONLY = 0, 1, 2


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (FP64, no FMA contraction, OpenMP)."""
    srcs = [os.path.join(_HERE, s) for s in _SOURCES]
    if not force and os.path.exists(_LIB_PATH):
        if all(os.path.getmtime(_LIB_PATH) >= os.path.getmtime(s) for s in srcs):
            return _LIB_PATH
    tmp = _LIB_PATH + f".tmp{os.getpid()}"
    cmd = ["gcc", "-O2", "-std=gnu11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
           "-fno-fast-math", "-o", tmp] + srcs
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def build_sanitized(path: str) -> str:
    """The same sources with AddressSanitizer and UndefinedBehaviorSanitizer
    (every finding fatal), for tests that run the oracle under them."""
    srcs = [os.path.join(_HERE, s) for s in _SOURCES]
    cmd = ["gcc", "-O1", "-g", "-std=gnu11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
           "-fno-omit-frame-pointer", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
           "-o", path] + srcs
    subprocess.run(cmd, check=True)
    return path


class _Grid(ctypes.Structure):
    _fields_ = [("origin_x", ctypes.c_int64), ("origin_y", ctypes.c_int64),
                ("tile_size", ctypes.c_int32), ("res", ctypes.c_int32), ("pad", ctypes.c_int32),
                ("tiles_x", ctypes.c_int32), ("tiles_y", ctypes.c_int32),
                ("scale_xy", ctypes.c_double), ("scale_z", ctypes.c_double), ("offset_z", ctypes.c_double)]


class _Pt(ctypes.Structure):
    _fields_ = [("u", ctypes.c_int64), ("v", ctypes.c_int64), ("z", ctypes.c_int32),
                ("rgb", ctypes.c_int32 * 3)]


PT_DTYPE = np.dtype([("u", np.int64), ("v", np.int64), ("z", np.int32), ("rgb", np.int32, (3,))], align=True)
assert PT_DTYPE.itemsize == ctypes.sizeof(_Pt)


def _load():
    global _lib
    with _lock:
        if _lib is None:
            if not _LIB_ENV:
                build(force=False)
            lib = ctypes.CDLL(_LIB_PATH)
            P = ctypes.c_void_p
            i32, i64, u64, dbl = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64, ctypes.c_double
            lib.ora_bin.restype = i64
            lib.ora_bin.argtypes = [ctypes.POINTER(_Grid), P, P, i64, P, i32, P, P, i64]
            lib.ora_canon.restype = ctypes.c_int
            lib.ora_canon.argtypes = [P, ctypes.c_int]
            lib.ora_nearest.restype = ctypes.c_int
            lib.ora_nearest.argtypes = [P, ctypes.c_int, i64, i64]
            lib.ora_delaunay.restype = ctypes.c_int
            lib.ora_delaunay.argtypes = [P, ctypes.c_int, u64, P, ctypes.c_int]
            lib.ora_recon_tile.restype = ctypes.c_int
            lib.ora_recon_tile.argtypes = [ctypes.POINTER(_Grid), P, ctypes.c_int, u64, P, P, P, P, P, P, P]
            lib.ora_recon_tiles.restype = ctypes.c_int
            lib.ora_recon_tiles.argtypes = [ctypes.POINTER(_Grid), P, P, P, P, i64, P, i32, P, P, P, ctypes.c_int]
            lib.ora_unet_num_params.restype = i64
            lib.ora_unet_forward.restype = ctypes.c_int
            lib.ora_unet_forward.argtypes = [P, P, ctypes.c_int, ctypes.c_int, ctypes.c_int, P, ctypes.c_int]
            lib.ora_unet_backward.restype = ctypes.c_int
            lib.ora_unet_backward.argtypes = [P, P, P, ctypes.c_int, ctypes.c_int, ctypes.c_int, P, P, ctypes.c_int]
            lib.ora_splat.restype = i64
            lib.ora_splat.argtypes = [i64, i64, i32, i32, i32, i32, P, P, P, P, i64, P, P]
            lib.ora_resolve.restype = None
            lib.ora_resolve.argtypes = [P, i64, dbl, dbl, P]
            lib.ora_splat_mean.restype = i64
            lib.ora_splat_mean.argtypes = [i64, i64, i32, i32, i32, i32, P, P, P, P, i64, P, P]
            lib.ora_resolve_mean.restype = None
            lib.ora_resolve_mean.argtypes = [P, i64, dbl, dbl, P]
            lib.ora_target_loss.restype = ctypes.c_int
            lib.ora_target_loss.argtypes = [P, P, P, i32, i32, dbl, ctypes.c_int, P, P]
            lib.ora_raster.restype = i64
            lib.ora_raster.argtypes = [P, i64, i64, dbl, dbl, dbl, i32, i32, P, P, P, P, i64, P]
            lib.ora_raster_resolve.restype = None
            lib.ora_pnet_num_params.restype = i64
            lib.ora_pnet_num_params.argtypes = [ctypes.c_int]
            lib.ora_pnet_forward.restype = ctypes.c_int
            lib.ora_pnet_forward.argtypes = [P, P, ctypes.c_int, ctypes.c_int, ctypes.c_int, P, ctypes.c_int]
            lib.ora_raster_resolve.argtypes = [P, i64, P]
            _lib = lib
    return _lib


def _p(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data) if a is not None else None


def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


def _grid(region) -> _Grid:
    return _Grid(region.origin_x, region.origin_y, region.tile_size, region.res, region.pad,
                 region.tiles_x, region.tiles_y, region.scale_xy, region.scale_z, region.offset_z)


def default_threads() -> int:
    return max(1, min(16, os.cpu_count() or 1))


# --------------------------------------------------------------------------
def bin_points(region, x, y, tile_list):
    """Tile + halo binning (Section 3.3: each patch's nearby chunk points).

    Returns (bin_off int64 [n_tiles+1], bin_idx int32) with, per listed tile,
    the indices of all points in its padded window, ascending."""
    lib = _load()
    x, y = _c(x, np.int32), _c(y, np.int32)
    tl = _c(tile_list, np.int32)
    g = _grid(region)
    off = np.zeros(len(tl) + 1, np.int64)
    total = lib.ora_bin(ctypes.byref(g), _p(x), _p(y), x.size, _p(tl), len(tl), _p(off), None, 0)
    idx = np.zeros(max(total, 1), np.int32)
    lib.ora_bin(ctypes.byref(g), _p(x), _p(y), x.size, _p(tl), len(tl), _p(off), _p(idx), total)
    return off, idx[:total]


def make_points(u, v, z, rgb) -> np.ndarray:
    pts = np.zeros(len(u), PT_DTYPE)
    pts["u"], pts["v"], pts["z"] = u, v, z
    pts["rgb"] = np.asarray(rgb).reshape(-1, 3)
    return pts


def canon(pts: np.ndarray) -> np.ndarray:
    """Sort by (v, u); one point per (u, v), keeping the largest (z, R, G, B)."""
    lib = _load()
    p = np.ascontiguousarray(pts.copy(), PT_DTYPE)
    m = lib.ora_canon(_p(p), len(p))
    return p[:m]


def nearest(pts: np.ndarray, qx: int, qy: int) -> int:
    """Index of the nearest point, ties by smallest (d^2, v, u) (Algorithm 1 NN)."""
    lib = _load()
    p = np.ascontiguousarray(pts, PT_DTYPE)
    return lib.ora_nearest(_p(p), len(p), int(qx), int(qy))


def delaunay(pts: np.ndarray, seed: int = 1) -> np.ndarray:
    """Delaunay triangulation (Algorithm 1 DelaunayTriangulate), CCW triples."""
    lib = _load()
    p = np.ascontiguousarray(pts, PT_DTYPE)
    cap = 2 * len(p) + 8
    tri = np.zeros((cap, 3), np.int32)
    nt = lib.ora_delaunay(_p(p), len(p), seed, _p(tri), cap)
    if nt < 0:
        raise RuntimeError("triangle buffer too small")
    return tri[:nt].copy()


def recon_tile(region, pts: np.ndarray, seed: int = 1) -> dict:
    """Algorithm 1 plus the Section 3.4 normalisation for one tile's points
    (tile-local raw coordinates).  Returns a dict of FP64 maps."""
    lib = _load()
    R = region.R
    p = np.ascontiguousarray(pts.copy(), PT_DTYPE)
    xo = np.zeros((R, R, 8))
    cz = np.zeros(1)
    hnn = np.zeros((R, R))
    hlin = np.zeros((R, R))
    nni = np.zeros((R, R), np.int32)
    ins = np.zeros((R, R), np.int8)
    nu = np.zeros(1, np.int32)
    g = _grid(region)
    st = lib.ora_recon_tile(ctypes.byref(g), _p(p), len(p), seed, _p(xo), _p(cz), _p(hnn), _p(hlin), _p(nni),
                            _p(ins), _p(nu))
    m = int(nu[0])
    return dict(x=xo, cz=float(cz[0]), hm_nn=hnn, hm_lin=hlin, nn_idx=nni, inside=ins.astype(bool),
                status=st, points=p[:m])


def tile_points(region, x, y, z, rgb, idx, tile_id) -> np.ndarray:
    """Gather a tile's binned points in tile-local coordinates."""
    S = region.tile_size
    cx = region.origin_x + (tile_id % region.tiles_x) * S + S // 2
    cy = region.origin_y + (tile_id // region.tiles_x) * S + S // 2
    idx = np.asarray(idx, np.int64)
    return make_points(np.asarray(x, np.int64)[idx] - cx, np.asarray(y, np.int64)[idx] - cy,
                       np.asarray(z)[idx], np.asarray(rgb).reshape(-1, 3)[idx])


def recon_tiles(region, x, y, z, rgb, tile_list, nthreads: int = 0):
    """Binning + Algorithm 1 + normalisation for a batch of tiles.

    Returns (x_out float64 [n][R][R][8], cz float64 [n], status int32 [n])."""
    lib = _load()
    x, y, z = _c(x, np.int32), _c(y, np.int32), _c(z, np.int32)
    rgb = _c(np.asarray(rgb).reshape(-1, 3), np.uint16)
    tl = _c(tile_list, np.int32)
    n = len(tl)
    R = region.R
    xo = np.zeros((n, R, R, 8))
    cz = np.zeros(n)
    st = np.zeros(n, np.int32)
    g = _grid(region)
    lib.ora_recon_tiles(ctypes.byref(g), _p(x), _p(y), _p(z), _p(rgb), x.size, _p(tl), n, _p(xo), _p(cz), _p(st),
                        nthreads or default_threads())
    return xo, cz, st


def num_params() -> int:
    return int(_load().ora_unet_num_params())


def unet_forward(w, x, res: int, pad: int, nthreads: int = 0) -> np.ndarray:
    """Refinement network forward (Section 3.4): x [n][R][R][8] -> y [n][res][res][4]."""
    lib = _load()
    w = _c(w, np.float64)
    x = _c(x, np.float64)
    n = x.shape[0]
    y = np.zeros((n, res, res, 4))
    rc = lib.ora_unet_forward(_p(w), _p(x), n, res, pad, _p(y), nthreads or default_threads())
    if rc:
        raise ValueError("res + 2*pad must be divisible by 4")
    return y


def unet_backward(w, x, dy, res: int, pad: int, want_gx: bool = False, nthreads: int = 0):
    """Adjoint of unet_forward: returns (gw [P], gx [n][R][R][8] or None)."""
    lib = _load()
    w = _c(w, np.float64)
    x = _c(x, np.float64)
    dy = _c(dy, np.float64)
    n = x.shape[0]
    gw = np.zeros(w.size)
    gx = np.zeros_like(x) if want_gx else None
    rc = lib.ora_unet_backward(_p(w), _p(x), _p(dy), n, res, pad, _p(gw), _p(gx) if want_gx else None,
                               nthreads or default_threads())
    if rc:
        raise ValueError("res + 2*pad must be divisible by 4")
    return gw, gx


def texture(y, cz, region) -> np.ndarray:
    """Denormalised texture: h = cz + r*y_h (metres), rgb clamped to [0, 1]."""
    H = region.tile_size // 2 + region.pad * region.cell
    r_m = H * region.scale_xy
    t = np.array(y, dtype=np.float64, copy=True)
    t[..., 0] = np.asarray(cz).reshape(-1, 1, 1) + r_m * t[..., 0]
    t[..., 1:] = np.clip(t[..., 1:], 0.0, 1.0)
    return t


def splat(region, x, y, z, rgb, tile_slot, n_slots: int, keys=None):
    """Per-texel max-key splat of full-resolution points (Sections 3.5/3.6).

    Returns (keys uint64 [n_slots][res][res], dropped)."""
    lib = _load()
    x, y, z = _c(x, np.int32), _c(y, np.int32), _c(z, np.int32)
    rgb = _c(np.asarray(rgb).reshape(-1, 3), np.uint16)
    ts = _c(tile_slot, np.int32)
    res = region.res
    if keys is None:
        keys = np.zeros((n_slots, res, res), np.uint64)
    else:
        keys = _c(keys, np.uint64).copy()
    dropped = lib.ora_splat(region.origin_x, region.origin_y, region.tile_size, res, region.tiles_x,
                            region.tiles_y, _p(x), _p(y), _p(z), _p(rgb), x.size, _p(ts), _p(keys))
    return keys, int(dropped)


def resolve(keys, tex, scale_z: float, offset_z: float) -> np.ndarray:
    """Resolve pass: overwrite texels holding a key with its height/colour."""
    lib = _load()
    keys = _c(keys, np.uint64)
    out = np.array(tex, dtype=np.float32, copy=True, order="C")
    lib.ora_resolve(_p(keys), keys.size, scale_z, offset_z, _p(out))
    return out


def splat_mean(region, x, y, z, rgb, tile_slot, n_slots: int, acc=None):
    """Ground-truth accumulation (Section 3.4, training data): per texel the
    sums of raw heights and 16-bit colours and the point count, in input
    order.  Returns (acc int64 [n_slots][res][res][5] = (sum z, sum R, sum G,
    sum B, count), dropped)."""
    lib = _load()
    x, y, z = _c(x, np.int32), _c(y, np.int32), _c(z, np.int32)
    rgb = _c(np.asarray(rgb).reshape(-1, 3), np.uint16)
    ts = _c(tile_slot, np.int32)
    res = region.res
    if acc is None:
        acc = np.zeros((n_slots, res, res, 5), np.int64)
    else:
        acc = _c(acc, np.int64).copy()
    dropped = lib.ora_splat_mean(region.origin_x, region.origin_y, region.tile_size, res, region.tiles_x,
                                 region.tiles_y, _p(x), _p(y), _p(z), _p(rgb), x.size, _p(ts), _p(acc))
    return acc, int(dropped)


def resolve_mean(acc, scale_z: float, offset_z: float) -> np.ndarray:
    """Mean texture [..., 4] (height in metres, colour in [0, 1]) from the
    sums; texels without points are NaN (gaps in the ground truth)."""
    lib = _load()
    acc = _c(acc, np.int64)
    n_cells = acc.size // 5
    out = np.empty(acc.shape[:-1] + (4,), np.float32)
    lib.ora_resolve_mean(_p(acc), n_cells, scale_z, offset_z, _p(out))
    return out


LOSS_CLIPPED_MSE, LOSS_L1 = 0, 1


def target_loss(y, tex, cz, region, kind: int = LOSS_CLIPPED_MSE):
    """Training loss of the normalised output y [n][res][res][4] against the
    target texture tex (metres / [0, 1], NaN = gap) (Section 3.4, training).
    Returns ((L, L_h, L_rgb), dL/dy as float64 [n][res][res][4])."""
    lib = _load()
    y = _c(y, np.float32)
    tex = _c(tex, np.float32)
    cz = _c(cz, np.float64)
    n, res = y.shape[0], y.shape[1]
    r_m = (region.tile_size // 2 + region.pad * region.cell) * region.scale_xy
    out = np.zeros(3)
    grad = np.zeros(y.shape)
    rc = lib.ora_target_loss(_p(y), _p(tex), _p(cz), n, res, r_m, kind, _p(out), _p(grad))
    if rc:
        raise ValueError("unknown loss kind")
    return tuple(float(v) for v in out), grad


def raster(M, origin, scale_xy: float, scale_z: float, offset_z: float, width: int, height: int, x, y, z, rgb,
           fb=None):
    """Point rasteriser (Section 3.6): nearest point per pixel through packed
    64-bit depth-and-colour keys.  M: 4 x 4 view-projection (row-major) on
    metres relative to origin = (ox, oy) raw.  Returns (fb uint64 [height][width],
    points drawn); fb accumulates when given (empty pixel = all ones)."""
    lib = _load()
    Mx = _c(np.asarray(M, np.float64).reshape(16), np.float64)
    x, y, z = _c(x, np.int32), _c(y, np.int32), _c(z, np.int32)
    rgb = _c(np.asarray(rgb).reshape(-1, 3), np.uint16)
    if fb is None:
        fb = np.full((height, width), np.iinfo(np.uint64).max, np.uint64)
    else:
        fb = _c(fb, np.uint64).copy()
    drawn = lib.ora_raster(_p(Mx), int(origin[0]), int(origin[1]), scale_xy, scale_z, offset_z, width, height,
                           _p(x), _p(y), _p(z), _p(rgb), x.size, _p(fb))
    return fb, int(drawn)


def raster_resolve(fb) -> np.ndarray:
    """RGBA8 words (alpha 255) of the nearest point per pixel; 0 = empty."""
    lib = _load()
    fb = _c(fb, np.uint64)
    out = np.zeros(fb.shape, np.uint32)
    lib.ora_raster_resolve(_p(fb), fb.size, _p(out))
    return out


def pnet_num_params(R: int = 96) -> int:
    """Parameters of the paper's refinement network at padded grid side R."""
    return int(_load().ora_pnet_num_params(R))


def pnet_forward(w, x, res: int, pad: int, nthreads: int = 0) -> np.ndarray:
    """The paper's refinement network (Section 3.4, architecture paragraph):
    x [n][R][R][8] -> y [n][res][res][4]."""
    lib = _load()
    w = _c(w, np.float64)
    x = _c(x, np.float64)
    n = x.shape[0]
    R = res + 2 * pad
    if w.size != pnet_num_params(R):
        raise ValueError(f"expected {pnet_num_params(R)} weights, got {w.size}")
    y = np.zeros((n, res, res, 4))
    if lib.ora_pnet_forward(_p(w), _p(x), n, res, pad, _p(y), nthreads or default_threads()):
        raise ValueError("res + 2*pad must be a multiple of 16")
    return y
