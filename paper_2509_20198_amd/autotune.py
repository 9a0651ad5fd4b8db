"""Autotuner for the convolution tilings of the refinement network.

Every (layer, precision, pass) has a small set of tilings (see
ls_conv_num_configs: direct / LDS-staged tile / pixel tiles per wave for
BF16, channel-block width for FP32, pixel-chunk count for the weight
gradient).  All tilings of a (layer, precision, pass) compute the same
result; they differ only in speed for a given shape.  The tuner times the
whole forward (pass 0) or forward + backward (passes 1, 2) on the real batch
shape with HIP events, changing one layer at a time (coordinate descent,
median of `reps` runs; the library's default, -1, is one of the
candidates), keeps the fastest tiling per layer and applies it.  If the
tuned set is not faster than the defaults on a final timing, the defaults
are kept.  The choice is cached in a JSON file keyed by device name, grid
shape, batch size, precision, passes and a hash of the built library, so a
rebuilt library is tuned again.
"""
from __future__ import annotations

import hashlib
import json
import os

import torch

from . import (BF16, FP32, LIB_PATH, OP_BACKWARD, OP_REFINE, Grid, act_bytes, alloc_workspace, conv_num_configs,
               get_conv_config, num_params, pack_weights_bf16, refine_backward, refine_tiles, set_conv_config,
               workspace_bytes)

N_LAYERS = 11


def default_cache_path() -> str:
    return os.environ.get("LS_AUTOTUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "lidarscout_mi355x", "autotune.json"))


_lib_hash = None


def library_hash() -> str:
    """First 16 hex digits of the SHA-256 of the built library."""
    global _lib_hash
    if _lib_hash is None:
        with open(LIB_PATH, "rb") as f:
            _lib_hash = hashlib.sha256(f.read()).hexdigest()[:16]
    return _lib_hash


def _key(g: Grid, n_tiles: int, precision: int, passes) -> str:
    name = torch.cuda.get_device_name() if torch.cuda.is_available() else "cpu"
    return (f"{name}|lib{library_hash()}|R{g.R}|res{g.res}|n{n_tiles}|{'bf16' if precision == BF16 else 'fp32'}"
            f"|passes{''.join(map(str, passes))}")


def _median_ms(fn, reps: int) -> float:
    fn()
    ts = []
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        fn()
        b.record()
        torch.cuda.synchronize()
        ts.append(a.elapsed_time(b))
    ts.sort()
    return ts[len(ts) // 2]


def apply(choice: dict, precision: int):
    for k, c in choice.items():
        layer, p = (int(v) for v in k.split(","))
        set_conv_config(layer, precision, p, int(c))


def reset(precision: int, passes=(0, 1, 2)):
    for p in passes:
        for layer in range(N_LAYERS):
            set_conv_config(layer, precision, p, -1)


def autotune(grid, n_tiles: int, precision: int = BF16, passes=(0,), reps: int = 5, cache_path: str | None = None,
             force: bool = False, seed: int = 0) -> dict:
    """Pick and apply the fastest tiling per layer; returns
    {"key", "choice": {"layer,pass": config}, "ms_default", "ms_tuned", "cached"}."""
    g = Grid.of(grid)
    passes = tuple(sorted(set(passes)))
    key = _key(g, n_tiles, precision, passes)
    path = cache_path or default_cache_path()
    cache = {}
    if os.path.exists(path):
        try:
            with open(path) as f:
                cache = json.load(f)
        except (OSError, ValueError):
            cache = {}
    if key in cache and not force:
        apply(cache[key]["choice"], precision)
        return dict(cache[key], cached=True)

    dev = torch.device("cuda")
    gen = torch.Generator(device=dev).manual_seed(seed)
    x = torch.randn((n_tiles, g.R, g.R, 8), device=dev, generator=gen) * 0.1
    w = torch.randn(num_params(), device=dev, generator=gen) * 0.05
    wb = pack_weights_bf16(w) if precision == BF16 else None
    backward = any(p > 0 for p in passes)
    ws = alloc_workspace(workspace_bytes(OP_BACKWARD if backward else OP_REFINE, g, n_tiles, 0, precision), dev)
    y_out = torch.empty((n_tiles, g.res, g.res, 4), device=dev)
    if backward:
        act = torch.empty(act_bytes(g, n_tiles, precision), dtype=torch.uint8, device=dev)
        gy = torch.randn((n_tiles, g.res, g.res, 4), device=dev, generator=gen)
        gw = torch.empty_like(w)

        def run():
            refine_tiles(w, x, None, g, precision, w_bf16=wb, y_out=y_out, want_tex=False, act_save=act, ws=ws)
            refine_backward(w, x, gy, g, precision, w_bf16=wb, act_save=act, grad_w=gw, ws=ws)
    else:
        def run():
            refine_tiles(w, x, None, g, precision, w_bf16=wb, y_out=y_out, want_tex=False, ws=ws)

    reset(precision, passes)
    ms_default = _median_ms(run, reps)
    choice = {}
    for p in passes:
        for layer in range(N_LAYERS):
            n = conv_num_configs(layer, precision, p)
            if n <= 1:
                continue
            best_c, best_t = -1, None
            for c in range(-1, n):
                set_conv_config(layer, precision, p, c)
                t = _median_ms(run, reps)
                if best_t is None or t < best_t:
                    best_c, best_t = c, t
            set_conv_config(layer, precision, p, best_c)
            choice[f"{layer},{p}"] = best_c
    ms_tuned = _median_ms(run, reps)
    kept_default = ms_tuned >= ms_default
    if kept_default:
        reset(precision, passes)
        choice = {k: -1 for k in choice}
        ms_tuned = ms_default
    out = {"key": key, "choice": choice, "ms_default": ms_default, "ms_tuned": ms_tuned,
           "kept_default": kept_default}
    cache[key] = out
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        with open(path, "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
    except OSError:
        pass
    return dict(out, cached=False)
