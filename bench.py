#!/usr/bin/env python3
"""Benchmark of the per-tile heightmap hot path on one MI355X.

A step is one pass of the whole reconstruction over the 1024-tile batch
(32 x 32 tiles of 640 m, 50-2000 sparse points per tile, log-uniform, the
same fBm terrain with per-tile seeds): tile binning, Algorithm 1 (nearest +
Delaunay-linear maps), normalisation and the refinement network with BF16
matrix-core convolutions, all captured in one HIP graph and replayed.  The
plain FP32 path (one launch per layer, no graph) is timed on the same
inputs for the comparison the metric asks for.

Printed: one JSON line.  `value` is BF16-batched tiles/s with inputs
resident in HBM.  `roofline` is for the dominant kernel group, timed live
with HIP events on its own stream; `cpu_baseline` is the FP64 oracle on a
bounded, strided sample of the same tiles (it also supplies the per-tile
error of the GPU result).  Secondary figures: the full-resolution splat
(100 M Morton-ordered points over 64 x 64 tiles) and the refinement backward
(256 tiles).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

import numpy as np
import torch

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import paper_2509_20198_amd as ls  # noqa: E402
import synth  # noqa: E402

METRIC = "heightmap tiles/s, BF16 batched vs FP32 plain at ≤0.05 m RMS vs FP64 oracle"
PEAK_BF16_TFLOPS = 2500.0
PEAK_FP32_TFLOPS = 157.3
PEAK_HBM_GBS = 8000.0


def recorded_traffic(kernel_source: str, profile: str):
    """HBM bytes per launch from a committed rocprofv3 counter summary, or
    None when the kernel source changed since the counters were taken."""
    try:
        with open(os.path.join(ROOT, "profiles", profile)) as f:
            text = f.read()
        with open(os.path.join(ROOT, "paper_2509_20198_amd", "csrc", kernel_source), "rb") as f:
            src = f.read()
    except OSError:
        return None
    sha = re.search(r"source_sha256: ([0-9a-f]{64})", text)
    val = re.search(r"traffic_bytes_per_launch: (\d+)", text)
    if not (sha and val) or hashlib.sha256(src).hexdigest() != sha.group(1):
        return None
    return int(val.group(1))


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def unet_flops(res: int, pad: int, inference: bool = True) -> float:
    """Multiply-add FLOPs (x2) of one tile's forward: every 3x3 conv on its
    plane, the head only on the res x res crop; for inference dec1a and
    dec1b only on the crop grown by the two and one texels the layers after
    them read (training keeps their whole planes for the backward)."""
    R = res + 2 * pad
    planes = [R, R, R // 2, R // 2, R // 4, R // 4, R // 2, R // 2, R, R]
    if inference:
        planes[8] = min(R, res + 4)
        planes[9] = min(R, res + 2)
    total = 0
    for (name, ci, co), hw in zip(synth.UNET_SHAPES[:-1], planes):
        total += 2 * hw * hw * co * 9 * ci
    _, ci, co = synth.UNET_SHAPES[-1]
    total += 2 * res * res * co * 9 * ci
    return float(total)


def train_flops(res: int, pad: int, grad_x: bool = False) -> float:
    """FLOPs one tile's training step cannot avoid: the forward as inference
    runs it (its output is the crop), then per layer the weight gradient
    over the pixels where the layer's output gradient can be nonzero and the
    input gradient over those where its input gradient can be (both grow by
    one texel per 3x3 conv from the crop, halve or double through the
    upsampling and the pools); the network input's gradient, and the head
    input skip's 8 channels, only with grad_x."""
    R = res + 2 * pad
    R2, R4 = R // 2, R // 4

    def grow(iv, n):
        return max(0, iv[0] - 1), min(n, iv[1] + 1)

    def half(iv, n):
        return iv[0] // 2, min(n, -(-iv[1] // 2))

    def dbl(iv, n):
        return 2 * iv[0], min(n, 2 * iv[1])

    def hull(a, b):
        return min(a[0], b[0]), max(a[1], b[1])

    def size(iv):
        return (iv[1] - iv[0]) ** 2

    crop = (pad, pad + res)
    g10 = grow(crop, R)
    g9 = grow(g10, R)
    gu1 = grow(g9, R)
    g8 = half(gu1, R2)
    g7 = grow(g8, R2)
    gu2 = grow(g7, R2)
    g6 = half(gu2, R4)
    g5 = grow(g6, R4)
    gp2 = grow(g5, R4)
    g4 = hull(gu2, dbl(gp2, R2))
    g3 = grow(g4, R2)
    gp1 = grow(g3, R2)
    g2 = hull(gu1, dbl(gp1, R))
    g1 = grow(g2, R)
    g0 = grow(g1, R)
    # per layer: (output-gradient window, input-gradient window or None)
    wins = [(g1, g0 if grad_x else None), (g2, g1), (g3, gp1), (g4, g3), (g5, gp2), (g6, g5), (g7, gu2), (g8, g7),
            (g9, gu1), (g10, g9), (crop, g10)]
    total = unet_flops(res, pad, inference=True)
    for l, ((_, ci, co), (wo, wi)) in enumerate(zip(synth.UNET_SHAPES, wins)):
        total += 2 * size(wo) * co * 9 * ci
        if wi is not None:
            total += 2 * size(wi) * (16 if l == len(wins) - 1 and not grad_x else ci) * 9 * co
    return float(total)


def unet_bytes(res: int, pad: int) -> float:
    """HBM bytes one tile's BF16 forward must move at least, as the library
    runs it: every layer up to dec1a reads its inputs once and writes its
    BF16 output once (and the fused 2x2 pool output of the two layers that
    feed a pool; the network input x is FP32); dec1b and the head run fused
    on the crop, reading A9 on the crop plus a two-texel halo and x on the
    crop plus one, and writing 4 FP32 channels."""
    R = res + 2 * pad
    f, h, q = R * R, (R // 2) ** 2, (R // 4) ** 2
    b16 = 2
    act = {"A1": 16 * f, "A2": 16 * f, "P1": 16 * h, "A3": 32 * h, "A4": 32 * h, "P2": 32 * q, "A5": 64 * q,
           "A6": 64 * q, "A7": 32 * h, "A8": 32 * h, "A9": 16 * f, "A10": 16 * f}
    layers = [  # (inputs, outputs) as activation names; "x" is the FP32 input
        (["x"], ["A1"]), (["A1"], ["A2", "P1"]), (["P1"], ["A3"]), (["A3"], ["A4", "P2"]), (["P2"], ["A5"]),
        (["A5"], ["A6"]), (["A6", "A4"], ["A7"]), (["A7"], ["A8"]), (["A8", "A2"], ["A9"])]
    total = 0
    for ins, outs in layers:
        for t in ins:
            total += 8 * f * 4 if t == "x" else act[t] * b16
        for t in outs:
            total += act[t] * b16
    total += (res + 4) ** 2 * 16 * b16 + (res + 2) ** 2 * 8 * 4 + res * res * 4 * 4  # dec1b + head
    return float(total)


class Timer:
    def __init__(self):
        self.a = torch.cuda.Event(enable_timing=True)
        self.b = torch.cuda.Event(enable_timing=True)

    def run(self, fn, steps, warmup):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        self.a.record()
        for _ in range(steps):
            fn()
        self.b.record()
        torch.cuda.synchronize()
        return self.a.elapsed_time(self.b) / steps


def achievable_peaks(dev):
    """What this GPU reaches on plain library work, beside the published
    peaks: a 1 GiB device copy (read + write) and an 8192^3 BF16 GEMM."""
    timer = Timer()
    a = torch.empty(1 << 28, dtype=torch.float32, device=dev)
    b = torch.empty_like(a)
    ms_copy = timer.run(lambda: b.copy_(a), 10, 3)
    del a, b
    n = 8192
    g = torch.Generator(device=dev).manual_seed(0)
    x = torch.randn((n, n), device=dev, generator=g).to(torch.bfloat16).contiguous()
    y = torch.randn((n, n), device=dev, generator=g).to(torch.bfloat16).contiguous()
    ms_mm = timer.run(lambda: torch.matmul(x, y), 10, 3)
    del x, y
    return {"hbm_copy_GBps": 2 * (1 << 30) / (ms_copy * 1e-3) / 1e9,
            "bf16_gemm_TFLOPs": 2 * n ** 3 / (ms_mm * 1e-3) / 1e12,
            "how": "torch copy_ of 1 GiB (bytes read + written); torch.matmul of two 8192x8192 BF16 matrices"}


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(work, sample_idx, gpu_tex_bf16, gpu_tex_fp32, weights64):
    """The FP64 oracle (recon + network forward) on a strided sample of the
    batch, timed on the host cores; also the GPU error on those tiles."""
    import oracle

    nthreads = oracle.default_threads()
    x, y, z, rgb = work.points.numpy()
    tl = work.tile_list[sample_idx]
    t0 = time.perf_counter()
    xo, cz, _ = oracle.recon_tiles(work.region, x, y, z, rgb, tl, nthreads=nthreads)
    yo = oracle.unet_forward(weights64, xo, work.region.res, work.region.pad, nthreads=nthreads)
    dt = time.perf_counter() - t0
    tex = oracle.texture(yo, cz, work.region)
    d16 = gpu_tex_bf16[..., 0].astype(np.float64) - tex[..., 0]
    d32 = gpu_tex_fp32[..., 0].astype(np.float64) - tex[..., 0]
    rms16 = np.sqrt((d16 ** 2).reshape(len(tl), -1).mean(1))
    base = oracle.texture(xo[:, work.region.pad:work.region.pad + work.region.res,
                             work.region.pad:work.region.pad + work.region.res][..., [0, 2, 3, 4]], cz, work.region)
    head_rms = np.sqrt(((tex[..., 0] - base[..., 0]) ** 2).reshape(len(tl), -1).mean(1))
    # one thread on a sub-sample (the figure comparable to a single-threaded CPU pipeline)
    tl1 = tl[:: max(1, len(tl) // 16)][:16]
    t1 = time.perf_counter()
    xo1, _, _ = oracle.recon_tiles(work.region, x, y, z, rgb, tl1, nthreads=1)
    oracle.unet_forward(weights64, xo1, work.region.res, work.region.pad, nthreads=1)
    dt1 = time.perf_counter() - t1
    return {
        "value": len(tl) / dt,
        "unit": "tiles/s",
        "cores": nthreads,
        "kind": "oracle",
        "sample": f"{len(tl)} tiles (every {len(work.tile_list) // len(tl)}th of the batch): FP64 binning, "
                  f"Algorithm 1, normalisation and network forward; wall {dt:.2f} s",
        "single_thread": {"tiles_per_s": len(tl1) / dt1, "ms_per_tile": dt1 / len(tl1) * 1e3,
                          "sample": f"{len(tl1)} of those tiles, one thread"},
        "cpu_model": cpu_model(),
        "host_threads": os.cpu_count(),
    }, {
        "bf16_rms_max_m": float(rms16.max()),
        "bf16_rms_mean_m": float(rms16.mean()),
        "bf16_abs_p99_m": float(np.quantile(np.abs(d16), 0.99)),
        "fp32_max_abs_m": float(np.abs(d32).max()),
        "head_rms_mean_m": float(head_rms.mean()),
        "tiles_checked": len(tl),
    }


def binning_rate(region, x, y, stage_ms: dict) -> dict:
    """Tile binning throughput: each sparse point's x, y read once (8 B) and
    one 4-byte point index written per window that holds it (a window is its
    tile grown by `pad` texels; every tile of the region is listed)."""
    ms = sum(stage_ms.get(k) or 0.0 for k in ("bin_count", "bin_scan", "bin_scatter"))
    if ms <= 0:
        return {}
    S, P = region.tile_size, region.pad * region.cell
    xs = x.detach().cpu().numpy().astype(np.int64) - region.origin_x
    ys = y.detach().cpu().numpy().astype(np.int64) - region.origin_y

    def windows(v, ntile):
        t, r = v // S, v % S
        return 1 + ((r < P) & (t > 0)) + ((r >= S - P) & (t < ntile - 1))

    member = int((windows(xs, region.tiles_x) * windows(ys, region.tiles_y)).sum())
    nbytes = 8 * xs.size + 4 * member
    return {"ms": ms, "points": int(xs.size), "memberships": member, "points_per_s": xs.size / (ms * 1e-3),
            "algorithmic_GBps": nbytes / (ms * 1e-3) / 1e9, "frac_hbm_peak": nbytes / (ms * 1e-3) / 1e9 / PEAK_HBM_GBS,
            "algorithmic_bytes": "8 B per point (x, y) + 4 B per point and window holding it",
            "kernels": "bin_count + bin_scan + bin_scatter"}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--cpu-tiles", type=int, default=256, help="oracle sample size (0 = skip)")
    ap.add_argument("--no-secondary", action="store_true", help="skip splat / backward figures")
    ap.add_argument("--no-backward", action="store_true", help="skip the backward / training figures")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="start with one plain 1 GiB device-to-device copy (reference for HBM counters)")
    ap.add_argument("--splat-points", type=int, default=100_000_000)
    ap.add_argument("--no-stream", action="store_true", help="skip the 16,384-tile streaming figures")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only (tiles are independent; how the path would shard over GPUs is "
              "described in the design notes); run with --gpus 1.", file=sys.stderr)
        sys.exit(2)
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    ls.load_library()
    if args.copy_calibration:
        src = torch.ones(1 << 28, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        log("copy calibration: 1 GiB read, 1 GiB written")

    # ---------------------------------------------------------------- inputs
    work = synth.batch_tiles(seed=2, device=dev)
    region = work.region
    g = ls.Grid.of(region)
    ps = work.points
    nt = len(work.tile_list)
    x, y, z = ps.x.contiguous(), ps.y.contiguous(), ps.z.contiguous()
    rgb = ps.rgb_u16()
    tl = torch.from_numpy(work.tile_list).to(dev)
    w64 = synth.unet_weights(0)
    w = torch.from_numpy(w64.astype(np.float32)).to(dev)
    wb = ls.pack_weights_bf16(w)
    R, res = g.R, g.res
    x_out = torch.empty((nt, R, R, 8), dtype=torch.float32, device=dev)
    cz = torch.empty(nt, dtype=torch.float64, device=dev)
    st = torch.empty(nt, dtype=torch.int32, device=dev)
    ws_recon = ls.alloc_workspace(ls.workspace_bytes(ls.OP_RECON, g, nt, ps.n), dev)
    ws16 = ls.alloc_workspace(ls.workspace_bytes(ls.OP_REFINE, g, nt, 0, ls.BF16), dev)
    ws32 = ls.alloc_workspace(ls.workspace_bytes(ls.OP_REFINE, g, nt, 0, ls.FP32), dev)
    tex16 = torch.empty((nt, res, res, 4), dtype=torch.float32, device=dev)
    tex32 = torch.empty_like(tex16)
    log(f"workload: {nt} tiles, {ps.n} sparse points")

    def step_bf16():
        ls.recon_tiles(g, x, y, z, rgb, tl, order=ls.ORDER_LONGEST_FIRST, x_out=x_out, cz_out=cz, status=st,
                       ws=ws_recon)
        ls.refine_tiles(w, x_out, cz, g, ls.BF16, w_bf16=wb, tex_out=tex16, want_y=False, ws=ws16)

    def step_fp32():
        ls.recon_tiles(g, x, y, z, rgb, tl, order=ls.ORDER_LONGEST_FIRST, x_out=x_out, cz_out=cz, status=st,
                       ws=ws_recon)
        ls.refine_tiles(w, x_out, cz, g, ls.FP32, tex_out=tex32, want_y=False, ws=ws32)

    # ---------------------------------------------------------------- conv tilings
    from paper_2509_20198_amd import autotune as AT

    tune = AT.autotune(g, nt, ls.BF16, passes=(0,), reps=5, force=True)
    log(f"autotuned BF16 forward tilings: {tune['ms_default']:.3f} -> {tune['ms_tuned']:.3f} ms")

    # ---------------------------------------------------------------- graph
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        for _ in range(2):
            step_bf16()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        step_bf16()
    torch.cuda.synchronize()
    log("graph captured")
    timer = Timer()
    ms16 = timer.run(graph.replay, args.steps, args.warmup)
    log(f"bf16 graph step {ms16:.3f} ms")
    ms32 = timer.run(step_fp32, max(3, args.steps // 4), 2)
    log(f"fp32 plain step {ms32:.3f} ms")
    graph.replay()
    torch.cuda.synchronize()
    status = st.cpu().numpy()

    # ---------------------------------------------------------------- per-kernel timing
    reps = 3
    ls.trace_enable(True)
    for _ in range(reps):
        step_bf16()
    torch.cuda.synchronize()
    rec = ls.trace_records()
    ls.trace_enable(False)
    per = {}
    for name, ms in rec:
        t, c = per.get(name, (0.0, 0))
        per[name] = (t + ms, c + 1)
    kernels = {k: {"ms_per_step": v[0] / reps, "launches_per_step": v[1] // reps} for k, v in per.items()}
    leaf = {k: v for k, v in kernels.items() if k != "recon_all"}
    dom = max(leaf, key=lambda k: leaf[k]["ms_per_step"])
    flops_tile = unet_flops(res, g.pad)
    if dom == "conv_bf16":
        ms_dom = kernels[dom]["ms_per_step"]
        ach = flops_tile * nt / (ms_dom * 1e-3) / 1e12
        roof = {"kernel": "conv_bf16 (every conv launch of a step)", "bound": "mfma", "achieved": ach,
                "peak": PEAK_BF16_TFLOPS, "unit": "TFLOP/s", "frac": ach / PEAK_BF16_TFLOPS, "traffic": None,
                "avg_launch_ms": ms_dom / kernels[dom]["launches_per_step"],
                "algorithmic_per_step": f"{flops_tile * nt / 1e9:.1f} GFLOP ({flops_tile / 1e9:.4f} GFLOP/tile)"}
    else:
        # recon: report the output-write bytes the kernel must move (HBM floor)
        ms_dom = kernels[dom]["ms_per_step"]
        bytes_step = nt * R * R * 8 * 4
        ach = bytes_step / (ms_dom * 1e-3) / 1e9
        traffic = recorded_traffic("ls_recon.hip", "recon_tile_batch_1024_traffic.md") if dom == "recon_tile" else None
        roof = {"kernel": dom, "bound": "hbm", "achieved": ach, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": ach / PEAK_HBM_GBS, "traffic": traffic, "traffic_unit": "HBM bytes per launch (counters)",
                "avg_launch_ms": ms_dom / kernels[dom]["launches_per_step"],
                "algorithmic_per_step": f"{bytes_step / 1e6:.1f} MB written (x_out)"}
    log(f"dominant kernel group: {dom} ({kernels[dom]['ms_per_step']:.3f} ms/step)")
    # the convolutions against the matrix-core peak, whatever group dominates
    conv_ms = kernels.get("conv_bf16", {}).get("ms_per_step", 0.0)
    conv_tf = flops_tile * nt / (conv_ms * 1e-3) / 1e12 if conv_ms > 0 else None
    conv_bytes = unet_bytes(res, g.pad) * nt
    conv_gbs = conv_bytes / (conv_ms * 1e-3) / 1e9 if conv_ms > 0 else None
    roof_conv = {"kernel": "conv_bf16 (every conv launch of a step)", "bound": "mfma", "achieved": conv_tf,
                 "peak": PEAK_BF16_TFLOPS, "unit": "TFLOP/s",
                 "frac": conv_tf / PEAK_BF16_TFLOPS if conv_tf else None, "ms_per_step": conv_ms,
                 "algorithmic_per_step": f"{flops_tile * nt / 1e9:.1f} GFLOP ({flops_tile / 1e9:.4f} GFLOP/tile)",
                 "hbm_algorithmic_GBps": conv_gbs, "hbm_frac": conv_gbs / PEAK_HBM_GBS if conv_gbs else None,
                 "hbm_algorithmic_per_step": f"{conv_bytes / 1e9:.2f} GB ({conv_bytes / nt / 1e6:.2f} MB/tile)"}

    out = {
        "metric": METRIC,
        "value": nt / (ms16 * 1e-3),
        "unit": "tiles/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms16,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16",
        "data": "synthetic",
        "config": {"workload": "batch_1024_tiles: 32x32 tiles of 640 m, 50-2000 sparse points per tile "
                               "(log-uniform), fBm terrain; recon + BF16 refine in one HIP graph",
                   "tiles": nt, "sparse_points": ps.n, "res": res, "pad": g.pad, "grid": f"{R}x{R}x8"},
        "roofline": roof,
        "roofline_conv": roof_conv,
        "sparse_points_per_s": ps.n / (ms16 * 1e-3),
        "fp32_plain": {"tiles_per_s": nt / (ms32 * 1e-3), "ms_per_step": ms32},
        "bf16_vs_fp32": ms32 / ms16,
        "kernels_ms_per_step": {k: round(v["ms_per_step"], 4) for k, v in sorted(kernels.items())},
        "binning": binning_rate(work.region, ps.x, ps.y, {k: v["ms_per_step"] for k, v in kernels.items()}),
        "autotune_bf16_forward": {"choice": tune["choice"], "refine_ms_default": tune["ms_default"],
                                  "refine_ms_tuned": tune["ms_tuned"],
                                  "configs": "0 direct (4 pixel tiles/wave), 1 LDS 16x16 tile, 2 direct (2 pixel tiles/wave), 3 LDS tile, persistent with patch prefetch, 4 (enc1b, head) fused with the layer before"},
        "tile_status_nonzero": int((status != 0).sum()),
    }
    try:
        peaks = achievable_peaks(dev)
        out["achievable_peaks"] = peaks
        if roof["unit"] == "GB/s":
            roof["frac_of_achievable"] = roof["achieved"] / peaks["hbm_copy_GBps"]
        if roof_conv["achieved"]:
            roof_conv["frac_of_achievable"] = roof_conv["achieved"] / peaks["bf16_gemm_TFLOPs"]
            roof_conv["hbm_frac_of_achievable"] = roof_conv["hbm_algorithmic_GBps"] / peaks["hbm_copy_GBps"]
    except Exception as e:  # secondary figure only
        out["achievable_peaks"] = {"error": repr(e)}

    # ---------------------------------------------------------------- secondary figures
    if not args.no_secondary:
        try:
            out["splat"] = bench_splat(args.splat_points, dev)
        except Exception as e:  # secondary figure only
            out["splat"] = {"error": repr(e)}
        try:
            out["point_kernels"] = bench_point_kernels(dev, args.splat_points)
        except Exception as e:  # secondary figure only
            out["point_kernels"] = {"error": repr(e)}
        try:
            out["lsnet"] = bench_lsnet(work, x_out, cz, dev)
        except Exception as e:  # secondary figure only
            out["lsnet"] = {"error": repr(e)}
        try:
            out["single_tile"] = bench_single_tile(dev)
        except Exception as e:  # secondary figure only
            out["single_tile"] = {"error": repr(e)}
        if not args.no_backward:
            try:
                out["backward"] = bench_training(dev)
            except Exception as e:
                out["backward"] = {"error": repr(e)}
        if not args.no_stream:
            try:
                out["stream"] = bench_stream(dev)
            except Exception as e:  # secondary figure only
                out["stream"] = {"error": repr(e)}

    # ---------------------------------------------------------------- CPU baseline (oracle)
    if args.cpu_tiles > 0:
        stride = max(1, nt // args.cpu_tiles)
        idx = np.arange(0, nt, stride)[: args.cpu_tiles]
        log(f"oracle baseline on {len(idx)} tiles")
        base, err = cpu_baseline(work, idx, tex16.cpu().numpy()[idx], tex32.cpu().numpy()[idx], w64)
        out["cpu_baseline"] = base
        out["accuracy"] = err
    print(json.dumps(out), flush=True)


def bench_splat(n_points: int, dev):
    region = synth.Region(tiles_x=64, tiles_y=64)
    g = ls.Grid.of(region)
    ps = synth.fullres_uniform(region, n_points, seed=3, device=dev)
    x, y, z = ps.x.contiguous(), ps.y.contiguous(), ps.z.contiguous()
    rgb = ps.rgb_u16()
    del ps
    nslots = 64 * 64
    ts = torch.arange(nslots, dtype=torch.int32, device=dev)
    keys = torch.zeros((nslots, 64, 64), dtype=torch.int64, device=dev)
    nd = torch.zeros(1, dtype=torch.int64, device=dev)
    torch.cuda.synchronize()
    fn = lambda: ls.splat_points(g, x, y, z, rgb, ts, nslots, keys=keys, n_dropped=nd)  # noqa: E731
    for _ in range(10):
        fn()
    torch.cuda.synchronize()
    ls.trace_enable(True)
    reps = 10
    for _ in range(reps):
        fn()
    torch.cuda.synchronize()
    times = sorted(t for n, t in ls.trace_records() if n == "splat")
    ls.trace_enable(False)
    ms = times[len(times) // 2]  # median launch
    alg_bytes = n_points * 18 + nslots * 64 * 64 * 8
    return {"workload": f"{n_points} points, 64x64 tiles, Morton-ordered", "ms": ms, "ms_min": times[0],
            "ms_mean": sum(times) / len(times),
            "points_per_s": n_points / (ms * 1e-3), "algorithmic_GBps": alg_bytes / (ms * 1e-3) / 1e9,
            "frac_hbm_peak": alg_bytes / (ms * 1e-3) / 1e9 / PEAK_HBM_GBS,
            "traffic": recorded_traffic("ls_splat.hip", "splat_100M_points_traffic.md")
            if n_points == 100_000_000 else None,
            "traffic_unit": "HBM bytes per launch (counters)"}


def training_set(dev, dense_per_tile: int = 2_000_000, chunk_tiles: int = 16):
    """256 tiles (16 x 16) with 200-800 sparse points each, reconstructed on
    the GPU, and two targets from `dense_per_tile` dense points per tile of
    the same terrain (no noise): the max-height splat (the configured target)
    and the per-texel mean (the paper's ground truth), both textures in
    metres / [0, 1]."""
    work = synth.train_tiles(seed=4, device=dev)
    region = work.region
    g = ls.Grid.of(region)
    ps = work.points
    tl = torch.from_numpy(work.tile_list).to(dev)
    x, cz, _ = ls.recon_tiles(g, ps.x, ps.y, ps.z, ps.rgb_u16(), tl)
    nt = len(work.tile_list)
    ids = np.asarray(work.tile_list, np.int64)
    slot = torch.full((region.tiles_x * region.tiles_y,), -1, dtype=torch.int32, device=dev)
    slot[torch.from_numpy(ids).to(dev)] = torch.arange(nt, dtype=torch.int32, device=dev)
    keys = torch.zeros((nt, region.res, region.res), dtype=torch.int64, device=dev)
    acc = torch.zeros((nt, region.res, region.res, 5), dtype=torch.int64, device=dev)
    nd = torch.zeros(1, dtype=torch.int64, device=dev)
    for c in range(0, nt, chunk_tiles):
        d = synth.fullres_points(region, ids[c:c + chunk_tiles], dense_per_tile, seed=1000 + c, noise_sigma_m=0.0,
                                 device=dev, terrain_seed=4)
        ls.splat_points(g, d.x, d.y, d.z, d.rgb_u16(), slot, nt, keys=keys, n_dropped=nd)
        ls.splat_mean(g, d.x, d.y, d.z, d.rgb_u16(), slot, nt, acc=acc, n_dropped=nd)
        del d
    tex_max = torch.zeros((nt, region.res, region.res, 4), dtype=torch.float32, device=dev)
    ls.resolve_keys(g, keys, tex_max)
    tex_mean = ls.resolve_mean(g, acc)
    torch.cuda.synchronize()
    return work, g, x, cz, tex_max, tex_mean, int((keys == 0).sum().item())


def bench_training(dev, train_steps: int = 60):
    """Refinement backward on the 256-tile training batch: FP32 and BF16
    forward + backward step times (BF16 also with activation recomputation),
    and short AdamW runs of the BF16 path from random weights: the configured
    L1 against max-height targets, and the paper's clipped MSE against mean
    targets."""
    from paper_2509_20198_amd import train as T

    t0 = time.perf_counter()
    work, g, x, cz, tex_max, tex_mean, empty = training_set(dev)
    log(f"training set ready in {time.perf_counter() - t0:.1f} s")
    nt = x.shape[0]
    w0 = torch.from_numpy(synth.unet_weights(1).astype(np.float32)).to(dev)
    gy = torch.randn((nt, g.res, g.res, 4), device=dev, generator=torch.Generator(device=dev).manual_seed(0))
    out = {"workload": f"{nt} tiles (16 x 16), 200-800 sparse points per tile; targets from 2,000,000 dense "
                       f"points per tile", "target_texels_without_points": empty}
    from paper_2509_20198_amd import autotune as AT

    for name, prec in (("fp32", ls.FP32), ("bf16", ls.BF16)):
        # conv tilings of forward, input gradient and weight gradient for this shape
        tune = AT.autotune(g, nt, prec, passes=(0, 1, 2), reps=3, force=True)
        log(f"autotuned {name} forward + backward tilings: {tune['ms_default']:.3f} -> {tune['ms_tuned']:.3f} ms")
        wb = ls.pack_weights_bf16(w0) if prec == ls.BF16 else None
        act = torch.empty(ls.act_bytes(g, nt, prec), dtype=torch.uint8, device=dev)
        ws = ls.alloc_workspace(ls.workspace_bytes(ls.OP_BACKWARD, g, nt, 0, prec), dev)
        gw = torch.empty_like(w0)

        def step():
            ls.refine_tiles(w0, x, cz, g, prec, w_bf16=wb, act_save=act, want_y=True, want_tex=False, ws=ws)
            ls.refine_backward(w0, x, gy, g, prec, w_bf16=wb, act_save=act, grad_w=gw, ws=ws)

        def step_recompute():
            ls.refine_tiles(w0, x, cz, g, prec, w_bf16=wb, want_y=True, want_tex=False, ws=ws)
            ls.refine_backward(w0, x, gy, g, prec, w_bf16=wb, grad_w=gw, ws=ws)

        ms = Timer().run(step, 5, 2)
        ms_rc = Timer().run(step_recompute, 5, 2)
        # forward + input gradient + weight gradient, each on whole planes
        flops = 3 * unet_flops(g.res, g.pad, inference=False) * nt
        # what the step cannot avoid (windows around the crop, no grad_x)
        flops_min = train_flops(g.res, g.pad) * nt
        peak = PEAK_BF16_TFLOPS if prec == ls.BF16 else PEAK_FP32_TFLOPS
        out[name] = {"fwd_bwd_ms": ms, "tiles_per_s": nt / (ms * 1e-3), "fwd_bwd_recompute_ms": ms_rc,
                     "achieved_TFLOPs": flops / (ms * 1e-3) / 1e12,
                     "frac_peak": flops / (ms * 1e-3) / 1e12 / peak,
                     "flops_per_tile": {"whole_planes_3x_forward": flops / nt, "unavoidable": flops_min / nt},
                     "achieved_TFLOPs_unavoidable": flops_min / (ms * 1e-3) / 1e12,
                     "frac_peak_unavoidable": flops_min / (ms * 1e-3) / 1e12 / peak,
                     "saved_activation_bytes": int(act.numel()),
                     "autotune": {"ms_default": tune["ms_default"], "ms_tuned": tune["ms_tuned"],
                                  "choice": tune["choice"]}}
        del act, ws
    # training: BF16 convolutions, FP32 weights and optimiser state
    for key, kind, tex in (("train_bf16", ls.LOSS_L1, tex_max), ("train_bf16_paper_loss", ls.LOSS_CLIPPED_MSE,
                                                                 tex_mean)):
        base = T.loss_value(T.linear_baseline(x, g.pad, g.res), tex, cz, g, kind)
        # one untimed step of a throwaway trainer first, so the timed steps
        # find the activation and workspace buffers in torch's caching allocator
        T.Trainer(w0, g, ls.BF16, save_acts=True, total_steps=train_steps, loss_kind=kind).step(x, tex, cz)
        tr = T.Trainer(w0, g, ls.BF16, save_acts=True, total_steps=train_steps, loss_kind=kind)
        losses = []
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(train_steps):
            losses.append(tr.step(x, tex, cz))
        torch.cuda.synchronize()
        dt = time.perf_counter() - t1
        losses = [float(v.item()) for v in losses]
        out[key] = {"steps": train_steps, "ms_per_step": dt / train_steps * 1e3,
                    "tiles_per_s_trained": nt * train_steps / dt, "loss_first": losses[0],
                    "loss_last": losses[-1], "loss_min": min(losses), "linear_baseline_loss": base,
                    "loss": "L1 vs max-height targets" if kind == ls.LOSS_L1 else
                    "NaN-masked clipped MSE vs per-texel mean targets",
                    "optimizer": "AdamW lr 1e-4 betas (0.9, 0.999) eps 1e-5 wd 1e-2, x0.1 at 1/3 and 2/3"}
    return out


def kernel_ms(fn, names, reps=10, warm=3):
    """Median per-call milliseconds of the named kernel groups (trace events)."""
    for _ in range(warm):
        fn()
    torch.cuda.synchronize()
    ls.trace_enable(True)
    for _ in range(reps):
        fn()
    torch.cuda.synchronize()
    rec = ls.trace_records()
    ls.trace_enable(False)
    out = {}
    for n in names:
        per = {}
        # group the records of each call: sum per call, then the median over calls
        ts = [t for name, t in rec if name == n]
        k = len(ts) // reps if reps else 0
        if k:
            sums = sorted(sum(ts[i * k:(i + 1) * k]) for i in range(reps))
            per = sums[len(sums) // 2]
        out[n] = per if k else None
    return out


def bench_single_tile(dev):
    """The single 400-point tile (plain FP32 path): microseconds per stage."""
    w = synth.single_tile(seed=1, n=400, device=dev)
    g = ls.Grid.of(w.region)
    ps = w.points
    tl = torch.from_numpy(w.tile_list).to(dev)
    x, cz, st = ls.recon_tiles(g, ps.x, ps.y, ps.z, ps.rgb_u16(), tl)
    wt = torch.from_numpy(synth.unet_weights(0).astype(np.float32)).to(dev)
    wb = ls.pack_weights_bf16(wt)
    ws_r = ls.alloc_workspace(ls.workspace_bytes(ls.OP_RECON, g, 1, ps.n), dev)
    ws32 = ls.alloc_workspace(ls.workspace_bytes(ls.OP_REFINE, g, 1, 0, ls.FP32), dev)
    ws16 = ls.alloc_workspace(ls.workspace_bytes(ls.OP_REFINE, g, 1, 0, ls.BF16), dev)
    tex = torch.empty((1, g.res, g.res, 4), dtype=torch.float32, device=dev)
    rec = kernel_ms(lambda: ls.recon_tiles(g, ps.x, ps.y, ps.z, ps.rgb_u16(), tl, x_out=x, cz_out=cz, status=st,
                                           ws=ws_r), ["bin_count", "bin_scan", "bin_scatter", "recon_tile",
                                                      "recon_all"], reps=50)
    f32 = Timer().run(lambda: ls.refine_tiles(wt, x, cz, g, ls.FP32, tex_out=tex, want_y=False, ws=ws32), 50, 5)
    b16 = Timer().run(lambda: ls.refine_tiles(wt, x, cz, g, ls.BF16, w_bf16=wb, tex_out=tex, want_y=False,
                                              ws=ws16), 50, 5)
    whole = Timer().run(lambda: (ls.recon_tiles(g, ps.x, ps.y, ps.z, ps.rgb_u16(), tl, x_out=x, cz_out=cz,
                                                status=st, ws=ws_r),
                                 ls.refine_tiles(wt, x, cz, g, ls.FP32, tex_out=tex, want_y=False, ws=ws32)), 50, 5)
    us = lambda v: None if v is None else round(v * 1e3, 1)  # noqa: E731
    return {"workload": "single_tile_400: one 640 m tile, 400 sparse points, 96 x 96 grid",
            "us_recon_kernel_groups": {k: us(v) for k, v in rec.items()},
            "us_refine_fp32": us(f32), "us_refine_bf16": us(b16), "us_recon_plus_fp32_refine": us(whole),
            "note": "latency-bound (one tile on 256 CUs); the paper's CPU triangulation and sampling take 16 ms "
                    "per patch and its CNN 4 ms on an RTX 3090 (context only, other hardware)"}


def bench_stream(dev, splat_points: int = 500_000_000, splat_tiles: int = 256):
    """The 16,384-tile streaming case (128 x 128 tiles, Pareto-distributed
    sparse counts, tiles sorted by distance to a random viewpoint): recon +
    BF16 refine of the whole set, the time at which the nearest tiles are
    finished when the list is processed as prioritised sub-batches, and the
    500 M-point full-resolution splat over the nearest tiles."""
    work = synth.stream_tiles(seed=5, device=dev)
    region = work.region
    g = ls.Grid.of(region)
    ps = work.points
    nt = len(work.tile_list)
    tl = torch.from_numpy(work.tile_list).to(dev)
    x, y, z, rgb = ps.x.contiguous(), ps.y.contiguous(), ps.z.contiguous(), ps.rgb_u16()
    w = torch.from_numpy(synth.unet_weights(0).astype(np.float32)).to(dev)
    wb = ls.pack_weights_bf16(w)
    R, res = g.R, g.res
    x_out = torch.empty((nt, R, R, 8), dtype=torch.float32, device=dev)
    cz = torch.empty(nt, dtype=torch.float64, device=dev)
    st = torch.empty(nt, dtype=torch.int32, device=dev)
    tex = torch.empty((nt, res, res, 4), dtype=torch.float32, device=dev)
    ws_r = ls.alloc_workspace(ls.workspace_bytes(ls.OP_RECON, g, nt, ps.n), dev)
    ws16 = ls.alloc_workspace(ls.workspace_bytes(ls.OP_REFINE, g, nt, 0, ls.BF16), dev)
    out = {"workload": f"stream_16384_tiles: 128 x 128 tiles (81.92 km), {ps.n} sparse points (Pareto 20-5000 "
                       "per tile), tiles sorted by distance to a viewpoint"}

    def whole(order):
        ls.recon_tiles(g, x, y, z, rgb, tl, order=order, x_out=x_out, cz_out=cz, status=st, ws=ws_r)
        ls.refine_tiles(w, x_out, cz, g, ls.BF16, w_bf16=wb, tex_out=tex, want_y=False, ws=ws16)

    for key, order in (("whole_longest_first", ls.ORDER_LONGEST_FIRST), ("whole_list_order", ls.ORDER_LIST)):
        ms = Timer().run(lambda: whole(order), 5, 2)
        out[key] = {"ms": ms, "tiles_per_s": nt / (ms * 1e-3), "sparse_points_per_s": ps.n / (ms * 1e-3)}
    stages = kernel_ms(lambda: whole(ls.ORDER_LONGEST_FIRST), ["bin_count", "bin_scan", "bin_scatter", "recon_tile",
                                                               "conv_bf16"], reps=3, warm=1)
    out["stage_ms"] = stages
    out["binning"] = binning_rate(region, x, y, stages)
    if stages.get("recon_tile"):
        out["recon_hbm_frac"] = nt * R * R * 8 * 4 / (stages["recon_tile"] * 1e-3) / 1e9 / PEAK_HBM_GBS
    if stages.get("conv_bf16"):
        out["conv_mfma_frac"] = unet_flops(res, g.pad) * nt / (stages["conv_bf16"] * 1e-3) / 1e12 / PEAK_BF16_TFLOPS
    # prioritised sub-batches: the nearest 256, the next 768, the rest
    bounds = [0, 256, 1024, nt]
    views = []
    for a, b in zip(bounds[:-1], bounds[1:]):
        views.append((tl[a:b], x_out[a:b], cz[a:b], st[a:b], tex[a:b]))
    wss = [(ls.alloc_workspace(ls.workspace_bytes(ls.OP_RECON, g, b - a, ps.n), dev),
            ls.alloc_workspace(ls.workspace_bytes(ls.OP_REFINE, g, b - a, 0, ls.BF16), dev))
           for a, b in zip(bounds[:-1], bounds[1:])]
    ev = [torch.cuda.Event(enable_timing=True) for _ in bounds]
    times = []
    for rep in range(4):
        torch.cuda.synchronize()
        ev[0].record()
        for k, ((tlk, xk, czk, stk, texk), (wr, wf)) in enumerate(zip(views, wss)):
            ls.recon_tiles(g, x, y, z, rgb, tlk, order=ls.ORDER_LIST, x_out=xk, cz_out=czk, status=stk, ws=wr)
            ls.refine_tiles(w, xk, czk, g, ls.BF16, w_bf16=wb, tex_out=texk, want_y=False, ws=wf)
            ev[k + 1].record()
        torch.cuda.synchronize()
        if rep > 0:
            times.append([ev[0].elapsed_time(e) for e in ev[1:]])
    med = np.median(np.asarray(times), 0)
    out["prioritised_sub_batches"] = {"ms_nearest_256_done": float(med[0]), "ms_nearest_1024_done": float(med[1]),
                                      "ms_all_done": float(med[2]),
                                      "how": "recon (tile-list order) + BF16 refine per sub-batch [256, 768, rest] "
                                             "of the distance-sorted list, events after each"}
    out["tile_status_nonzero"] = int((st != 0).sum().item())
    del x_out, ws_r, ws16, wss, views
    # full-resolution splat over the nearest tiles
    ids = np.asarray(work.tile_list[:splat_tiles], np.int64)
    per = splat_points // splat_tiles
    n = per * splat_tiles
    bx = torch.empty(n, dtype=torch.int32, device=dev)
    by, bz = torch.empty_like(bx), torch.empty_like(bx)
    brgb = torch.empty((n, 3), dtype=torch.int16, device=dev)
    step = 16
    for c in range(0, splat_tiles, step):
        d = synth.fullres_points(region, ids[c:c + step], per, seed=5000 + c, device=dev, terrain_seed=5)
        a0, a1 = c * per, (c + len(ids[c:c + step])) * per
        bx[a0:a1], by[a0:a1], bz[a0:a1], brgb[a0:a1] = d.x, d.y, d.z, d.rgb_u16()
        del d
    slot = torch.full((region.tiles_x * region.tiles_y,), -1, dtype=torch.int32, device=dev)
    slot[torch.from_numpy(ids).to(dev)] = torch.arange(splat_tiles, dtype=torch.int32, device=dev)
    keys = torch.zeros((splat_tiles, res, res), dtype=torch.int64, device=dev)
    nd = torch.zeros(1, dtype=torch.int64, device=dev)
    ms = kernel_ms(lambda: ls.splat_points(g, bx, by, bz, brgb, slot, splat_tiles, keys=keys, n_dropped=nd),
                   ["splat"], reps=5, warm=2)["splat"]
    alg = n * 18 + splat_tiles * res * res * 8
    out["splat"] = {"points": n, "tiles": splat_tiles, "ms": ms, "points_per_s": n / (ms * 1e-3),
                    "algorithmic_GBps": alg / (ms * 1e-3) / 1e9, "frac_hbm_peak": alg / (ms * 1e-3) / 1e9 / PEAK_HBM_GBS}
    del bx, by, bz, brgb
    return out


def lsnet_flops(res: int, pad: int) -> float:
    """Multiply-add FLOPs (x2) of one tile through the paper's network as the
    library runs it (the first encoder layers as one 8 -> 64 conv, the FC1
    pair as one GEMM with its zero blocks; the decoders' last layer and the
    final CNN only on the crop grown by the halo the layers after them read:
    3, 2, 1 and 0 texels)."""
    R = res + 2 * pad

    def win(halo):
        return min(R, res + 2 * halo) ** 2

    L = (R // 16) ** 2 * 32
    f = 2 * R * R * 64 * 9 * 8
    f += 4 * 2 * (R // 2) ** 2 * 32 * 9 * 16 + 4 * 2 * (R // 4) ** 2 * 32 * 9 * 32 + 4 * 2 * (R // 8) ** 2 * 32 * 9 * 32
    f += 2 * 512 * 4 * L + 2 * 2 * L * 512
    f += 2 * (2 * (R // 8) ** 2 * 32 * 9 * 32 + 2 * (R // 4) ** 2 * 32 * 9 * 32 + 2 * (R // 2) ** 2 * 16 * 9 * 32
              + 2 * win(3) * 16 * 9 * 16)
    f += 2 * win(2) * 32 * 9 * 40 + 2 * win(1) * 32 * 9 * 32 + 2 * win(0) * 4 * 9 * 32
    return float(f)


def bench_lsnet(work, x_out, cz, dev):
    """The paper's refinement network on the 1024-tile batch: BF16 and FP32."""
    g = ls.Grid.of(work.region)
    nt = x_out.shape[0]
    w = torch.from_numpy(synth.pnet_weights(0, R=g.R).astype(np.float32)).to(dev)
    out = {"network": f"the paper's architecture, {ls.lsnet_num_params(g)} parameters"}
    for name, prec in (("bf16", ls.BF16), ("fp32", ls.FP32)):
        ws = ls.alloc_workspace(ls.workspace_bytes(ls.OP_REFINE_LSNET, g, nt, 0, prec), dev)
        tex = torch.empty((nt, g.res, g.res, 4), dtype=torch.float32, device=dev)
        ms = Timer().run(lambda: ls.lsnet_refine_tiles(w, x_out, cz, g, prec, tex_out=tex, want_y=False, ws=ws),
                         5 if prec == ls.BF16 else 2, 1)
        tf = lsnet_flops(g.res, g.pad) * nt / (ms * 1e-3) / 1e12
        out[name] = {"ms": ms, "tiles_per_s": nt / (ms * 1e-3), "TFLOPs": tf,
                     "frac_peak": tf / (PEAK_BF16_TFLOPS if prec == ls.BF16 else PEAK_FP32_TFLOPS)}
        del ws
    return out


def bench_point_kernels(dev, n_points: int = 100_000_000):
    """Mean splat (ground truth) and point rasteriser on the 100 M-point
    full-resolution set over 64 x 64 tiles."""
    region = synth.Region(tiles_x=64, tiles_y=64)
    g = ls.Grid.of(region)
    ps = synth.fullres_uniform(region, n_points, seed=3, device=dev)
    x, y, z = ps.x.contiguous(), ps.y.contiguous(), ps.z.contiguous()
    rgb = ps.rgb_u16()
    del ps
    nslots = 64 * 64
    ts = torch.arange(nslots, dtype=torch.int32, device=dev)
    acc = torch.zeros((nslots, 64, 64, 5), dtype=torch.int64, device=dev)
    nd = torch.zeros(1, dtype=torch.int64, device=dev)
    ms = kernel_ms(lambda: ls.splat_mean(g, x, y, z, rgb, ts, nslots, acc=acc, n_dropped=nd), ["splat_mean"],
                   reps=5, warm=2)["splat_mean"]
    alg = n_points * 18 + nslots * 4096 * 40
    out = {"splat_mean": {"workload": f"{n_points} points, 64 x 64 tiles, Morton-ordered", "ms": ms,
                          "points_per_s": n_points / (ms * 1e-3), "algorithmic_GBps": alg / (ms * 1e-3) / 1e9,
                          "frac_hbm_peak": alg / (ms * 1e-3) / 1e9 / PEAK_HBM_GBS,
                          "algorithmic_bytes": "18 B per point + 40 B of sums per texel",
                          "traffic": recorded_traffic("ls_target.hip", "splat_mean_100M_points_traffic.md"),
                          "traffic_unit": "HBM bytes per launch (counters)"}}
    del acc
    # a perspective view over the region from 3 km up, 1920 x 1080
    side = 64 * 640.0
    f = 1.2
    M = np.array([[f, 0, 0, -side / 2 * f], [0, f * 16 / 9, 0, -side / 2 * f * 16 / 9], [0, 0, 0, 0],
                  [0, 0, -1, 3000.0]]) / 20000.0
    view = ls.View(m=M, width=1920, height=1080)
    fb = torch.full((1080, 1920), -1, dtype=torch.int64, device=dev)
    nd = torch.zeros(1, dtype=torch.int64, device=dev)
    ms = kernel_ms(lambda: ls.raster_points(view, x, y, z, rgb, fb=fb, n_drawn=nd), ["raster"], reps=5,
                   warm=2)["raster"]
    drawn = int(nd.item()) // 7
    alg = n_points * 18 + 1920 * 1080 * 8
    out["raster"] = {"workload": f"{n_points} points, 1920 x 1080 frame buffer, {drawn} drawn", "ms": ms,
                     "points_per_s": n_points / (ms * 1e-3), "algorithmic_GBps": alg / (ms * 1e-3) / 1e9,
                     "frac_hbm_peak": alg / (ms * 1e-3) / 1e9 / PEAK_HBM_GBS,
                     "traffic": recorded_traffic("ls_raster.hip", "raster_100M_points_traffic.md")
                     if n_points == 100_000_000 else None,
                     "traffic_unit": "HBM bytes per launch (counters)"}
    return out


if __name__ == "__main__":
    main()
