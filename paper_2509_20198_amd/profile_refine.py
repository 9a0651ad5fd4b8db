"""Per-launch times of the refinement network on synthetic tiles, for
profilers: the BF16 forward of the 1024-tile batch (after its
reconstruction) and the BF16 forward + backward of the 256-tile training
batch, each repeated a few times with the default tilings, so that a
kernel trace or counter run sees exactly these launches.

    python -m paper_2509_20198_amd.profile_refine [--reps N] [--part forward|backward|both]

Prints one JSON line per part: the median time of each traced launch group
(HIP events on the library's stream) and their sum.
"""
from __future__ import annotations

import argparse
import json
import os
import sys

import numpy as np
import torch

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))

import paper_2509_20198_amd as ls  # noqa: E402
import synth  # noqa: E402


def _traced(fn, reps: int):
    for _ in range(2):
        fn()
    torch.cuda.synchronize()
    ls.trace_enable(True)
    for _ in range(reps):
        fn()
    torch.cuda.synchronize()
    rec = ls.trace_records()
    ls.trace_enable(False)
    per = len(rec) // reps
    t = np.array([ms for _, ms in rec[:per * reps]]).reshape(reps, per)
    med = np.median(t, 0)
    groups: dict = {}
    for (n, _), m in zip(rec[:per], med):
        groups[n] = groups.get(n, 0.0) + float(m)
    return {"total_ms": round(float(med.sum()), 4), "launches": per,
            "by_group_ms": {k: round(v, 4) for k, v in sorted(groups.items(), key=lambda kv: -kv[1])},
            "sequence": [(n, round(float(m), 4)) for (n, _), m in zip(rec[:per], med)]}


def forward(dev, reps: int):
    work = synth.batch_tiles(seed=2, device=dev)
    g = ls.Grid.of(work.region)
    ps = work.points
    tl = torch.from_numpy(work.tile_list).to(dev)
    nt = len(work.tile_list)
    x, cz, _ = ls.recon_tiles(g, ps.x, ps.y, ps.z, ps.rgb_u16(), tl)
    w = torch.from_numpy(synth.unet_weights(0).astype(np.float32)).to(dev)
    wb = ls.pack_weights_bf16(w)
    ws = ls.alloc_workspace(ls.workspace_bytes(ls.OP_REFINE, g, nt, 0, ls.BF16), dev)
    tex = torch.empty((nt, g.res, g.res, 4), device=dev)
    out = _traced(lambda: ls.refine_tiles(w, x, cz, g, ls.BF16, w_bf16=wb, tex_out=tex, want_y=False, ws=ws), reps)
    return {"part": "forward", "workload": f"{nt} tiles (batch_1024_tiles), BF16", **out}


def backward(dev, reps: int):
    work = synth.train_tiles(seed=4, device=dev)
    g = ls.Grid.of(work.region)
    ps = work.points
    tl = torch.from_numpy(work.tile_list).to(dev)
    nt = len(work.tile_list)
    x, cz, _ = ls.recon_tiles(g, ps.x, ps.y, ps.z, ps.rgb_u16(), tl)
    w0 = torch.from_numpy(synth.unet_weights(1).astype(np.float32)).to(dev)
    wb = ls.pack_weights_bf16(w0)
    gy = torch.randn((nt, g.res, g.res, 4), device=dev, generator=torch.Generator(device=dev).manual_seed(0))
    act = torch.empty(ls.act_bytes(g, nt, ls.BF16), dtype=torch.uint8, device=dev)
    ws = ls.alloc_workspace(ls.workspace_bytes(ls.OP_BACKWARD, g, nt, 0, ls.BF16), dev)
    gw = torch.empty_like(w0)

    def step():
        ls.refine_tiles(w0, x, cz, g, ls.BF16, w_bf16=wb, act_save=act, want_y=True, want_tex=False, ws=ws)
        ls.refine_backward(w0, x, gy, g, ls.BF16, w_bf16=wb, act_save=act, grad_w=gw, ws=ws)

    out = _traced(step, reps)
    return {"part": "backward", "workload": f"{nt} tiles (train_256_tiles), BF16 forward + backward", **out}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--part", choices=("forward", "backward", "both"), default="both")
    args = ap.parse_args()
    if not torch.cuda.is_available():
        print("profile_refine needs a GPU", file=sys.stderr)
        sys.exit(2)
    dev = torch.device("cuda:0")
    ls.load_library()
    if args.part in ("forward", "both"):
        print(json.dumps(forward(dev, args.reps)), flush=True)
    if args.part in ("backward", "both"):
        print(json.dumps(backward(dev, args.reps)), flush=True)


if __name__ == "__main__":
    main()
