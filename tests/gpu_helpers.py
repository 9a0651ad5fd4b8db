"""Shared helpers for the GPU parity tests (inputs to device, oracle runs)."""
import numpy as np
import torch

import oracle
import synth

R_M = 480.0  # padded half side in metres (64000/2 + 16*1000 raw at 0.01 m)


def dev():
    return torch.device("cuda:0")


def points_to_dev(ps: synth.PointSet):
    d = dev()
    return (ps.x.to(d).contiguous(), ps.y.to(d).contiguous(), ps.z.to(d).contiguous(),
            ps.rgb_u16().to(d).contiguous())


def arrays_to_dev(x, y, z, rgb):
    d = dev()
    r = np.asarray(rgb).reshape(-1, 3).astype(np.int32)
    r = np.where(r >= 32768, r - 65536, r).astype(np.int16)
    return (torch.from_numpy(np.ascontiguousarray(x, np.int32)).to(d),
            torch.from_numpy(np.ascontiguousarray(y, np.int32)).to(d),
            torch.from_numpy(np.ascontiguousarray(z, np.int32)).to(d),
            torch.from_numpy(np.ascontiguousarray(r)).to(d))


def oracle_recon(region, ps_numpy, tile_list):
    x, y, z, rgb = ps_numpy
    return oracle.recon_tiles(region, x, y, z, rgb, tile_list)


def rms_per_tile(a, b):
    d = (np.asarray(a, np.float64) - np.asarray(b, np.float64))
    return np.sqrt((d ** 2).reshape(d.shape[0], -1).mean(1))
