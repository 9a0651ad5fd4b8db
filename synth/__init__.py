"""Seeded synthetic inputs shaped like LidarScout's workloads.

This module is the one place both the FP64 oracle and the HIP path take
their inputs from.  It holds none of the method's arithmetic (no binning,
interpolation, network or splat): only terrain, point sets, tile lists and
network weights, all derived from counter-based hashes so that the same
seed gives bit-identical integers on the CPU and on the GPU.

Every random draw goes through splitmix64 (Vigna's published 64-bit mixer:
add the golden-ratio increment, then two xor-shift-multiply rounds and a
final xor-shift).  torch int64 arithmetic wraps modulo 2**64, which is the
unsigned arithmetic the mixer is defined in; right shifts are made logical
by masking.

Terrain (all lengths in LAS raw units, 1 raw = 1 cm):
  z_m(x, y) = 50 * sum_{o=0..3} 0.5**o * V_o(x, y) / 1.875   [metres]
with V_o value noise of wavelength 20000 / 2**o raw (200 m down to 25 m),
lattice values uniform in [-1, 1) from splitmix64 of (octave, i, j, seed),
bilinear blending with a smoothstep fade.  z_raw = rint(100 * z_m), ties to
even.  Colour is a uint8 height ramp v = clamp(round((z_m + 50) / 100 * 255))
stored as 16-bit LAS colour (R, G, B) = (v, 255 - v, 128) * 257.

The paper's data sets (airborne LIDAR and photogrammetry scans, Table 1 of
Section 3.1) are not available; these point sets stand in for them.  Sparse
per-tile counts span the paper's chunk-point densities (one point per
50,000, Section 3.2) and full-resolution sizes match the 50-300 million
points a close-up loads (Section 3.5).
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np
import torch

# ----------------------------------------------------------------------------
# counter-based hashing (splitmix64) on int64 tensors
# ----------------------------------------------------------------------------
_MASK64 = (1 << 64) - 1


def _s64(v: int) -> int:
    """Reinterpret an unsigned 64-bit constant as a signed int64."""
    v &= _MASK64
    return v - (1 << 64) if v >= (1 << 63) else v


_GOLDEN = _s64(0x9E3779B97F4A7C15)
_MIX1 = _s64(0xBF58476D1CE4E5B9)
_MIX2 = _s64(0x94D049BB133111EB)


def _srl(x: torch.Tensor, k: int) -> torch.Tensor:
    return (x >> k) & ((1 << (64 - k)) - 1)


def splitmix64(x: torch.Tensor) -> torch.Tensor:
    """splitmix64 output function applied elementwise to an int64 tensor."""
    z = x + _GOLDEN
    z = (z ^ _srl(z, 30)) * _MIX1
    z = (z ^ _srl(z, 27)) * _MIX2
    return z ^ _srl(z, 31)


def splitmix64_int(x: int) -> int:
    """Scalar splitmix64 on Python ints (unsigned result)."""
    z = (x + 0x9E3779B97F4A7C15) & _MASK64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _MASK64
    return z ^ (z >> 31)


def hash2(seed: int, k: torch.Tensor) -> torch.Tensor:
    """Hash of (seed, counter): splitmix64(seed ^ splitmix64(k))."""
    return splitmix64(splitmix64(k) ^ _s64(seed))


def uniform01(h: torch.Tensor) -> torch.Tensor:
    """Top 53 bits of a hash as a float64 in [0, 1)."""
    return _srl(h, 11).to(torch.float64) * (2.0 ** -53)


def tile_seed(base_seed: int, tile_id: int) -> int:
    return splitmix64_int((base_seed ^ tile_id) & _MASK64)


# ----------------------------------------------------------------------------
# terrain
# ----------------------------------------------------------------------------
TERRAIN_AMPLITUDE_M = 50.0
TERRAIN_OCTAVES = 4
TERRAIN_BASE_WAVELENGTH = 20000  # raw units (200 m)


def _lattice(seed: int, octave: int, i: torch.Tensor, j: torch.Tensor) -> torch.Tensor:
    so = splitmix64_int((seed * 0x100000001B3 + octave) & _MASK64)
    key = (i << 32) ^ (j & 0xFFFFFFFF)
    h = splitmix64(splitmix64(key) ^ _s64(so))
    return uniform01(h) * 2.0 - 1.0


def terrain_m(x: torch.Tensor, y: torch.Tensor, seed: int) -> torch.Tensor:
    """fBm value-noise height in metres at integer raw coordinates (int64)."""
    x = x.to(torch.int64)
    y = y.to(torch.int64)
    total = torch.zeros(x.shape, dtype=torch.float64, device=x.device)
    for o in range(TERRAIN_OCTAVES):
        lam = TERRAIN_BASE_WAVELENGTH >> o
        i = torch.div(x, lam, rounding_mode="floor")
        j = torch.div(y, lam, rounding_mode="floor")
        fx = (x - i * lam).to(torch.float64) / lam
        fy = (y - j * lam).to(torch.float64) / lam
        sx = fx * fx * (3.0 - 2.0 * fx)
        sy = fy * fy * (3.0 - 2.0 * fy)
        l00 = _lattice(seed, o, i, j)
        l10 = _lattice(seed, o, i + 1, j)
        l01 = _lattice(seed, o, i, j + 1)
        l11 = _lattice(seed, o, i + 1, j + 1)
        a = l00 * (1.0 - sx) + l10 * sx
        b = l01 * (1.0 - sx) + l11 * sx
        total = total + (0.5 ** o) * (a * (1.0 - sy) + b * sy)
    return TERRAIN_AMPLITUDE_M * total / 1.875


def ramp_rgb(z_m: torch.Tensor) -> torch.Tensor:
    """uint8 height ramp stored as 16-bit colour, shape [n, 3] (int32 values)."""
    v = torch.clamp(torch.round((z_m + 50.0) / 100.0 * 255.0), 0, 255).to(torch.int32)
    rgb = torch.stack([v, 255 - v, torch.full_like(v, 128)], dim=1) * 257
    return rgb


def gaussian(seed: int, k: torch.Tensor) -> torch.Tensor:
    """Box-Muller standard normal from two hashed uniforms per counter."""
    u1 = 1.0 - uniform01(hash2(seed, 2 * k))
    u2 = uniform01(hash2(seed, 2 * k + 1))
    return torch.sqrt(-2.0 * torch.log(u1)) * torch.cos(2.0 * math.pi * u2)


# ----------------------------------------------------------------------------
# region / point sets
# ----------------------------------------------------------------------------
@dataclasses.dataclass
class Region:
    origin_x: int = 0
    origin_y: int = 0
    tile_size: int = 64000  # raw units (640 m)
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

    @property
    def cell(self) -> int:
        return self.tile_size // self.res


@dataclasses.dataclass
class PointSet:
    """SoA point arrays: int32 x, y, z and uint16 colour stored as int32 [n, 3]."""
    x: torch.Tensor
    y: torch.Tensor
    z: torch.Tensor
    rgb: torch.Tensor

    @property
    def n(self) -> int:
        return int(self.x.numel())

    def to(self, device) -> "PointSet":
        return PointSet(self.x.to(device), self.y.to(device), self.z.to(device), self.rgb.to(device))

    def rgb_u16(self) -> torch.Tensor:
        """Colour as uint16 bit patterns in an int16 tensor (for device upload)."""
        r = self.rgb.to(torch.int32)
        return torch.where(r >= 32768, r - 65536, r).to(torch.int16).contiguous()

    def numpy(self):
        return (self.x.cpu().numpy().astype(np.int32), self.y.cpu().numpy().astype(np.int32),
                self.z.cpu().numpy().astype(np.int32), self.rgb.cpu().numpy().astype(np.uint16))


def _points_in_tiles(region: Region, tile_ids: np.ndarray, counts: np.ndarray, seed: int,
                     terrain_seed: int, noise_sigma_m: float, device) -> PointSet:
    """Uniform integer xy inside each listed tile, terrain z (plus optional noise)."""
    counts = np.asarray(counts, dtype=np.int64)
    tile_ids = np.asarray(tile_ids, dtype=np.int64)
    n = int(counts.sum())
    seeds = np.array([_s64(tile_seed(seed, int(t))) for t in tile_ids], dtype=np.int64)
    dev = torch.device(device)
    cnt = torch.from_numpy(counts).to(dev)
    tid = torch.from_numpy(tile_ids).to(dev)
    sd = torch.from_numpy(seeds).to(dev)
    owner = torch.repeat_interleave(torch.arange(len(counts), device=dev), cnt)
    start = torch.cumsum(cnt, 0) - cnt
    k = torch.arange(n, device=dev, dtype=torch.int64) - start[owner]
    s = sd[owner]
    hx = splitmix64(splitmix64(2 * k) ^ s)
    hy = splitmix64(splitmix64(2 * k + 1) ^ s)
    S = region.tile_size
    tx = tid[owner] % region.tiles_x
    ty = tid[owner] // region.tiles_x
    x = region.origin_x + tx * S + _srl(hx, 1) % S
    y = region.origin_y + ty * S + _srl(hy, 1) % S
    zm = terrain_m(x, y, terrain_seed)
    if noise_sigma_m > 0:
        g = gaussian(seed ^ 0x5EED, torch.arange(n, device=dev, dtype=torch.int64))
        zm = zm + noise_sigma_m * g
    z = torch.round(zm * 100.0).to(torch.int32)
    rgb = ramp_rgb(zm)
    return PointSet(x.to(torch.int32), y.to(torch.int32), z, rgb)


def shuffle(ps: PointSet, seed: int) -> PointSet:
    """Global seeded permutation (so binning cannot exploit input order)."""
    dev = ps.x.device
    key = hash2(seed, torch.arange(ps.n, device=dev, dtype=torch.int64))
    perm = torch.argsort(key, stable=True)
    return PointSet(ps.x[perm], ps.y[perm], ps.z[perm], ps.rgb[perm])


def _spread_bits(v: torch.Tensor) -> torch.Tensor:
    v = v & 0xFFFF
    v = (v | (v << 8)) & 0x00FF00FF
    v = (v | (v << 4)) & 0x0F0F0F0F
    v = (v | (v << 2)) & 0x33333333
    v = (v | (v << 1)) & 0x55555555
    return v


def morton_sort(ps: PointSet, region: Region, seed: int) -> PointSet:
    """Order by Morton code of the global texel cell, ties by a seeded shuffle."""
    dev = ps.x.device
    C = region.cell
    gx = torch.div(ps.x.to(torch.int64) - region.origin_x, C, rounding_mode="floor").clamp(0, 65535)
    gy = torch.div(ps.y.to(torch.int64) - region.origin_y, C, rounding_mode="floor").clamp(0, 65535)
    code = _spread_bits(gx) | (_spread_bits(gy) << 1)
    tie = _srl(hash2(seed, torch.arange(ps.n, device=dev, dtype=torch.int64)), 44)
    perm = torch.argsort((code << 20) | tie, stable=True)
    return PointSet(ps.x[perm], ps.y[perm], ps.z[perm], ps.rgb[perm])


# ----------------------------------------------------------------------------
# per-tile sparse counts
# ----------------------------------------------------------------------------
def _u(seed: int, t: int, stream: int) -> float:
    return (splitmix64_int((tile_seed(seed, t) ^ (0xC0FFEE + stream)) & _MASK64) >> 11) * 2.0 ** -53


def counts_loguniform(seed: int, n_tiles: int, lo: int = 50, ratio: float = 40.0) -> np.ndarray:
    """n_t = floor(lo * ratio**u): log-uniform in [lo, lo*ratio)."""
    return np.array([int(math.floor(lo * ratio ** _u(seed, t, 0))) for t in range(n_tiles)], np.int64)


def counts_uniform(seed: int, n_tiles: int, lo: int, hi: int) -> np.ndarray:
    """n_t uniform integer in [lo, hi]."""
    return np.array([lo + int(_u(seed, t, 1) * (hi - lo + 1)) for t in range(n_tiles)], np.int64)


def counts_pareto(seed: int, n_tiles: int, xmin: int = 20, alpha: float = 1.5, cap: int = 5000) -> np.ndarray:
    """n_t = min(cap, floor(xmin * u**(-1/alpha))), u in (0, 1]."""
    out = []
    for t in range(n_tiles):
        u = 1.0 - _u(seed, t, 2)
        out.append(min(cap, int(math.floor(xmin * u ** (-1.0 / alpha)))))
    return np.array(out, np.int64)


# ----------------------------------------------------------------------------
# network weights (pinned 3-level U-Net, 119,844 parameters)
# ----------------------------------------------------------------------------
#: (name, Cin, Cout) per 3x3 layer, in storage order; each layer stores
#: W[Cout][3][3][Cin] followed by b[Cout].
UNET_SHAPES = [
    ("enc1a", 8, 16), ("enc1b", 16, 16),
    ("enc2a", 16, 32), ("enc2b", 32, 32),
    ("bot_a", 32, 64), ("bot_b", 64, 64),
    ("dec2a", 96, 32), ("dec2b", 32, 32),
    ("dec1a", 48, 16), ("dec1b", 16, 16),
    ("head", 24, 4),
]
N_PARAMS = sum(co * 9 * ci + co for _, ci, co in UNET_SHAPES)


def unet_weights(seed: int = 0, head_std: Optional[float] = None, bias_std: float = 0.0) -> np.ndarray:
    """Kaiming-normal (fan_in, gain sqrt 2) hidden layers, small-normal head, biases 0.

    head_std defaults to 0.01 / sqrt(216).  bias_std > 0 draws N(0, bias_std^2)
    biases (used by tests so that bias arithmetic is exercised).
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    parts = []
    for name, ci, co in UNET_SHAPES:
        fan_in = 9 * ci
        std = (0.01 / math.sqrt(216.0) if head_std is None else head_std) if name == "head" \
            else math.sqrt(2.0 / fan_in)
        parts.append(rng.standard_normal(co * fan_in) * std)
        if bias_std > 0:
            parts.append(rng.standard_normal(co) * bias_std)
        else:
            parts.append(np.zeros(co))
    w = np.concatenate(parts)
    assert w.size == N_PARAMS
    return w


# ----------------------------------------------------------------------------
# workload configurations
# ----------------------------------------------------------------------------
@dataclasses.dataclass
class SparseWorkload:
    name: str
    region: Region
    points: PointSet
    tile_list: np.ndarray  # int32 linear tile ids in processing (priority) order
    counts: np.ndarray     # own-tile sparse counts, indexed by linear tile id


def sparse_workload(name: str, tiles_x: int, tiles_y: int, counts: np.ndarray, seed: int,
                    order: str = "desc", viewpoint=None, pad: int = 16, res: int = 64,
                    device="cpu", tile_size: int = 64000) -> SparseWorkload:
    region = Region(tiles_x=tiles_x, tiles_y=tiles_y, pad=pad, res=res, tile_size=tile_size)
    ids = np.arange(tiles_x * tiles_y, dtype=np.int64)
    ps = _points_in_tiles(region, ids, counts, seed, terrain_seed=seed, noise_sigma_m=0.0, device=device)
    ps = shuffle(ps, seed ^ 0xABCDEF)
    if order == "desc":
        tl = sorted(ids.tolist(), key=lambda t: (-int(counts[t]), t))
    elif order == "view":
        vx, vy = viewpoint
        S = region.tile_size
        def d2(t):
            cx = (t % tiles_x) * S + S // 2
            cy = (t // tiles_x) * S + S // 2
            return ((cx - vx) ** 2 + (cy - vy) ** 2, t)
        tl = sorted(ids.tolist(), key=d2)
    else:
        tl = ids.tolist()
    return SparseWorkload(name, region, ps, np.asarray(tl, np.int32), counts)


def single_tile(seed: int = 1, n: int = 400, pad: int = 16, res: int = 64, device="cpu") -> SparseWorkload:
    """One 640 m tile, n sparse points (400 for the single-tile case)."""
    return sparse_workload("single_tile_400", 1, 1, np.array([n]), seed, order="id", pad=pad, res=res,
                           device=device)


def batch_tiles(seed: int = 2, tiles_x: int = 32, tiles_y: int = 32, device="cpu", pad: int = 16) -> SparseWorkload:
    """32x32 tiles, log-uniform sparse counts in [50, 2000), processed in descending count."""
    counts = counts_loguniform(seed, tiles_x * tiles_y)
    return sparse_workload(f"batch_{tiles_x * tiles_y}_tiles", tiles_x, tiles_y, counts, seed,
                           order="desc", pad=pad, device=device)


def train_tiles(seed: int = 4, tiles_x: int = 16, tiles_y: int = 16, device="cpu") -> SparseWorkload:
    counts = counts_uniform(seed, tiles_x * tiles_y, 200, 800)
    return sparse_workload(f"train_{tiles_x * tiles_y}_tiles", tiles_x, tiles_y, counts, seed,
                           order="id", device=device)


def stream_tiles(seed: int = 5, tiles_x: int = 128, tiles_y: int = 128, device="cpu") -> SparseWorkload:
    counts = counts_pareto(seed, tiles_x * tiles_y)
    S = 64000
    vx = int(_u(seed, 0, 7) * tiles_x * S)
    vy = int(_u(seed, 0, 8) * tiles_y * S)
    return sparse_workload(f"stream_{tiles_x * tiles_y}_tiles", tiles_x, tiles_y, counts, seed,
                           order="view", viewpoint=(vx, vy), device=device)


def fullres_points(region: Region, tile_ids, n_per_tile: int, seed: int, noise_sigma_m: float = 0.1,
                   device="cpu", terrain_seed: Optional[int] = None) -> PointSet:
    """Dense points, uniform xy within each listed tile, Morton-ordered by 10 m cell."""
    tile_ids = np.asarray(tile_ids, dtype=np.int64)
    counts = np.full(len(tile_ids), n_per_tile, dtype=np.int64)
    ps = _points_in_tiles(region, tile_ids, counts, seed,
                          terrain_seed=seed if terrain_seed is None else terrain_seed,
                          noise_sigma_m=noise_sigma_m, device=device)
    return morton_sort(ps, region, seed ^ 0x77)


def fullres_uniform(region: Region, n: int, seed: int, noise_sigma_m: float = 0.1, device="cpu") -> PointSet:
    """n dense points uniform over the whole region, Morton-ordered by 10 m cell."""
    dev = torch.device(device)
    k = torch.arange(n, device=dev, dtype=torch.int64)
    W = region.tiles_x * region.tile_size
    H = region.tiles_y * region.tile_size
    x = region.origin_x + _srl(hash2(seed, 2 * k), 1) % W
    y = region.origin_y + _srl(hash2(seed, 2 * k + 1), 1) % H
    zm = terrain_m(x, y, seed)
    if noise_sigma_m > 0:
        zm = zm + noise_sigma_m * gaussian(seed ^ 0x5EED, k)
    ps = PointSet(x.to(torch.int32), y.to(torch.int32), torch.round(zm * 100.0).to(torch.int32), ramp_rgb(zm))
    return morton_sort(ps, region, seed ^ 0x77)


# ----------------------------------------------------------------------------
# the paper's refinement network: layer list and random initialisation
# ----------------------------------------------------------------------------
def pnet_layers(R: int = 96):
    """[(name, kind, cin, cout)] in weight order; kind "conv" (3x3) or "fc"."""
    F = (R // 16) ** 2 * 32
    out = []
    for i, (nm, c0) in enumerate((("hlin", 1), ("hnn", 1), ("rgblin", 3), ("rgbnn", 3))):
        ch = [c0, 16, 32, 32, 32]
        out += [(f"enc_{nm}{k + 1}", "conv", ch[k], ch[k + 1]) for k in range(4)]
    out += [("fc1_h", "fc", 2 * F, 256), ("fc1_c", "fc", 2 * F, 256), ("fc2_h", "fc", 512, F), ("fc2_t", "fc", 512, F)]
    d = [32, 32, 32, 16, 16]
    out += [(f"dec_h{k + 1}", "conv", d[k], d[k + 1]) for k in range(4)]
    out += [(f"dec_t{k + 1}", "conv", d[k], d[k + 1]) for k in range(4)]
    out += [("fin1", "conv", 40, 32), ("fin2", "conv", 32, 32), ("fin3", "conv", 32, 4)]
    return out


def pnet_layer_size(kind: str, cin: int, cout: int) -> int:
    return cout * 9 * cin + cout if kind == "conv" else cout * cin + cout


def pnet_weights(seed: int = 0, R: int = 96, final_std: Optional[float] = None, bias_std: float = 0.0) -> np.ndarray:
    """Kaiming-normal (fan_in, gain sqrt 2) hidden layers, small-normal final
    layer (default 0.01 / sqrt(288)), biases 0 (or N(0, bias_std^2))."""
    rng = np.random.Generator(np.random.PCG64(seed))
    parts = []
    layers = pnet_layers(R)
    for name, kind, ci, co in layers:
        fan_in = 9 * ci if kind == "conv" else ci
        std = (0.01 / math.sqrt(288.0) if final_std is None else final_std) if name == "fin3" \
            else math.sqrt(2.0 / fan_in)
        n_w = co * 9 * ci if kind == "conv" else co * ci
        parts.append(rng.standard_normal(n_w) * std)
        parts.append(rng.standard_normal(co) * bias_std if bias_std > 0 else np.zeros(co))
    return np.concatenate(parts)
