// Streaming of full-resolution points (SoA int32 x, y, z + uint16 rgb[3],
// 18 bytes per point) for the per-point kernels: the max-key splat, the
// ground-truth mean splat and the point rasteriser.  A workgroup of
// PT_THREADS lanes takes a batch of PT_BATCH consecutive points, each lane
// PT_PPT of them as PT_PPT/4 quads (coalesced, non-temporal 16-byte loads
// when the arrays are aligned, point-by-point bounds-checked loads for the
// ragged last batch).
#pragma once

#include "ls_common.hpp"

namespace lsp {

constexpr int PT_THREADS = 256;
#ifndef LS_SPLAT_PPT
#define LS_SPLAT_PPT 8
#endif
constexpr int PT_PPT = LS_SPLAT_PPT;             // points per thread per batch (multiple of 4)
constexpr int PT_QPT = PT_PPT / 4;               // point quads per thread per batch
constexpr int PT_BATCH = PT_THREADS * PT_PPT;    // points per batch
static_assert(PT_PPT % 4 == 0, "points are loaded in quads");

typedef int v4i __attribute__((ext_vector_type(4)));
typedef unsigned int v2u __attribute__((ext_vector_type(2)));

// floor(n / d) for 0 <= n < 2^31 as a multiply-high and shift (Granlund and
// Montgomery, 1994): with l = ceil(log2 d) and m = ceil(2^(31+l) / d) < 2^32,
// floor(n / d) = floor(n * m / 2^(31+l)) exactly over that range.
struct MagicDiv {
  uint32_t m;
  int s;  // 31 + l
  __device__ __forceinline__ int operator()(int64_t n) const {
    return (int)(((uint64_t)(uint32_t)n * m) >> s);
  }
};

static inline MagicDiv magic_div(uint32_t d) {
  int l = 0;
  while ((1ull << l) < d) ++l;
  MagicDiv r;
  r.m = (uint32_t)(((1ull << (31 + l)) + d - 1) / d);
  r.s = 31 + l;
  return r;
}

__device__ __forceinline__ uint32_t spread16(uint32_t v) {
  v &= 0xFFFF;
  v = (v | (v << 8)) & 0x00FF00FF;
  v = (v | (v << 4)) & 0x0F0F0F0F;
  v = (v | (v << 2)) & 0x33333333;
  v = (v | (v << 1)) & 0x55555555;
  return v;
}

__device__ __forceinline__ uint32_t compact16(uint32_t v) {
  v &= 0x55555555;
  v = (v | (v >> 1)) & 0x33333333;
  v = (v | (v >> 2)) & 0x0F0F0F0F;
  v = (v | (v >> 4)) & 0x00FF00FF;
  v = (v | (v >> 8)) & 0x0000FFFF;
  return v;
}

// The point arrays of one call.
struct PointStream {
  int64_t n;
  const int32_t* x;
  const int32_t* y;
  const int32_t* z;
  const uint16_t* rgb;
  int32_t vec_ok;    // x, y, z 16-byte and rgb 8-byte aligned: quad vector loads
  int32_t vec16_ok;  // also rgb 16-byte aligned: 16-byte colour loads
};

static inline PointStream point_stream(const int32_t* x, const int32_t* y, const int32_t* z, const uint16_t* rgb,
                                       int64_t n) {
  auto al = [](const void* q, uintptr_t a) { return (reinterpret_cast<uintptr_t>(q) % a) == 0; };
  PointStream s;
  s.n = n;
  s.x = x;
  s.y = y;
  s.z = z;
  s.rgb = rgb;
  s.vec_ok = (al(x, 16) && al(y, 16) && al(z, 16) && al(rgb, 8)) ? 1 : 0;
  s.vec16_ok = (s.vec_ok && al(rgb, 16)) ? 1 : 0;
  return s;
}

// Raw fields of the PT_PPT points a thread owns in one batch.
struct PointRegs {
  int x[PT_PPT], y[PT_PPT], z[PT_PPT];
  uint32_t c[PT_PPT * 3 / 2];  // 16-bit colours of each quad, two per dword, in input order
  uint32_t valid;              // bit s: point s exists (ragged last batch)
};

// Thread t owns the quads base/4 + k*PT_THREADS + t (k < PT_QPT).  The
// points are streamed once: non-temporal loads keep the output arrays
// resident in the caches instead.
__device__ __forceinline__ void load_points(const PointStream& p, int64_t base, int tid, PointRegs& r) {
  const int64_t q0 = base / 4 + tid;
  if (p.vec_ok && base + PT_BATCH <= p.n) {
#pragma unroll
    for (int k = 0; k < PT_QPT; ++k) {
      const int64_t q = q0 + (int64_t)k * PT_THREADS;
      const v4i xv = __builtin_nontemporal_load(reinterpret_cast<const v4i*>(p.x) + q);
      const v4i yv = __builtin_nontemporal_load(reinterpret_cast<const v4i*>(p.y) + q);
      const v4i zv = __builtin_nontemporal_load(reinterpret_cast<const v4i*>(p.z) + q);
      const v2u* cp = reinterpret_cast<const v2u*>(p.rgb) + 3 * q;
      const v2u c0 = __builtin_nontemporal_load(cp), c1 = __builtin_nontemporal_load(cp + 1),
                c2 = __builtin_nontemporal_load(cp + 2);
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        r.x[4 * k + e] = xv[e];
        r.y[4 * k + e] = yv[e];
        r.z[4 * k + e] = zv[e];
      }
      r.c[6 * k + 0] = c0.x;
      r.c[6 * k + 1] = c0.y;
      r.c[6 * k + 2] = c1.x;
      r.c[6 * k + 3] = c1.y;
      r.c[6 * k + 4] = c2.x;
      r.c[6 * k + 5] = c2.y;
    }
    r.valid = (PT_PPT == 32) ? 0xFFFFFFFFu : ((1u << PT_PPT) - 1u);
    return;
  }
  // ragged or unaligned batch: point by point, bounds-checked
  r.valid = 0;
#pragma unroll
  for (int k = 0; k < PT_QPT; ++k) {
#pragma unroll
    for (int w = 0; w < 6; ++w) r.c[6 * k + w] = 0;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int64_t i = 4 * (q0 + (int64_t)k * PT_THREADS) + e;
      const int s = 4 * k + e;
      r.x[s] = r.y[s] = r.z[s] = 0;
      if (i >= p.n) continue;
      r.valid |= 1u << s;
      r.x[s] = p.x[i];
      r.y[s] = p.y[i];
      r.z[s] = p.z[i];
#pragma unroll
      for (int ch = 0; ch < 3; ++ch) {
        const int v = 3 * e + ch;  // colour value index within the quad
        r.c[6 * k + v / 2] |= (uint32_t)p.rgb[3 * i + ch] << (16 * (v & 1));
      }
    }
  }
}

// Same fields, but thread t owns the PT_PPT consecutive points base +
// PT_PPT*t + s (two 16-byte loads per coordinate array, three for the
// colours): runs of points on one texel stay within a thread, so a kernel
// can sum them in registers first.  point_colour reads both layouts.
__device__ __forceinline__ void load_points_consecutive(const PointStream& p, int64_t base, int tid, PointRegs& r) {
  static_assert(PT_PPT == 8, "two quads per thread");
  const int64_t first = base + (int64_t)PT_PPT * tid;
  if (p.vec16_ok && base + PT_BATCH <= p.n) {
    const int64_t q = first / 4;
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      const v4i xv = __builtin_nontemporal_load(reinterpret_cast<const v4i*>(p.x) + q + k);
      const v4i yv = __builtin_nontemporal_load(reinterpret_cast<const v4i*>(p.y) + q + k);
      const v4i zv = __builtin_nontemporal_load(reinterpret_cast<const v4i*>(p.z) + q + k);
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        r.x[4 * k + e] = xv[e];
        r.y[4 * k + e] = yv[e];
        r.z[4 * k + e] = zv[e];
      }
    }
    // 8 points x 3 colours x 2 bytes = 48 bytes at a 16-byte aligned offset
    typedef unsigned int v4u __attribute__((ext_vector_type(4)));
    const v4u* cp = reinterpret_cast<const v4u*>(p.rgb + 3 * first);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const v4u cv = __builtin_nontemporal_load(cp + k);
#pragma unroll
      for (int e = 0; e < 4; ++e) r.c[4 * k + e] = cv[e];
    }
    r.valid = (1u << PT_PPT) - 1u;
    return;
  }
  r.valid = 0;
#pragma unroll
  for (int w = 0; w < PT_PPT * 3 / 2; ++w) r.c[w] = 0;
#pragma unroll
  for (int s = 0; s < PT_PPT; ++s) {
    const int64_t i = first + s;
    r.x[s] = r.y[s] = r.z[s] = 0;
    if (i >= p.n) continue;
    r.valid |= 1u << s;
    r.x[s] = p.x[i];
    r.y[s] = p.y[i];
    r.z[s] = p.z[i];
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) {
      const int v = 3 * s + ch;
      r.c[v / 2] |= (uint32_t)p.rgb[3 * i + ch] << (16 * (v & 1));
    }
  }
}

// 16-bit colour channel ch of point s.
__device__ __forceinline__ uint32_t point_colour(const PointRegs& r, int s, int ch) {
  const int k = s >> 2, v = 3 * (s & 3) + ch;
  const uint32_t w = r.c[6 * k + v / 2];
  return (v & 1) ? (w >> 16) : (w & 0xFFFFu);
}

// Texel grid of a region: texel (gx, gy) = floor((x - ox) / C), floor((y -
// oy) / C); its tile (gx / res, gy / res) has an output slot or -1.
struct TexelGrid {
  int64_t ox, oy;
  int32_t C, res, tiles_x, tiles_y;
  MagicDiv divC, divR;
  int32_t gw, gh;     // global texel extent
  int32_t n_slots;
  int32_t morton_ok;  // gw, gh <= 65536: 16-bit Morton halves
  const int32_t* tile_slot;
};

// Fills the grid from the host description; LS_ERANGE when texel
// coordinates times the cell would not fit 31 bits.
static inline int texel_grid(const LsGridInfo& gi, const int32_t* tile_slot, int32_t n_slots, TexelGrid& t) {
  t.ox = gi.ox;
  t.oy = gi.oy;
  t.C = gi.C;
  t.res = gi.res;
  t.divC = magic_div((uint32_t)gi.C);
  t.divR = magic_div((uint32_t)gi.res);
  t.tiles_x = gi.tx;
  t.tiles_y = gi.ty;
  const int64_t gw = (int64_t)gi.tx * gi.res, gh = (int64_t)gi.ty * gi.res;
  if (gw * gi.C >= 0x7fffffffLL || gh * gi.C >= 0x7fffffffLL) return LS_ERANGE;
  t.gw = (int32_t)gw;
  t.gh = (int32_t)gh;
  t.n_slots = n_slots;
  t.morton_ok = (gw <= 65536 && gh <= 65536) ? 1 : 0;
  t.tile_slot = tile_slot;
  return LS_OK;
}

// Texel of a point; false (dropped) outside the region or in an unmapped
// tile.
__device__ __forceinline__ bool point_texel(const TexelGrid& p, int xi, int yi, int& gx, int& gy) {
  const int64_t dx = (int64_t)xi - p.ox, dy = (int64_t)yi - p.oy;
  if (dx < 0 || dy < 0) return false;
  if (dx >= (int64_t)p.gw * p.C || dy >= (int64_t)p.gh * p.C) return false;
  gx = p.divC(dx);
  gy = p.divC(dy);
  const int tx = p.divR(gx), ty = p.divR(gy);
  const int32_t s = p.tile_slot[ty * p.tiles_x + tx];
  return s >= 0 && s < p.n_slots;
}

// Index of texel (gx, gy) in the [slot][res][res] arrays; the tile must be
// mapped.
__device__ __forceinline__ int64_t texel_index(const TexelGrid& p, int gx, int gy) {
  const int tx = p.divR(gx), ty = p.divR(gy);
  const int s = p.tile_slot[ty * p.tiles_x + tx];
  return ((int64_t)s * p.res + (gy - ty * p.res)) * p.res + (gx - tx * p.res);
}

// Block-wide minimum and maximum of per-thread values (256 lanes), returned
// as wave-uniform values so that barriers after it stay in uniform flow.
// s_lo, s_hi hold 2 x 4 words: consecutive calls (batches) alternate halves
// (parity), so a wave that runs ahead into the next batch cannot overwrite
// a value another wave has yet to read (there is one barrier per call).
__device__ __forceinline__ void block_min_max(uint32_t& lo, uint32_t& hi, uint32_t* s_lo, uint32_t* s_hi,
                                              int parity) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  constexpr int NW = PT_THREADS / 64;
  s_lo += parity * NW;
  s_hi += parity * NW;
  for (int o = 32; o > 0; o >>= 1) {
    lo = min(lo, (uint32_t)__shfl_xor((int)lo, o, 64));
    hi = max(hi, (uint32_t)__shfl_xor((int)hi, o, 64));
  }
  if (lane == 0) {
    s_lo[wave] = lo;
    s_hi[wave] = hi;
  }
  __syncthreads();
  uint32_t blo = s_lo[0], bhi = s_hi[0];
#pragma unroll
  for (int w = 1; w < NW; ++w) {
    blo = min(blo, s_lo[w]);
    bhi = max(bhi, s_hi[w]);
  }
  lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)blo);
  hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)bhi);
}

// Adds a per-thread count into *dst with one global atomic per workgroup.
__device__ __forceinline__ void block_count_add(unsigned long long v, unsigned long long* s_part,
                                                unsigned long long* dst) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int o = 32; o > 0; o >>= 1) v += (unsigned long long)__shfl_xor((long long)v, o, 64);
  if (lane == 0) s_part[wave] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long d = 0;
    for (int w = 0; w < PT_THREADS / 64; ++w) d += s_part[w];
    if (d && dst) atomicAdd(dst, d);
  }
}

}  // namespace lsp
