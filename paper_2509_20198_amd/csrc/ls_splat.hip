// Full-resolution splat into the heightmap textures and the resolve pass
// (LidarScout Sections 3.5-3.6) for gfx950.
//
// Each point becomes a 64-bit key, orderable height in the high word and
// 8-bit colour below it, and every texel keeps the maximum key (its highest
// point), the packed-atomic idea the paper uses for its point rasteriser.
// The maximum is commutative, so the result is bit-exact for any order.
//
// k_splat: a workgroup takes a batch of SPLAT_BATCH consecutive points
// (coalesced, non-temporal SoA quad loads).  When the batch's texels fall in
// a short range of Morton codes (the case for Morton-ordered full-resolution
// chunks), the batch is first reduced in LDS with 64-bit max (one slot per
// Morton code) and then flushed with one global 64-bit atomic max per
// touched texel; otherwise every point goes straight to a global atomic max.
// The small window (16 KB) lets several workgroups share a CU,
// so the loads of some overlap the LDS phases of others.
#include <algorithm>

#include "ls_common.hpp"

namespace {

constexpr int SPLAT_THREADS = 256;
#ifndef LS_SPLAT_PPT
#define LS_SPLAT_PPT 8
#endif
#ifndef LS_SPLAT_WIN
#define LS_SPLAT_WIN 2048
#endif
constexpr int SPLAT_PPT = LS_SPLAT_PPT;                 // points per thread per batch (multiple of 4)
constexpr int SPLAT_QPT = SPLAT_PPT / 4;                // point quads per thread per batch
constexpr int SPLAT_BATCH = SPLAT_THREADS * SPLAT_PPT;  // points per batch
constexpr int SPLAT_WIN = LS_SPLAT_WIN;                 // LDS window of 64-bit keys
static_assert(SPLAT_PPT % 4 == 0, "points are loaded in quads");

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

static MagicDiv magic_div(uint32_t d) {
  int l = 0;
  while ((1ull << l) < d) ++l;
  MagicDiv r;
  r.m = (uint32_t)(((1ull << (31 + l)) + d - 1) / d);
  r.s = 31 + l;
  return r;
}

struct SplatParams {
  int64_t ox, oy;
  int32_t C, res, tiles_x, tiles_y;
  MagicDiv divC, divR;
  int32_t gw, gh;  // global texel extent
  int32_t n_slots;
  int32_t morton_ok;
  int32_t vec_ok;  // x, y, z 16-byte and rgb 8-byte aligned: quad vector loads
  int64_t n;
  const int32_t* x;
  const int32_t* y;
  const int32_t* z;
  const uint16_t* rgb;
  const int32_t* tile_slot;
  unsigned long long* keys;
  unsigned long long* n_dropped;
};

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

// texel index of (gx, gy) in the key array; the tile must be mapped
__device__ __forceinline__ int64_t cell_of(const SplatParams& p, int gx, int gy) {
  const int tx = p.divR(gx), ty = p.divR(gy);
  const int s = p.tile_slot[ty * p.tiles_x + tx];
  return ((int64_t)s * p.res + (gy - ty * p.res)) * p.res + (gx - tx * p.res);
}

// Key and texel of one point; returns false (dropped) outside the region or
// in an unmapped tile.
__device__ __forceinline__ bool point_key(const SplatParams& p, int xi, int yi, int zi, uint32_t r, uint32_t g,
                                          uint32_t b, unsigned long long& key, int& gx, int& gy) {
  const int64_t dx = (int64_t)xi - p.ox, dy = (int64_t)yi - p.oy;
  if (dx < 0 || dy < 0) return false;
  if (dx >= (int64_t)p.gw * p.C || dy >= (int64_t)p.gh * p.C) return false;
  gx = p.divC(dx);
  gy = p.divC(dy);
  const int tx = p.divR(gx), ty = p.divR(gy);
  const int32_t s = p.tile_slot[ty * p.tiles_x + tx];
  if (s < 0 || s >= p.n_slots) return false;
  const uint32_t zz = (uint32_t)zi ^ 0x80000000u;
  key = ((unsigned long long)zz << 32) | ((unsigned long long)(r >> 8) << 24) | ((unsigned long long)(g >> 8) << 16) |
        ((unsigned long long)(b >> 8) << 8) | 0xFFull;
  return true;
}

// Raw fields of the SPLAT_PPT points a thread owns in one batch.
struct SplatRegs {
  int x[SPLAT_PPT], y[SPLAT_PPT], z[SPLAT_PPT];
  uint32_t c[SPLAT_PPT * 3 / 2];  // 16-bit colours of each quad, two per dword, in input order
  uint32_t valid;                 // bit s: point s exists (ragged last batch)
};

// Thread t owns the quads base/4 + k*SPLAT_THREADS + t (k < SPLAT_QPT).  The
// points are streamed once: non-temporal loads keep the key array resident
// in the caches instead.
__device__ __forceinline__ void splat_load(const SplatParams& p, int64_t base, int tid, SplatRegs& r) {
  const int64_t q0 = base / 4 + tid;
  if (p.vec_ok && base + SPLAT_BATCH <= p.n) {
#pragma unroll
    for (int k = 0; k < SPLAT_QPT; ++k) {
      const int64_t q = q0 + (int64_t)k * SPLAT_THREADS;
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
    r.valid = (SPLAT_PPT == 32) ? 0xFFFFFFFFu : ((1u << SPLAT_PPT) - 1u);
    return;
  }
  // ragged or unaligned batch: point by point, bounds-checked
  r.valid = 0;
#pragma unroll
  for (int k = 0; k < SPLAT_QPT; ++k) {
#pragma unroll
    for (int w = 0; w < 6; ++w) r.c[6 * k + w] = 0;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int64_t i = 4 * (q0 + (int64_t)k * SPLAT_THREADS) + e;
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

__device__ __forceinline__ uint32_t splat_colour(const SplatRegs& r, int s, int ch) {
  const int k = s >> 2, v = 3 * (s & 3) + ch;
  const uint32_t w = r.c[6 * k + v / 2];
  return (v & 1) ? (w >> 16) : (w & 0xFFFFu);
}

// One workgroup per batch of SPLAT_BATCH consecutive points (grid-stride, so
// any grid size is correct).
// When the batch's texels span fewer than SPLAT_WIN Morton codes, keys are
// first max-reduced in an LDS window indexed by Morton code and flushed with
// one global 64-bit atomic max per touched texel; otherwise every point
// goes straight to a global atomic max.
// At most 64 VGPRs (eight waves per SIMD): the loads of more workgroups are
// in flight at once, which pays more than the one register spilled.
__global__ void __launch_bounds__(SPLAT_THREADS, 8) k_splat(SplatParams p) {
  __shared__ unsigned long long s_win[SPLAT_WIN];
  __shared__ uint32_t s_lo[SPLAT_THREADS / 64], s_hi[SPLAT_THREADS / 64];
  __shared__ unsigned long long s_drop[SPLAT_THREADS / 64];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  unsigned long long dropped = 0;
  // invariant: the window is all zero when a batch starts (the flush clears
  // the slots it reads)
  for (int w = tid; w < SPLAT_WIN; w += SPLAT_THREADS) s_win[w] = 0;
  for (int64_t base = (int64_t)blockIdx.x * SPLAT_BATCH; base < p.n; base += (int64_t)gridDim.x * SPLAT_BATCH) {
    SplatRegs r;
    splat_load(p, base, tid, r);
    unsigned long long key[SPLAT_PPT];
    uint32_t mcs[SPLAT_PPT];  // Morton code of each point's texel
    uint32_t lo = 0xFFFFFFFFu, hi = 0;
#pragma unroll
    for (int s = 0; s < SPLAT_PPT; ++s) {
      key[s] = 0;
      mcs[s] = 0;
      if (!((r.valid >> s) & 1u)) continue;
      int gx, gy;
      unsigned long long kk;
      if (!point_key(p, r.x[s], r.y[s], r.z[s], splat_colour(r, s, 0), splat_colour(r, s, 1), splat_colour(r, s, 2),
                     kk, gx, gy)) {
        ++dropped;
        continue;
      }
      if (!p.morton_ok) {
        // texel grid too wide for 16-bit Morton halves: straight to the key array
        atomicMax(&p.keys[cell_of(p, gx, gy)], kk);
        continue;
      }
      key[s] = kk;
      const uint32_t mc = spread16((uint32_t)gx) | (spread16((uint32_t)gy) << 1);
      mcs[s] = mc;
      lo = min(lo, mc);
      hi = max(hi, mc);
    }
    if (p.morton_ok) {
      // block min / max of the Morton codes: wave shuffles, then one value per wave
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
      for (int w = 1; w < SPLAT_THREADS / 64; ++w) {
        blo = min(blo, s_lo[w]);
        bhi = max(bhi, s_hi[w]);
      }
      // uniform by construction; readfirstlane keeps the barriers below in
      // provably uniform control flow
      blo = (uint32_t)__builtin_amdgcn_readfirstlane((int)blo);
      bhi = (uint32_t)__builtin_amdgcn_readfirstlane((int)bhi);
      if (bhi >= blo && (bhi - blo) < (uint32_t)SPLAT_WIN) {
#pragma unroll
        for (int s = 0; s < SPLAT_PPT; ++s)
          if (key[s]) atomicMax(&s_win[mcs[s] - blo], key[s]);
        __syncthreads();
        const int span = (int)(bhi - blo) + 1;
        for (int w = tid; w < span; w += SPLAT_THREADS) {
          const unsigned long long kv = s_win[w];
          if (!kv) continue;
          s_win[w] = 0;
          const uint32_t code = blo + (uint32_t)w;
          atomicMax(&p.keys[cell_of(p, (int)compact16(code), (int)compact16(code >> 1))], kv);
        }
        // the next batch's first barrier (or the kernel's end) orders these
        // clears before the window is used again
      } else {
#pragma unroll
        for (int s = 0; s < SPLAT_PPT; ++s)
          if (key[s])
            atomicMax(&p.keys[cell_of(p, (int)compact16(mcs[s]), (int)compact16(mcs[s] >> 1))], key[s]);
      }
    }
  }
  // one global atomic per workgroup for the dropped count
  for (int o = 32; o > 0; o >>= 1) dropped += (unsigned long long)__shfl_xor((long long)dropped, o, 64);
  if (lane == 0) s_drop[wave] = dropped;
  __syncthreads();
  if (tid == 0) {
    unsigned long long d = 0;
    for (int w = 0; w < SPLAT_THREADS / 64; ++w) d += s_drop[w];
    if (d) atomicAdd(p.n_dropped, d);
  }
}

__global__ void k_resolve(const unsigned long long* __restrict__ keys, int64_t n_cells, double scale_z,
                          double offset_z, float4* __restrict__ tex) {
#pragma clang fp contract(off)
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n_cells; i += (int64_t)gridDim.x * blockDim.x) {
    const unsigned long long k = keys[i];
    if (!k) continue;
    const int32_t zr = (int32_t)((uint32_t)(k >> 32) ^ 0x80000000u);
    // separate multiply and add, each correctly rounded (no contraction);
    // float division is IEEE-correct with the library's compile flags
    const double hm = (double)zr * scale_z;
    const double h = hm + offset_z;
    tex[i] = make_float4((float)h, (float)((k >> 24) & 0xFF) / 255.0f, (float)((k >> 16) & 0xFF) / 255.0f,
                         (float)((k >> 8) & 0xFF) / 255.0f);
  }
}

}  // namespace

int ls_resolve_impl(const LsGridInfo& gi, const uint64_t* keys, int32_t n_slots, float* tex_inout, hipStream_t st) {
  const int64_t cells = (int64_t)n_slots * gi.res * gi.res;
  if (cells <= 0) return LS_OK;
  const int blocks = (int)std::min<int64_t>((cells + 255) / 256, 16384);
  LS_TRACE("resolve", st);
  hipLaunchKernelGGL(k_resolve, dim3(blocks), dim3(256), 0, st, reinterpret_cast<const unsigned long long*>(keys),
                     cells, gi.scale_z, gi.offset_z, reinterpret_cast<float4*>(tex_inout));
  LS_LAUNCH_CHECK();
  return LS_OK;
}

int ls_splat_impl(const LsGridInfo& gi, const int32_t* x, const int32_t* y, const int32_t* z, const uint16_t* rgb,
                  int64_t n, const int32_t* tile_slot, int32_t n_slots, uint64_t* keys, float* tex_inout,
                  uint64_t* n_dropped, hipStream_t st) {
  SplatParams p;
  p.ox = gi.ox;
  p.oy = gi.oy;
  p.C = gi.C;
  p.res = gi.res;
  p.divC = magic_div((uint32_t)gi.C);
  p.divR = magic_div((uint32_t)gi.res);
  p.tiles_x = gi.tx;
  p.tiles_y = gi.ty;
  const int64_t gw = (int64_t)gi.tx * gi.res, gh = (int64_t)gi.ty * gi.res;
  if (gw * gi.C >= 0x7fffffffLL || gh * gi.C >= 0x7fffffffLL) return LS_ERANGE;
  p.gw = (int32_t)gw;
  p.gh = (int32_t)gh;
  p.n_slots = n_slots;
  p.morton_ok = (gw <= 65536 && gh <= 65536) ? 1 : 0;
  auto al = [](const void* q, uintptr_t a) { return (reinterpret_cast<uintptr_t>(q) % a) == 0; };
  p.vec_ok = (al(x, 16) && al(y, 16) && al(z, 16) && al(rgb, 8)) ? 1 : 0;
  p.n = n;
  p.x = x;
  p.y = y;
  p.z = z;
  p.rgb = rgb;
  p.tile_slot = tile_slot;
  p.keys = reinterpret_cast<unsigned long long*>(keys);
  p.n_dropped = reinterpret_cast<unsigned long long*>(n_dropped);
  if (n > 0) {
    const int64_t batches = (n + SPLAT_BATCH - 1) / SPLAT_BATCH;
    // one workgroup per batch: finished workgroups are replaced at once,
    // which balances better than a persistent grid (measured)
    const int blocks = (int)std::min<int64_t>(batches, 0x7fffffff);
    LS_TRACE("splat", st);
    hipLaunchKernelGGL(k_splat, dim3(blocks), dim3(SPLAT_THREADS), 0, st, p);
    LS_LAUNCH_CHECK();
  }
  if (tex_inout) return ls_resolve_impl(gi, keys, n_slots, tex_inout, st);
  return LS_OK;
}
