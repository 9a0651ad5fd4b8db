// Full-resolution splat into the heightmap textures and the resolve pass
// (LidarScout Sections 3.5-3.6) for gfx950.
//
// Each point becomes a 64-bit key, orderable height in the high word and
// 8-bit colour below it, and every texel keeps the maximum key (its highest
// point), the packed-atomic idea the paper uses for its point rasteriser.
// The maximum is commutative, so the result is bit-exact for any order.
//
// k_splat: a workgroup takes a batch of SPLAT_BATCH consecutive points
// (coalesced SoA loads).  When the batch's texels fall in a short range of
// Morton codes (the case for Morton-ordered full-resolution chunks), the
// batch is first reduced in LDS with 64-bit max (one slot per Morton code)
// and then flushed with one global 64-bit atomic max per touched texel;
// otherwise every point goes straight to a global atomic max.
#include <algorithm>

#include "ls_common.hpp"

namespace {

constexpr int SPLAT_THREADS = 256;
constexpr int SPLAT_PAIRS = 8;                                   // point pairs per thread per batch
constexpr int SPLAT_PPT = 2 * SPLAT_PAIRS;                       // points per thread per batch
constexpr int SPLAT_BATCH = SPLAT_THREADS * SPLAT_PPT;           // points per batch
constexpr int SPLAT_WIN = 8192;                                  // LDS window (64 KB of keys)

struct SplatParams {
  int64_t ox, oy;
  int32_t C, res, tiles_x, tiles_y;
  double inv_C, inv_res;
  int32_t gw, gh;  // global texel extent
  int32_t n_slots;
  int32_t morton_ok;
  int32_t vec_ok;  // x, y, z 8-byte aligned and rgb 4-byte aligned: pairwise vector loads
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

// floor(a / b) for 0 <= a < 2^31, b > 0, from a double reciprocal plus a
// one-step correction (the product is within one of the quotient)
__device__ __forceinline__ int udiv(int64_t a, int b, double inv) {
  int q = (int)((double)a * inv);
  if ((int64_t)q * b > a) --q;
  else if ((int64_t)(q + 1) * b <= a) ++q;
  return q;
}

// texel index of (gx, gy) in the key array; the tile must be mapped
__device__ __forceinline__ int64_t cell_of(const SplatParams& p, int gx, int gy) {
  const int tx = udiv(gx, p.res, p.inv_res), ty = udiv(gy, p.res, p.inv_res);
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
  gx = udiv(dx, p.C, p.inv_C);
  gy = udiv(dy, p.C, p.inv_C);
  const int tx = udiv(gx, p.res, p.inv_res), ty = udiv(gy, p.res, p.inv_res);
  const int32_t s = p.tile_slot[ty * p.tiles_x + tx];
  if (s < 0 || s >= p.n_slots) return false;
  const uint32_t zz = (uint32_t)zi ^ 0x80000000u;
  key = ((unsigned long long)zz << 32) | ((unsigned long long)(r >> 8) << 24) | ((unsigned long long)(g >> 8) << 16) |
        ((unsigned long long)(b >> 8) << 8) | 0xFFull;
  return true;
}

__global__ void __launch_bounds__(SPLAT_THREADS) k_splat(SplatParams p) {
  __shared__ unsigned long long s_win[SPLAT_WIN];
  __shared__ uint32_t s_lo[SPLAT_THREADS / 64], s_hi[SPLAT_THREADS / 64];
  __shared__ unsigned long long s_drop[SPLAT_THREADS / 64];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  unsigned long long dropped = 0;
  for (int64_t base = (int64_t)blockIdx.x * SPLAT_BATCH; base < p.n; base += (int64_t)gridDim.x * SPLAT_BATCH) {
    unsigned long long key[SPLAT_PPT];
    int gxs[SPLAT_PPT], gys[SPLAT_PPT];
    uint32_t lo = 0xFFFFFFFFu, hi = 0;
    const int64_t pbase = base >> 1;
#pragma unroll
    for (int k = 0; k < SPLAT_PAIRS; ++k) {
      const int64_t pr = pbase + (int64_t)k * SPLAT_THREADS + tid;
      const int64_t i0 = 2 * pr;
      int xv[2], yv[2], zv[2];
      uint32_t rv[2], gv[2], bv[2];
      int nv = 0;
      if (p.vec_ok && i0 + 1 < p.n) {
        const int2 x2 = reinterpret_cast<const int2*>(p.x)[pr];
        const int2 y2 = reinterpret_cast<const int2*>(p.y)[pr];
        const int2 z2 = reinterpret_cast<const int2*>(p.z)[pr];
        const uint32_t* c = reinterpret_cast<const uint32_t*>(p.rgb) + 3 * pr;
        const uint32_t c0 = c[0], c1 = c[1], c2 = c[2];
        xv[0] = x2.x; xv[1] = x2.y;
        yv[0] = y2.x; yv[1] = y2.y;
        zv[0] = z2.x; zv[1] = z2.y;
        rv[0] = c0 & 0xFFFF; gv[0] = c0 >> 16; bv[0] = c1 & 0xFFFF;
        rv[1] = c1 >> 16; gv[1] = c2 & 0xFFFF; bv[1] = c2 >> 16;
        nv = 2;
      } else {
        for (int q = 0; q < 2; ++q) {
          const int64_t i = i0 + q;
          if (i >= p.n) break;
          xv[q] = p.x[i];
          yv[q] = p.y[i];
          zv[q] = p.z[i];
          rv[q] = p.rgb[3 * i];
          gv[q] = p.rgb[3 * i + 1];
          bv[q] = p.rgb[3 * i + 2];
          nv = q + 1;
        }
      }
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        const int slot = 2 * k + q;
        key[slot] = 0;
        if (q >= nv) continue;
        int gx, gy;
        if (!point_key(p, xv[q], yv[q], zv[q], rv[q], gv[q], bv[q], key[slot], gx, gy)) {
          key[slot] = 0;
          ++dropped;
          continue;
        }
        gxs[slot] = gx;
        gys[slot] = gy;
        if (p.morton_ok) {
          const uint32_t mc = spread16((uint32_t)gx) | (spread16((uint32_t)gy) << 1);
          lo = min(lo, mc);
          hi = max(hi, mc);
        }
      }
    }
    bool use_lds = false;
    if (p.morton_ok) {
      // block min / max of the Morton codes: wave shuffles, then 4 values
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
      // uniform by construction; readfirstlane lets the compiler keep the
      // barriers below in uniform control flow
      blo = (uint32_t)__builtin_amdgcn_readfirstlane((int)blo);
      bhi = (uint32_t)__builtin_amdgcn_readfirstlane((int)bhi);
      use_lds = bhi >= blo && (bhi - blo) < (uint32_t)SPLAT_WIN;
      if (use_lds) {
        const int span = (int)(bhi - blo) + 1;
        for (int w = tid; w < span; w += SPLAT_THREADS) s_win[w] = 0;
        __syncthreads();
#pragma unroll
        for (int k = 0; k < SPLAT_PPT; ++k)
          if (key[k]) {
            const uint32_t mc = spread16((uint32_t)gxs[k]) | (spread16((uint32_t)gys[k]) << 1);
            atomicMax(&s_win[mc - blo], key[k]);
          }
        __syncthreads();
        for (int w = tid; w < span; w += SPLAT_THREADS) {
          const unsigned long long kv = s_win[w];
          if (!kv) continue;
          const uint32_t code = blo + (uint32_t)w;
          atomicMax(&p.keys[cell_of(p, (int)compact16(code), (int)compact16(code >> 1))], kv);
        }
      }
      __syncthreads();
    }
    if (!use_lds) {
#pragma unroll
      for (int k = 0; k < SPLAT_PPT; ++k)
        if (key[k]) atomicMax(&p.keys[cell_of(p, gxs[k], gys[k])], key[k]);
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
    // float division is IEEE-correct in this build
    const double hm = (double)zr * scale_z;
    const double h = hm + offset_z;
    tex[i] = make_float4((float)h, (float)((k >> 24) & 0xFF) / 255.0f, (float)((k >> 16) & 0xFF) / 255.0f,
                         (float)((k >> 8) & 0xFF) / 255.0f);
  }
}

int g_cus = 0;
int cus() {
  if (g_cus <= 0) {
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0)
      g_cus = v;
    else
      g_cus = 256;
  }
  return g_cus;
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
  p.inv_C = 1.0 / gi.C;
  p.inv_res = 1.0 / gi.res;
  p.tiles_x = gi.tx;
  p.tiles_y = gi.ty;
  const int64_t gw = (int64_t)gi.tx * gi.res, gh = (int64_t)gi.ty * gi.res;
  if (gw * gi.C >= 0x7fffffffLL || gh * gi.C >= 0x7fffffffLL) return LS_ERANGE;
  p.gw = (int32_t)gw;
  p.gh = (int32_t)gh;
  p.n_slots = n_slots;
  p.morton_ok = (gw <= 65536 && gh <= 65536) ? 1 : 0;
  auto al = [](const void* q, uintptr_t a) { return (reinterpret_cast<uintptr_t>(q) % a) == 0; };
  p.vec_ok = (al(x, 8) && al(y, 8) && al(z, 8) && al(rgb, 4)) ? 1 : 0;
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
    const int blocks = (int)std::min<int64_t>(batches, 8 * cus());
    LS_TRACE("splat", st);
    hipLaunchKernelGGL(k_splat, dim3(blocks), dim3(SPLAT_THREADS), 0, st, p);
    LS_LAUNCH_CHECK();
  }
  if (tex_inout) return ls_resolve_impl(gi, keys, n_slots, tex_inout, st);
  return LS_OK;
}
