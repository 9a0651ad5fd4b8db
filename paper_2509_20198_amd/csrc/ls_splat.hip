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
constexpr int SPLAT_PPT = 16;
constexpr int SPLAT_BATCH = SPLAT_THREADS * SPLAT_PPT;  // points per batch
constexpr int SPLAT_WIN = 8192;                         // LDS window (64 KB of keys)

struct SplatParams {
  int64_t ox, oy;
  int32_t C, res, tiles_x, tiles_y;
  int32_t gw, gh;  // global texel extent
  int32_t n_slots;
  int32_t morton_ok;
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

__device__ __forceinline__ int64_t fdiv(int64_t a, int64_t b) {
  int64_t q = a / b;
  if ((a % b != 0) && ((a < 0) != (b < 0))) --q;
  return q;
}

// texel index of (gx, gy) in the key array, or -1 if its tile is unmapped
__device__ __forceinline__ int64_t cell_of(const SplatParams& p, int gx, int gy) {
  const int tx = gx / p.res, ty = gy / p.res;
  const int s = p.tile_slot[ty * p.tiles_x + tx];
  if (s < 0 || s >= p.n_slots) return -1;
  return ((int64_t)s * p.res + (gy - ty * p.res)) * p.res + (gx - tx * p.res);
}

__global__ void __launch_bounds__(SPLAT_THREADS) k_splat(SplatParams p) {
  __shared__ unsigned long long s_win[SPLAT_WIN];
  __shared__ uint32_t s_lo, s_hi;
  __shared__ unsigned long long s_drop;
  const int tid = threadIdx.x;
  unsigned long long dropped = 0;
  for (int64_t base = (int64_t)blockIdx.x * SPLAT_BATCH; base < p.n; base += (int64_t)gridDim.x * SPLAT_BATCH) {
    uint32_t mc[SPLAT_PPT];
    unsigned long long key[SPLAT_PPT];
    int gxs[SPLAT_PPT], gys[SPLAT_PPT];
    uint32_t lo = 0xFFFFFFFFu, hi = 0;
#pragma unroll
    for (int k = 0; k < SPLAT_PPT; ++k) {
      const int64_t i = base + (int64_t)k * SPLAT_THREADS + tid;
      key[k] = 0;
      gxs[k] = -1;
      gys[k] = -1;
      if (i >= p.n) continue;
      const int64_t gx = fdiv((int64_t)p.x[i] - p.ox, p.C), gy = fdiv((int64_t)p.y[i] - p.oy, p.C);
      if (gx < 0 || gy < 0 || gx >= p.gw || gy >= p.gh) {
        ++dropped;
        continue;
      }
      const int32_t slot = p.tile_slot[(gy / p.res) * p.tiles_x + gx / p.res];
      if (slot < 0 || slot >= p.n_slots) {
        ++dropped;
        continue;
      }
      const uint16_t* c = p.rgb + 3 * i;
      const uint32_t zz = (uint32_t)p.z[i] ^ 0x80000000u;
      key[k] = ((unsigned long long)zz << 32) | ((unsigned long long)(c[0] >> 8) << 24) |
               ((unsigned long long)(c[1] >> 8) << 16) | ((unsigned long long)(c[2] >> 8) << 8) | 0xFFull;
      gxs[k] = (int)gx;
      gys[k] = (int)gy;
      mc[k] = spread16((uint32_t)gx) | (spread16((uint32_t)gy) << 1);
      lo = min(lo, mc[k]);
      hi = max(hi, mc[k]);
    }
    bool use_lds = false;
    if (p.morton_ok) {
      if (tid == 0) {
        s_lo = 0xFFFFFFFFu;
        s_hi = 0;
      }
      __syncthreads();
      if (hi >= lo) {
        atomicMin(&s_lo, lo);
        atomicMax(&s_hi, hi);
      }
      __syncthreads();
      const uint32_t blo = s_lo, bhi = s_hi;
      use_lds = bhi >= blo && (bhi - blo) < (uint32_t)SPLAT_WIN;
      if (use_lds) {
        const int span = (int)(bhi - blo) + 1;
        for (int w = tid; w < span; w += SPLAT_THREADS) s_win[w] = 0;
        __syncthreads();
#pragma unroll
        for (int k = 0; k < SPLAT_PPT; ++k)
          if (key[k]) atomicMax(&s_win[mc[k] - blo], key[k]);
        __syncthreads();
        for (int w = tid; w < span; w += SPLAT_THREADS) {
          const unsigned long long kv = s_win[w];
          if (!kv) continue;
          const uint32_t code = blo + (uint32_t)w;
          const int gx = (int)compact16(code), gy = (int)compact16(code >> 1);
          const int64_t cell = cell_of(p, gx, gy);
          atomicMax(&p.keys[cell], kv);
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
  // one atomic per workgroup for the dropped count
  if (tid == 0) s_drop = 0;
  __syncthreads();
  if (dropped) atomicAdd(&s_drop, dropped);
  __syncthreads();
  if (tid == 0 && s_drop) atomicAdd(p.n_dropped, s_drop);
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
  p.tiles_x = gi.tx;
  p.tiles_y = gi.ty;
  const int64_t gw = (int64_t)gi.tx * gi.res, gh = (int64_t)gi.ty * gi.res;
  if (gw > 0x7fffffff || gh > 0x7fffffff) return LS_ERANGE;
  p.gw = (int32_t)gw;
  p.gh = (int32_t)gh;
  p.n_slots = n_slots;
  p.morton_ok = (gw <= 65536 && gh <= 65536) ? 1 : 0;
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
    hipLaunchKernelGGL(k_splat, dim3(blocks), dim3(SPLAT_THREADS), 0, st, p);
    LS_LAUNCH_CHECK();
  }
  if (tex_inout) return ls_resolve_impl(gi, keys, n_slots, tex_inout, st);
  return LS_OK;
}
