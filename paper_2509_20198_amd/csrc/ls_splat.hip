// Full-resolution splat into the heightmap textures and the resolve pass
// (LidarScout Sections 3.5-3.6) for gfx950.
//
// Each point becomes a 64-bit key, orderable height in the high word and
// 8-bit colour below it, and every texel keeps the maximum key (its highest
// point), the packed-atomic idea the paper uses for its point rasteriser.
// The maximum is commutative, so the result is bit-exact for any order.
//
// k_splat: a workgroup takes a batch of PT_BATCH consecutive points
// (coalesced, non-temporal SoA quad loads).  When the batch's texels fall in
// a short range of Morton codes (the case for Morton-ordered full-resolution
// chunks), the batch is first reduced in LDS with 64-bit max (one slot per
// Morton code) and then flushed with one global 64-bit atomic max per
// touched texel; otherwise every point goes straight to a global atomic max.
// The small window (16 KB) lets several workgroups share a CU,
// so the loads of some overlap the LDS phases of others.
#include <algorithm>

#include "ls_common.hpp"
#include "ls_points.hpp"

namespace {

using namespace lsp;

#ifndef LS_SPLAT_WIN
#define LS_SPLAT_WIN 2048
#endif
constexpr int SPLAT_WIN = LS_SPLAT_WIN;  // LDS window of 64-bit keys

struct SplatParams {
  PointStream pts;
  TexelGrid grid;
  unsigned long long* keys;
  unsigned long long* n_dropped;
};

// Key of one point: orderable height above 8-bit colour.
__device__ __forceinline__ unsigned long long point_key(int zi, uint32_t r, uint32_t g, uint32_t b) {
  const uint32_t zz = (uint32_t)zi ^ 0x80000000u;
  return ((unsigned long long)zz << 32) | ((unsigned long long)(r >> 8) << 24) | ((unsigned long long)(g >> 8) << 16) |
         ((unsigned long long)(b >> 8) << 8) | 0xFFull;
}

// One workgroup per batch of PT_BATCH consecutive points (grid-stride, so
// any grid size is correct).
// When the batch's texels span fewer than SPLAT_WIN Morton codes, keys are
// first max-reduced in an LDS window indexed by Morton code and flushed with
// one global 64-bit atomic max per touched texel; otherwise every point
// goes straight to a global atomic max.
// At most 64 VGPRs (eight waves per SIMD): the loads of more workgroups are
// in flight at once, which pays more than the one register spilled.
__global__ void __launch_bounds__(PT_THREADS, 8) k_splat(SplatParams p) {
  __shared__ unsigned long long s_win[SPLAT_WIN];
  __shared__ uint32_t s_lo[2 * PT_THREADS / 64], s_hi[2 * PT_THREADS / 64];
  __shared__ unsigned long long s_drop[PT_THREADS / 64];
  const int tid = threadIdx.x;
  const TexelGrid& G = p.grid;
  unsigned long long dropped = 0;
  int parity = 0;
  // invariant: the window is all zero when a batch starts (the flush clears
  // the slots it reads)
  for (int w = tid; w < SPLAT_WIN; w += PT_THREADS) s_win[w] = 0;
  for (int64_t base = (int64_t)blockIdx.x * PT_BATCH; base < p.pts.n; base += (int64_t)gridDim.x * PT_BATCH) {
    PointRegs r;
    load_points(p.pts, base, tid, r);
    unsigned long long key[PT_PPT];
    uint32_t mcs[PT_PPT];  // Morton code of each point's texel
    uint32_t lo = 0xFFFFFFFFu, hi = 0;
#pragma unroll
    for (int s = 0; s < PT_PPT; ++s) {
      key[s] = 0;
      mcs[s] = 0;
      if (!((r.valid >> s) & 1u)) continue;
      int gx, gy;
      if (!point_texel(G, r.x[s], r.y[s], gx, gy)) {
        ++dropped;
        continue;
      }
      const unsigned long long kk = point_key(r.z[s], point_colour(r, s, 0), point_colour(r, s, 1),
                                              point_colour(r, s, 2));
      if (!G.morton_ok) {
        // texel grid too wide for 16-bit Morton halves: straight to the key array
        atomicMax(&p.keys[texel_index(G, gx, gy)], kk);
        continue;
      }
      key[s] = kk;
      const uint32_t mc = spread16((uint32_t)gx) | (spread16((uint32_t)gy) << 1);
      mcs[s] = mc;
      lo = min(lo, mc);
      hi = max(hi, mc);
    }
    if (G.morton_ok) {
      block_min_max(lo, hi, s_lo, s_hi, parity);
      parity ^= 1;
      if (hi >= lo && (hi - lo) < (uint32_t)SPLAT_WIN) {
#pragma unroll
        for (int s = 0; s < PT_PPT; ++s)
          if (key[s]) atomicMax(&s_win[mcs[s] - lo], key[s]);
        __syncthreads();
        const int span = (int)(hi - lo) + 1;
        for (int w = tid; w < span; w += PT_THREADS) {
          const unsigned long long kv = s_win[w];
          if (!kv) continue;
          s_win[w] = 0;
          const uint32_t code = lo + (uint32_t)w;
          atomicMax(&p.keys[texel_index(G, (int)compact16(code), (int)compact16(code >> 1))], kv);
        }
        // the next batch's first barrier (or the kernel's end) orders these
        // clears before the window is used again
      } else {
#pragma unroll
        for (int s = 0; s < PT_PPT; ++s)
          if (key[s])
            atomicMax(&p.keys[texel_index(G, (int)compact16(mcs[s]), (int)compact16(mcs[s] >> 1))], key[s]);
      }
    }
  }
  block_count_add(dropped, s_drop, p.n_dropped);
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
  if (texel_grid(gi, tile_slot, n_slots, p.grid) != LS_OK) return LS_ERANGE;
  p.pts = point_stream(x, y, z, rgb, n);
  p.keys = reinterpret_cast<unsigned long long*>(keys);
  p.n_dropped = reinterpret_cast<unsigned long long*>(n_dropped);
  if (n > 0) {
    const int64_t batches = (n + PT_BATCH - 1) / PT_BATCH;
    // one workgroup per batch: finished workgroups are replaced at once,
    // which balances better than a persistent grid (measured)
    const int blocks = (int)std::min<int64_t>(batches, 0x7fffffff);
    LS_TRACE("splat", st);
    hipLaunchKernelGGL(k_splat, dim3(blocks), dim3(PT_THREADS), 0, st, p);
    LS_LAUNCH_CHECK();
  }
  if (tex_inout) return ls_resolve_impl(gi, keys, n_slots, tex_inout, st);
  return LS_OK;
}
