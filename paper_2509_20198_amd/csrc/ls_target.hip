// Ground-truth heightmaps and the training loss (LidarScout Section 3.4,
// training data and training paragraphs) for gfx950.
//
// k_splat_mean: every full-resolution point adds its raw height, its three
// 16-bit colours and a count of one to its texel.  The sums are integers,
// so any order gives the same bits.  A workgroup takes a batch of PT_BATCH
// consecutive points, each thread PT_PPT consecutive ones, whose runs on one
// texel (the common case in Morton order) are summed in registers first.
// When the batch's texels fall in a short range of Morton codes, the runs
// are then summed in an LDS window (64-bit height sums, 32-bit colour sums
// and counts, which cannot overflow within one batch) and flushed with one
// global 64-bit atomic add per touched texel and field; otherwise every run
// adds straight to the global sums.
//
// k_resolve_mean: texel mean = sum / count in double precision (IEEE
// division), height scaled and offset to metres, colour / 65535; texels
// without points are NaN (gaps in the ground truth).
//
// k_target_loss: per element of the normalised network output, the clipped
// squared error or the absolute error against the target (NaN = no target:
// zero loss and gradient), its gradient written in place, and per-block
// partial sums reduced in a fixed order by a second kernel (deterministic).
#include <algorithm>
#include <math.h>

#include "ls_common.hpp"
#include "ls_points.hpp"

namespace {

using namespace lsp;

constexpr int MEAN_WIN = 1024;  // LDS window of texels (24 KB)

struct MeanParams {
  PointStream pts;
  TexelGrid grid;
  unsigned long long* acc;  // [cells][5]: sum z (two's complement), sum R, G, B, count
  unsigned long long* n_dropped;
};

__device__ __forceinline__ void add_global(unsigned long long* a, long long z, uint32_t r, uint32_t g, uint32_t b,
                                           uint32_t cnt) {
  atomicAdd(a + 0, (unsigned long long)z);
  atomicAdd(a + 1, (unsigned long long)r);
  atomicAdd(a + 2, (unsigned long long)g);
  atomicAdd(a + 3, (unsigned long long)b);
  atomicAdd(a + 4, (unsigned long long)cnt);
}

// Sum of the points of one run (consecutive points of a thread on one texel).
struct Run {
  long long z;
  uint32_t r, g, b, n;
};

__global__ void __launch_bounds__(PT_THREADS) k_splat_mean(MeanParams p) {
  __shared__ unsigned long long s_z[MEAN_WIN];
  __shared__ uint32_t s_c[MEAN_WIN][4];  // R, G, B sums and count
  __shared__ uint32_t s_lo[2 * PT_THREADS / 64], s_hi[2 * PT_THREADS / 64];
  __shared__ unsigned long long s_drop[PT_THREADS / 64];
  const int tid = threadIdx.x;
  const TexelGrid& G = p.grid;
  unsigned long long dropped = 0;
  int parity = 0;
  // invariant: the window is all zero when a batch starts (the flush clears
  // the slots it reads)
  for (int w = tid; w < MEAN_WIN; w += PT_THREADS) {
    s_z[w] = 0;
    s_c[w][0] = s_c[w][1] = s_c[w][2] = s_c[w][3] = 0;
  }
  for (int64_t base = (int64_t)blockIdx.x * PT_BATCH; base < p.pts.n; base += (int64_t)gridDim.x * PT_BATCH) {
    PointRegs r;
    load_points_consecutive(p.pts, base, tid, r);
    // texel key of every point: its Morton code, or its array index when the
    // grid is too wide for 16-bit Morton halves
    int64_t key[PT_PPT];
    uint32_t ok = 0;  // bit s: point s lands in a mapped texel
    uint32_t lo = 0xFFFFFFFFu, hi = 0;
#pragma unroll
    for (int s = 0; s < PT_PPT; ++s) {
      key[s] = -1;
      if (!((r.valid >> s) & 1u)) continue;
      int gx, gy;
      if (!point_texel(G, r.x[s], r.y[s], gx, gy)) {
        ++dropped;
        continue;
      }
      ok |= 1u << s;
      if (G.morton_ok) {
        const uint32_t mc = spread16((uint32_t)gx) | (spread16((uint32_t)gy) << 1);
        key[s] = mc;
        lo = min(lo, mc);
        hi = max(hi, mc);
      } else {
        key[s] = texel_index(G, gx, gy);
      }
    }
    bool window = false;
    if (G.morton_ok) {
      block_min_max(lo, hi, s_lo, s_hi, parity);
      parity ^= 1;
      window = hi >= lo && (hi - lo) < (uint32_t)MEAN_WIN;  // uniform
    }
    // runs of equal keys, summed in registers, then added to the LDS window
    // or straight to the global sums
    auto flush = [&](int64_t k, const Run& u) {
      if (window) {
        const uint32_t w = (uint32_t)k - lo;
        atomicAdd(&s_z[w], (unsigned long long)u.z);
        atomicAdd(&s_c[w][0], u.r);
        atomicAdd(&s_c[w][1], u.g);
        atomicAdd(&s_c[w][2], u.b);
        atomicAdd(&s_c[w][3], u.n);
      } else {
        const int64_t cell = G.morton_ok ? texel_index(G, (int)compact16((uint32_t)k), (int)compact16((uint32_t)k >> 1))
                                         : k;
        add_global(p.acc + 5 * cell, u.z, u.r, u.g, u.b, u.n);
      }
    };
    Run u = {0, 0, 0, 0, 0};
    int64_t cur = -1;
#pragma unroll
    for (int s = 0; s < PT_PPT; ++s) {
      if (!((ok >> s) & 1u)) continue;
      if (key[s] != cur) {
        if (u.n) flush(cur, u);
        cur = key[s];
        u = Run{0, 0, 0, 0, 0};
      }
      u.z += r.z[s];
      u.r += point_colour(r, s, 0);
      u.g += point_colour(r, s, 1);
      u.b += point_colour(r, s, 2);
      u.n += 1;
    }
    if (u.n) flush(cur, u);
    if (window) {
      __syncthreads();
      // one lane per (texel, field): the lanes of one atomic instruction
      // cover whole 40-byte texel records rather than one field of 64
      // texels spread over eight rows
      const int span = (int)(hi - lo) + 1;
      for (int i = tid; i < 5 * span; i += PT_THREADS) {
        const int w = i / 5, f = i - 5 * w;
        if (!s_c[w][3]) continue;
        const uint32_t code = lo + (uint32_t)w;
        const unsigned long long v = f == 0 ? s_z[w] : (unsigned long long)s_c[w][f - 1];
        atomicAdd(p.acc + 5 * texel_index(G, (int)compact16(code), (int)compact16(code >> 1)) + f, v);
      }
      __syncthreads();
      for (int w = tid; w < span; w += PT_THREADS) {
        s_z[w] = 0;
        s_c[w][0] = s_c[w][1] = s_c[w][2] = s_c[w][3] = 0;
      }
      // the next batch's first barrier (or the kernel's end) orders these
      // clears before the window is used again
    }
  }
  block_count_add(dropped, s_drop, p.n_dropped);
}

__global__ void k_resolve_mean(const unsigned long long* __restrict__ acc, int64_t n_cells, double scale_z,
                               double offset_z, float4* __restrict__ tex) {
#pragma clang fp contract(off)
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n_cells; i += (int64_t)gridDim.x * blockDim.x) {
    const unsigned long long* a = acc + 5 * i;
    const unsigned long long cnt = a[4];
    if (!cnt) {
      tex[i] = make_float4(NAN, NAN, NAN, NAN);
      continue;
    }
    const double c = (double)cnt;
    // each operation correctly rounded: division, then multiply, then add
    const double zm = (double)(long long)a[0] / c;
    const double hm = zm * scale_z;
    const double h = hm + offset_z;
    const double r = ((double)a[1] / c) / 65535.0, g = ((double)a[2] / c) / 65535.0, b = ((double)a[3] / c) / 65535.0;
    tex[i] = make_float4((float)h, (float)r, (float)g, (float)b);
  }
}

constexpr int LOSS_THREADS = 256;
constexpr int LOSS_BLOCKS = 1024;

// Elements are taken as float4 texels (h, r, g, b).  Per texel: target
// height normalised with the tile's cz and r_m, d = y - target in double;
// clipped MSE: e = min(d^2, 1), g = d / N where d^2 <= 1; L1: e = |d|,
// g = sign(d) / (2 N); N = texels (height) or 3 * texels (colour).
__global__ void __launch_bounds__(LOSS_THREADS) k_target_loss(const float4* __restrict__ y,
                                                              const float4* __restrict__ t,
                                                              const double* __restrict__ cz, int64_t n_texels,
                                                              int32_t px_per_tile, double r_m, int kind,
                                                              float4* __restrict__ grad, double* __restrict__ part) {
#pragma clang fp contract(off)
  __shared__ double s_h[LOSS_THREADS], s_c[LOSS_THREADS];
  const double Nh = (double)n_texels, Nc = 3.0 * Nh;
  double sh = 0.0, sc = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)LOSS_THREADS + threadIdx.x; i < n_texels;
       i += (int64_t)gridDim.x * LOSS_THREADS) {
    const float4 yv = y[i], tv = t[i];
    const double czt = cz[i / px_per_tile];
    const float ya[4] = {yv.x, yv.y, yv.z, yv.w}, ta[4] = {tv.x, tv.y, tv.z, tv.w};
    float ga[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      double e = 0.0, g = 0.0;
      if (!isnan(ta[c])) {
        const double target = c == 0 ? ((double)ta[c] - czt) / r_m : (double)ta[c];
        const double d = (double)ya[c] - target;
        const double N = c == 0 ? Nh : Nc;
        if (kind == 0) {
          const double sq = d * d;
          if (sq <= 1.0) {
            e = sq;
            g = d / N;
          } else {
            e = 1.0;
          }
        } else {
          e = fabs(d);
          g = (d > 0.0 ? 1.0 : (d < 0.0 ? -1.0 : 0.0)) / (2.0 * N);
        }
      }
      if (c == 0)
        sh += e;
      else
        sc += e;
      ga[c] = (float)g;
    }
    if (grad) grad[i] = make_float4(ga[0], ga[1], ga[2], ga[3]);
  }
  s_h[threadIdx.x] = sh;
  s_c[threadIdx.x] = sc;
  __syncthreads();
  for (int o = LOSS_THREADS / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) {
      s_h[threadIdx.x] += s_h[threadIdx.x + o];
      s_c[threadIdx.x] += s_c[threadIdx.x + o];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = s_h[0];
    part[2 * blockIdx.x + 1] = s_c[0];
  }
}

// One workgroup sums the per-block partials in a fixed order:
// out = (L, L_h, L_rgb) with L_h = sum_h / N_h, L_rgb = sum_c / (3 N_h),
// L = (L_h + L_rgb) / 2.
__global__ void __launch_bounds__(LOSS_THREADS) k_loss_final(const double* __restrict__ part, int nblk,
                                                             int64_t n_texels, double* __restrict__ out) {
#pragma clang fp contract(off)
  __shared__ double s_h[LOSS_THREADS], s_c[LOSS_THREADS];
  double sh = 0.0, sc = 0.0;
  for (int b = threadIdx.x; b < nblk; b += LOSS_THREADS) {
    sh += part[2 * b];
    sc += part[2 * b + 1];
  }
  s_h[threadIdx.x] = sh;
  s_c[threadIdx.x] = sc;
  __syncthreads();
  for (int o = LOSS_THREADS / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) {
      s_h[threadIdx.x] += s_h[threadIdx.x + o];
      s_c[threadIdx.x] += s_c[threadIdx.x + o];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double Nh = (double)n_texels;
    const double lh = s_h[0] / Nh, lc = s_c[0] / (3.0 * Nh);
    out[0] = 0.5 * (lh + lc);
    out[1] = lh;
    out[2] = lc;
  }
}

}  // namespace

int ls_splat_mean_impl(const LsGridInfo& gi, const int32_t* x, const int32_t* y, const int32_t* z,
                       const uint16_t* rgb, int64_t n, const int32_t* tile_slot, int32_t n_slots, int64_t* acc,
                       uint64_t* n_dropped, hipStream_t st) {
  MeanParams p;
  if (texel_grid(gi, tile_slot, n_slots, p.grid) != LS_OK) return LS_ERANGE;
  p.pts = point_stream(x, y, z, rgb, n);
  p.acc = reinterpret_cast<unsigned long long*>(acc);
  p.n_dropped = reinterpret_cast<unsigned long long*>(n_dropped);
  if (n <= 0) return LS_OK;
  const int64_t batches = (n + PT_BATCH - 1) / PT_BATCH;
  const int blocks = (int)std::min<int64_t>(batches, 0x7fffffff);
  LS_TRACE("splat_mean", st);
  hipLaunchKernelGGL(k_splat_mean, dim3(blocks), dim3(PT_THREADS), 0, st, p);
  LS_LAUNCH_CHECK();
  return LS_OK;
}

int ls_resolve_mean_impl(const LsGridInfo& gi, const int64_t* acc, int32_t n_slots, float* tex, hipStream_t st) {
  const int64_t cells = (int64_t)n_slots * gi.res * gi.res;
  if (cells <= 0) return LS_OK;
  const int blocks = (int)std::min<int64_t>((cells + 255) / 256, 16384);
  LS_TRACE("resolve_mean", st);
  hipLaunchKernelGGL(k_resolve_mean, dim3(blocks), dim3(256), 0, st,
                     reinterpret_cast<const unsigned long long*>(acc), cells, gi.scale_z, gi.offset_z,
                     reinterpret_cast<float4*>(tex));
  LS_LAUNCH_CHECK();
  return LS_OK;
}

size_t ls_loss_ws_bytes() { return (size_t)LOSS_BLOCKS * 2 * sizeof(double); }

int ls_target_loss_impl(const float* y, const float* t, const double* cz, int32_t n_tiles, const LsGridInfo& gi,
                        int kind, double* loss_out, float* grad, void* ws, size_t ws_bytes, hipStream_t st) {
  if (ws_bytes < ls_loss_ws_bytes() || !ws) return LS_EWORKSPACE;
  const int64_t px = (int64_t)gi.res * gi.res;
  const int64_t n_texels = (int64_t)n_tiles * px;
  const double r_m = ((double)gi.H) * gi.scale_xy;
  double* part = reinterpret_cast<double*>(ws);
  const int blocks = (int)std::max<int64_t>(1, std::min<int64_t>((n_texels + LOSS_THREADS - 1) / LOSS_THREADS,
                                                                  LOSS_BLOCKS));
  LS_TRACE("target_loss", st);
  hipLaunchKernelGGL(k_target_loss, dim3(blocks), dim3(LOSS_THREADS), 0, st, reinterpret_cast<const float4*>(y),
                     reinterpret_cast<const float4*>(t), cz, n_texels, (int32_t)px, r_m, kind,
                     reinterpret_cast<float4*>(grad), part);
  LS_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_loss_final, dim3(1), dim3(LOSS_THREADS), 0, st, part, blocks, n_texels, loss_out);
  LS_LAUNCH_CHECK();
  return LS_OK;
}
