// Point rasteriser with packed 64-bit depth-and-colour keys (LidarScout
// Section 3.6, point rendering) for gfx950.
//
// Every point is moved to metres relative to the view origin, transformed by
// the 4 x 4 view-projection matrix in double precision (each row summed
// left to right, no contraction), kept when w > 0 and both normalised
// device coordinates lie in [-1, 1), and mapped to pixel
// floor(((ndc + 1) / 2) * size).  Its key is the FP32 bit pattern of w
// (positive floats order like their bit patterns, so the smallest key is
// the nearest point) above alpha | B8 | G8 | R8, and each pixel keeps the
// smallest key with a 64-bit atomic minimum; the minimum is commutative, so
// the frame buffer is bit-exact for any point order.  A pixel's current key
// is read first and the atomic skipped when it cannot lower it (keys only
// decrease, so the skip is exact).  The resolve pass writes the colour word
// of each covered pixel and 0 for empty ones.
#include <algorithm>
#include <math.h>

#include "ls_common.hpp"
#include "ls_points.hpp"

namespace {

using namespace lsp;

struct RasterParams {
  PointStream pts;
  double m[16];
  int64_t ox, oy;
  double sx, sz, oz;
  int32_t width, height;
  unsigned long long* fb;
  unsigned long long* n_drawn;
};

__device__ __forceinline__ double row_dot(const double* m, double X, double Y, double Z) {
#pragma clang fp contract(off)
  double a = m[0] * X;
  a = a + m[1] * Y;
  a = a + m[2] * Z;
  a = a + m[3];
  return a;
}

// Key and pixel of one point; false when it is culled.
__device__ __forceinline__ bool raster_point(const RasterParams& p, int xi, int yi, int zi, uint32_t r, uint32_t g,
                                             uint32_t b, unsigned long long& key, int64_t& pix) {
#pragma clang fp contract(off)
  const double X = (double)((int64_t)xi - p.ox) * p.sx;
  const double Y = (double)((int64_t)yi - p.oy) * p.sx;
  double Z = (double)zi * p.sz;
  Z = Z + p.oz;
  const double cx = row_dot(p.m, X, Y, Z), cy = row_dot(p.m + 4, X, Y, Z), cw = row_dot(p.m + 12, X, Y, Z);
  if (!(cw > 0.0)) return false;
  const double nx = cx / cw, ny = cy / cw;
  if (!(nx >= -1.0 && nx < 1.0 && ny >= -1.0 && ny < 1.0)) return false;
  const double fx = floor(((nx + 1.0) * 0.5) * (double)p.width);
  const double fy = floor(((ny + 1.0) * 0.5) * (double)p.height);
  if (!(fx >= 0.0 && fx < (double)p.width && fy >= 0.0 && fy < (double)p.height)) return false;
  pix = (int64_t)fy * p.width + (int64_t)fx;
  const uint32_t db = __builtin_bit_cast(uint32_t, (float)cw);
  key = ((unsigned long long)db << 32) | (0xFFull << 24) | ((unsigned long long)(b >> 8) << 16) |
        ((unsigned long long)(g >> 8) << 8) | (unsigned long long)(r >> 8);
  return true;
}

__global__ void __launch_bounds__(PT_THREADS) k_raster(RasterParams p) {
  __shared__ unsigned long long s_part[PT_THREADS / 64];
  unsigned long long drawn = 0;
  for (int64_t base = (int64_t)blockIdx.x * PT_BATCH; base < p.pts.n; base += (int64_t)gridDim.x * PT_BATCH) {
    PointRegs r;
    load_points(p.pts, base, threadIdx.x, r);
#pragma unroll
    for (int s = 0; s < PT_PPT; ++s) {
      if (!((r.valid >> s) & 1u)) continue;
      unsigned long long key;
      int64_t pix;
      if (!raster_point(p, r.x[s], r.y[s], r.z[s], point_colour(r, s, 0), point_colour(r, s, 1),
                        point_colour(r, s, 2), key, pix))
        continue;
      ++drawn;
      if (key < __atomic_load_n(p.fb + pix, __ATOMIC_RELAXED)) atomicMin(p.fb + pix, key);
    }
  }
  block_count_add(drawn, s_part, p.n_drawn);
}

__global__ void k_raster_resolve(const unsigned long long* __restrict__ fb, int64_t n, uint32_t* __restrict__ rgba) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const unsigned long long k = fb[i];
    rgba[i] = k == ~0ull ? 0u : (uint32_t)(k & 0xFFFFFFFFull);
  }
}

}  // namespace

int ls_raster_impl(const ls_view& v, const int32_t* x, const int32_t* y, const int32_t* z, const uint16_t* rgb,
                   int64_t n, uint64_t* fb, uint64_t* n_drawn, hipStream_t st) {
  RasterParams p;
  p.pts = point_stream(x, y, z, rgb, n);
  for (int i = 0; i < 16; ++i) p.m[i] = v.m[i];
  p.ox = v.origin_x;
  p.oy = v.origin_y;
  p.sx = v.scale_xy;
  p.sz = v.scale_z;
  p.oz = v.offset_z;
  p.width = v.width;
  p.height = v.height;
  p.fb = reinterpret_cast<unsigned long long*>(fb);
  p.n_drawn = reinterpret_cast<unsigned long long*>(n_drawn);
  if (n <= 0) return LS_OK;
  const int64_t batches = (n + PT_BATCH - 1) / PT_BATCH;
  const int blocks = (int)std::min<int64_t>(batches, 0x7fffffff);
  LS_TRACE("raster", st);
  hipLaunchKernelGGL(k_raster, dim3(blocks), dim3(PT_THREADS), 0, st, p);
  LS_LAUNCH_CHECK();
  return LS_OK;
}

int ls_raster_resolve_impl(const uint64_t* fb, int64_t n_pixels, uint32_t* rgba, hipStream_t st) {
  if (n_pixels <= 0) return LS_OK;
  const int blocks = (int)std::min<int64_t>((n_pixels + 255) / 256, 16384);
  LS_TRACE("raster_resolve", st);
  hipLaunchKernelGGL(k_raster_resolve, dim3(blocks), dim3(256), 0, st,
                     reinterpret_cast<const unsigned long long*>(fb), n_pixels, rgba);
  LS_LAUNCH_CHECK();
  return LS_OK;
}
