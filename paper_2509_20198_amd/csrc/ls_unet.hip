// Refinement network (LidarScout Section 3.4) forward and backward for
// gfx950: the 3-level U-Net with input-skip head described in lidarscout.h.
//
// Every 3x3 convolution reads its input through a ConvSrc descriptor that
// folds the glue of the network into the load addressing: nearest x2
// upsampling, channel concatenation of two tensors, embedding a smaller
// tensor at an offset (the head's crop window, seen from the backward), and
// the ReLU mask of the backward (a value counts only where the forward
// activation was positive).  Average pooling writes its own small tensor.
//
// FP32 path ("plain"): one launch per layer over the whole batch, each lane
// one output pixel x COB output channels, weights read as wave-uniform
// scalars from a [tap][cin][cout] copy.  BF16 path: see ls_unet_bf16.hip.
#include <algorithm>
#include <vector>

#include "ls_common.hpp"
#include "ls_unet.hpp"

namespace {

constexpr int CT = 256;

__global__ void k_prep_weights(const float* __restrict__ w, float* __restrict__ wt, float* __restrict__ wd) {
  // one thread per weight element of all layers
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  int64_t off = 0;
  for (int l = 0; l < LS_NLAYER; ++l) {
    const int cin = LS_LAYERS[l].cin, cout = LS_LAYERS[l].cout;
    const int64_t nw = (int64_t)cout * 9 * cin;
    if (i >= off && i < off + nw) {
      const int64_t r = i - off;
      const int co = (int)(r / (9 * cin));
      const int tap = (int)((r / cin) % 9);
      const int ci = (int)(r % cin);
      const float v = w[i];
      wt[off + ((int64_t)tap * cin + ci) * cout + co] = v;
      wd[off + ((int64_t)(8 - tap) * cout + co) * cin + ci] = v;
      return;
    }
    off += nw + cout;
  }
}

__device__ __forceinline__ float4 ld4(const float* p) { return *reinterpret_cast<const float4*>(p); }

// Pixel (yy, xx) of the conv input, channels [c, c+4) of source part `which`.
template <bool MASK>
__device__ __forceinline__ float4 src_load4(const ConvSrc& s, int b, int yy, int xx, int c, bool& ok) {
  const SrcPart& p = c < s.a.c ? s.a : s.b;
  const int cc = c < s.a.c ? c : c - s.a.c;
  int sy, sx;
  if (p.up) {
    sy = yy >> 1;
    sx = xx >> 1;
  } else {
    sy = yy - p.oy;
    sx = xx - p.ox;
  }
  ok = sy >= 0 && sx >= 0 && sy < p.h && sx < p.w;
  if (!ok) return make_float4(0.f, 0.f, 0.f, 0.f);
  const int64_t o = (((int64_t)b * p.h + sy) * p.w + sx) * p.stride + p.coff + cc;
  float4 v = ld4(p.f32 + o);
  if (MASK && p.mask) {
    const float4 m = ld4(p.mask + o);
    v.x = m.x > 0.f ? v.x : 0.f;
    v.y = m.y > 0.f ? v.y : 0.f;
    v.z = m.z > 0.f ? v.z : 0.f;
    v.w = m.w > 0.f ? v.w : 0.f;
  }
  return v;
}

// Generic FP32 direct conv: out[b][y0+i][x0+j][co] for i < Ho, j < Wo over an
// H x W input plane with zero padding.
template <int COB, bool MASK>
__global__ void __launch_bounds__(CT) k_conv_f32(ConvArgs A) {
  const int64_t pix = blockIdx.x * (int64_t)CT + threadIdx.x;
  const int64_t npix = (int64_t)A.B * A.Ho * A.Wo;
  if (pix >= npix) return;
  const int b = (int)(pix / ((int64_t)A.Ho * A.Wo));
  const int r = (int)(pix - (int64_t)b * A.Ho * A.Wo);
  const int oy = r / A.Wo, ox = r - oy * A.Wo;
  const int y = A.y0 + oy, x = A.x0 + ox;
  const int co0 = blockIdx.y * COB;
  const int cin = A.src.a.c + A.src.b.c;
  float acc[COB];
#pragma unroll
  for (int c = 0; c < COB; ++c) acc[c] = A.bias ? A.bias[co0 + c] : 0.f;
  for (int ky = 0; ky < 3; ++ky) {
    const int yy = y + ky - 1;
    if (yy < 0 || yy >= A.H) continue;
    for (int kx = 0; kx < 3; ++kx) {
      const int xx = x + kx - 1;
      if (xx < 0 || xx >= A.W) continue;
      const float* wrow = A.wt + (int64_t)(ky * 3 + kx) * cin * A.cout + co0;
      for (int ci = 0; ci < cin; ci += 4) {
        bool ok;
        const float4 v = src_load4<MASK>(A.src, b, yy, xx, ci, ok);
        if (!ok) continue;
        const float* w0 = wrow + (int64_t)ci * A.cout;
#pragma unroll
        for (int c = 0; c < COB; ++c) {
          float s = acc[c];
          s = fmaf(v.x, w0[c], s);
          s = fmaf(v.y, w0[A.cout + c], s);
          s = fmaf(v.z, w0[2 * A.cout + c], s);
          s = fmaf(v.w, w0[3 * A.cout + c], s);
          acc[c] = s;
        }
      }
    }
  }
  float* o = A.out + pix * A.out_stride + A.out_coff + co0;
#pragma unroll
  for (int c = 0; c < COB; ++c) o[c] = A.relu ? fmaxf(acc[c], 0.f) : acc[c];
}

// out = avgpool2x2(in), NHWC, C multiple of 4
__global__ void k_avgpool_f32(const float* __restrict__ in, float* __restrict__ out, int B, int H, int W, int C) {
  const int64_t n = (int64_t)B * (H / 2) * (W / 2) * (C / 4);
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int c4 = (int)(i % (C / 4));
  int64_t r = i / (C / 4);
  const int x = (int)(r % (W / 2));
  r /= (W / 2);
  const int y = (int)(r % (H / 2));
  const int b = (int)(r / (H / 2));
  const float* p = in + (((int64_t)b * H + 2 * y) * W + 2 * x) * C + 4 * c4;
  const float4 a = ld4(p), bq = ld4(p + C), c = ld4(p + (int64_t)W * C), d = ld4(p + (int64_t)W * C + C);
  float4 o;
  o.x = 0.25f * ((a.x + bq.x) + (c.x + d.x));
  o.y = 0.25f * ((a.y + bq.y) + (c.y + d.y));
  o.z = 0.25f * ((a.z + bq.z) + (c.z + d.z));
  o.w = 0.25f * ((a.w + bq.w) + (c.w + d.w));
  reinterpret_cast<float4*>(out)[i] = o;
}

// Head epilogue: y = crop(x[..., {0,2,3,4}]) + head, texture.
__global__ void k_head_epilogue(const float* __restrict__ head, const float* __restrict__ x, const double* __restrict__ cz,
                                int B, int res, int pad, double r_m, float* __restrict__ y_out,
                                float* __restrict__ tex_out) {
  const int64_t n = (int64_t)B * res * res;
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int b = (int)(i / ((int64_t)res * res));
  const int r = (int)(i - (int64_t)b * res * res);
  const int R = res + 2 * pad;
  const int yy = r / res + pad, xx = r % res + pad;
  const float* xp = x + (((int64_t)b * R + yy) * R + xx) * 8;
  const float4 h = ld4(head + 4 * i);
  const float4 v = make_float4(xp[0] + h.x, xp[2] + h.y, xp[3] + h.z, xp[4] + h.w);
  if (y_out) reinterpret_cast<float4*>(y_out)[i] = v;
  if (tex_out) {
    const double hm = cz[b] + r_m * (double)v.x;
    reinterpret_cast<float4*>(tex_out)[i] =
        make_float4((float)hm, fminf(fmaxf(v.y, 0.f), 1.f), fminf(fmaxf(v.z, 0.f), 1.f), fminf(fmaxf(v.w, 0.f), 1.f));
  }
}

// ---------------------------------------------------------------- backward
// dW partials as a register-tiled product: dW[co][n] = sum over pixels of
// dZ(p, co) * I(p, n), with n = tap*cin + ci the im2col column and column
// n = 9*cin standing for the bias (I = 1).  dZ(p, co) = dA[p][co] masked by
// A[p][co] > 0 (or a pre-masked BF16 copy), defined on the output window;
// I is read through the forward ConvSrc.  A workgroup owns one pixel chunk
// (blockIdx.y) and WG_COLS columns (blockIdx.x) for all output channels;
// slabs of WG_KP pixels are staged in LDS and every thread accumulates a
// 4x4 block (4 channels x 4 columns) in FP32, in a fixed order.
constexpr int WG_KP = 32;

__device__ __forceinline__ float bf16_round(float f) {
  return __builtin_bit_cast(float, (uint32_t)__builtin_bit_cast(unsigned short, static_cast<__bf16>(f)) << 16);
}

__device__ __forceinline__ float4 bf16x4_to_f32(uint2 v) {
  return make_float4(__builtin_bit_cast(float, v.x << 16), __builtin_bit_cast(float, v.x & 0xFFFF0000u),
                     __builtin_bit_cast(float, v.y << 16), __builtin_bit_cast(float, v.y & 0xFFFF0000u));
}

// channels cc..cc+3 of part p at input-plane pixel (yy, xx); zero outside
__device__ __forceinline__ float4 wg_load4(const SrcPart& p, int b, int yy, int xx, int cc, int H, int W, int rnd) {
  const float4 z = make_float4(0.f, 0.f, 0.f, 0.f);
  if (yy < 0 || xx < 0 || yy >= H || xx >= W) return z;
  int sy, sx;
  if (p.up) {
    sy = yy >> 1;
    sx = xx >> 1;
  } else {
    sy = yy - p.oy;
    sx = xx - p.ox;
  }
  if (sy < 0 || sx < 0 || sy >= p.h || sx >= p.w) return z;
  const int64_t o = (((int64_t)b * p.h + sy) * p.w + sx) * p.stride + p.coff + cc;
  if (p.bf16) return bf16x4_to_f32(*reinterpret_cast<const uint2*>(p.bf16 + o));
  float4 v = *reinterpret_cast<const float4*>(p.f32 + o);
  if (rnd) {
    v.x = bf16_round(v.x);
    v.y = bf16_round(v.y);
    v.z = bf16_round(v.z);
    v.w = bf16_round(v.w);
  }
  return v;
}

template <int MWG>
__global__ void __launch_bounds__(CT) k_wgrad_tiled(WgradArgs A) {
  constexpr int TM = MWG / 4;            // threads along the channel axis
  constexpr int NWG4 = CT / TM;          // float4 columns per workgroup
  __shared__ float4 s_g[WG_KP][TM];
  __shared__ float4 s_x[WG_KP][NWG4];
  const int tid = threadIdx.x;
  const int tm = tid % TM, tn = tid / TM;
  const int cin = A.src.a.c + A.src.b.c;
  const int N = 9 * cin;
  const int nb = blockIdx.x * NWG4 * 4;
  const int64_t npix = (int64_t)A.B * A.Ho * A.Wo;
  const int64_t p0 = npix * blockIdx.y / gridDim.y, p1 = npix * (blockIdx.y + 1) / gridDim.y;
  const int64_t hw = (int64_t)A.Ho * A.Wo;
  float acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = 0.f;
  for (int64_t ps = p0; ps < p1; ps += WG_KP) {
    for (int e = tid; e < WG_KP * TM; e += CT) {
      const int kk = e / TM, c4 = e - kk * TM;
      const int64_t p = ps + kk;
      float4 g = make_float4(0.f, 0.f, 0.f, 0.f);
      if (p < p1 && 4 * c4 < A.cout) {
        const int64_t o = p * A.d_stride + 4 * c4;
        if (A.g_bf16) {
          g = bf16x4_to_f32(*reinterpret_cast<const uint2*>(A.g_bf16 + o));
        } else {
          g = *reinterpret_cast<const float4*>(A.dA + o);
          if (A.mask) {
            const float4 m = *reinterpret_cast<const float4*>(A.mask + o);
            g.x = m.x > 0.f ? g.x : 0.f;
            g.y = m.y > 0.f ? g.y : 0.f;
            g.z = m.z > 0.f ? g.z : 0.f;
            g.w = m.w > 0.f ? g.w : 0.f;
          }
        }
      }
      s_g[kk][c4] = g;
    }
    for (int e = tid; e < WG_KP * NWG4; e += CT) {
      const int kk = e / NWG4, n4 = e - kk * NWG4;
      const int64_t p = ps + kk;
      const int n = nb + 4 * n4;
      float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
      if (p < p1) {
        if (n < N) {
          const int tap = n / cin, ci = n - tap * cin;
          const int ky = tap / 3, kx = tap - 3 * ky;
          const int b = (int)(p / hw);
          const int r = (int)(p - (int64_t)b * hw);
          const int yy = A.y0 + r / A.Wo + ky - 1, xx = A.x0 + r % A.Wo + kx - 1;
          const bool in_a = ci < A.src.a.c;
          v = wg_load4(in_a ? A.src.a : A.src.b, b, yy, xx, in_a ? ci : ci - A.src.a.c, A.H, A.W, A.round_in);
        } else if (n == N) {
          v.x = 1.f;
        }
      }
      s_x[kk][n4] = v;
    }
    __syncthreads();
#pragma unroll 8
    for (int kk = 0; kk < WG_KP; ++kk) {
      const float4 g = s_g[kk][tm], x = s_x[kk][tn];
      const float gv[4] = {g.x, g.y, g.z, g.w}, xv[4] = {x.x, x.y, x.z, x.w};
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = fmaf(gv[i], xv[j], acc[i][j]);
    }
    __syncthreads();
  }
  float* out = A.partial + (int64_t)blockIdx.y * ((int64_t)A.cout * N + A.cout);
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int co = 4 * tm + i;
    if (co >= A.cout) continue;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int n = nb + 4 * tn + j;
      if (n < N)
        out[(int64_t)co * N + n] = acc[i][j];
      else if (n == N)
        out[(int64_t)A.cout * N + co] = acc[i][j];
    }
  }
}

// The same dW partials on the matrix cores for the BF16 path (gradient
// already masked and rounded to BF16, inputs rounded to BF16):
// D[co][n] += A[co][32 pixels] * B[32 pixels][n] per
// v_mfma_f32_16x16x32_bf16, FP32 accumulation.  A 32-pixel slab is staged in
// LDS pixel-contiguous (transposed: one row of 32 pixels per channel and per
// im2col column), so every A and B fragment (8 consecutive pixels of one
// row) is a single 16-byte read; rows are 80 bytes apart, which keeps the 16
// rows of a fragment in distinct banks.  Wave w owns column tiles
// [w * CTW, (w + 1) * CTW) of the workgroup's 64 * CTW columns for all
// channel tiles; the bias is the column of ones n = 9 * cin.
constexpr int WM_PITCH = 40;  // BF16 elements per staged row (32 pixels + pad)
typedef __bf16 wm_bf16x8 __attribute__((ext_vector_type(8)));
typedef float wm_f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned short wm_u16x8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ uint32_t wm_pack(float lo, float hi) {
  return (uint32_t)__builtin_bit_cast(unsigned short, static_cast<__bf16>(lo)) |
         ((uint32_t)__builtin_bit_cast(unsigned short, static_cast<__bf16>(hi)) << 16);
}

// channels cc..cc+7 of part p at input-plane pixel (yy, xx) as BF16 bits
// (FP32-stored parts rounded to nearest even); zero outside
// The fields of one of a conv's two input parts, chosen per lane and held
// in registers (a per-lane choice between two SrcPart references is read
// through memory at every use, one dependent load after another).
struct PartR {
  const uint16_t* bf16;
  const float* f32;
  int h, w, stride, coff, up, oy, ox;
};
__device__ __forceinline__ PartR part_pick(bool first, const SrcPart& a, const SrcPart& b) {
  PartR r;
  r.bf16 = first ? a.bf16 : b.bf16;
  r.f32 = first ? a.f32 : b.f32;
  r.h = first ? a.h : b.h;
  r.w = first ? a.w : b.w;
  r.stride = first ? a.stride : b.stride;
  r.coff = first ? a.coff : b.coff;
  r.up = first ? a.up : b.up;
  r.oy = first ? a.oy : b.oy;
  r.ox = first ? a.ox : b.ox;
  return r;
}

// Element offset of channels cc .. cc + 7 of part p at input pixel (yy, xx)
// of image b, or -1 where the input is zero padding.
__device__ __forceinline__ int64_t wm_offset8(const PartR& p, int b, int yy, int xx, int cc, int H, int W) {
  if (yy < 0 || xx < 0 || yy >= H || xx >= W) return -1;
  const int sy = p.up ? (yy >> 1) : yy - p.oy, sx = p.up ? (xx >> 1) : xx - p.ox;
  if (sy < 0 || sx < 0 || sy >= p.h || sx >= p.w) return -1;
  return (((int64_t)b * p.h + sy) * p.w + sx) * p.stride + p.coff + cc;
}

__device__ __forceinline__ uint4 wm_load8(const PartR& p, int b, int yy, int xx, int cc, int H, int W) {
  const uint4 z = make_uint4(0u, 0u, 0u, 0u);
  if (yy < 0 || xx < 0 || yy >= H || xx >= W) return z;
  const int sy = p.up ? (yy >> 1) : yy - p.oy, sx = p.up ? (xx >> 1) : xx - p.ox;
  if (sy < 0 || sx < 0 || sy >= p.h || sx >= p.w) return z;
  const int64_t o = (((int64_t)b * p.h + sy) * p.w + sx) * p.stride + p.coff + cc;
  if (p.bf16) return *reinterpret_cast<const uint4*>(p.bf16 + o);
  const float4 f0 = *reinterpret_cast<const float4*>(p.f32 + o);
  const float4 f1 = *reinterpret_cast<const float4*>(p.f32 + o + 4);
  return make_uint4(wm_pack(f0.x, f0.y), wm_pack(f0.z, f0.w), wm_pack(f1.x, f1.y), wm_pack(f1.z, f1.w));
}

template <int MT, int CTW, bool XF32>
__global__ void __launch_bounds__(CT) k_wgrad_mfma(WgradArgs A) {
  constexpr int COLS = 4 * CTW * 16;
  constexpr int NJ = COLS / 128;  // column octets a thread stages per slab
  __shared__ __align__(16) uint16_t s_g[MT * 16][WM_PITCH];
  __shared__ __align__(16) uint16_t s_x[COLS][WM_PITCH];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int r16 = lane & 15, g = lane >> 4;
  const int cin = A.src.a.c + A.src.b.c;
  const int N = 9 * cin;
  const int nb = blockIdx.x * COLS;
  const int64_t npix = (int64_t)A.B * A.Ho * A.Wo;
  const int64_t p0 = npix * blockIdx.y / gridDim.y, p1 = npix * (blockIdx.y + 1) / gridDim.y;
  // A thread always stages the same pixel pair of a slab and the same
  // column octets, so their decoding is done once: column octet j is an
  // input octet (tap ky, kx; part; channel), the bias octet, or zero.
  const int pp = tid & 15;
  int cdesc[NJ];
#pragma unroll
  for (int j = 0; j < NJ; ++j) {
    const int n = nb + 8 * ((tid >> 4) + 16 * j);
    if (n < N) {
      const int tap = n / cin, ci = n - tap * cin;
      const int ky = tap / 3, kx = tap - 3 * ky;
      const bool in_a = ci < A.src.a.c;
      cdesc[j] = (in_a ? 0 : (1 << 24)) | (ky << 20) | (kx << 18) | (in_a ? ci : ci - A.src.a.c);
    } else {
      cdesc[j] = n == N ? (2 << 24) : (3 << 24);
    }
  }
  // output pixel (b, oy, ox) of the pair's two pixels, advanced slab by slab
  int pb[2], py[2], px[2];
  const int64_t hw = (int64_t)A.Ho * A.Wo;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int64_t p = p0 + 2 * pp + h;
    pb[h] = (int)(p / hw);
    const int r = (int)(p - (int64_t)pb[h] * hw);
    py[h] = r / A.Wo;
    px[h] = r - py[h] * A.Wo;
  }
  wm_f32x4 acc[MT][CTW];
#pragma unroll
  for (int mt = 0; mt < MT; ++mt)
#pragma unroll
    for (int ct = 0; ct < CTW; ++ct) acc[mt][ct] = wm_f32x4{0.f, 0.f, 0.f, 0.f};
  for (int64_t ps = p0; ps < p1; ps += 32) {
    // all loads of the slab first (gradient: thread = (pixel pair, 4
    // channels); im2col: thread = (pixel pair, 8 columns of one tap)), then
    // the LDS writes, so the slab costs one memory round trip
    constexpr int NGE = (16 * MT * 4 + CT - 1) / CT;
    uint2 gv[NGE][2];
#pragma unroll
    for (int i = 0; i < NGE; ++i) {
      const int e = tid + CT * i, cq = e >> 4;
      gv[i][0] = make_uint2(0u, 0u);
      gv[i][1] = make_uint2(0u, 0u);
      if (e < 16 * MT * 4 && 4 * cq < A.cout) {
        const int64_t pa = ps + 2 * pp;
        if (pa < p1) gv[i][0] = *reinterpret_cast<const uint2*>(A.g_bf16 + pa * A.d_stride + 4 * cq);
        if (pa + 1 < p1) gv[i][1] = *reinterpret_cast<const uint2*>(A.g_bf16 + (pa + 1) * A.d_stride + 4 * cq);
      }
    }
    uint32_t xv[NJ][2][8];
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
      const int d = cdesc[j], kind = d >> 24;
#pragma unroll
      for (int h = 0; h < 2; ++h) {
#pragma unroll
        for (int k = 0; k < 8; ++k) xv[j][h][k] = 0u;
        if (ps + 2 * pp + h < p1) {
          if (kind < 2) {
            const int ky = (d >> 20) & 3, kx = (d >> 18) & 3, cc = d & 0x3FFFF;
            const PartR part = part_pick(kind == 0, A.src.a, A.src.b);
            const int64_t o = wm_offset8(part, pb[h], A.y0 + py[h] + ky - 1, A.x0 + px[h] + kx - 1, cc, A.H, A.W);
            if (o >= 0) {
              // one address for both kinds (a BF16 part reads its 16 bytes twice)
              const bool f32 = XF32 && part.f32 != nullptr;
              const uint4* q = reinterpret_cast<const uint4*>(
                  (f32 ? reinterpret_cast<const char*>(part.f32) : reinterpret_cast<const char*>(part.bf16)) +
                  o * (f32 ? 4 : 2));
              const uint4 q0 = q[0], q1 = XF32 ? *(f32 ? q + 1 : q) : q0;
              xv[j][h][0] = q0.x;
              xv[j][h][1] = q0.y;
              xv[j][h][2] = q0.z;
              xv[j][h][3] = q0.w;
              xv[j][h][4] = q1.x;
              xv[j][h][5] = q1.y;
              xv[j][h][6] = q1.z;
              xv[j][h][7] = q1.w;
            }
          } else if (kind == 2) {
            xv[j][h][0] = 0x3F80u;  // BF16 1.0 in column N
          }
        }
      }
    }
#pragma unroll
    for (int i = 0; i < NGE; ++i) {
      const int e = tid + CT * i, cq = e >> 4;
      if (e < 16 * MT * 4) {
        const uint2 v0 = gv[i][0], v1 = gv[i][1];
        uint32_t* row = reinterpret_cast<uint32_t*>(&s_g[4 * cq][2 * pp]);
        row[0 * WM_PITCH / 2] = (v0.x & 0xFFFFu) | (v1.x << 16);
        row[1 * WM_PITCH / 2] = (v0.x >> 16) | (v1.x & 0xFFFF0000u);
        row[2 * WM_PITCH / 2] = (v0.y & 0xFFFFu) | (v1.y << 16);
        row[3 * WM_PITCH / 2] = (v0.y >> 16) | (v1.y & 0xFFFF0000u);
      }
    }
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
      const int co8 = (tid >> 4) + 16 * j;
      const int d = cdesc[j], kind = d >> 24;
      uint32_t a[2][4];
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const bool f32 = XF32 && kind < 2 && (kind == 0 ? A.src.a.f32 : A.src.b.f32) != nullptr;
#pragma unroll
        for (int k = 0; k < 4; ++k)
          a[h][k] = f32 ? wm_pack(__uint_as_float(xv[j][h][2 * k]), __uint_as_float(xv[j][h][2 * k + 1])) : xv[j][h][k];
      }
      uint32_t* row = reinterpret_cast<uint32_t*>(&s_x[8 * co8][2 * pp]);
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        row[(2 * c) * WM_PITCH / 2] = (a[0][c] & 0xFFFFu) | (a[1][c] << 16);
        row[(2 * c + 1) * WM_PITCH / 2] = (a[0][c] >> 16) | (a[1][c] & 0xFFFF0000u);
      }
    }
    __syncthreads();
    wm_bf16x8 af[MT];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
      af[mt] = __builtin_bit_cast(wm_bf16x8, *reinterpret_cast<const wm_u16x8*>(&s_g[mt * 16 + r16][8 * g]));
#pragma unroll
    for (int ct = 0; ct < CTW; ++ct) {
      const wm_bf16x8 bf =
          __builtin_bit_cast(wm_bf16x8, *reinterpret_cast<const wm_u16x8*>(&s_x[(wave * CTW + ct) * 16 + r16][8 * g]));
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) acc[mt][ct] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[mt], bf, acc[mt][ct], 0, 0, 0);
    }
    // next slab: advance both pixels by 32 (rows of any width, images)
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      px[h] += 32;
      while (px[h] >= A.Wo) {
        px[h] -= A.Wo;
        if (++py[h] == A.Ho) {
          py[h] = 0;
          ++pb[h];
        }
      }
    }
    __syncthreads();
  }
  float* out = A.partial + (int64_t)blockIdx.y * ((int64_t)A.cout * N + A.cout);
#pragma unroll
  for (int mt = 0; mt < MT; ++mt)
#pragma unroll
    for (int ct = 0; ct < CTW; ++ct) {
      const int n = nb + (wave * CTW + ct) * 16 + r16;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int co = mt * 16 + 4 * g + i;
        if (co >= A.cout) continue;
        if (n < N)
          out[(int64_t)co * N + n] = acc[mt][ct][i];
        else if (n == N)
          out[(int64_t)A.cout * N + co] = acc[mt][ct][i];
      }
    }
}

// out[i] = sum over chunks of partial[c][i], in a fixed order: RED_SEG
// consecutive runs of chunks are summed in parallel (each run in chunk
// order), then the run sums in run order.  A workgroup covers RED_OUT
// outputs, so enough workgroups run even for a few thousand outputs.
// Weight gradient of a 3x3 conv by 16 x 16 output tiles on the matrix cores
// (BF16 path).  For an output tile the masked BF16 gradient (256 pixels x
// cout) is staged in LDS transposed, one row of 256 pixels per channel, and
// the input patch (18 x 18 pixels) of 8 input channels at a time in three
// copies shifted by the tap's column offset kx = 0, 1, 2 (16 columns each, a
// row of 16 pixels per channel and patch row).  Every MFMA operand -- 8
// consecutive pixels of one gradient channel, or of one input channel at
// one tap -- is then one aligned 16-byte LDS read, and the input is staged
// once per tile instead of once per tap as the im2col form does.  Columns
// are enumerated per 8-channel group as 5 tiles of 16 (taps 2t and 2t + 1 x
// 8 channels; tap 9 is zero padding), and the first column chunk also owns a
// bias tile (a column of ones).  A workgroup takes the groups of one column
// chunk (WT_GROUPS groups) for the spatial tiles x, x + gridDim.x, ...;
// wave w multiplies pixel rows 4w .. 4w + 3 of each tile (two K steps of 32
// pixels), and the four waves' sums are added in LDS in a fixed order at
// the end, so the partial sums are deterministic.
constexpr int WT_GROUPS = 2;            // 8-channel input groups per workgroup
constexpr int WT_PITCH = 256 + 8;       // staged gradient row: 256 pixels + pad (BF16)
constexpr int WT_TILES = 5 * WT_GROUPS + 1;  // column tiles per workgroup (+ bias)

template <int MT, bool XF32>
__global__ void __launch_bounds__(CT) k_wgrad_tile(WgradArgs A) {
  constexpr int NGI = (128 * MT * 4 + CT - 1) / CT;         // gradient items per thread
  constexpr int NXI = (WT_GROUPS * 18 * 18 + CT - 1) / CT;  // input items per thread
  static_assert(MT * WT_TILES * 64 * 4 * 4 <= WT_GROUPS * 3 * 8 * 18 * 16 * 2, "reduction fits the patch LDS");
  __shared__ __align__(16) uint16_t s_g[MT * 16][WT_PITCH];
  __shared__ __align__(16) uint16_t s_x[WT_GROUPS][3][8][18][16];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int r16 = lane & 15, g = lane >> 4;
  const int cin = A.src.a.c + A.src.b.c;
  const int N = 9 * cin;
  const int ng8 = cin / 8;
  const int gbase = blockIdx.y * WT_GROUPS;
  const int ngr = min(WT_GROUPS, ng8 - gbase);
  const bool bias = blockIdx.y == 0;
  const int tiles_x = (A.Wo + 15) / 16, tiles_y = (A.Ho + 15) / 16;
  const int per_img = tiles_x * tiles_y, ntiles = A.B * per_img;
  wm_f32x4 acc[MT][WT_TILES];
#pragma unroll
  for (int mt = 0; mt < MT; ++mt)
#pragma unroll
    for (int t = 0; t < WT_TILES; ++t) acc[mt][t] = wm_f32x4{0.f, 0.f, 0.f, 0.f};
  wm_u16x8 ones;
#pragma unroll
  for (int j = 0; j < 8; ++j) ones[j] = 0x3F80u;  // BF16 1.0
  for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const int b = tile / per_img, tt = tile - b * per_img;
    const int ty0 = (tt / tiles_x) * 16, tx0 = (tt % tiles_x) * 16;
    // Every load of the tile is issued before any LDS write, so the tile
    // costs one memory round trip: gradient items (a pixel pair of a row, 4
    // channels) and input items (one pixel of one 8-channel group, 16 bytes,
    // 32 for an FP32 part, rounded when written).
    uint2 gv[NGI][2];
#pragma unroll
    for (int i = 0; i < NGI; ++i) {
      const int e = tid + CT * i;
      gv[i][0] = make_uint2(0u, 0u);
      gv[i][1] = make_uint2(0u, 0u);
      const int pp = e & 127, cq = e >> 7;
      const int r = pp >> 3, c = 2 * (pp & 7);
      const int oy = ty0 + r, ox = tx0 + c;
      if (e < 128 * MT * 4 && 4 * cq < A.cout && oy < A.Ho) {
        const int64_t o = (((int64_t)b * A.Ho + oy) * A.Wo + ox) * A.d_stride + 4 * cq;
        if (ox < A.Wo) gv[i][0] = *reinterpret_cast<const uint2*>(A.g_bf16 + o);
        if (ox + 1 < A.Wo) gv[i][1] = *reinterpret_cast<const uint2*>(A.g_bf16 + o + A.d_stride);
      }
    }
    uint32_t xv[NXI][8];
#pragma unroll
    for (int i = 0; i < NXI; ++i) {
      const int e = tid + CT * i;
#pragma unroll
      for (int k = 0; k < 8; ++k) xv[i][k] = 0u;
      if (e < ngr * 18 * 18) {
        const int gi = e / 324, pix = e - gi * 324;
        const int pr = pix / 18, pc = pix - pr * 18;
        const int g8 = gbase + gi;
        const bool in_a = 8 * g8 < A.src.a.c;
        const PartR part = part_pick(in_a, A.src.a, A.src.b);
        const int64_t o = wm_offset8(part, b, A.y0 + ty0 + pr - 1, A.x0 + tx0 + pc - 1,
                                     in_a ? 8 * g8 : 8 * g8 - A.src.a.c, A.H, A.W);
        if (o >= 0) {
          // one address for both kinds: 16 bytes, and 16 more for FP32
          const bool f32 = XF32 && part.f32 != nullptr;
          const uint4* q = reinterpret_cast<const uint4*>(
              (f32 ? reinterpret_cast<const char*>(part.f32) : reinterpret_cast<const char*>(part.bf16)) +
              o * (f32 ? 4 : 2));
          // (a BF16 part reads its 16 bytes twice: no branch, so nothing
          // that uses the data is moved up between the loads)
          const uint4 q0 = q[0], q1 = *(f32 ? q + 1 : q);
          xv[i][0] = q0.x;
          xv[i][1] = q0.y;
          xv[i][2] = q0.z;
          xv[i][3] = q0.w;
          xv[i][4] = q1.x;
          xv[i][5] = q1.y;
          xv[i][6] = q1.z;
          xv[i][7] = q1.w;
        }
      }
    }
#pragma unroll
    for (int i = 0; i < NGI; ++i) {
      const int e = tid + CT * i;
      if (e < 128 * MT * 4) {
        const int pp = e & 127, cq = e >> 7;
        const int r = pp >> 3, c = 2 * (pp & 7);
        const uint2 v0 = gv[i][0], v1 = gv[i][1];
        uint32_t* row = reinterpret_cast<uint32_t*>(&s_g[4 * cq][r * 16 + c]);
        row[0 * WT_PITCH / 2] = (v0.x & 0xFFFFu) | (v1.x << 16);
        row[1 * WT_PITCH / 2] = (v0.x >> 16) | (v1.x & 0xFFFF0000u);
        row[2 * WT_PITCH / 2] = (v0.y & 0xFFFFu) | (v1.y << 16);
        row[3 * WT_PITCH / 2] = (v0.y >> 16) | (v1.y & 0xFFFF0000u);
      }
    }
    // input patch of each group in its three shifted copies
#pragma unroll
    for (int i = 0; i < NXI; ++i) {
      const int e = tid + CT * i;
      if (e < ngr * 18 * 18) {
        const int gi = e / 324, pix = e - gi * 324;
        const int pr = pix / 18, pc = pix - pr * 18;
        const int g8 = gbase + gi;
        const bool f32 = XF32 && (8 * g8 < A.src.a.c ? A.src.a.f32 : A.src.b.f32) != nullptr;
        uint32_t w4[4];
#pragma unroll
        for (int k = 0; k < 4; ++k)
          w4[k] = f32 ? wm_pack(__uint_as_float(xv[i][2 * k]), __uint_as_float(xv[i][2 * k + 1])) : xv[i][k];
#pragma unroll
        for (int kx = 0; kx < 3; ++kx) {
          const int col = pc - kx;
          if (col < 0 || col >= 16) continue;
#pragma unroll
          for (int ci = 0; ci < 8; ++ci)
            s_x[gi][kx][ci][pr][col] = (uint16_t)((ci & 1) ? (w4[ci >> 1] >> 16) : (w4[ci >> 1] & 0xFFFFu));
        }
      }
    }
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < 2; ++ks) {
      const int kstep = 2 * wave + ks;  // pixel rows 2 kstep, 2 kstep + 1
      wm_bf16x8 af[MT];
#pragma unroll
      for (int mt = 0; mt < MT; ++mt)
        af[mt] = __builtin_bit_cast(wm_bf16x8, *reinterpret_cast<const wm_u16x8*>(&s_g[mt * 16 + r16][kstep * 32 + 8 * g]));
      if (bias) {
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
          acc[mt][WT_TILES - 1] =
              __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[mt], __builtin_bit_cast(wm_bf16x8, ones), acc[mt][WT_TILES - 1], 0, 0, 0);
      }
      const int orow = 2 * kstep + (g >> 1), ocol = 8 * (g & 1), ci = r16 & 7;
#pragma unroll
      for (int gi = 0; gi < WT_GROUPS; ++gi) {
        if (gi >= ngr) break;
#pragma unroll
        for (int t = 0; t < 5; ++t) {
          const int tap = 2 * t + (r16 >> 3);
          wm_u16x8 bv = {0, 0, 0, 0, 0, 0, 0, 0};
          if (tap < 9) {
            const int ky = tap / 3, kx = tap - 3 * ky;
            bv = *reinterpret_cast<const wm_u16x8*>(&s_x[gi][kx][ci][orow + ky][ocol]);
          }
          const wm_bf16x8 bf = __builtin_bit_cast(wm_bf16x8, bv);
#pragma unroll
          for (int mt = 0; mt < MT; ++mt)
            acc[mt][gi * 5 + t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[mt], bf, acc[mt][gi * 5 + t], 0, 0, 0);
        }
      }
    }
    __syncthreads();  // every wave is done with the staged tile
  }
  // the four waves' sums in a fixed order, through the patch LDS
  float* red = reinterpret_cast<float*>(&s_x[0][0][0][0][0]);
  for (int w = 0; w < 4; ++w) {
    if (wave == w) {
#pragma unroll
      for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int t = 0; t < WT_TILES; ++t) {
          float* q = red + (((mt * WT_TILES + t) * 64) + lane) * 4;
#pragma unroll
          for (int i = 0; i < 4; ++i) q[i] = (w == 0 ? 0.f : q[i]) + acc[mt][t][i];
        }
    }
    __syncthreads();
  }
  // partial sums of this workgroup's pixels: D[co][n], rows co = mt*16 + 4g + i
  float* out = A.partial + (int64_t)blockIdx.x * ((int64_t)A.cout * N + A.cout);
  for (int e = tid; e < MT * WT_TILES * 64; e += CT) {
    const int l = e & 63, mtt = e >> 6;
    const int mt = mtt / WT_TILES, t = mtt - mt * WT_TILES;
    const int lr16 = l & 15, lg = l >> 4;
    const float* q = red + (size_t)e * 4;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int co = mt * 16 + 4 * lg + i;
      if (co >= A.cout) continue;
      if (t == WT_TILES - 1) {
        if (bias && lr16 == 0) out[(int64_t)A.cout * N + co] = q[i];
        continue;
      }
      const int gi = t / 5, tp = t - 5 * gi;
      const int tap = 2 * tp + (lr16 >> 3);
      if (gi >= ngr || tap >= 9) continue;
      const int n = tap * cin + 8 * (gbase + gi) + (lr16 & 7);
      out[(int64_t)co * N + n] = q[i];
    }
  }
}

constexpr int RED_OUT = 16, RED_SEG = CT / RED_OUT, RED_BATCH = 16;
__global__ void __launch_bounds__(CT) k_reduce_partials(const float* __restrict__ partial, int nchunk, int64_t n,
                                                      float* __restrict__ out) {
  __shared__ float s_run[RED_SEG][RED_OUT];
  const int o = threadIdx.x % RED_OUT, seg = threadIdx.x / RED_OUT;
  const int64_t i = blockIdx.x * (int64_t)RED_OUT + o;
  const int len = (nchunk + RED_SEG - 1) / RED_SEG;
  const int c0 = seg * len, c1 = min(nchunk, c0 + len);
  float s = 0.f;
  if (i < n) {
    // the run's values are loaded RED_BATCH at a time before they are added
    // (in chunk order, as a plain loop would), so a run costs about one
    // memory round trip per batch instead of one per chunk
    const float* p = partial + (int64_t)c0 * n + i;
    const int cnt = c1 - c0;
    int c = 0;
    for (; c + RED_BATCH <= cnt; c += RED_BATCH) {
      float v[RED_BATCH];
#pragma unroll
      for (int j = 0; j < RED_BATCH; ++j) v[j] = p[(int64_t)(c + j) * n];
#pragma unroll
      for (int j = 0; j < RED_BATCH; ++j) s += v[j];
    }
    for (; c < cnt; ++c) s += p[(int64_t)c * n];
  }
  s_run[seg][o] = s;
  __syncthreads();
  if (seg == 0 && i < n) {
    float t = 0.f;
    for (int r = 0; r < RED_SEG; ++r) t += s_run[r][o];
    out[i] = t;
  }
}

// dLow[b][y][x][c] = sum of the 2x2 block of dHigh (first `c_low` channels of
// a `stride`-channel tensor): adjoint of nearest x2 upsampling.
__global__ void k_up_adjoint(const float* __restrict__ dhigh, int stride, float* __restrict__ dlow, int B, int h, int w,
                             int c_low) {
  const int64_t n = (int64_t)B * h * w * c_low;
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int c = (int)(i % c_low);
  int64_t r = i / c_low;
  const int x = (int)(r % w);
  r /= w;
  const int y = (int)(r % h);
  const int b = (int)(r / h);
  const int W = 2 * w;
  const float* p = dhigh + (((int64_t)b * 2 * h + 2 * y) * W + 2 * x) * stride + c;
  dlow[i] = (p[0] + p[stride]) + (p[(int64_t)W * stride] + p[(int64_t)W * stride + stride]);
}

// dst[p][c] = (accumulate ? dst : 0) + src[p*stride + coff + c]
__global__ void k_copy_channels(const float* __restrict__ src, int stride, int coff, float* __restrict__ dst, int C,
                                int64_t npix, int accumulate) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= npix * C) return;
  const int64_t p = i / C;
  const int c = (int)(i - p * C);
  const float v = src[p * stride + coff + c];
  dst[i] = accumulate ? dst[i] + v : v;
}

// dst[b][y0 + y][y0 + x][c] += src[b][y][x][c]: a window tensor of C
// channels added into the H x H plane
__global__ void k_add_window(const float* __restrict__ src, int n, int y0, float* __restrict__ dst, int H, int B,
                             int C) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= (int64_t)B * n * n * C) return;
  const int c = (int)(i % C);
  int64_t r = i / C;
  const int x = (int)(r % n);
  r /= n;
  const int y = (int)(r % n);
  const int b = (int)(r / n);
  dst[(((int64_t)b * H + y0 + y) * H + y0 + x) * C + c] += src[i];
}

// dHigh += 0.25 * spread(dLow): adjoint of 2x2 average pooling
__global__ void k_pool_adjoint_add(const float* __restrict__ dlow, float* __restrict__ dhigh, int B, int H, int W, int C) {
  const int64_t n = (int64_t)B * H * W * C;
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int c = (int)(i % C);
  int64_t r = i / C;
  const int x = (int)(r % W);
  r /= W;
  const int y = (int)(r % H);
  const int b = (int)(r / H);
  dhigh[i] += 0.25f * dlow[(((int64_t)b * (H / 2) + y / 2) * (W / 2) + x / 2) * C + c];
}

// dX[crop][{0,2,3,4}] += dY (residual path)
__global__ void k_residual_adjoint(const float* __restrict__ dy, float* __restrict__ dx, int B, int res, int pad) {
  const int64_t n = (int64_t)B * res * res;
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int b = (int)(i / ((int64_t)res * res));
  const int r = (int)(i - (int64_t)b * res * res);
  const int R = res + 2 * pad;
  float* p = dx + (((int64_t)b * R + r / res + pad) * R + r % res + pad) * 8;
  const float4 g = ld4(dy + 4 * i);
  p[0] += g.x;
  p[2] += g.y;
  p[3] += g.z;
  p[4] += g.w;
}

inline int nblk(int64_t n) { return (int)((n + CT - 1) / CT); }

}  // namespace

// ------------------------------------------------------------------ host side
SrcPart src_plain(const float* p, int c, int h, int w, int stride, int coff, const float* mask) {
  SrcPart s;
  s.f32 = p;
  s.bf16 = nullptr;
  s.mask = mask;
  s.c = c;
  s.h = h;
  s.w = w;
  s.stride = stride;
  s.coff = coff;
  s.up = 0;
  s.oy = 0;
  s.ox = 0;
  return s;
}

SrcPart src_none() { return src_plain(nullptr, 0, 0, 0, 0, 0, nullptr); }

int ls_conv_f32(const ConvArgs& a, hipStream_t st) {
  const int64_t npix = (int64_t)a.B * a.Ho * a.Wo;
  const bool mask = (a.src.a.mask != nullptr) || (a.src.b.mask != nullptr);
  const int cap = a.cob_max > 0 ? a.cob_max : 32;
  int cob = 4;
  for (int c = 32; c >= 4; c /= 2)
    if (c <= cap && a.cout % c == 0) {
      cob = c;
      break;
    }
  if (a.cout % 4) return LS_ENOTIMPL;
  dim3 grid(nblk(npix), a.cout / cob);
  LS_TRACE("conv_f32", st);
#define LS_CONV_CASE(N)                                                                   \
  if (cob == N) {                                                                          \
    if (mask) hipLaunchKernelGGL((k_conv_f32<N, true>), grid, dim3(CT), 0, st, a);         \
    else hipLaunchKernelGGL((k_conv_f32<N, false>), grid, dim3(CT), 0, st, a);             \
  }
  LS_CONV_CASE(32) LS_CONV_CASE(16) LS_CONV_CASE(8) LS_CONV_CASE(4)
#undef LS_CONV_CASE
  LS_LAUNCH_CHECK();
  return LS_OK;
}

int ls_avgpool_f32(const float* in, float* out, int B, int H, int W, int C, hipStream_t st) {
  const int64_t n = (int64_t)B * (H / 2) * (W / 2) * (C / 4);
  LS_TRACE("avgpool_f32", st);
  hipLaunchKernelGGL(k_avgpool_f32, dim3(nblk(n)), dim3(CT), 0, st, in, out, B, H, W, C);
  LS_LAUNCH_CHECK();
  return LS_OK;
}

int ls_head_epilogue(const float* head, const float* x, const double* cz, int B, int res, int pad, double r_m,
                     float* y_out, float* tex_out, hipStream_t st) {
  const int64_t n = (int64_t)B * res * res;
  LS_TRACE("head_epilogue", st);
  hipLaunchKernelGGL(k_head_epilogue, dim3(nblk(n)), dim3(CT), 0, st, head, x, cz, B, res, pad, r_m, y_out, tex_out);
  LS_LAUNCH_CHECK();
  return LS_OK;
}

int ls_prep_weights(const float* w, float* wt, float* wd, hipStream_t st) {
  LS_TRACE("prep_weights", st);
  hipLaunchKernelGGL(k_prep_weights, dim3(nblk(LS_NUM_PARAMS)), dim3(CT), 0, st, w, wt, wd);
  LS_LAUNCH_CHECK();
  return LS_OK;
}

int ls_wgrad_f32(const WgradArgs& a, float* grad_w_layer, hipStream_t st) {
  const int cin = a.src.a.c + a.src.b.c;
  const int64_t n = (int64_t)a.cout * 9 * cin + a.cout;
  // every part and the gradient are read four channels at a time
  if (a.cout % 4 || a.src.a.c % 4 || a.src.b.c % 4 || a.d_stride % 4) return LS_ENOTIMPL;
  const int mwg = a.cout <= 16 ? 16 : (a.cout <= 32 ? 32 : 64);
  if (a.cout > 64) return LS_ENOTIMPL;
  LS_TRACE("wgrad", st);
  // the tile kernel: 16 x 16 output tiles, the input staged once per tile
  if (a.mfma == 2 && a.g_bf16 && a.src.a.c % 8 == 0 && a.src.b.c % 8 == 0 && a.cout <= 32 && a.d_stride % 4 == 0) {
    const int ng8 = cin / 8;
    dim3 grid((unsigned)a.nchunk, (unsigned)((ng8 + WT_GROUPS - 1) / WT_GROUPS));
    // an FP32-stored part needs the rounding at staging, compiled in only where used
    const bool xf32 = (a.src.a.c > 0 && a.src.a.f32) || (a.src.b.c > 0 && a.src.b.f32);
    if (a.cout <= 16) {
      if (xf32)
        hipLaunchKernelGGL((k_wgrad_tile<1, true>), grid, dim3(CT), 0, st, a);
      else
        hipLaunchKernelGGL((k_wgrad_tile<1, false>), grid, dim3(CT), 0, st, a);
    } else {
      if (xf32)
        hipLaunchKernelGGL((k_wgrad_tile<2, true>), grid, dim3(CT), 0, st, a);
      else
        hipLaunchKernelGGL((k_wgrad_tile<2, false>), grid, dim3(CT), 0, st, a);
    }
  } else if (a.mfma && a.g_bf16 && a.src.a.c % 8 == 0 && a.src.b.c % 8 == 0) {
    // the matrix-core kernel stages 8 channels of one part at a time
    // column tiles per wave: the fewest that cover the columns in one
    // workgroup, at most 8 (more workgroups along x beyond that)
    const int tiles = (9 * cin + 1 + 15) / 16;
    const int ctw = tiles <= 8 ? 2 : (tiles <= 16 ? 4 : 8);
    dim3 grid((unsigned)((9 * cin + 1 + 64 * ctw - 1) / (64 * ctw)), (unsigned)a.nchunk);
    const bool xf32 = (a.src.a.c > 0 && a.src.a.f32) || (a.src.b.c > 0 && a.src.b.f32);
#define LS_WM(M, C)                                                            \
  do {                                                                         \
    if (xf32)                                                                  \
      hipLaunchKernelGGL((k_wgrad_mfma<M, C, true>), grid, dim3(CT), 0, st, a);  \
    else                                                                       \
      hipLaunchKernelGGL((k_wgrad_mfma<M, C, false>), grid, dim3(CT), 0, st, a); \
  } while (0)
    const int mt = (a.cout + 15) / 16;
    if (mt == 1) {
      if (ctw == 2) LS_WM(1, 2); else if (ctw == 4) LS_WM(1, 4); else LS_WM(1, 8);
    } else if (mt == 2) {
      if (ctw == 2) LS_WM(2, 2); else if (ctw == 4) LS_WM(2, 4); else LS_WM(2, 8);
    } else {
      if (ctw == 2) LS_WM(4, 2); else if (ctw == 4) LS_WM(4, 4); else LS_WM(4, 8);
    }
#undef LS_WM
  } else {
    const int cols = 4 * (CT / (mwg / 4));
    dim3 grid((unsigned)((9 * cin + 1 + cols - 1) / cols), (unsigned)a.nchunk);
    switch (mwg) {
      case 16: hipLaunchKernelGGL(k_wgrad_tiled<16>, grid, dim3(CT), 0, st, a); break;
      case 32: hipLaunchKernelGGL(k_wgrad_tiled<32>, grid, dim3(CT), 0, st, a); break;
      default: hipLaunchKernelGGL(k_wgrad_tiled<64>, grid, dim3(CT), 0, st, a); break;
    }
  }
  hipLaunchKernelGGL(k_reduce_partials, dim3((unsigned)((n + RED_OUT - 1) / RED_OUT)), dim3(CT), 0, st, a.partial,
                     a.nchunk, n, grad_w_layer);
  LS_LAUNCH_CHECK();
  return LS_OK;
}

int ls_up_adjoint(const float* dhigh, int stride, float* dlow, int B, int h, int w, int c_low, hipStream_t st) {
  LS_TRACE("up_adjoint", st);
  const int64_t n = (int64_t)B * h * w * c_low;
  hipLaunchKernelGGL(k_up_adjoint, dim3(nblk(n)), dim3(CT), 0, st, dhigh, stride, dlow, B, h, w, c_low);
  LS_LAUNCH_CHECK();
  return LS_OK;
}

int ls_copy_channels(const float* src, int stride, int coff, float* dst, int C, int64_t npix, int acc, hipStream_t st) {
  LS_TRACE("copy_channels", st);
  hipLaunchKernelGGL(k_copy_channels, dim3(nblk(npix * C)), dim3(CT), 0, st, src, stride, coff, dst, C, npix, acc);
  LS_LAUNCH_CHECK();
  return LS_OK;
}

int ls_add_window(const float* src, int n, int y0, float* dst, int H, int B, int C, hipStream_t st) {
  if (n <= 0 || B <= 0) return LS_OK;
  if (y0 < 0 || y0 + n > H) return LS_EINVAL;
  LS_TRACE("copy_channels", st);
  hipLaunchKernelGGL(k_add_window, dim3(nblk((int64_t)B * n * n * C)), dim3(CT), 0, st, src, n, y0, dst, H, B, C);
  LS_LAUNCH_CHECK();
  return LS_OK;
}

int ls_pool_adjoint_add(const float* dlow, float* dhigh, int B, int H, int W, int C, hipStream_t st) {
  LS_TRACE("pool_adjoint", st);
  const int64_t n = (int64_t)B * H * W * C;
  hipLaunchKernelGGL(k_pool_adjoint_add, dim3(nblk(n)), dim3(CT), 0, st, dlow, dhigh, B, H, W, C);
  LS_LAUNCH_CHECK();
  return LS_OK;
}

int ls_residual_adjoint(const float* dy, float* dx, int B, int res, int pad, hipStream_t st) {
  LS_TRACE("residual_adjoint", st);
  const int64_t n = (int64_t)B * res * res;
  hipLaunchKernelGGL(k_residual_adjoint, dim3(nblk(n)), dim3(CT), 0, st, dy, dx, B, res, pad);
  LS_LAUNCH_CHECK();
  return LS_OK;
}
