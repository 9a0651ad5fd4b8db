// BF16 refinement-network forward on the gfx950 matrix cores.
//
// Each 3x3 conv is an implicit GEMM: rows = output pixels (NHWC order),
// columns = output channels, reduction k = tap*cin + ci (tap-major, so a run
// of 8 consecutive k is 8 consecutive channels of one input pixel: one
// 16-byte load).  A wave owns 16*MT pixels x all output channels and issues
// v_mfma_f32_16x16x32_bf16 (FP32 accumulation); lane l supplies A row l%16
// and B column l%16 with k in [8*(l/16), 8*(l/16)+8) of each 32-wide step,
// and receives D rows 4*(l/16)..+3 of column l%16.  Bias and ReLU are
// applied in FP32, activations are stored as BF16 (round to nearest even).
// The head keeps its FP32 result for the FP32 residual and denormalisation.
#include <algorithm>

#include "ls_common.hpp"
#include "ls_unet_bf16.hpp"

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));

constexpr int WAVES = 4;
constexpr int MT = 4;  // 16-pixel tiles per wave

struct ConvArgsB {
  ConvSrc src;
  int B, H, W;
  int y0, x0, Ho, Wo;
  const uint16_t* wp;  // packed [Npad][Kpad]
  int Kpad;
  const float* bias;
  int cout;            // channels stored
  int relu;
  uint16_t* out_bf16;  // [B][Ho][Wo][out_stride] or null
  float* out_f32;
  int out_stride;
};

__device__ __forceinline__ unsigned short f2bf(float f) {
  return __builtin_bit_cast(unsigned short, static_cast<__bf16>(f));
}

__device__ __forceinline__ float bf2f(unsigned short h) {
  return __builtin_bit_cast(float, (uint32_t)h << 16);
}

// 8 consecutive channels of input pixel (yy, xx) as BF16 bits; zero outside.
__device__ __forceinline__ u16x8 load8(const ConvSrc& s, int b, int yy, int xx, int ci, int H, int W) {
  u16x8 z = {0, 0, 0, 0, 0, 0, 0, 0};
  if (yy < 0 || xx < 0 || yy >= H || xx >= W) return z;
  const bool in_a = ci < s.a.c;
  const SrcPart& p = in_a ? s.a : s.b;
  const int cc = in_a ? ci : ci - s.a.c;
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
  if (p.bf16) return *reinterpret_cast<const u16x8*>(p.bf16 + o);
  const float4 f0 = *reinterpret_cast<const float4*>(p.f32 + o);
  const float4 f1 = *reinterpret_cast<const float4*>(p.f32 + o + 4);
  u16x8 r;
  r[0] = f2bf(f0.x);
  r[1] = f2bf(f0.y);
  r[2] = f2bf(f0.z);
  r[3] = f2bf(f0.w);
  r[4] = f2bf(f1.x);
  r[5] = f2bf(f1.y);
  r[6] = f2bf(f1.z);
  r[7] = f2bf(f1.w);
  return r;
}

template <int NT>
__global__ void __launch_bounds__(64 * WAVES) k_conv_bf16(ConvArgsB A) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t npix = (int64_t)A.B * A.Ho * A.Wo;
  const int64_t wbase = ((int64_t)blockIdx.x * WAVES + wave) * (16 * MT);
  if (wbase >= npix) return;
  const int r16 = lane & 15, g = lane >> 4;
  const int cin = A.src.a.c + A.src.b.c;
  const int K = 9 * cin;
  int pb[MT], py[MT], px[MT];
  bool pv[MT];
#pragma unroll
  for (int mt = 0; mt < MT; ++mt) {
    const int64_t p = wbase + mt * 16 + r16;
    pv[mt] = p < npix;
    const int64_t pp = pv[mt] ? p : 0;
    const int b = (int)(pp / ((int64_t)A.Ho * A.Wo));
    const int r = (int)(pp - (int64_t)b * A.Ho * A.Wo);
    pb[mt] = b;
    py[mt] = A.y0 + r / A.Wo;
    px[mt] = A.x0 + r % A.Wo;
  }
  f32x4 acc[MT][NT];
#pragma unroll
  for (int mt = 0; mt < MT; ++mt)
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) acc[mt][nt] = f32x4{0.f, 0.f, 0.f, 0.f};
  const int KS = A.Kpad / 32;
  for (int ks = 0; ks < KS; ++ks) {
    const int k = ks * 32 + 8 * g;
    bf16x8 bfr[NT];
#pragma unroll
    for (int nt = 0; nt < NT; ++nt)
      bfr[nt] = __builtin_bit_cast(bf16x8,
                                   *reinterpret_cast<const u16x8*>(A.wp + (int64_t)(nt * 16 + r16) * A.Kpad + k));
    const bool kv = k < K;
    const int tap = kv ? k / cin : 0;
    const int ci = k - tap * cin;
    const int ky = tap / 3, kx = tap - 3 * (tap / 3);
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) {
      u16x8 a = {0, 0, 0, 0, 0, 0, 0, 0};
      if (kv && pv[mt]) a = load8(A.src, pb[mt], py[mt] + ky - 1, px[mt] + kx - 1, ci, A.H, A.W);
      const bf16x8 ab = __builtin_bit_cast(bf16x8, a);
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) acc[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ab, bfr[nt], acc[mt][nt], 0, 0, 0);
    }
  }
  // epilogue: D rows 4*g + r (pixels), column r16 (channel)
#pragma unroll
  for (int nt = 0; nt < NT; ++nt) {
    const int co = nt * 16 + r16;
    if (co >= A.cout) continue;
    const float bias = A.bias ? A.bias[co] : 0.f;
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t p = wbase + mt * 16 + 4 * g + r;
        if (p >= npix) continue;
        float v = acc[mt][nt][r] + bias;
        if (A.relu) v = fmaxf(v, 0.f);
        if (A.out_bf16) A.out_bf16[p * A.out_stride + co] = f2bf(v);
        else A.out_f32[p * A.out_stride + co] = v;
      }
  }
}

__global__ void k_avgpool_bf16(const uint16_t* __restrict__ in, uint16_t* __restrict__ out, int B, int H, int W, int C) {
  const int64_t n = (int64_t)B * (H / 2) * (W / 2) * C;
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int c = (int)(i % C);
  int64_t r = i / C;
  const int x = (int)(r % (W / 2));
  r /= (W / 2);
  const int y = (int)(r % (H / 2));
  const int b = (int)(r / (H / 2));
  const uint16_t* p = in + (((int64_t)b * H + 2 * y) * W + 2 * x) * C + c;
  const float s = (bf2f(p[0]) + bf2f(p[C])) + (bf2f(p[(int64_t)W * C]) + bf2f(p[(int64_t)W * C + C]));
  out[i] = f2bf(0.25f * s);
}

__global__ void k_pack_weights_bf16(const uint16_t* __restrict__ w, uint16_t* __restrict__ packed) {
  // one thread per packed element of all layers
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  int64_t off = 0, woff = 0;
  for (int l = 0; l < LS_NLAYER; ++l) {
    const int cin = LS_LAYERS[l].cin, cout = LS_LAYERS[l].cout;
    const int K = 9 * cin, Kpad = (K + 31) / 32 * 32, Npad = (cout + 15) / 16 * 16;
    const int64_t n = (int64_t)Npad * Kpad;
    if (i >= off && i < off + n) {
      const int co = (int)((i - off) / Kpad), k = (int)((i - off) % Kpad);
      packed[i] = (co < cout && k < K) ? w[woff + (int64_t)co * K + k] : (uint16_t)0;
      return;
    }
    off += n;
    woff += (int64_t)cout * K + cout;
  }
}

__global__ void k_round_bf16(const float* __restrict__ w, uint16_t* __restrict__ out, int64_t n) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) out[i] = f2bf(w[i]);
}

}  // namespace

int ls_bf16_kpad(int l) { return (9 * LS_LAYERS[l].cin + 31) / 32 * 32; }

size_t ls_bf16_packed_offset(int l) {
  size_t off = 0;
  for (int k = 0; k < l; ++k) off += (size_t)((LS_LAYERS[k].cout + 15) / 16 * 16) * ls_bf16_kpad(k);
  return off;
}

size_t ls_bf16_packed_total() { return ls_bf16_packed_offset(LS_NLAYER); }

int ls_pack_bf16(const float* w, uint16_t* out, int64_t n, hipStream_t st) {
  hipLaunchKernelGGL(k_round_bf16, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, w, out, n);
  LS_LAUNCH_CHECK();
  return LS_OK;
}

int ls_bf16_prep_weights(const uint16_t* w_bf16, uint16_t* packed, hipStream_t st) {
  const int64_t n = (int64_t)ls_bf16_packed_total();
  hipLaunchKernelGGL(k_pack_weights_bf16, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, w_bf16, packed);
  LS_LAUNCH_CHECK();
  return LS_OK;
}

namespace {

int conv_bf16(const ConvSrc& s, int B, int H, int l, const uint16_t* packed, const float* w, uint16_t* out_bf16,
              float* out_f32, int relu, int y0, int x0, int Ho, int Wo, hipStream_t st) {
  ConvArgsB a;
  a.src = s;
  a.B = B;
  a.H = H;
  a.W = H;
  a.y0 = y0;
  a.x0 = x0;
  a.Ho = Ho;
  a.Wo = Wo;
  a.wp = packed + ls_bf16_packed_offset(l);
  a.Kpad = ls_bf16_kpad(l);
  a.bias = w + ls_layer_b_offset(l);
  a.cout = LS_LAYERS[l].cout;
  a.relu = relu;
  a.out_bf16 = out_bf16;
  a.out_f32 = out_f32;
  a.out_stride = a.cout;
  const int64_t npix = (int64_t)B * Ho * Wo;
  const int64_t per_block = 16 * MT * WAVES;
  dim3 grid((unsigned)((npix + per_block - 1) / per_block));
  const int nt = (a.cout + 15) / 16;
  switch (nt) {
    case 1: hipLaunchKernelGGL(k_conv_bf16<1>, grid, dim3(64 * WAVES), 0, st, a); break;
    case 2: hipLaunchKernelGGL(k_conv_bf16<2>, grid, dim3(64 * WAVES), 0, st, a); break;
    case 4: hipLaunchKernelGGL(k_conv_bf16<4>, grid, dim3(64 * WAVES), 0, st, a); break;
    default: return LS_ENOTIMPL;
  }
  LS_LAUNCH_CHECK();
  return LS_OK;
}

SrcPart bpart(const uint16_t* p, int c, int hw) {
  SrcPart s = src_none();
  s.bf16 = p;
  s.c = c;
  s.h = hw;
  s.w = hw;
  s.stride = c;
  return s;
}

ConvSrc cs(SrcPart a, SrcPart b) {
  ConvSrc s;
  s.a = a;
  s.b = b;
  return s;
}

int pool_bf16(const uint16_t* in, uint16_t* out, int B, int H, int C, hipStream_t st) {
  const int64_t n = (int64_t)B * (H / 2) * (H / 2) * C;
  hipLaunchKernelGGL(k_avgpool_bf16, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, in, out, B, H, H, C);
  LS_LAUNCH_CHECK();
  return LS_OK;
}

}  // namespace

#define LS_TRYB(expr)              \
  do {                             \
    int rc_ = (expr);              \
    if (rc_ != LS_OK) return rc_;  \
  } while (0)

int ls_bf16_forward(const float* w, const uint16_t* packed, const float* x, int B, const LsGridInfo& gi,
                    uint16_t* acts, float* head, hipStream_t st) {
  const int R = gi.R, R2 = R / 2, R4 = R / 4;
  const int64_t f = (int64_t)R * R, h = f / 4, q = f / 16;
  // same activation order and sizes as the FP32 layout
  uint16_t* A1 = acts;
  uint16_t* A2 = A1 + 16 * f * B;
  uint16_t* P1 = A2 + 16 * f * B;
  uint16_t* A3 = P1 + 16 * h * B;
  uint16_t* A4 = A3 + 32 * h * B;
  uint16_t* P2 = A4 + 32 * h * B;
  uint16_t* A5 = P2 + 32 * q * B;
  uint16_t* A6 = A5 + 64 * q * B;
  uint16_t* A7 = A6 + 64 * q * B;
  uint16_t* A8 = A7 + 32 * h * B;
  uint16_t* A9 = A8 + 32 * h * B;
  uint16_t* A10 = A9 + 16 * f * B;
  SrcPart X = src_plain(x, 8, R, R, 8, 0, nullptr);
  const SrcPart none = src_none();
  auto full = [&](const ConvSrc& s, int H, int l, uint16_t* out) {
    return conv_bf16(s, B, H, l, packed, w, out, nullptr, 1, 0, 0, H, H, st);
  };
  SrcPart u6 = bpart(A6, 64, R4);
  u6.up = 1;
  SrcPart u8 = bpart(A8, 32, R2);
  u8.up = 1;
  LS_TRYB(full(cs(X, none), R, 0, A1));
  LS_TRYB(full(cs(bpart(A1, 16, R), none), R, 1, A2));
  LS_TRYB(pool_bf16(A2, P1, B, R, 16, st));
  LS_TRYB(full(cs(bpart(P1, 16, R2), none), R2, 2, A3));
  LS_TRYB(full(cs(bpart(A3, 32, R2), none), R2, 3, A4));
  LS_TRYB(pool_bf16(A4, P2, B, R2, 32, st));
  LS_TRYB(full(cs(bpart(P2, 32, R4), none), R4, 4, A5));
  LS_TRYB(full(cs(bpart(A5, 64, R4), none), R4, 5, A6));
  LS_TRYB(full(cs(u6, bpart(A4, 32, R2)), R2, 6, A7));
  LS_TRYB(full(cs(bpart(A7, 32, R2), none), R2, 7, A8));
  LS_TRYB(full(cs(u8, bpart(A2, 16, R)), R, 8, A9));
  LS_TRYB(full(cs(bpart(A9, 16, R), none), R, 9, A10));
  return conv_bf16(cs(bpart(A10, 16, R), X), B, R, 10, packed, w, nullptr, head, 0, gi.pad, gi.pad, gi.res, gi.res,
                   st);
}
