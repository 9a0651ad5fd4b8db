// BF16 refinement-network forward on the gfx950 matrix cores.
//
// Each 3x3 conv is an implicit GEMM: rows = output pixels (NHWC order),
// columns = output channels, reduction k = tap*cin + ci (tap-major, so a run
// of 8 consecutive k is 8 consecutive channels of one input pixel: one
// 16-byte load).  A wave owns 16*MT pixels (MT = 2 or 4) x all output channels and issues
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
  const uint16_t* mask;  // BF16 output: zero where this activation (same layout) is not positive, or null
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

int launch_direct(const ConvArgsB& a, int nt, int mt, int64_t npix, hipStream_t st);

// Workgroups are dealt to the 8 XCDs round-robin (workgroup i to XCD i % 8),
// each XCD with its own L2.  This renumbering hands every XCD a contiguous
// run of output tiles, so the halo rows two neighbouring tiles share are
// fetched from HBM once, into the one L2 that serves both.
constexpr int N_XCD = 8;
__device__ __forceinline__ int xcd_block() {
  const int nb = gridDim.x, bid = blockIdx.x;
  const int per = nb / N_XCD, rem = nb - per * N_XCD;
  const int x = bid % N_XCD, i = bid / N_XCD;
  return x * per + min(x, rem) + i;
}

// NT 16-channel output tiles, MT 16-pixel tiles per wave
template <int NT, int MT>
__global__ void __launch_bounds__(64 * WAVES) k_conv_bf16(ConvArgsB A) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t npix = (int64_t)A.B * A.Ho * A.Wo;
  const int64_t wbase = ((int64_t)xcd_block() * WAVES + wave) * (16 * MT);
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
        if (A.mask && !(bf2f(A.mask[p * A.out_stride + co]) > 0.f)) v = 0.f;
        if (A.out_bf16) A.out_bf16[p * A.out_stride + co] = f2bf(v);
        else A.out_f32[p * A.out_stride + co] = v;
      }
  }
}

// ---------------------------------------------------------------------------
// LDS-staged variant: a workgroup owns a 16 x 16 output tile of one image.
// The 18 x 18 x cin input patch (zero padded, upsampling / concatenation /
// FP32->BF16 folded in) is loaded once into LDS with an odd number of 16-byte
// units per pixel, so the 16 lanes of an MFMA row read 16 distinct bank
// groups.  Each wave computes 4 output rows (4 MFMA row tiles of 16 pixels)
// for all output channels.  The result goes back through LDS so every lane
// stores whole 16-byte channel groups, and the layers that feed an average
// pool also write the pooled 8 x 8 tile.
constexpr int TT = 16;       // output tile side
constexpr int PT = TT + 2;   // input patch side
constexpr size_t LDS_MAX = 160 * 1024;  // LDS per workgroup on gfx950

__host__ __device__ __forceinline__ int patch_pitch(int cin) {
  const int u = cin / 8;
  return 8 * (u + ((u & 1) ? 0 : 1));  // bf16 elements per pixel, odd number of 16-byte units
}

// Bias, ReLU and the store of one 16 x 16 output tile (and its 8 x 8 average
// pool): the accumulators go through LDS so every lane stores whole 16-byte
// channel groups.  All threads call it after the last MFMA.
template <int NT>
__device__ __forceinline__ void conv_tile_store(const ConvTileArgs& A, f32x4 (&acc)[4][NT], int b, int ty0, int tx0,
                                                int wave, int g, int r16, unsigned char* s_raw) {
  __syncthreads();  // the patch is dead; the same LDS now holds the output tile
  const int cout = A.cout;
  if (A.out_f32) {
    float* s_of = reinterpret_cast<float*>(s_raw);
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
      const int co = nt * 16 + r16;
      if (co >= cout) continue;
      const float bias = A.bias ? A.bias[co] : 0.f;
#pragma unroll
      for (int mt = 0; mt < 4; ++mt)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          float v = acc[mt][nt][r] + bias;
          if (A.relu) v = fmaxf(v, 0.f);
          s_of[((wave * 4 + mt) * TT + 4 * g + r) * cout + co] = v;
        }
    }
    __syncthreads();
    for (int e = threadIdx.x; e < TT * TT * cout / 4; e += 256) {
      const int pix = e / (cout / 4), c4 = e - pix * (cout / 4);
      const int oy = ty0 + pix / TT, ox = tx0 + pix % TT;
      if (oy >= A.Ho || ox >= A.Wo) continue;
      *reinterpret_cast<float4*>(A.out_f32 + (((int64_t)b * A.Ho + oy) * A.Wo + ox) * A.out_stride + A.out_coff +
                                 4 * c4) = *reinterpret_cast<const float4*>(s_of + pix * cout + 4 * c4);
    }
    return;
  }
  uint16_t* s_o = reinterpret_cast<uint16_t*>(s_raw);
#pragma unroll
  for (int nt = 0; nt < NT; ++nt) {
    const int co = nt * 16 + r16;
    if (co >= cout) continue;
    const float bias = A.bias ? A.bias[co] : 0.f;
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        float v = acc[mt][nt][r] + bias;
        if (A.relu) v = fmaxf(v, 0.f);
        s_o[((wave * 4 + mt) * TT + 4 * g + r) * cout + co] = f2bf(v);
      }
  }
  __syncthreads();
  const int c8n = cout / 8;
  if (A.out_bf16)
    for (int e = threadIdx.x; e < TT * TT * c8n; e += 256) {
      const int pix = e / c8n, c8 = e - pix * c8n;
      const int oy = ty0 + pix / TT, ox = tx0 + pix % TT;
      if (oy >= A.Ho || ox >= A.Wo) continue;
      *reinterpret_cast<u16x8*>(A.out_bf16 + (((int64_t)b * A.Ho + oy) * A.Wo + ox) * A.out_stride + A.out_coff +
                                8 * c8) = *reinterpret_cast<const u16x8*>(s_o + pix * cout + 8 * c8);
    }
  if (A.pool_out) {
    const int Hp = A.Ho / 2, Wp = A.Wo / 2;
    for (int e = threadIdx.x; e < (TT / 2) * (TT / 2) * cout; e += 256) {
      const int pp = e / cout, c = e - pp * cout;
      const int py = pp / (TT / 2), px = pp % (TT / 2);
      const uint16_t* q = s_o + ((2 * py) * TT + 2 * px) * cout + c;
      const float s = (bf2f(q[0]) + bf2f(q[cout])) + (bf2f(q[TT * cout]) + bf2f(q[TT * cout + cout]));
      const int oy = ty0 / 2 + py, ox = tx0 / 2 + px;
      if (oy >= Hp || ox >= Wp) continue;
      A.pool_out[(((int64_t)b * Hp + oy) * Wp + ox) * A.pool_stride + A.pool_coff + c] = f2bf(0.25f * s);
    }
  }
}

template <int NT>
__global__ void __launch_bounds__(256) k_conv_bf16_lds(ConvTileArgs A) {
  extern __shared__ __align__(16) unsigned char s_raw[];
  uint16_t* s_in = reinterpret_cast<uint16_t*>(s_raw);
  const int cin = A.src.a.c + A.src.b.c;
  const int pitch = patch_pitch(cin);
  const int per_img = A.tiles_x * A.tiles_y;
  const int blk = xcd_block();
  const int b = blk / per_img;
  const int t = blk - b * per_img;
  const int ty0 = (t / A.tiles_x) * TT, tx0 = (t % A.tiles_x) * TT;
  const int iy0 = A.y0 + ty0 - 1, ix0 = A.x0 + tx0 - 1;
  const int chunks = cin / 8;
  for (int e = threadIdx.x; e < PT * PT * chunks; e += 256) {
    const int pix = e / chunks, ch = e - pix * chunks;
    const int py = pix / PT, px = pix - py * PT;
    *reinterpret_cast<u16x8*>(s_in + pix * pitch + ch * 8) = load8(A.src, b, iy0 + py, ix0 + px, ch * 8, A.H, A.W);
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int r16 = lane & 15, g = lane >> 4;
  const int K = 9 * cin, KS = A.Kpad / 32;
  f32x4 acc[4][NT];
#pragma unroll
  for (int mt = 0; mt < 4; ++mt)
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) acc[mt][nt] = f32x4{0.f, 0.f, 0.f, 0.f};
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
    const uint16_t* base = s_in + ((wave * 4 + ky) * PT + r16 + kx) * pitch + ci;
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) {
      u16x8 a = {0, 0, 0, 0, 0, 0, 0, 0};
      if (kv) a = *reinterpret_cast<const u16x8*>(base + mt * PT * pitch);
      const bf16x8 ab = __builtin_bit_cast(bf16x8, a);
#pragma unroll
      for (int nt = 0; nt < NT; ++nt)
        acc[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ab, bfr[nt], acc[mt][nt], 0, 0, 0);
    }
  }
  conv_tile_store<NT>(A, acc, b, ty0, tx0, wave, g, r16, s_raw);
}

constexpr int pitch_c(int cin) { return 8 * (cin / 8 + ((cin / 8) & 1 ? 0 : 1)); }

// 8 consecutive FP32 values rounded to BF16 bits.
__device__ __forceinline__ u16x8 f32x8_to_bf16(const float* p) {
  const float4 f0 = *reinterpret_cast<const float4*>(p);
  const float4 f1 = *reinterpret_cast<const float4*>(p + 4);
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

// The channels of one stored part at input-plane pixel (yy, xx) into LDS
// (zeros outside the plane or the part), C channels, 16 bytes at a time.
template <int C, bool UP, bool F32>
__device__ __forceinline__ void load_part(const SrcPart& p, int b, int yy, int xx, bool in_plane, uint16_t* dst) {
  int sy, sx;
  if (UP) {
    sy = yy >> 1;
    sx = xx >> 1;
  } else {
    sy = yy - p.oy;
    sx = xx - p.ox;
  }
  const bool ok = in_plane && sy >= 0 && sx >= 0 && sy < p.h && sx < p.w;
  const int64_t o = (((int64_t)b * p.h + sy) * p.w + sx) * p.stride + p.coff;
#pragma unroll
  for (int c = 0; c < C / 8; ++c) {
    u16x8 v = {0, 0, 0, 0, 0, 0, 0, 0};
    if (ok) v = F32 ? f32x8_to_bf16(p.f32 + o + 8 * c) : *reinterpret_cast<const u16x8*>(p.bf16 + o + 8 * c);
    *reinterpret_cast<u16x8*>(dst + 8 * c) = v;
  }
}

// Bias, ReLU and the store of one 16 x 16 output tile computed with the MFMA
// operands swapped (D = channels x pixels): lane (g, r16) holds output pixel
// (wave * 4 + mt, r16) of the tile with channels nt * 16 + 4g .. + 3, so
// every lane stores 4 consecutive channels of one pixel (8 bytes as BF16, 16
// as FP32) and a wave covers 16 whole pixels per store: no LDS staging.  The
// 2 x 2 average pool pairs rows mt, mt + 1 inside the lane and columns r16,
// r16 ^ 1 across lanes, adding in the order of the staged epilogue (top pair,
// bottom pair, then their sum), so both epilogues give identical bits.
// The bias of the 4 channels lane (g, r16) stores for each channel tile.
template <int NT>
__device__ __forceinline__ void load_bias_t(const ConvTileArgs& A, int g, float (&bias)[NT][4]) {
#pragma unroll
  for (int nt = 0; nt < NT; ++nt)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int c = nt * 16 + 4 * g + r;
      bias[nt][r] = (A.bias && c < A.cout) ? A.bias[c] : 0.f;
    }
}

template <int NT>
__device__ __forceinline__ void conv_tile_store_t(const ConvTileArgs& A, const f32x4 (&acc)[4][NT],
                                                  const float (&bias)[NT][4], int b, int ty0, int tx0, int wave,
                                                  int g, int r16) {
  const int cout = A.cout;
  const int ox = tx0 + r16, oy0 = ty0 + wave * 4;
  // a whole tile inside the output needs no per-row test
  const bool full = ty0 + TT <= A.Ho && tx0 + TT <= A.Wo;
  const int64_t pix0 = ((int64_t)b * A.Ho + oy0) * A.Wo + ox;  // output pixel of row mt = 0
  const int ostr = A.out_stride;
#pragma unroll
  for (int nt = 0; nt < NT; ++nt) {
    const int c0 = nt * 16 + 4 * g;
    if (c0 >= cout) continue;  // only the 4-channel head leaves lanes idle
    float q[4][4];
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        float v = acc[mt][nt][r] + bias[nt][r];
        if (A.relu) v = fmaxf(v, 0.f);
        q[mt][r] = v;
      }
    if (A.up_out && c0 < A.up_c) {
      // 2 x 2 block sums, in the order of the separate upsampling adjoint:
      // (top left + top right) + (bottom left + bottom right)
      const int Hp = A.Ho / 2, Wp = A.Wo / 2;
#pragma unroll
      for (int pr = 0; pr < 2; ++pr) {
        float sum[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const float tl = q[2 * pr][r], bl = q[2 * pr + 1][r];
          const float tr = __shfl_xor(tl, 1, 64), br = __shfl_xor(bl, 1, 64);
          sum[r] = (tl + tr) + (bl + br);
        }
        const int py = (oy0 + 2 * pr) / 2, px = ox / 2;
        if ((r16 & 1) == 0 && (full || (py < Hp && px < Wp)))
          *reinterpret_cast<float4*>(A.up_out + (((int64_t)b * Hp + py) * Wp + px) * A.up_c + c0) =
              make_float4(sum[0], sum[1], sum[2], sum[3]);
      }
      continue;
    }
    if (A.out2_f32 && c0 >= A.split) {
      const int s2 = cout - A.split;
#pragma unroll
      for (int mt = 0; mt < 4; ++mt)
        if (full || (oy0 + mt < A.Ho && ox < A.Wo))
          *reinterpret_cast<float4*>(A.out2_f32 + (pix0 + (int64_t)mt * A.Wo) * s2 + (c0 - A.split)) =
              make_float4(q[mt][0], q[mt][1], q[mt][2], q[mt][3]);
      continue;
    }
    const int64_t off0 = pix0 * ostr + A.out_coff + c0, row = (int64_t)A.Wo * ostr;
    if (A.out_f32) {
#pragma unroll
      for (int mt = 0; mt < 4; ++mt)
        if (full || (oy0 + mt < A.Ho && ox < A.Wo))
          *reinterpret_cast<float4*>(A.out_f32 + off0 + mt * row) = make_float4(q[mt][0], q[mt][1], q[mt][2], q[mt][3]);
      continue;
    }
    if (A.mask) {
      // the backward's ReLU' of the layer below, 4 channels of each pixel
      const int64_t moff = A.mask_w ? (((int64_t)b * A.mask_h + oy0 + A.mask_y0) * A.mask_w + ox + A.mask_x0) * ostr + c0
                                    : off0;
      const int64_t mrow = A.mask_w ? (int64_t)A.mask_w * ostr : row;
#pragma unroll
      for (int mt = 0; mt < 4; ++mt)
        if (full || (oy0 + mt < A.Ho && ox < A.Wo)) {
          const uint2 mv = *reinterpret_cast<const uint2*>(A.mask + moff + mt * mrow);
          const uint32_t mw[2] = {mv.x, mv.y};
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const unsigned short m = (unsigned short)((r & 1) ? (mw[r >> 1] >> 16) : (mw[r >> 1] & 0xFFFFu));
            if (!(bf2f(m) > 0.f)) q[mt][r] = 0.f;
          }
        }
    }
    unsigned short h[4][4];
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) {
#pragma unroll
      for (int r = 0; r < 4; ++r) h[mt][r] = f2bf(q[mt][r]);
      if (A.out_bf16 && (full || (oy0 + mt < A.Ho && ox < A.Wo))) {
        uint2 u;
        u.x = (uint32_t)h[mt][0] | ((uint32_t)h[mt][1] << 16);
        u.y = (uint32_t)h[mt][2] | ((uint32_t)h[mt][3] << 16);
        *reinterpret_cast<uint2*>(A.out_bf16 + off0 + mt * row) = u;
      }
    }
    if (A.pool_out) {
      const int Hp = A.Ho / 2, Wp = A.Wo / 2;
#pragma unroll
      for (int pr = 0; pr < 2; ++pr) {
        unsigned short pv[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const float tl = bf2f(h[2 * pr][r]), bl = bf2f(h[2 * pr + 1][r]);
          const float tr = __shfl_xor(tl, 1, 64), br = __shfl_xor(bl, 1, 64);
          pv[r] = f2bf(0.25f * ((tl + tr) + (bl + br)));
        }
        const int py = (ty0 + wave * 4 + 2 * pr) / 2, px = ox / 2;
        if ((r16 & 1) == 0 && (full || (py < Hp && px < Wp))) {
          uint2 u;
          u.x = (uint32_t)pv[0] | ((uint32_t)pv[1] << 16);
          u.y = (uint32_t)pv[2] | ((uint32_t)pv[3] << 16);
          *reinterpret_cast<uint2*>(A.pool_out + (((int64_t)b * Hp + py) * Wp + px) * A.pool_stride + A.pool_coff +
                                    c0) = u;
        }
      }
    }
  }
}

// k_conv_bf16_lds specialised at compile time on the layer's input: CA
// channels from part a (nearest-upsampled if UPA, FP32-stored if F32A) and
// CB from part b.  Patch coordinates are computed once per pixel, the K loop
// is unrolled with the tap and channel of every step known up to the lane's
// 8-channel group, and the MFMA sequence per output is the generic kernel's
// with the operands swapped (weights as A, pixels as B), so each lane ends
// with 4 channels of one pixel and the epilogue needs no LDS.
template <int NT, int CA, int CB, bool UPA, bool F32A, bool F32B>
__global__ void __launch_bounds__(256) k_conv_bf16_lds_t(ConvTileArgs A) {
  constexpr int CIN = CA + CB, PITCH = pitch_c(CIN), K = 9 * CIN, KS = (K + 31) / 32, KPAD = KS * 32;
  extern __shared__ __align__(16) unsigned char s_raw[];
  uint16_t* s_in = reinterpret_cast<uint16_t*>(s_raw);
  const int per_img = A.tiles_x * A.tiles_y;
  const int blk = xcd_block();
  const int b = blk / per_img;
  const int t = blk - b * per_img;
  const int ty0 = (t / A.tiles_x) * TT, tx0 = (t % A.tiles_x) * TT;
  const int iy0 = A.y0 + ty0 - 1, ix0 = A.x0 + tx0 - 1;
  for (int pix = threadIdx.x; pix < PT * PT; pix += 256) {
    const int py = pix / PT, px = pix - py * PT;
    const int yy = iy0 + py, xx = ix0 + px;
    const bool in_plane = yy >= 0 && xx >= 0 && yy < A.H && xx < A.W;
    uint16_t* dst = s_in + pix * PITCH;
    load_part<CA, UPA, F32A>(A.src.a, b, yy, xx, in_plane, dst);
    if (CB > 0) load_part<CB, false, F32B>(A.src.b, b, yy, xx, in_plane, dst + CA);
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int r16 = lane & 15, g = lane >> 4;
  f32x4 acc[4][NT];
#pragma unroll
  for (int mt = 0; mt < 4; ++mt)
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) acc[mt][nt] = f32x4{0.f, 0.f, 0.f, 0.f};
  const uint16_t* wrow = A.wp + (int64_t)r16 * KPAD + 8 * g;
  const uint16_t* base = s_in + (wave * 4 * PT + r16) * PITCH;
#pragma unroll
  for (int ks = 0; ks < KS; ++ks) {
    const int k = ks * 32 + 8 * g;
    bf16x8 bfr[NT];
#pragma unroll
    for (int nt = 0; nt < NT; ++nt)
      bfr[nt] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const u16x8*>(wrow + nt * 16 * KPAD + ks * 32));
    const bool kv = k < K;
    const int tap = kv ? k / CIN : 0;
    const int ci = k - tap * CIN;
    const int ky = tap / 3, kx = tap - 3 * ky;
    const uint16_t* pb = base + (ky * PT + kx) * PITCH + ci;
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) {
      u16x8 a = {0, 0, 0, 0, 0, 0, 0, 0};
      if (kv) a = *reinterpret_cast<const u16x8*>(pb + mt * PT * PITCH);
      const bf16x8 ab = __builtin_bit_cast(bf16x8, a);
#pragma unroll
      for (int nt = 0; nt < NT; ++nt)
        acc[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bfr[nt], ab, acc[mt][nt], 0, 0, 0);
    }
  }
  float bias[NT][4];
  load_bias_t<NT>(A, g, bias);
  conv_tile_store_t<NT>(A, acc, bias, b, ty0, tx0, wave, g, r16);
}

// Packed weight rows in LDS: KPAD elements padded to an odd number of
// 16-byte units, so the 16 rows a B fragment reads fall in distinct banks.
constexpr int wpitch_c(int kpad) { return kpad + ((kpad / 8) % 2 == 0 ? 8 : 0); }

// LDS bytes of k_conv_bf16_pipe: the input patch, then the layer's weights.
constexpr size_t pipe_lds_bytes(int nt, int cin) {
  return (size_t)PT * PT * pitch_c(cin) * 2 + (size_t)nt * 16 * wpitch_c((9 * cin + 31) / 32 * 32) * 2;
}

// MINW is the layer's register budget as waves per SIMD (measured per layer:
// the narrow layers gain from more waves, the widest spill below one).
// Persistent form of k_conv_bf16_lds_t: each workgroup copies the layer's
// packed weights into LDS once, then walks the output tiles tile,
// tile + gridDim.x, ...; while one tile is multiplied and stored, the next
// tile's patch is already being loaded into registers (NJ 16-byte units per
// thread, 32 bytes for units of an FP32 source, converted to BF16 when they
// are written to LDS), so neither the patch nor the weights are waited for
// inside the MFMA loop.  Same MFMA sequence and epilogue as
// k_conv_bf16_lds_t, hence identical results.
template <int NT, int CA, int CB, bool UPA, bool F32A, bool F32B, int MINW>
__global__ void __launch_bounds__(256, MINW) k_conv_bf16_pipe(ConvTileArgs A) {
  constexpr int CIN = CA + CB, C8 = CIN / 8, PITCH = pitch_c(CIN), K = 9 * CIN, KS = (K + 31) / 32, KPAD = KS * 32;
  constexpr int NU = PT * PT * C8, NJ = (NU + 255) / 256;
  constexpr int WPITCH = wpitch_c(KPAD), WU = NT * 16 * (KPAD / 8);
  constexpr bool F32 = F32A || F32B;
  constexpr int RW = F32 ? 8 : 4;  // 32-bit registers per unit
  extern __shared__ __align__(16) unsigned char s_raw[];
  uint16_t* s_in = reinterpret_cast<uint16_t*>(s_raw);
  uint16_t* s_w = s_in + PT * PT * PITCH;
  for (int u = threadIdx.x; u < WU; u += 256) {
    const int row = u / (KPAD / 8), c8 = u - row * (KPAD / 8);
    *reinterpret_cast<u16x8*>(s_w + row * WPITCH + 8 * c8) =
        *reinterpret_cast<const u16x8*>(A.wp + (int64_t)row * KPAD + 8 * c8);
  }
  const int per_img = A.tiles_x * A.tiles_y, ntiles = A.B * per_img;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int r16 = lane & 15, g = lane >> 4;
  uint32_t pf[NJ][RW];
  auto fetch = [&](int tile) {
    const int b = tile / per_img, t = tile - b * per_img;
    const int iy0 = A.y0 + (t / A.tiles_x) * TT - 1, ix0 = A.x0 + (t % A.tiles_x) * TT - 1;
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
#pragma unroll
      for (int r = 0; r < RW; ++r) pf[j][r] = 0u;
      const int u = threadIdx.x + 256 * j;
      if (u < NU) {
        const int pix = u / C8, ch = u - pix * C8;
        const int py = pix / PT, px = pix - py * PT;
        const int yy = iy0 + py, xx = ix0 + px;
        const bool ina = ch < CA / 8;
        const SrcPart& p = ina ? A.src.a : A.src.b;
        const int cc = ina ? ch * 8 : ch * 8 - CA;
        const bool up = ina && UPA;
        const int sy = up ? (yy >> 1) : yy - p.oy, sx = up ? (xx >> 1) : xx - p.ox;
        if (yy >= 0 && xx >= 0 && yy < A.H && xx < A.W && sy >= 0 && sx >= 0 && sy < p.h && sx < p.w) {
          const int64_t o = (((int64_t)b * p.h + sy) * p.w + sx) * p.stride + p.coff + cc;
          if ((ina && F32A) || (!ina && F32B)) {
            const uint4 f0 = *reinterpret_cast<const uint4*>(p.f32 + o);
            const uint4 f1 = *reinterpret_cast<const uint4*>(p.f32 + o + 4);
            pf[j][0] = f0.x;
            pf[j][1] = f0.y;
            pf[j][2] = f0.z;
            pf[j][3] = f0.w;
            pf[j][RW - 4] = f1.x;
            pf[j][RW - 3] = f1.y;
            pf[j][RW - 2] = f1.z;
            pf[j][RW - 1] = f1.w;
          } else {
            const uint4 v = *reinterpret_cast<const uint4*>(p.bf16 + o);
            pf[j][0] = v.x;
            pf[j][1] = v.y;
            pf[j][2] = v.z;
            pf[j][3] = v.w;
          }
        }
      }
    }
  };
  int tile = xcd_block();
  if (tile >= ntiles) return;
  fetch(tile);
  float bias[NT][4];
  load_bias_t<NT>(A, g, bias);
  const uint16_t* wrow = s_w + r16 * WPITCH + 8 * g;
  const uint16_t* base = s_in + (wave * 4 * PT + r16) * PITCH;
  for (;;) {
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
      const int u = threadIdx.x + 256 * j;
      if (u < NU) {
        const int pix = u / C8, ch = u - pix * C8;
        const bool ina = ch < CA / 8;
        u16x8 v;
        if ((ina && F32A) || (!ina && F32B)) {
#pragma unroll
          for (int r = 0; r < 8; ++r) v[r] = f2bf(__builtin_bit_cast(float, pf[j][r]));
        } else {
          const uint4 q = make_uint4(pf[j][0], pf[j][1], pf[j][2], pf[j][3]);
          v = __builtin_bit_cast(u16x8, q);
        }
        *reinterpret_cast<u16x8*>(s_in + pix * PITCH + ch * 8) = v;
      }
    }
    __syncthreads();
    const int b = tile / per_img, t = tile - b * per_img;
    const int ty0 = (t / A.tiles_x) * TT, tx0 = (t % A.tiles_x) * TT;
    const int next = tile + (int)gridDim.x;
    if (next < ntiles) fetch(next);
    f32x4 acc[4][NT];
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) acc[mt][nt] = f32x4{0.f, 0.f, 0.f, 0.f};
    // The operands of K step ks + 1 are read from LDS before the products of
    // step ks are issued (scheduling barriers keep the two groups apart), so
    // each product waits only for reads issued a step earlier.
    bf16x8 wf[2][NT], pf8[2][4];
    auto operands = [&](int ks, bf16x8 (&w)[NT], bf16x8 (&px)[4]) {
      const int k = ks * 32 + 8 * g;
#pragma unroll
      for (int nt = 0; nt < NT; ++nt)
        w[nt] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const u16x8*>(wrow + nt * 16 * WPITCH + ks * 32));
      const bool kv = k < K;
      const int tap = kv ? k / CIN : 0;
      const int ci = k - tap * CIN;
      const int ky = tap / 3, kx = tap - 3 * ky;
      const uint16_t* pb = base + (ky * PT + kx) * PITCH + ci;
#pragma unroll
      for (int mt = 0; mt < 4; ++mt) {
        u16x8 a = {0, 0, 0, 0, 0, 0, 0, 0};
        if (kv) a = *reinterpret_cast<const u16x8*>(pb + mt * PT * PITCH);
        px[mt] = __builtin_bit_cast(bf16x8, a);
      }
    };
    operands(0, wf[0], pf8[0]);
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      const int cur = ks & 1;
      if (ks + 1 < KS) operands(ks + 1, wf[cur ^ 1], pf8[cur ^ 1]);
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int mt = 0; mt < 4; ++mt)
#pragma unroll
        for (int nt = 0; nt < NT; ++nt)
          acc[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wf[cur][nt], pf8[cur][mt], acc[mt][nt], 0, 0, 0);
      __builtin_amdgcn_sched_barrier(0);
    }
    conv_tile_store_t<NT>(A, acc, bias, b, ty0, tx0, wave, g, r16);
    if (next >= ntiles) break;
    tile = next;
    __syncthreads();  // every wave is done reading the patch before it is overwritten
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

// 8 values per thread: two 16-byte loads, one 16-byte store
__global__ void k_round8_bf16(const float* __restrict__ w, uint16_t* __restrict__ out, int64_t n8) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n8) *reinterpret_cast<u16x8*>(out + 8 * i) = f32x8_to_bf16(w + 8 * i);
}

__global__ void k_round_bf16(const float* __restrict__ w, uint16_t* __restrict__ out, int64_t n) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) out[i] = f2bf(w[i]);
}

// Gradient channels the dgrad of layer l reads: cout, except the head whose
// 4-channel output gradient is stored padded to 8 (one 16-byte load).
__host__ __device__ __forceinline__ int dgrad_cg(int l) { return l == LS_NLAYER - 1 ? 8 : LS_LAYERS[l].cout; }
__host__ __device__ __forceinline__ int dgrad_kpad(int l) { return (9 * dgrad_cg(l) + 31) / 32 * 32; }

// dgrad weights, per layer [ceil16(cin)][Kpad']: row ci, k = tap' * cg + co
// holds W[co][8 - tap'][ci] (the kernel turned by 180 degrees and
// transposed), zero for padding.
__global__ void k_pack_dgrad_bf16(const uint16_t* __restrict__ w, uint16_t* __restrict__ packed) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  int64_t off = 0, woff = 0;
  for (int l = 0; l < LS_NLAYER; ++l) {
    const int cin = LS_LAYERS[l].cin, cout = LS_LAYERS[l].cout, cg = dgrad_cg(l);
    const int Kpad = dgrad_kpad(l), Npad = (cin + 15) / 16 * 16;
    const int64_t n = (int64_t)Npad * Kpad;
    if (i >= off && i < off + n) {
      const int ci = (int)((i - off) / Kpad), k = (int)((i - off) % Kpad);
      uint16_t v = 0;
      if (ci < cin && k < 9 * cg) {
        const int tf = k / cg, co = k - tf * cg;
        if (co < cout) v = w[woff + ((int64_t)co * 9 + (8 - tf)) * cin + ci];
      }
      packed[i] = v;
      return;
    }
    off += n;
    woff += (int64_t)cout * 9 * cin + cout;
  }
}

// out = BF16(g where the forward activation is positive, else 0)
__global__ void k_mask_round_bf16(const float* __restrict__ g, const uint16_t* __restrict__ act,
                                  uint16_t* __restrict__ out, int64_t n) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) out[i] = f2bf(bf2f(act[i]) > 0.f ? g[i] : 0.f);
}

// out[p][c] = BF16(g where act[p][c] > 0, else 0) for C channels per
// pixel, 8 per thread, with g = src[p][coff + c] of a `stride`-channel
// tensor, plus (low given) the 2x2 average-pool adjoint 0.25 * low[p / 2][c]
// of a half-resolution gradient: the channel split, the pool adjoint and the
// masking of the backward in one pass.
__global__ void k_mask_round_ex(const float* __restrict__ src, int stride, int coff, const uint16_t* __restrict__ act,
                                const float* __restrict__ low, int B, int H, int W, int C, int sy0, int sn,
                                uint16_t* __restrict__ out) {
  const int c8n = C / 8;
  const int64_t n = (int64_t)B * H * W * c8n;
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int c0 = 8 * (int)(i % c8n);
  const int64_t p = i / c8n;
  const int x = (int)(p % W);
  const int64_t r = p / W;
  const int y = (int)(r % H);
  const int b = (int)(r / H);
  float g[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  // src: the whole plane (sn = 0) or the window [sy0, sy0 + sn)^2, zero outside
  const int wy = y - sy0, wx = x - sy0;
  if (sn == 0 || (wy >= 0 && wx >= 0 && wy < sn && wx < sn)) {
    const int64_t si = sn == 0 ? p : ((int64_t)b * sn + wy) * sn + wx;
    const float* sp = src + si * stride + coff + c0;
    const float4 a0 = *reinterpret_cast<const float4*>(sp), a1 = *reinterpret_cast<const float4*>(sp + 4);
    g[0] = a0.x;
    g[1] = a0.y;
    g[2] = a0.z;
    g[3] = a0.w;
    g[4] = a1.x;
    g[5] = a1.y;
    g[6] = a1.z;
    g[7] = a1.w;
  }
  if (low) {
    const float* lp = low + (((int64_t)b * (H / 2) + y / 2) * (W / 2) + x / 2) * C + c0;
    const float4 l0 = *reinterpret_cast<const float4*>(lp), l1 = *reinterpret_cast<const float4*>(lp + 4);
    const float lv[8] = {l0.x, l0.y, l0.z, l0.w, l1.x, l1.y, l1.z, l1.w};
#pragma unroll
    for (int k = 0; k < 8; ++k) g[k] += 0.25f * lv[k];
  }
  const u16x8 av = *reinterpret_cast<const u16x8*>(act + p * C + c0);
  u16x8 o;
#pragma unroll
  for (int k = 0; k < 8; ++k) o[k] = f2bf(bf2f(av[k]) > 0.f ? g[k] : 0.f);
  *reinterpret_cast<u16x8*>(out + p * C + c0) = o;
}

// [npix][4] FP32 -> [npix][8] BF16 with channels 4..7 zero
// one pixel per thread: its 4 FP32 channels in, 8 BF16 channels (the last 4
// zero) out as one 16-byte store
__global__ void k_embed8_bf16(const float* __restrict__ g, uint16_t* __restrict__ out, int64_t npix) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= npix) return;
  const float4 v = *reinterpret_cast<const float4*>(g + 4 * i);
  uint4 o;
  o.x = (uint32_t)f2bf(v.x) | ((uint32_t)f2bf(v.y) << 16);
  o.y = (uint32_t)f2bf(v.z) | ((uint32_t)f2bf(v.w) << 16);
  o.z = 0u;
  o.w = 0u;
  *reinterpret_cast<uint4*>(out + 8 * i) = o;
}

// the same, one output element per thread (any alignment)
__global__ void k_embed8_bf16_s(const float* __restrict__ g, uint16_t* __restrict__ out, int64_t npix) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= npix * 8) return;
  const int c = (int)(i & 7);
  out[i] = c < 4 ? f2bf(g[(i >> 3) * 4 + c]) : (uint16_t)0;
}

}  // namespace

size_t ls_bf16_dpacked_offset(int l) {
  size_t off = 0;
  for (int k = 0; k < l; ++k) off += (size_t)((LS_LAYERS[k].cin + 15) / 16 * 16) * dgrad_kpad(k);
  return off;
}

size_t ls_bf16_dpacked_total() { return ls_bf16_dpacked_offset(LS_NLAYER); }

int ls_bf16_prep_dgrad_weights(const uint16_t* w_bf16, uint16_t* packed, hipStream_t st) {
  const int64_t n = (int64_t)ls_bf16_dpacked_total();
  hipLaunchKernelGGL(k_pack_dgrad_bf16, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, w_bf16, packed);
  LS_LAUNCH_CHECK();
  return LS_OK;
}

int ls_bf16_mask_round(const float* g, const uint16_t* act, uint16_t* out, int64_t n, hipStream_t st) {
  LS_TRACE("mask_round", st);
  hipLaunchKernelGGL(k_mask_round_bf16, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, g, act, out, n);
  LS_LAUNCH_CHECK();
  return LS_OK;
}

int ls_bf16_mask_round_ex(const float* src, int stride, int coff, const uint16_t* act, const float* low, int B,
                          int H, int C, uint16_t* out, hipStream_t st, int sy0, int sn) {
  if (C % 8 || stride % 4 || coff % 4) return LS_ENOTIMPL;
  LS_TRACE("mask_round", st);
  const int64_t n = (int64_t)B * H * H * (C / 8);
  if (sn < 0 || sy0 < 0 || sy0 + sn > H) return LS_EINVAL;
  hipLaunchKernelGGL(k_mask_round_ex, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, src, stride, coff, act, low,
                     B, H, H, C, sy0, sn, out);
  LS_LAUNCH_CHECK();
  return LS_OK;
}

int ls_bf16_embed8(const float* g, uint16_t* out, int64_t npix, hipStream_t st) {
  LS_TRACE("embed8", st);
  if (reinterpret_cast<uintptr_t>(g) % 16 || reinterpret_cast<uintptr_t>(out) % 16)
    hipLaunchKernelGGL(k_embed8_bf16_s, dim3((unsigned)((npix * 8 + 255) / 256)), dim3(256), 0, st, g, out, npix);
  else
    hipLaunchKernelGGL(k_embed8_bf16, dim3((unsigned)((npix + 255) / 256)), dim3(256), 0, st, g, out, npix);
  LS_LAUNCH_CHECK();
  return LS_OK;
}

// Input gradient of layer l over the whole H x H plane: the conv of the
// (masked, BF16) output gradient `s` with the turned weights, FP32 result
// [B][H][H][cin].
int ls_bf16_dgrad(const ConvSrc& s, int B, int H, int l, const uint16_t* dpacked, float* out, const uint16_t* mask,
                  uint16_t* out_masked, hipStream_t st) {
  const int cin = LS_LAYERS[l].cin;
  if (s.a.c + s.b.c != dgrad_cg(l)) return LS_EINVAL;
  // config 0 / 1: direct operand fetch with 4 / 2 pixel tiles per wave;
  // 2 and the default: the persistent LDS-tiled form
  const int cfg = ls_conv_config_get(l, LS_BF16, 1);
  if (cfg < 0 || cfg == 2) {
    ConvTileArgs a;
    a.src = s;
    a.B = B;
    a.H = H;
    a.W = H;
    a.y0 = 0;
    a.x0 = 0;
    a.Ho = H;
    a.Wo = H;
    a.tiles_x = (H + TT - 1) / TT;
    a.tiles_y = (H + TT - 1) / TT;
    a.wp = dpacked + ls_bf16_dpacked_offset(l);
    a.Kpad = dgrad_kpad(l);
    a.bias = nullptr;
    a.cout = cin;
    a.relu = 0;
    a.out_bf16 = mask ? out_masked : nullptr;
    a.out_f32 = mask ? nullptr : out;
    a.out_stride = cin;
    a.out_coff = 0;
    a.pool_out = nullptr;
    a.pool_stride = 0;
    a.pool_coff = 0;
    a.mask = mask;
    const int rc = ls_bf16_conv_pipe(a, (cin + 15) / 16, s.a.c, s.b.c, s.a.up != 0, s.a.f32 != nullptr,
                                     s.b.c > 0 && s.b.f32 != nullptr, st, "dgrad_bf16");
    if (rc != LS_ENOTIMPL) return rc;
  }
  ConvArgsB a;
  a.src = s;
  a.B = B;
  a.H = H;
  a.W = H;
  a.y0 = 0;
  a.x0 = 0;
  a.Ho = H;
  a.Wo = H;
  a.wp = dpacked + ls_bf16_dpacked_offset(l);
  a.Kpad = dgrad_kpad(l);
  a.bias = nullptr;
  a.cout = cin;
  a.relu = 0;
  // FP32 input gradient, or (mask given) the BF16 operand of the next layer
  // down: the gradient zeroed where that layer's activation is not positive
  a.out_bf16 = mask ? out_masked : nullptr;
  a.out_f32 = mask ? nullptr : out;
  a.out_stride = cin;
  a.mask = mask;
  LS_TRACE("dgrad_bf16", st);
  const int mt = cfg == 1 ? 2 : 4;
  return launch_direct(a, (cin + 15) / 16, mt, (int64_t)B * H * H, st);
}

int ls_bf16_dgrad_split(const ConvSrc& s, int B, int H, int l, const uint16_t* dpacked, float* out, float* up_out,
                        int up_c, const uint16_t* mask, uint16_t* out_masked, int split, hipStream_t st, int y0,
                        int n) {
  const int cin = LS_LAYERS[l].cin;
  if (s.a.c + s.b.c != dgrad_cg(l)) return LS_EINVAL;
  if (n == 0) {
    y0 = 0;
    n = H;
  }
  if (y0 < 0 || n < 0 || y0 + n > H) return LS_EINVAL;
  const int cfg = ls_conv_config_get(l, LS_BF16, 1);
  if (!(cfg < 0 || cfg == 2)) return LS_ENOTIMPL;
  // whole 16-channel tiles on each side of the split; even windows for the
  // 2 x 2 sums; the masked split only on the whole plane
  if (up_c > 0 ? (up_c % 16 || up_c >= cin || y0 % 2 || n % 2)
               : (split <= 0 || split % 16 || split >= cin || !mask || n != H))
    return LS_ENOTIMPL;
  ConvTileArgs a;
  a.src = s;
  a.B = B;
  a.H = H;
  a.W = H;
  a.y0 = y0;
  a.x0 = y0;
  a.Ho = n;
  a.Wo = n;
  a.tiles_x = (n + TT - 1) / TT;
  a.tiles_y = (n + TT - 1) / TT;
  a.wp = dpacked + ls_bf16_dpacked_offset(l);
  a.Kpad = dgrad_kpad(l);
  a.bias = nullptr;
  a.cout = cin;
  a.relu = 0;
  a.pool_out = nullptr;
  a.pool_stride = 0;
  a.pool_coff = 0;
  if (up_c > 0) {
    // channels from up_c on: FP32, cin - up_c per pixel
    a.out_bf16 = nullptr;
    a.out_f32 = out;
    a.out_stride = cin - up_c;
    a.out_coff = -up_c;
    a.mask = nullptr;
    a.up_out = up_out;
    a.up_c = up_c;
  } else {
    // channels below split: masked BF16, split per pixel; the others FP32,
    // or not computed at all when out is null
    a.out_bf16 = out_masked;
    a.out_f32 = nullptr;
    a.out_stride = split;
    a.out_coff = 0;
    a.mask = mask;
    a.split = split;
    a.out2_f32 = out;
    if (!out) a.cout = split;
  }
  return ls_bf16_conv_pipe(a, (a.cout + 15) / 16, s.a.c, s.b.c, s.a.up != 0, s.a.f32 != nullptr,
                           s.b.c > 0 && s.b.f32 != nullptr, st, "dgrad_bf16");
}

int ls_bf16_dgrad_win(const ConvSrc& s, int B, int H, int l, const uint16_t* dpacked, int y0, int x0, int n,
                      const uint16_t* mask, int mask_n, int mask_o, uint16_t* out_masked, int split, float* out2,
                      hipStream_t st) {
  const int cin = LS_LAYERS[l].cin;
  if (s.a.c + s.b.c != dgrad_cg(l)) return LS_EINVAL;
  if (y0 < 0 || x0 < 0 || n <= 0 || y0 + n > H || x0 + n > H || !mask || !out_masked) return LS_EINVAL;
  if (y0 < mask_o || x0 < mask_o || y0 + n > mask_o + mask_n || x0 + n > mask_o + mask_n) return LS_EINVAL;
  const int cfg = ls_conv_config_get(l, LS_BF16, 1);
  if (!(cfg < 0 || cfg == 2) || split <= 0 || split % 16 || split > cin || (out2 && split == cin)) return LS_ENOTIMPL;
  ConvTileArgs a;
  a.src = s;
  a.B = B;
  a.H = H;
  a.W = H;
  a.y0 = y0;
  a.x0 = x0;
  a.Ho = n;
  a.Wo = n;
  a.tiles_x = (n + TT - 1) / TT;
  a.tiles_y = (n + TT - 1) / TT;
  a.wp = dpacked + ls_bf16_dpacked_offset(l);
  a.Kpad = dgrad_kpad(l);
  a.bias = nullptr;
  a.cout = out2 ? cin : split;
  a.relu = 0;
  a.out_bf16 = out_masked;
  a.out_f32 = nullptr;
  a.out_stride = split;
  a.out_coff = 0;
  a.pool_out = nullptr;
  a.pool_stride = 0;
  a.pool_coff = 0;
  a.mask = mask;
  a.mask_h = mask_n;
  a.mask_w = mask_n;
  a.mask_y0 = y0 - mask_o;
  a.mask_x0 = x0 - mask_o;
  if (out2) {
    a.split = split;
    a.out2_f32 = out2;
  }
  return ls_bf16_conv_pipe(a, (a.cout + 15) / 16, s.a.c, s.b.c, s.a.up != 0, s.a.f32 != nullptr,
                           s.b.c > 0 && s.b.f32 != nullptr, st, "dgrad_bf16");
}

bool ls_bf16_lvl1_windowed() {
  auto pipe = [](int l) {
    const int c = ls_conv_config_get(l, LS_BF16, 1);
    return c < 0 || c == 2;
  };
  return pipe(LS_NLAYER - 1) && pipe(LS_NLAYER - 2);
}

int ls_bf16_kpad(int l) { return (9 * LS_LAYERS[l].cin + 31) / 32 * 32; }

size_t ls_bf16_packed_offset(int l) {
  size_t off = 0;
  for (int k = 0; k < l; ++k) off += (size_t)((LS_LAYERS[k].cout + 15) / 16 * 16) * ls_bf16_kpad(k);
  return off;
}

size_t ls_bf16_packed_total() { return ls_bf16_packed_offset(LS_NLAYER); }

int ls_pack_bf16(const float* w, uint16_t* out, int64_t n, hipStream_t st) {
  if (n % 8 == 0 && (reinterpret_cast<uintptr_t>(w) % 16) == 0 && (reinterpret_cast<uintptr_t>(out) % 16) == 0) {
    const int64_t n8 = n / 8;
    hipLaunchKernelGGL(k_round8_bf16, dim3((unsigned)((n8 + 255) / 256)), dim3(256), 0, st, w, out, n8);
  } else {
    hipLaunchKernelGGL(k_round_bf16, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, w, out, n);
  }
  LS_LAUNCH_CHECK();
  return LS_OK;
}

int ls_bf16_prep_weights(const uint16_t* w_bf16, uint16_t* packed, hipStream_t st) {
  const int64_t n = (int64_t)ls_bf16_packed_total();
  LS_TRACE("pack_bf16", st);
  hipLaunchKernelGGL(k_pack_weights_bf16, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, w_bf16, packed);
  LS_LAUNCH_CHECK();
  return LS_OK;
}

namespace {

// Direct kernel over npix output pixels: nt channel tiles, mt pixel tiles per wave.
int launch_direct(const ConvArgsB& a, int nt, int mt, int64_t npix, hipStream_t st) {
  const int64_t per_block = 16 * mt * WAVES;
  dim3 grid((unsigned)((npix + per_block - 1) / per_block));
#define LS_DIRECT(N, M) hipLaunchKernelGGL((k_conv_bf16<N, M>), grid, dim3(64 * WAVES), 0, st, a)
  if (mt == 2) {
    switch (nt) {
      case 1: LS_DIRECT(1, 2); break;
      case 2: LS_DIRECT(2, 2); break;
      case 3: LS_DIRECT(3, 2); break;
      case 4: LS_DIRECT(4, 2); break;
      case 6: LS_DIRECT(6, 2); break;
      default: return LS_ENOTIMPL;
    }
  } else {
    switch (nt) {
      case 1: LS_DIRECT(1, 4); break;
      case 2: LS_DIRECT(2, 4); break;
      case 3: LS_DIRECT(3, 4); break;
      case 4: LS_DIRECT(4, 4); break;
      case 6: LS_DIRECT(6, 4); break;
      default: return LS_ENOTIMPL;
    }
  }
#undef LS_DIRECT
  LS_LAUNCH_CHECK();
  return LS_OK;
}

int conv_bf16(const ConvSrc& s, int B, int H, int l, const uint16_t* packed, const float* w, uint16_t* out_bf16,
              float* out_f32, int relu, int y0, int x0, int Ho, int Wo, int mt, hipStream_t st) {
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
  a.mask = nullptr;
  const int nt = (a.cout + 15) / 16;
  LS_TRACE("conv_bf16", st);
  return launch_direct(a, nt, mt, (int64_t)B * Ho * Wo, st);
}

int conv_bf16_lds(const ConvSrc& s, int B, int H, int l, const uint16_t* packed, const float* w, uint16_t* out_bf16,
                  float* out_f32, uint16_t* pool_out, int relu, int y0, int x0, int Ho, int Wo, bool pipe,
                  hipStream_t st) {
  ConvTileArgs a;
  a.src = s;
  a.B = B;
  a.H = H;
  a.W = H;
  a.y0 = y0;
  a.x0 = x0;
  a.Ho = Ho;
  a.Wo = Wo;
  a.tiles_x = (Wo + TT - 1) / TT;
  a.tiles_y = (Ho + TT - 1) / TT;
  a.wp = packed + ls_bf16_packed_offset(l);
  a.Kpad = ls_bf16_kpad(l);
  a.bias = w + ls_layer_b_offset(l);
  a.cout = LS_LAYERS[l].cout;
  a.relu = relu;
  a.out_bf16 = out_bf16;
  a.out_f32 = out_f32;
  a.pool_out = pool_out;
  a.out_stride = a.cout;
  a.out_coff = 0;
  a.pool_stride = a.cout;
  a.pool_coff = 0;
  a.mask = nullptr;
  if (pool_out && (Ho % TT || Wo % TT)) return LS_ENOTIMPL;
  const int cin = s.a.c + s.b.c;
  const size_t patch = (size_t)PT * PT * patch_pitch(cin) * 2;
  const size_t otile = (size_t)TT * TT * a.cout * (out_f32 ? 4 : 2);
  const size_t lds = patch > otile ? patch : otile;
  const dim3 grid((unsigned)(B * a.tiles_x * a.tiles_y));
  const int nt = (a.cout + 15) / 16;
  LS_TRACE("conv_bf16", st);
  // the layer's own specialisation when the sources are the network's
  auto is = [&](int ca, int cb, bool upa, bool f32a, bool f32b) {
    return s.a.c == ca && s.b.c == cb && (s.a.up != 0) == upa && (s.a.f32 != nullptr) == f32a &&
           (cb == 0 || ((s.b.f32 != nullptr) == f32b && !s.b.up));
  };
  // persistent pipelined form: as many workgroups as fit on the device at once
#define LS_PIPE(L, N, CA, CB, UPA, F32A, F32B, W)                                                        \
  if (pipe && l == L && nt == N && is(CA, CB, UPA, F32A, F32B)) {                                        \
    auto* fn = &k_conv_bf16_pipe<N, CA, CB, UPA, F32A, F32B, W>;                                         \
    constexpr size_t plds = pipe_lds_bytes(N, CA + CB);                                                  \
    static_assert(plds <= LDS_MAX, "pipelined tile exceeds LDS");                                       \
    if (plds > 65536)                                                                                    \
      LS_HOST_CHECK(hipFuncSetAttribute(reinterpret_cast<const void*>(fn),                               \
                                        hipFuncAttributeMaxDynamicSharedMemorySize, (int)plds));         \
    int per_cu = 0, dev = 0, cus = 0;                                                                    \
    LS_HOST_CHECK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, 256, plds));                \
    LS_HOST_CHECK(hipGetDevice(&dev));                                                                   \
    LS_HOST_CHECK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));             \
    const int64_t want = (int64_t)std::max(per_cu, 1) * std::max(cus, 1);                                \
    const dim3 pgrid((unsigned)std::min<int64_t>(want, (int64_t)grid.x));                               \
    hipLaunchKernelGGL((k_conv_bf16_pipe<N, CA, CB, UPA, F32A, F32B, W>), pgrid, dim3(256), plds, st, a); \
    LS_LAUNCH_CHECK();                                                                                   \
    return LS_OK;                                                                                        \
  }
  LS_PIPE(0, 1, 8, 0, false, true, false, 1)
  LS_PIPE(1, 1, 16, 0, false, false, false, 2)
  LS_PIPE(2, 2, 16, 0, false, false, false, 2)
  LS_PIPE(3, 2, 32, 0, false, false, false, 2)
  LS_PIPE(4, 4, 32, 0, false, false, false, 2)
  LS_PIPE(5, 4, 64, 0, false, false, false, 1)
  LS_PIPE(6, 2, 64, 32, true, false, false, 1)
  LS_PIPE(7, 2, 32, 0, false, false, false, 2)
  LS_PIPE(8, 1, 32, 16, true, false, false, 2)
  LS_PIPE(9, 1, 16, 0, false, false, false, 2)
  LS_PIPE(10, 1, 16, 8, false, false, true, 2)
#undef LS_PIPE
#define LS_SPEC(L, N, CA, CB, UPA, F32A, F32B)                                                          \
  if (l == L && nt == N && is(CA, CB, UPA, F32A, F32B)) {                                            \
    if (patch > 65536)                                                                               \
      LS_HOST_CHECK(hipFuncSetAttribute(                                                             \
          reinterpret_cast<const void*>(&k_conv_bf16_lds_t<N, CA, CB, UPA, F32A, F32B>),             \
          hipFuncAttributeMaxDynamicSharedMemorySize, (int)patch));                                  \
    hipLaunchKernelGGL((k_conv_bf16_lds_t<N, CA, CB, UPA, F32A, F32B>), grid, dim3(256), patch, st, a); \
    LS_LAUNCH_CHECK();                                                                               \
    return LS_OK;                                                                                    \
  }
  LS_SPEC(0, 1, 8, 0, false, true, false)
  LS_SPEC(1, 1, 16, 0, false, false, false)
  LS_SPEC(2, 2, 16, 0, false, false, false)
  LS_SPEC(3, 2, 32, 0, false, false, false)
  LS_SPEC(4, 4, 32, 0, false, false, false)
  LS_SPEC(5, 4, 64, 0, false, false, false)
  LS_SPEC(6, 2, 64, 32, true, false, false)
  LS_SPEC(7, 2, 32, 0, false, false, false)
  LS_SPEC(8, 1, 32, 16, true, false, false)
  LS_SPEC(9, 1, 16, 0, false, false, false)
  LS_SPEC(10, 1, 16, 8, false, false, true)
#undef LS_SPEC
  auto generic = [&](const void* f) -> int {
    if (lds > 65536) LS_HOST_CHECK(hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    return LS_OK;
  };
  switch (nt) {
    case 1:
      if (generic(reinterpret_cast<const void*>(&k_conv_bf16_lds<1>)) != LS_OK) return LS_EHIP;
      hipLaunchKernelGGL(k_conv_bf16_lds<1>, grid, dim3(256), lds, st, a);
      break;
    case 2:
      if (generic(reinterpret_cast<const void*>(&k_conv_bf16_lds<2>)) != LS_OK) return LS_EHIP;
      hipLaunchKernelGGL(k_conv_bf16_lds<2>, grid, dim3(256), lds, st, a);
      break;
    case 4:
      if (generic(reinterpret_cast<const void*>(&k_conv_bf16_lds<4>)) != LS_OK) return LS_EHIP;
      hipLaunchKernelGGL(k_conv_bf16_lds<4>, grid, dim3(256), lds, st, a);
      break;
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

// Two 3x3 convs in one pass, for inference: layer l1 (CIN1 input channels,
// 16 outputs, ReLU) on a 16 x 16 region, kept in LDS as BF16, then layer l2
// on it (with CB2 more channels of a second part staged beside it) for the
// 14 x 14 outputs whose 3 x 3 windows the region covers.  l1's activation
// never goes to HBM, which is what bounds these full-resolution 16-channel
// layers; the region's halo costs 31 % more matrix work.  l1's outputs
// outside the plane are zero (l2's zero padding), so both layers compute
// exactly what the separate launches compute: same MFMA sequences, same
// rounding points, identical bits.
constexpr int FT = TT - 2;  // fused output tile side

struct Conv2Args {
  SrcPart a1;  // l1's input (CIN1 channels)
  SrcPart b2;  // l2's second part (CB2 channels), if any
  int B, H, W;
  int y0, x0, Ho, Wo;  // l2's output window in the plane
  int tiles_x, tiles_y;
  const uint16_t* wp1;  // packed l1 weights [16][KPAD1]
  const float* bias1;
  const uint16_t* wp2;  // packed l2 weights [16 * NT2][KPAD2]
  const float* bias2;
  int cout2, relu2;
  uint16_t* out_bf16;  // l2 output [B][Ho][Wo][cout2], or null
  float* out_f32;      // same layout, or null
  uint16_t* pool_out;  // 2 x 2 average pool of the BF16 output [B][Ho/2][Wo/2][cout2], or null
  // out_bf16 is stored only on [st0, st1)^2 of the output window (the rest
  // is never read; the pool still sees every pixel)
  int st0 = 0, st1 = 1 << 30;
};

// Products of one 16 x 16 output tile from a staged 18 x 18 patch (pitch
// PITCH, CIN channels) with weights staged in LDS (rows of WPITCH): the K
// order and accumulation of k_conv_bf16_lds_t.
template <int NT, int CIN, int WPITCH>
__device__ __forceinline__ void patch_mfma(const uint16_t* s_w, const uint16_t* s_patch, int wave, int g, int r16,
                                           f32x4 (&acc)[4][NT]) {
  constexpr int PITCH = pitch_c(CIN), K = 9 * CIN, KS = (K + 31) / 32;
#pragma unroll
  for (int mt = 0; mt < 4; ++mt)
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) acc[mt][nt] = f32x4{0.f, 0.f, 0.f, 0.f};
  const uint16_t* wrow = s_w + r16 * WPITCH + 8 * g;
  const uint16_t* base = s_patch + (wave * 4 * PT + r16) * PITCH;
#pragma unroll
  for (int ks = 0; ks < KS; ++ks) {
    const int k = ks * 32 + 8 * g;
    bf16x8 bfr[NT];
#pragma unroll
    for (int nt = 0; nt < NT; ++nt)
      bfr[nt] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const u16x8*>(wrow + nt * 16 * WPITCH + ks * 32));
    const bool kv = k < K;
    const int tap = kv ? k / CIN : 0;
    const int ci = k - tap * CIN;
    const int ky = tap / 3, kx = tap - 3 * ky;
    const uint16_t* pb = base + (ky * PT + kx) * PITCH + ci;
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) {
      u16x8 a = {0, 0, 0, 0, 0, 0, 0, 0};
      if (kv) a = *reinterpret_cast<const u16x8*>(pb + mt * PT * PITCH);
      const bf16x8 ab = __builtin_bit_cast(bf16x8, a);
#pragma unroll
      for (int nt = 0; nt < NT; ++nt)
        acc[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bfr[nt], ab, acc[mt][nt], 0, 0, 0);
    }
  }
}

// Persistent like k_conv_bf16_pipe: both layers' packed weights are copied
// into LDS once per workgroup, which then walks the tiles tile, tile +
// gridDim.x, ...; the next tile's input units (16 bytes each, 32 for an FP32
// part, rounded to BF16 when written to LDS) are loaded into registers while
// the current tile is multiplied.
template <int CIN1, bool F32A, int CB2, bool F32B, int NT2, int MINW>
__global__ void __launch_bounds__(256, MINW) k_conv2_bf16(Conv2Args A) {
  constexpr int P1 = pitch_c(CIN1), CIN2 = 16 + CB2, P2 = pitch_c(CIN2);
  constexpr int KPAD1 = (9 * CIN1 + 31) / 32 * 32, KPAD2 = (9 * CIN2 + 31) / 32 * 32;
  constexpr int WP1 = wpitch_c(KPAD1), WP2 = wpitch_c(KPAD2);
  constexpr int NU1 = PT * PT * (CIN1 / 8), NJ1 = (NU1 + 255) / 256, RW1 = F32A ? 8 : 4;
  constexpr int C82 = CB2 > 0 ? CB2 / 8 : 1;  // 8-channel units per pixel of the second part
  constexpr int NU2 = PT * PT * (CB2 / 8), NJ2 = CB2 > 0 ? (NU2 + 255) / 256 : 0, RW2 = F32B ? 8 : 4;
  __shared__ __align__(16) uint16_t s1[PT * PT * P1];
  __shared__ __align__(16) uint16_t s2[PT * PT * P2];
  __shared__ __align__(16) uint16_t w1[16 * WP1];
  __shared__ __align__(16) uint16_t w2[NT2 * 16 * WP2];
  for (int u = threadIdx.x; u < 16 * (KPAD1 / 8); u += 256) {
    const int row = u / (KPAD1 / 8), c8 = u - row * (KPAD1 / 8);
    *reinterpret_cast<u16x8*>(w1 + row * WP1 + 8 * c8) = *reinterpret_cast<const u16x8*>(A.wp1 + (int64_t)row * KPAD1 + 8 * c8);
  }
  for (int u = threadIdx.x; u < NT2 * 16 * (KPAD2 / 8); u += 256) {
    const int row = u / (KPAD2 / 8), c8 = u - row * (KPAD2 / 8);
    *reinterpret_cast<u16x8*>(w2 + row * WP2 + 8 * c8) = *reinterpret_cast<const u16x8*>(A.wp2 + (int64_t)row * KPAD2 + 8 * c8);
  }
  // l1 padding of l2's patch (rows and columns 16, 17): zero for good
  for (int pix = threadIdx.x; pix < PT * PT; pix += 256) {
    const int py = pix / PT, px = pix - py * PT;
    if (py >= TT || px >= TT) {
      const u16x8 z = {0, 0, 0, 0, 0, 0, 0, 0};
      *reinterpret_cast<u16x8*>(s2 + pix * P2) = z;
      *reinterpret_cast<u16x8*>(s2 + pix * P2 + 8) = z;
    }
  }
  const int per_img = A.tiles_x * A.tiles_y, ntiles = A.B * per_img;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int r16 = lane & 15, g = lane >> 4;
  uint32_t pf1[NJ1][RW1];
  uint32_t pf2[NJ2 > 0 ? NJ2 : 1][RW2];
  // the input units of a tile: l1's patch at (oy0 - 2, ox0 - 2), l2's second
  // part at (oy0 - 1, ox0 - 1)
  auto fetch_part = [&](const SrcPart& p, int b, int py0, int px0, int u, int C8, bool f32, uint32_t* r) {
    const int pix = u / C8, ch = u - pix * C8;
    const int py = pix / PT, px = pix - py * PT;
    const int yy = py0 + py, xx = px0 + px;
    const int sy = yy - p.oy, sx = xx - p.ox;
    if (yy >= 0 && xx >= 0 && yy < A.H && xx < A.W && sy >= 0 && sx >= 0 && sy < p.h && sx < p.w) {
      const int64_t o = (((int64_t)b * p.h + sy) * p.w + sx) * p.stride + p.coff + 8 * ch;
      if (f32) {
        const uint4 f0 = *reinterpret_cast<const uint4*>(p.f32 + o);
        const uint4 f1 = *reinterpret_cast<const uint4*>(p.f32 + o + 4);
        r[0] = f0.x;
        r[1] = f0.y;
        r[2] = f0.z;
        r[3] = f0.w;
        r[4] = f1.x;
        r[5] = f1.y;
        r[6] = f1.z;
        r[7] = f1.w;
      } else {
        const uint4 v = *reinterpret_cast<const uint4*>(p.bf16 + o);
        r[0] = v.x;
        r[1] = v.y;
        r[2] = v.z;
        r[3] = v.w;
      }
    }
  };
  auto fetch = [&](int tile) {
    const int b = tile / per_img, t = tile - b * per_img;
    const int oy0 = A.y0 + (t / A.tiles_x) * FT, ox0 = A.x0 + (t % A.tiles_x) * FT;
#pragma unroll
    for (int j = 0; j < NJ1; ++j) {
#pragma unroll
      for (int r = 0; r < RW1; ++r) pf1[j][r] = 0u;
      const int u = threadIdx.x + 256 * j;
      if (u < NU1) fetch_part(A.a1, b, oy0 - 2, ox0 - 2, u, CIN1 / 8, F32A, pf1[j]);
    }
#pragma unroll
    for (int j = 0; j < NJ2; ++j) {
#pragma unroll
      for (int r = 0; r < RW2; ++r) pf2[j][r] = 0u;
      const int u = threadIdx.x + 256 * j;
      if (u < NU2) fetch_part(A.b2, b, oy0 - 1, ox0 - 1, u, C82, F32B, pf2[j]);
    }
  };
  auto to_lds = [&](const uint32_t* r, bool f32, uint16_t* dst) {
    u16x8 v;
    if (f32) {
#pragma unroll
      for (int k = 0; k < 8; ++k) v[k] = f2bf(__builtin_bit_cast(float, r[k]));
    } else {
      v = __builtin_bit_cast(u16x8, make_uint4(r[0], r[1], r[2], r[3]));
    }
    *reinterpret_cast<u16x8*>(dst) = v;
  };
  int tile = xcd_block();
  if (tile >= ntiles) return;
  const int cout = A.cout2;
  float bias1[4], bias2[NT2][4];
#pragma unroll
  for (int r = 0; r < 4; ++r) bias1[r] = A.bias1[4 * g + r];
#pragma unroll
  for (int nt = 0; nt < NT2; ++nt)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int c = nt * 16 + 4 * g + r;
      bias2[nt][r] = c < cout ? A.bias2[c] : 0.f;
    }
  // the biases and weights have landed before any tile's loads are in
  // flight, so no wait for them inside the loop also waits for a prefetch
  __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0)
  fetch(tile);
  for (;;) {
#pragma unroll
    for (int j = 0; j < NJ1; ++j) {
      const int u = threadIdx.x + 256 * j;
      if (u < NU1) {
        const int pix = u / (CIN1 / 8), ch = u - pix * (CIN1 / 8);
        to_lds(pf1[j], F32A, s1 + pix * P1 + 8 * ch);
      }
    }
#pragma unroll
    for (int j = 0; j < NJ2; ++j) {
      const int u = threadIdx.x + 256 * j;
      if (u < NU2) {
        const int pix = u / C82, ch = u - pix * C82;
        to_lds(pf2[j], F32B, s2 + pix * P2 + 16 + 8 * ch);
      }
    }
    __syncthreads();
    const int b = tile / per_img, t = tile - b * per_img;
    const int ry0 = (t / A.tiles_x) * FT, rx0 = (t % A.tiles_x) * FT;  // tile origin in the output window
    const int oy0 = A.y0 + ry0, ox0 = A.x0 + rx0;                      // ... in the plane
    const int next = tile + (int)gridDim.x;
    if (next < ntiles) fetch(next);
    {
      f32x4 acc[4][1];
      patch_mfma<1, CIN1, WP1>(w1, s1, wave, g, r16, acc);
#pragma unroll
      for (int mt = 0; mt < 4; ++mt) {
        const int row = wave * 4 + mt, col = r16;
        const int yy = oy0 - 1 + row, xx = ox0 - 1 + col;
        const bool in = yy >= 0 && xx >= 0 && yy < A.H && xx < A.W;
        unsigned short h[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) h[r] = in ? f2bf(fmaxf(acc[mt][0][r] + bias1[r], 0.f)) : (unsigned short)0;
        uint2 u;
        u.x = (uint32_t)h[0] | ((uint32_t)h[1] << 16);
        u.y = (uint32_t)h[2] | ((uint32_t)h[3] << 16);
        *reinterpret_cast<uint2*>(s2 + (row * PT + col) * P2 + 4 * g) = u;
      }
    }
    __syncthreads();
    f32x4 acc[4][NT2];
    patch_mfma<NT2, CIN2, WP2>(w2, s2, wave, g, r16, acc);
    // l2's epilogue: rows and columns below FT and inside the window
    const int r0 = wave * 4, c = r16;
    const int oyr = ry0 + r0, oxr = rx0 + c;  // window coordinates of row mt = 0
#pragma unroll
    for (int nt = 0; nt < NT2; ++nt) {
      const int c0 = nt * 16 + 4 * g;
      if (c0 >= cout) continue;
      float q[4][4];
#pragma unroll
      for (int mt = 0; mt < 4; ++mt)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          float v = acc[mt][nt][r] + bias2[nt][r];
          if (A.relu2) v = fmaxf(v, 0.f);
          q[mt][r] = v;
        }
      auto ok = [&](int mt) { return r0 + mt < FT && c < FT && oyr + mt < A.Ho && oxr < A.Wo; };
      const int64_t off0 = (((int64_t)b * A.Ho + oyr) * A.Wo + oxr) * cout + c0, row = (int64_t)A.Wo * cout;
      if (A.out_f32) {
#pragma unroll
        for (int mt = 0; mt < 4; ++mt)
          if (ok(mt))
            *reinterpret_cast<float4*>(A.out_f32 + off0 + mt * row) = make_float4(q[mt][0], q[mt][1], q[mt][2], q[mt][3]);
        continue;
      }
      unsigned short h[4][4];
#pragma unroll
      for (int mt = 0; mt < 4; ++mt) {
#pragma unroll
        for (int r = 0; r < 4; ++r) h[mt][r] = f2bf(q[mt][r]);
        if (A.out_bf16 && ok(mt) && oyr + mt >= A.st0 && oyr + mt < A.st1 && oxr >= A.st0 && oxr < A.st1) {
          uint2 u;
          u.x = (uint32_t)h[mt][0] | ((uint32_t)h[mt][1] << 16);
          u.y = (uint32_t)h[mt][2] | ((uint32_t)h[mt][3] << 16);
          *reinterpret_cast<uint2*>(A.out_bf16 + off0 + mt * row) = u;
        }
      }
      if (A.pool_out) {
        // same pairing and order as the separate epilogue: rows mt, mt + 1
        // in the lane, columns c, c ^ 1 across lanes (tile origins are even)
        const int Hp = A.Ho / 2, Wp = A.Wo / 2;
#pragma unroll
        for (int pr = 0; pr < 2; ++pr) {
          unsigned short pv[4];
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const float tl = bf2f(h[2 * pr][r]), bl = bf2f(h[2 * pr + 1][r]);
            const float tr = __shfl_xor(tl, 1, 64), br = __shfl_xor(bl, 1, 64);
            pv[r] = f2bf(0.25f * ((tl + tr) + (bl + br)));
          }
          const int pyr = (oyr + 2 * pr) / 2, pxr = oxr / 2;
          if ((c & 1) == 0 && r0 + 2 * pr < FT && c < FT && pyr < Hp && pxr < Wp) {
            uint2 u;
            u.x = (uint32_t)pv[0] | ((uint32_t)pv[1] << 16);
            u.y = (uint32_t)pv[2] | ((uint32_t)pv[3] << 16);
            *reinterpret_cast<uint2*>(A.pool_out + (((int64_t)b * Hp + pyr) * Wp + pxr) * cout + c0) = u;
          }
        }
      }
    }
    if (next >= ntiles) break;
    tile = next;
    __syncthreads();  // every wave is done with both patches before they are overwritten
  }
}

// Layers l1 and l2 fused (k_conv2_bf16) for the input shapes that have a
// compiled form; LS_ENOTIMPL otherwise.
int conv2_bf16(const SrcPart& a1, const SrcPart& b2, int B, int H, int l1, int l2, const uint16_t* packed,
               const float* w, uint16_t* out_bf16, float* out_f32, uint16_t* pool_out, int relu2, int y0, int x0,
               int Ho, int Wo, hipStream_t st, int st0 = 0, int st1 = 1 << 30) {
  if (LS_LAYERS[l1].cout != 16 || LS_LAYERS[l2].cin != 16 + b2.c || a1.c != LS_LAYERS[l1].cin) return LS_ENOTIMPL;
  if (a1.up || b2.up || (pool_out && (Ho % 2 || Wo % 2))) return LS_ENOTIMPL;
  Conv2Args a;
  a.a1 = a1;
  a.b2 = b2;
  a.B = B;
  a.H = H;
  a.W = H;
  a.y0 = y0;
  a.x0 = x0;
  a.Ho = Ho;
  a.Wo = Wo;
  a.tiles_x = (Wo + FT - 1) / FT;
  a.tiles_y = (Ho + FT - 1) / FT;
  a.wp1 = packed + ls_bf16_packed_offset(l1);
  a.bias1 = w + ls_layer_b_offset(l1);
  a.wp2 = packed + ls_bf16_packed_offset(l2);
  a.bias2 = w + ls_layer_b_offset(l2);
  a.cout2 = LS_LAYERS[l2].cout;
  a.relu2 = relu2;
  a.out_bf16 = out_bf16;
  a.out_f32 = out_f32;
  a.pool_out = pool_out;
  a.st0 = st0;
  a.st1 = st1;
  const int64_t nblk = (int64_t)B * a.tiles_x * a.tiles_y;
  if (nblk <= 0) return LS_OK;
  if (nblk >= ((int64_t)1 << 31)) return LS_ENOTIMPL;
  const bool f32a = a1.f32 != nullptr, f32b = b2.c > 0 && b2.f32 != nullptr;
  LS_TRACE("conv_bf16", st);
  // persistent: as many workgroups as fit on the device at once
  auto launch = [&](auto* fn) {
    int per_cu = 0, dev = 0, cus = 0;
    LS_HOST_CHECK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, 256, 0));
    LS_HOST_CHECK(hipGetDevice(&dev));
    LS_HOST_CHECK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    const int64_t want = (int64_t)std::max(per_cu, 1) * std::max(cus, 1);
    hipLaunchKernelGGL(fn, dim3((unsigned)std::min<int64_t>(want, nblk)), dim3(256), 0, st, a);
    LS_LAUNCH_CHECK();
    return LS_OK;
  };
  if (a1.c == 8 && f32a && b2.c == 0 && a.cout2 <= 16) return launch(&k_conv2_bf16<8, true, 0, false, 1, 2>);
  if (a1.c == 16 && !f32a && b2.c == 8 && f32b && a.cout2 <= 16) return launch(&k_conv2_bf16<16, false, 8, true, 1, 2>);
  return LS_ENOTIMPL;
}

int pool_bf16(const uint16_t* in, uint16_t* out, int B, int H, int C, hipStream_t st) {
  const int64_t n = (int64_t)B * (H / 2) * (H / 2) * C;
  LS_TRACE("avgpool_bf16", st);
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
                    uint16_t* acts, float* head, bool fuse, hipStream_t st) {
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
  // per layer: tiling variant 0 = direct (operands from global memory, 4 pixel
  // tiles per wave), 1 = LDS-staged 16 x 16 tile, 2 = direct with 2
  // pixel tiles per wave, 3 = the LDS tile in persistent workgroups that
  // prefetch the next patch
  auto variant = [&](int l) {
    const int c = ls_conv_config_get(l, LS_BF16, 0);
    return c >= 0 && c <= 3 ? c : 3;  // default: the persistent tile
  };
  // layer pairs (enc1a, enc1b) and (dec1b, head) in one pass when their
  // first activation is not kept: config 4 of the pair's second layer, the
  // default for the head (measured on 1024 tiles: dec1b + head 0.230 ->
  // 0.170 ms; enc1a + enc1b 0.261 -> 0.267 ms, so separate by default)
  auto fused = [&](int l2) {
    const int c = ls_conv_config_get(l2, LS_BF16, 0);
    return fuse && (c == 4 || (c < 0 && l2 == LS_NLAYER - 1));
  };
  // a layer feeding an average pool writes the pooled tensor too when it uses the LDS tile
  auto conv = [&](const ConvSrc& s, int H, int l, uint16_t* out, uint16_t* pooled) -> int {
    const int cin_l = LS_LAYERS[l].cin;
    if ((variant(l) == 1 || variant(l) == 3) && (size_t)PT * PT * patch_pitch(cin_l) * 2 <= LDS_MAX) {
      const bool fuse = pooled && H % TT == 0;
      LS_TRYB(conv_bf16_lds(s, B, H, l, packed, w, out, nullptr, fuse ? pooled : nullptr, 1, 0, 0, H, H,
                            variant(l) == 3, st));
      if (pooled && !fuse) return pool_bf16(out, pooled, B, H, LS_LAYERS[l].cout, st);
      return LS_OK;
    }
    LS_TRYB(conv_bf16(s, B, H, l, packed, w, out, nullptr, 1, 0, 0, H, H, variant(l) == 2 ? 2 : 4, st));
    if (pooled) return pool_bf16(out, pooled, B, H, LS_LAYERS[l].cout, st);
    return LS_OK;
  };
  SrcPart u6 = bpart(A6, 64, R4);
  u6.up = 1;
  SrcPart u8 = bpart(A8, 32, R2);
  u8.up = 1;
  int rc01 = LS_ENOTIMPL;
  // with the head pair fused (inference), A2 is read only by dec1a on its
  // window grown by one texel: the fused enc1a + enc1b stores just that part
  int a2_0 = 0, a2_1 = 1 << 30;
  const int64_t head_tiles = (int64_t)B * ((gi.res + FT - 1) / FT) * ((gi.res + FT - 1) / FT);
  if (fused(10) && head_tiles < ((int64_t)1 << 31)) {  // the fused head pair then runs (no whole-plane dec1a)
    a2_0 = std::max(0, gi.pad - 3);
    a2_1 = std::min(R, gi.pad + gi.res + 3);
  }
  if (fused(1)) rc01 = conv2_bf16(X, none, B, R, 0, 1, packed, w, A2, nullptr, P1, 1, 0, 0, R, R, st, a2_0, a2_1);
  if (rc01 == LS_ENOTIMPL) {
    LS_TRYB(conv(cs(X, none), R, 0, A1, nullptr));
    LS_TRYB(conv(cs(bpart(A1, 16, R), none), R, 1, A2, P1));
  } else {
    LS_TRYB(rc01);
  }
  LS_TRYB(conv(cs(bpart(P1, 16, R2), none), R2, 2, A3, nullptr));
  LS_TRYB(conv(cs(bpart(A3, 32, R2), none), R2, 3, A4, P2));
  LS_TRYB(conv(cs(bpart(P2, 32, R4), none), R4, 4, A5, nullptr));
  LS_TRYB(conv(cs(bpart(A5, 64, R4), none), R4, 5, A6, nullptr));
  LS_TRYB(conv(cs(u6, bpart(A4, 32, R2)), R2, 6, A7, nullptr));
  LS_TRYB(conv(cs(bpart(A7, 32, R2), none), R2, 7, A8, nullptr));
  if (fused(10)) {
    // dec1a only where the fused dec1b + head read it, the crop and a
    // two-texel halo (clipped to the plane), stored as a window tensor
    const int w0 = std::max(0, gi.pad - 2), w1 = std::min(R, gi.pad + gi.res + 2), Hw = w1 - w0;
    if (variant(8) == 1 || variant(8) == 3)
      LS_TRYB(conv_bf16_lds(cs(u8, bpart(A2, 16, R)), B, R, 8, packed, w, A9, nullptr, nullptr, 1, w0, w0, Hw, Hw,
                            variant(8) == 3, st));
    else
      LS_TRYB(conv_bf16(cs(u8, bpart(A2, 16, R)), B, R, 8, packed, w, A9, nullptr, 1, w0, w0, Hw, Hw,
                        variant(8) == 2 ? 2 : 4, st));
    SrcPart a9 = bpart(A9, 16, Hw);
    a9.oy = w0;
    a9.ox = w0;
    const int rc = conv2_bf16(a9, X, B, R, 9, 10, packed, w, nullptr, head, nullptr, 0, gi.pad, gi.pad, gi.res, gi.res,
                              st);
    if (rc != LS_ENOTIMPL) return rc;
  }
  // the window conv of layer l from s into `out`, output [y0, y0 + n)^2
  auto conv_win = [&](const ConvSrc& s, int l, uint16_t* out, int y0, int n) -> int {
    if ((variant(l) == 1 || variant(l) == 3) && (size_t)PT * PT * patch_pitch(LS_LAYERS[l].cin) * 2 <= LDS_MAX)
      return conv_bf16_lds(s, B, R, l, packed, w, out, nullptr, nullptr, 1, y0, y0, n, n, variant(l) == 3, st);
    return conv_bf16(s, B, R, l, packed, w, out, nullptr, 1, y0, y0, n, n, variant(l) == 2 ? 2 : 4, st);
  };
  SrcPart a10 = bpart(A10, 16, R);
  if (!fuse && ls_bf16_lvl1_windowed()) {
    // saved for the backward, which then runs decoder level 1 on the same
    // windows: A9 and A10 only where the head's output and its gradient
    // reach, stored as window tensors
    const Lvl1Win lw = ls_lvl1_windows(R, gi.pad, gi.res);
    LS_TRYB(conv_win(cs(u8, bpart(A2, 16, R)), 8, A9, lw.d0, lw.dn));
    SrcPart a9 = bpart(A9, 16, lw.dn);
    a9.oy = lw.d0;
    a9.ox = lw.d0;
    LS_TRYB(conv_win(cs(a9, none), 9, A10, lw.h0, lw.hn));
    a10 = bpart(A10, 16, lw.hn);
    a10.oy = lw.h0;
    a10.ox = lw.h0;
  } else {
    LS_TRYB(conv(cs(u8, bpart(A2, 16, R)), R, 8, A9, nullptr));
    LS_TRYB(conv(cs(bpart(A9, 16, R), none), R, 9, A10, nullptr));
  }
  if ((variant(10) == 1 || variant(10) == 3) && (size_t)PT * PT * patch_pitch(24) * 2 <= LDS_MAX)
    return conv_bf16_lds(cs(a10, X), B, R, 10, packed, w, nullptr, head, nullptr, 0, gi.pad, gi.pad, gi.res, gi.res,
                         variant(10) == 3, st);
  return conv_bf16(cs(a10, X), B, R, 10, packed, w, nullptr, head, 0, gi.pad, gi.pad, gi.res, gi.res,
                   variant(10) == 2 ? 2 : 4, st);
}

int ls_bf16_conv_pipe(const ConvTileArgs& a, int nt, int ca, int cb, bool upa, bool f32a, bool f32b,
                      hipStream_t st, const char* trace) {
  if (a.B <= 0 || a.tiles_x <= 0 || a.tiles_y <= 0) return LS_OK;
  const int64_t ntile = (int64_t)a.B * a.tiles_x * a.tiles_y;
  LS_TRACE(trace, st);
  // one persistent form per input shape: as many workgroups as fit on the
  // device at once, each walking tiles tile, tile + grid, ...
#define LS_PIPE_G(N, CA, CB, UPA, F32A, F32B, W)                                                         \
  if (nt == N && ca == CA && cb == CB && upa == UPA && f32a == F32A && f32b == F32B) {                  \
    auto* fn = &k_conv_bf16_pipe<N, CA, CB, UPA, F32A, F32B, W>;                                         \
    constexpr size_t plds = pipe_lds_bytes(N, CA + CB);                                                  \
    static_assert(plds <= LDS_MAX, "pipelined tile exceeds LDS");                                       \
    if (plds > 65536)                                                                                    \
      LS_HOST_CHECK(hipFuncSetAttribute(reinterpret_cast<const void*>(fn),                               \
                                        hipFuncAttributeMaxDynamicSharedMemorySize, (int)plds));         \
    int per_cu = 0, dev = 0, cus = 0;                                                                    \
    LS_HOST_CHECK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, 256, plds));                \
    LS_HOST_CHECK(hipGetDevice(&dev));                                                                   \
    LS_HOST_CHECK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));             \
    const int64_t want = (int64_t)std::max(per_cu, 1) * std::max(cus, 1);                                \
    const dim3 pgrid((unsigned)std::min<int64_t>(want, ntile));                                          \
    hipLaunchKernelGGL((k_conv_bf16_pipe<N, CA, CB, UPA, F32A, F32B, W>), pgrid, dim3(256), plds, st, a); \
    LS_LAUNCH_CHECK();                                                                                   \
    return LS_OK;                                                                                        \
  }
  // the shapes of the paper's refinement network (per-input encoders, decoders, final CNN)
  LS_PIPE_G(4, 8, 0, false, true, false, 1)
  LS_PIPE_G(2, 16, 0, false, false, false, 2)
  LS_PIPE_G(2, 32, 0, false, false, false, 2)
  LS_PIPE_G(2, 32, 0, true, false, false, 2)
  LS_PIPE_G(1, 32, 0, true, false, false, 2)
  LS_PIPE_G(1, 16, 0, true, false, false, 2)
  LS_PIPE_G(2, 32, 8, false, false, true, 2)
  LS_PIPE_G(1, 32, 0, false, false, false, 2)
  // the input gradients of the U-Net (gradient channels -> layer input channels)
  LS_PIPE_G(2, 8, 0, false, false, false, 2)
  LS_PIPE_G(1, 8, 0, false, false, false, 2)
  LS_PIPE_G(1, 16, 0, false, false, false, 2)
  LS_PIPE_G(3, 16, 0, false, false, false, 2)
  LS_PIPE_G(6, 32, 0, false, false, false, 1)
  LS_PIPE_G(4, 64, 0, false, false, false, 1)
  LS_PIPE_G(2, 64, 0, false, false, false, 1)
#undef LS_PIPE_G
  return LS_ENOTIMPL;
}
