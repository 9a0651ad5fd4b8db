// The paper's refinement network (LidarScout Section 3.4, architecture
// paragraph) on gfx950: per-input convolutional encoders, a two-step fully
// connected merge, separate height and texture decoders, a skip of the
// original inputs into a final CNN, and the centre res x res crop added to
// the linear input.  Layer sizes (the figure is missing; this is the
// reading the library implements, 2,528,708 parameters at R = 96):
//
//   inputs  I0 = h_lin (x channel 0), I1 = h_nn (1), I2 = rgb_lin (2-4),
//           I3 = rgb_nn (5-7)
//   encoder i: four times e = avgpool2(relu(conv3x3(e))), c_i->16->32->32->32
//   FC1     z_h = relu(W [F_0, F_1] + b), z_c = relu(W [F_2, F_3] + b), 256 each
//   FC2     d_h, d_t = relu(W [z_h, z_c] + b), each an R/16 x R/16 x 32 image
//   decoder k: four times a = relu(conv3x3(up2(a))), 32->32->32->16->16
//   final   f = relu(conv(relu(conv([a_h, a_t, x])))) 40->32->32, then a
//           3x3 conv 32->4 without ReLU on the crop; y = crop(x_lin) + f
//
// Flat weights in the order above: conv W[Cout][3][3][Cin] then b[Cout];
// fully connected W[N][K] then b[N] (K = position in the concatenated
// input, feature images flattened row, column, channel).
//
// MI355X mapping.  The four encoders run as grouped convolutions: their
// first layers together as one 8 -> 64 conv over the whole input tile
// (block-diagonal weights: each encoder's 16 outputs see only its own input
// channels, the other weights are exact zeros), the later layers as one
// launch per encoder reading its 16 or 32 channels out of the shared tensor
// and writing its slice of the next one; the BF16 path fuses every pool into
// the conv epilogue, so only pooled encoder activations are stored.  The two
// FC1 layers are one GEMM over the interleaved encoder features (zero
// blocks where an FC1 layer does not read an encoder), and the two FC2
// layers one GEMM whose output columns are permuted so that it is directly
// the decoders' shared 64-channel input image.  Convolutions use the
// library's conv kernels (FP32 vector, or BF16 on the matrix cores with FP32
// accumulation); the fully connected layers have their own kernels
// (tiled FP32, or BF16 on v_mfma_f32_16x16x32_bf16).  The batch is taken in
// chunks so the workspace stays bounded.
#include <algorithm>

#include "ls_common.hpp"
#include "ls_unet.hpp"
#include "ls_unet_bf16.hpp"

namespace {

// ------------------------------------------------------------------ layers
enum LayerKind { CONV = 0, FC = 1 };
struct NetLayer {
  int kind, cin, cout;
};
constexpr int NL = 31;
constexpr int L_ENC = 0, L_FC1H = 16, L_FC1C = 17, L_FC2H = 18, L_FC2T = 19, L_DECH = 20, L_DECT = 24, L_FIN1 = 28,
              L_FIN2 = 29, L_FIN3 = 30;
constexpr int ENC_CIN0[4] = {1, 1, 3, 3};

struct Net {
  int R, L;  // padded side, features per encoder (R/16)^2 * 32
  NetLayer layer[NL];
  int64_t woff[NL], boff[NL];
  int64_t total;
};

Net make_net(int R) {
  Net n;
  n.R = R;
  n.L = (R / 16) * (R / 16) * 32;
  for (int i = 0; i < 4; ++i) {
    const int c[5] = {ENC_CIN0[i], 16, 32, 32, 32};
    for (int k = 0; k < 4; ++k) n.layer[L_ENC + 4 * i + k] = {CONV, c[k], c[k + 1]};
  }
  n.layer[L_FC1H] = {FC, 2 * n.L, 256};
  n.layer[L_FC1C] = {FC, 2 * n.L, 256};
  n.layer[L_FC2H] = {FC, 512, n.L};
  n.layer[L_FC2T] = {FC, 512, n.L};
  const int d[5] = {32, 32, 32, 16, 16};
  for (int k = 0; k < 4; ++k) {
    n.layer[L_DECH + k] = {CONV, d[k], d[k + 1]};
    n.layer[L_DECT + k] = {CONV, d[k], d[k + 1]};
  }
  n.layer[L_FIN1] = {CONV, 40, 32};
  n.layer[L_FIN2] = {CONV, 32, 32};
  n.layer[L_FIN3] = {CONV, 32, 4};
  int64_t off = 0;
  for (int k = 0; k < NL; ++k) {
    const NetLayer& l = n.layer[k];
    const int64_t nw = l.kind == CONV ? (int64_t)l.cout * 9 * l.cin : (int64_t)l.cout * l.cin;
    n.woff[k] = off;
    n.boff[k] = off + nw;
    off += nw + l.cout;
  }
  n.total = off;
  return n;
}

// ------------------------------------------------------------------ weight preparation
// Every derived weight array is one segment; a thread per destination
// element finds its segment and computes the element.
enum SegKind {
  S_CONV_T = 0,   // FP32 [tap][cin][cout] from W[cout][tap][cin]
  S_ENC1_T = 1,   // FP32 [tap][8][64], the four first encoder layers block-diagonally
  S_ENC1_B = 2,   // FP32 [64] their biases
  S_FC1_T = 3,    // FP32 [4L][512] (K x N) of the joint FC1
  S_FC1_B = 4,    // FP32 [512]
  S_FC2_T = 5,    // FP32 [512][2L] of the joint FC2, output columns permuted
  S_FC2_B = 6,    // FP32 [2L]
  S_CONV_P = 7,   // BF16 [Npad][Kpad] from W (k = tap*cin + ci)
  S_ENC1_P = 8,   // BF16 [64][96] block-diagonal
  S_FC1_P = 9,    // BF16 [512][4L] (N x K)
  S_FC2_P = 10,   // BF16 [2L][512]
};
struct Seg {
  int kind, layer, cin, cout, kpad;
  int64_t dst, count;  // destination element offset (in FP32 or BF16 elements) and size
};
constexpr int MAX_SEG = 40;
struct PrepArgs {
  const float* w;
  float* f32;
  uint16_t* bf16;
  int L;
  int inputs;  // bit i: input I_i present (absent inputs are zero)
  int nseg;
  int64_t woff[NL], boff[NL];
  Seg seg[MAX_SEG];
};

__device__ __forceinline__ unsigned short f2bf(float f) {
  return __builtin_bit_cast(unsigned short, static_cast<__bf16>(f));
}

// Value of the joint FC1 matrix at output n, input k: k indexes the
// interleaved features [pixel][encoder][32], n < 256 is the height FC1 (reads
// encoders 0, 1), n >= 256 the colour FC1 (encoders 2, 3).
__device__ __forceinline__ float fc1_value(const PrepArgs& A, int n, int64_t k) {
  const int p = (int)(k / 128), r = (int)(k % 128), e = r / 32, c = r % 32;
  const bool hgt = n < 256;
  if (hgt != (e < 2)) return 0.f;
  const int layer = hgt ? L_FC1H : L_FC1C;
  const int nn = hgt ? n : n - 256;
  const int64_t kk = (int64_t)(e % 2) * A.L + (int64_t)p * 32 + c;
  return A.w[A.woff[layer] + (int64_t)nn * (2 * A.L) + kk];
}

// Joint FC2 at output column n' = pixel*64 + decoder*32 + c, input k.
__device__ __forceinline__ float fc2_value(const PrepArgs& A, int64_t n, int k) {
  const int p = (int)(n / 64), r = (int)(n % 64), dk = r / 32, c = r % 32;
  const int layer = dk == 0 ? L_FC2H : L_FC2T;
  return A.w[A.woff[layer] + ((int64_t)p * 32 + c) * 512 + k];
}

// First encoder layers as one 8 -> 64 conv: output co = 16*e + j reads only
// encoder e's input channels.
__device__ __forceinline__ float enc1_value(const PrepArgs& A, int co, int tap, int ci) {
  const int e = co / 16, j = co % 16;
  if (!((A.inputs >> e) & 1)) return 0.f;  // an absent input reads as zero
  const int c0 = e == 0 ? 0 : (e == 1 ? 1 : (e == 2 ? 2 : 5));
  const int cn = e < 2 ? 1 : 3;
  if (ci < c0 || ci >= c0 + cn) return 0.f;
  return A.w[A.woff[L_ENC + 4 * e] + ((int64_t)j * 9 + tap) * cn + (ci - c0)];
}

// Input I_i that x channel ch belongs to: 0 h_lin, 1 h_nn, 2 rgb_lin, 3 rgb_nn.
__device__ __forceinline__ int input_of_channel(int ch) { return ch == 0 ? 0 : (ch == 1 ? 1 : (ch < 5 ? 2 : 3)); }

// Weight of conv layer `layer` at (co, tap, ci); the final CNN's first
// layer sees an absent input's skip channels as zero.
__device__ __forceinline__ float conv_value(const PrepArgs& A, int layer, int cin, int co, int tap, int ci) {
  if (layer == L_FIN1 && ci >= 32 && !((A.inputs >> input_of_channel(ci - 32)) & 1)) return 0.f;
  return A.w[A.woff[layer] + ((int64_t)co * 9 + tap) * cin + ci];
}

__global__ void k_lsnet_prep(PrepArgs A) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  int64_t base = 0;
  for (int s = 0; s < A.nseg; ++s) {
    const Seg& g = A.seg[s];
    if (i < base + g.count) {
      const int64_t r = i - base;
      const int cin = g.cin, cout = g.cout;
      switch (g.kind) {
        case S_CONV_T: {
          const int tap = (int)(r / ((int64_t)cin * cout)), ci = (int)((r / cout) % cin), co = (int)(r % cout);
          A.f32[g.dst + r] = conv_value(A, g.layer, cin, co, tap, ci);
          break;
        }
        case S_ENC1_T: {
          const int tap = (int)(r / (8 * 64)), ci = (int)((r / 64) % 8), co = (int)(r % 64);
          A.f32[g.dst + r] = enc1_value(A, co, tap, ci);
          break;
        }
        case S_ENC1_B: {
          const int e = (int)r / 16, j = (int)r % 16;
          A.f32[g.dst + r] = A.w[A.boff[L_ENC + 4 * e] + j];
          break;
        }
        case S_FC1_T: {
          const int64_t k = r / 512;
          const int n = (int)(r % 512);
          A.f32[g.dst + r] = fc1_value(A, n, k);
          break;
        }
        case S_FC1_B: {
          const int n = (int)r;
          A.f32[g.dst + r] = n < 256 ? A.w[A.boff[L_FC1H] + n] : A.w[A.boff[L_FC1C] + n - 256];
          break;
        }
        case S_FC2_T: {
          const int k = (int)(r / (2 * A.L));
          const int64_t n = r % (2 * A.L);
          A.f32[g.dst + r] = fc2_value(A, n, k);
          break;
        }
        case S_FC2_B: {
          const int p = (int)(r / 64), q = (int)(r % 64), dk = q / 32, c = q % 32;
          A.f32[g.dst + r] = A.w[A.boff[dk == 0 ? L_FC2H : L_FC2T] + p * 32 + c];
          break;
        }
        case S_CONV_P: {
          const int n = (int)(r / g.kpad), k = (int)(r % g.kpad);
          float v = 0.f;
          if (n < cout && k < 9 * cin) v = conv_value(A, g.layer, cin, n, k / cin, k % cin);
          A.bf16[g.dst + r] = f2bf(v);
          break;
        }
        case S_ENC1_P: {
          const int n = (int)(r / g.kpad), k = (int)(r % g.kpad);
          A.bf16[g.dst + r] = f2bf(k < 72 ? enc1_value(A, n, k / 8, k % 8) : 0.f);
          break;
        }
        case S_FC1_P: {
          const int64_t K = 4 * (int64_t)A.L;
          A.bf16[g.dst + r] = f2bf(fc1_value(A, (int)(r / K), r % K));
          break;
        }
        case S_FC2_P: {
          A.bf16[g.dst + r] = f2bf(fc2_value(A, r / 512, (int)(r % 512)));
          break;
        }
        default: break;
      }
      return;
    }
    base += g.count;
  }
}

// ------------------------------------------------------------------ fully connected layers
// FP32: C[M][N] = act(A[M][K] B[K][N] + bias), a 64 x 64 block per
// workgroup, 4 x 4 outputs per thread, K in steps of 16 through LDS.
// N % 64 == 0 and K % 16 == 0; rows beyond M are masked.
constexpr int FC_T = 256;
__global__ void __launch_bounds__(FC_T) k_fc_f32(const float* __restrict__ A, const float* __restrict__ B,
                                                 const float* __restrict__ bias, float* __restrict__ C, int M, int N,
                                                 int K, int relu) {
  __shared__ float sA[16][64 + 4];
  __shared__ float sB[16][64];
  const int tid = threadIdx.x;
  const int m0 = blockIdx.y * 64, n0 = blockIdx.x * 64;
  const int tm = tid / 16, tn = tid % 16;  // 4 rows tm*4.., 4 cols tn*4..
  float acc[4][4] = {};
  for (int k0 = 0; k0 < K; k0 += 16) {
    for (int e = tid; e < 64 * 16; e += FC_T) {
      const int r = e / 16, kk = e % 16;
      const int m = m0 + r;
      sA[kk][r] = m < M ? A[(int64_t)m * K + k0 + kk] : 0.f;
    }
    for (int e = tid; e < 16 * 64; e += FC_T) {
      const int kk = e / 64, c = e % 64;
      sB[kk][c] = B[(int64_t)(k0 + kk) * N + n0 + c];
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < 16; ++kk) {
      float a[4], b[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = sA[kk][tm * 4 + i];
#pragma unroll
      for (int j = 0; j < 4; ++j) b[j] = sB[kk][tn * 4 + j];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = fmaf(a[i], b[j], acc[i][j]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int m = m0 + tm * 4 + i;
    if (m >= M) continue;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int n = n0 + tn * 4 + j;
      float v = acc[i][j] + bias[n];
      if (relu) v = fmaxf(v, 0.f);
      C[(int64_t)m * N + n] = v;
    }
  }
}

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));

// BF16 on the matrix cores: C[M][N] = act(A[M][K] W[N][K]^T + bias) with
// FP32 accumulation, stored as BF16.  A workgroup (4 waves) owns 64 rows x 64
// columns, each wave 16 rows x 4 column tiles; per 32-wide K step lane l
// loads row (l % 16) of A and of W at k = 8 * (l / 16) (16-byte loads).
// K % 32 == 0, N % 64 == 0; rows beyond M read zeros and are not stored.
__global__ void __launch_bounds__(256) k_fc_bf16(const uint16_t* __restrict__ A, const uint16_t* __restrict__ W,
                                                 const float* __restrict__ bias, uint16_t* __restrict__ C, int M,
                                                 int N, int K, int relu) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int r16 = lane & 15, g = lane >> 4;
  const int m0 = blockIdx.y * 64 + wave * 16, n0 = blockIdx.x * 64;
  const int m = m0 + r16;
  const bool mv = m < M;
  const uint16_t* ap = A + (int64_t)(mv ? m : 0) * K + 8 * g;
  const uint16_t* wp = W + (int64_t)(n0 + r16) * K + 8 * g;
  f32x4 acc[4];
#pragma unroll
  for (int nt = 0; nt < 4; ++nt) acc[nt] = f32x4{0.f, 0.f, 0.f, 0.f};
  for (int k = 0; k < K; k += 32) {
    u16x8 a = {0, 0, 0, 0, 0, 0, 0, 0};
    if (mv) a = *reinterpret_cast<const u16x8*>(ap + k);
    const bf16x8 ab = __builtin_bit_cast(bf16x8, a);
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
      const bf16x8 bb = __builtin_bit_cast(bf16x8, *reinterpret_cast<const u16x8*>(wp + (int64_t)nt * 16 * K + k));
      acc[nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ab, bb, acc[nt], 0, 0, 0);
    }
  }
  // D rows 4g + i (A rows), column r16 (W rows)
#pragma unroll
  for (int nt = 0; nt < 4; ++nt) {
    const int n = n0 + nt * 16 + r16;
    const float b = bias[n];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int mm = m0 + 4 * g + i;
      if (mm >= M) continue;
      float v = acc[nt][i] + b;
      if (relu) v = fmaxf(v, 0.f);
      C[(int64_t)mm * N + n] = f2bf(v);
    }
  }
}

// y = crop(x_lin) + head, with an absent linear input read as zero, and the
// texture h = cz + r * y_h (double), colour clamped to [0, 1].
__global__ void k_lsnet_epilogue(const float* __restrict__ head, const float* __restrict__ x,
                                 const double* __restrict__ cz, int B, int res, int pad, double r_m, int inputs,
                                 float* __restrict__ y_out, float* __restrict__ tex_out) {
  const int64_t n = (int64_t)B * res * res;
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int b = (int)(i / ((int64_t)res * res));
  const int r = (int)(i - (int64_t)b * res * res);
  const int R = res + 2 * pad;
  const int yy = r / res + pad, xx = r % res + pad;
  const float* xp = x + (((int64_t)b * R + yy) * R + xx) * 8;
  const float4 h = reinterpret_cast<const float4*>(head)[i];
  const bool lh = inputs & 1, lc = (inputs >> 2) & 1;
  const float4 v = make_float4((lh ? xp[0] : 0.f) + h.x, (lc ? xp[2] : 0.f) + h.y, (lc ? xp[3] : 0.f) + h.z,
                               (lc ? xp[4] : 0.f) + h.w);
  if (y_out) reinterpret_cast<float4*>(y_out)[i] = v;
  if (tex_out) {
    const double hm = cz[b] + r_m * (double)v.x;
    reinterpret_cast<float4*>(tex_out)[i] =
        make_float4((float)hm, fminf(fmaxf(v.y, 0.f), 1.f), fminf(fmaxf(v.z, 0.f), 1.f), fminf(fmaxf(v.w, 0.f), 1.f));
  }
}

// ------------------------------------------------------------------ host side
struct Derived {
  // FP32 path
  int64_t conv_t[NL];  // per conv layer (except the first encoder layers), [9][cin][cout]
  int64_t enc1_t, enc1_b, fc1_t, fc1_b, fc2_t, fc2_b;
  int64_t n_f32;
  // BF16 path
  int64_t conv_p[NL];
  int kpad[NL];
  int64_t enc1_p, fc1_p, fc2_p;
  int64_t n_bf16;
  Seg seg[MAX_SEG];
  int nseg;
};

Derived derive(const Net& n, int precision) {
  Derived d{};
  const int64_t L = n.L;
  int64_t f = 0, h = 0;
  auto seg = [&](int kind, int layer, int cin, int cout, int kpad, int64_t dst, int64_t count) {
    d.seg[d.nseg++] = Seg{kind, layer, cin, cout, kpad, dst, count};
  };
  // the combined biases are FP32 in both paths
  d.enc1_b = f;
  seg(S_ENC1_B, 0, 0, 0, 0, f, 64);
  f += 64;
  d.fc1_b = f;
  seg(S_FC1_B, 0, 0, 0, 0, f, 512);
  f += 512;
  d.fc2_b = f;
  seg(S_FC2_B, 0, 0, 0, 0, f, 2 * L);
  f += 2 * L;
  if (precision == LS_FP32) {
    d.enc1_t = f;
    seg(S_ENC1_T, 0, 8, 64, 0, f, 9 * 8 * 64);
    f += 9 * 8 * 64;
    for (int k = 0; k < NL; ++k) {
      const NetLayer& l = n.layer[k];
      const bool first_enc = k < L_FC1H && k % 4 == 0;
      if (l.kind != CONV || first_enc) continue;
      d.conv_t[k] = f;
      seg(S_CONV_T, k, l.cin, l.cout, 0, f, 9LL * l.cin * l.cout);
      f += 9LL * l.cin * l.cout;
    }
    d.fc1_t = f;
    seg(S_FC1_T, 0, 0, 0, 0, f, 4 * L * 512);
    f += 4 * L * 512;
    d.fc2_t = f;
    seg(S_FC2_T, 0, 0, 0, 0, f, 512 * 2 * L);
    f += 512 * 2 * L;
  } else {
    d.enc1_p = h;
    seg(S_ENC1_P, 0, 8, 64, 96, h, 64 * 96);
    h += 64 * 96;
    for (int k = 0; k < NL; ++k) {
      const NetLayer& l = n.layer[k];
      const bool first_enc = k < L_FC1H && k % 4 == 0;
      if (l.kind != CONV || first_enc) continue;
      const int kp = (9 * l.cin + 31) / 32 * 32, np = (l.cout + 15) / 16 * 16;
      d.kpad[k] = kp;
      d.conv_p[k] = h;
      seg(S_CONV_P, k, l.cin, l.cout, kp, h, (int64_t)np * kp);
      h += (int64_t)np * kp;
    }
    d.fc1_p = h;
    seg(S_FC1_P, 0, 0, 0, 0, h, 512 * 4 * L);
    h += 512 * 4 * L;
    d.fc2_p = h;
    seg(S_FC2_P, 0, 0, 0, 0, h, 2 * L * 512);
    h += 2 * L * 512;
  }
  d.n_f32 = f;
  d.n_bf16 = h;
  return d;
}

constexpr int CHUNK_F32 = 256, CHUNK_BF16 = 1024;

// Activation elements per tile (FP32 path stores the full-resolution encoder
// outputs before pooling; the BF16 path pools in the conv epilogue).
struct Acts {
  int64_t e1, p1, e2, p2, e3, p3, e4, feat, z, d, dd1, dd2, dd3, aht, f1, f2, head, total;
};

Acts acts_per_tile(int R, int res, bool full_enc) {
  Acts a{};
  const int64_t r2 = (int64_t)R * R;
  int64_t o = 0;
  auto take = [&](int64_t n) {
    const int64_t at = o;
    o += (n + 63) / 64 * 64;
    return at;
  };
  if (full_enc) a.e1 = take(r2 * 64);
  a.p1 = take(r2 / 4 * 64);
  if (full_enc) a.e2 = take(r2 / 4 * 128);
  a.p2 = take(r2 / 16 * 128);
  if (full_enc) a.e3 = take(r2 / 16 * 128);
  a.p3 = take(r2 / 64 * 128);
  if (full_enc) a.e4 = take(r2 / 64 * 128);
  a.feat = take(r2 / 256 * 128);
  a.z = take(512);
  a.d = take(r2 / 256 * 64);
  a.dd1 = take(r2 / 64 * 64);
  a.dd2 = take(r2 / 16 * 64);
  a.dd3 = take(r2 / 4 * 32);
  a.aht = take(r2 * 32);
  a.f1 = take(r2 * 32);
  a.f2 = take(r2 * 32);
  a.head = take((int64_t)res * res * 4);  // FP32 in both paths
  a.total = o;
  return a;
}

size_t ws_bytes(const LsGridInfo& gi, int32_t n_tiles, int precision) {
  const Net n = make_net(gi.R);
  const Derived d = derive(n, precision);
  const int chunk = std::max(1, std::min<int>(n_tiles, precision == LS_FP32 ? CHUNK_F32 : CHUNK_BF16));
  const Acts a = acts_per_tile(gi.R, gi.res, precision == LS_FP32);
  const size_t el = precision == LS_FP32 ? 4 : 2;
  return ls_align((size_t)d.n_f32 * 4) + ls_align((size_t)d.n_bf16 * 2) + ls_align((size_t)a.total * el * chunk) +
         ls_align((size_t)gi.res * gi.res * 4 * 4 * chunk) + 1024;
}

#define LS_TRYN(expr)             \
  do {                            \
    int rc_ = (expr);             \
    if (rc_ != LS_OK) return rc_; \
  } while (0)

int fc_f32(const float* A, const float* B, const float* bias, float* C, int M, int N, int K, hipStream_t st) {
  if (N % 64 || K % 16) return LS_ENOTIMPL;
  dim3 grid((unsigned)(N / 64), (unsigned)((M + 63) / 64));
  LS_TRACE("fc_f32", st);
  hipLaunchKernelGGL(k_fc_f32, grid, dim3(FC_T), 0, st, A, B, bias, C, M, N, K, 1);
  LS_LAUNCH_CHECK();
  return LS_OK;
}

int fc_bf16(const uint16_t* A, const uint16_t* W, const float* bias, uint16_t* C, int M, int N, int K,
            hipStream_t st) {
  if (N % 64 || K % 32) return LS_ENOTIMPL;
  dim3 grid((unsigned)(N / 64), (unsigned)((M + 63) / 64));
  LS_TRACE("fc_bf16", st);
  hipLaunchKernelGGL(k_fc_bf16, grid, dim3(256), 0, st, A, W, bias, C, M, N, K, 1);
  LS_LAUNCH_CHECK();
  return LS_OK;
}

SrcPart part_f32(const float* p, int c, int hw, int stride, int coff, bool up) {
  SrcPart s = src_plain(p, c, hw, hw, stride, coff, nullptr);
  s.up = up ? 1 : 0;
  return s;
}

SrcPart part_bf16(const uint16_t* p, int c, int hw, int stride, int coff, bool up) {
  SrcPart s = src_none();
  s.bf16 = p;
  s.c = c;
  s.h = hw;
  s.w = hw;
  s.stride = stride;
  s.coff = coff;
  s.up = up ? 1 : 0;
  return s;
}

// FP32 conv over a whole H x H plane (or the crop window) into a channel slice.
int conv32(const ConvSrc& s, int B, int H, const float* wt, const float* bias, int cout, int relu, float* out,
           int out_stride, int out_coff, int y0, int x0, int Ho, hipStream_t st) {
  ConvArgs a;
  a.src = s;
  a.B = B;
  a.H = H;
  a.W = H;
  a.y0 = y0;
  a.x0 = x0;
  a.Ho = Ho;
  a.Wo = Ho;
  a.wt = wt;
  a.bias = bias;
  a.cout = cout;
  a.relu = relu;
  a.out = out;
  a.out_stride = out_stride;
  a.out_coff = out_coff;
  a.cob_max = 32;
  return ls_conv_f32(a, st);
}

// BF16 conv over a whole H x H plane (or the crop window): output slice
// and/or fused 2 x 2 average pool slice.
int conv16(const ConvSrc& s, int B, int H, const uint16_t* wp, int kpad, const float* bias, int cout, int relu,
           uint16_t* out, int out_stride, int out_coff, uint16_t* pool, int pool_stride, int pool_coff, float* out_f32,
           int y0, int x0, int Ho, hipStream_t st) {
  ConvTileArgs a;
  a.src = s;
  a.B = B;
  a.H = H;
  a.W = H;
  a.y0 = y0;
  a.x0 = x0;
  a.Ho = Ho;
  a.Wo = Ho;
  a.tiles_x = (Ho + 15) / 16;
  a.tiles_y = (Ho + 15) / 16;
  a.wp = wp;
  a.Kpad = kpad;
  a.bias = bias;
  a.cout = cout;
  a.relu = relu;
  a.out_bf16 = out;
  a.out_f32 = out_f32;
  a.out_stride = out_stride;
  a.out_coff = out_coff;
  a.pool_out = pool;
  a.pool_stride = pool_stride;
  a.pool_coff = pool_coff;
  a.mask = nullptr;
  const int nt = (cout + 15) / 16;
  const bool f32b = s.b.c > 0 && s.b.f32 != nullptr;
  return ls_bf16_conv_pipe(a, nt, s.a.c, s.b.c, s.a.up != 0, s.a.f32 != nullptr, f32b, st);
}

// A square window [y0, y0 + n) of the plane (both axes): the part of a
// full-resolution layer's output that the layers after it read, here the
// crop grown by `halo` texels and clipped to the plane.
struct Window {
  int y0, n;
};
Window crop_window(int R, int pad, int res, int halo) {
  const int a = std::max(0, pad - halo), b = std::min(R, pad + res + halo);
  return Window{a, b - a};
}
// a tensor stored for a window only, read as part of the plane
SrcPart window_part(SrcPart p, const Window& w) {
  p.oy = w.y0;
  p.ox = w.y0;
  return p;
}

ConvSrc src1(SrcPart a) {
  ConvSrc s;
  s.a = a;
  s.b = src_none();
  return s;
}

}  // namespace

int64_t ls_lsnet_params(int R) {
  if (R <= 0 || R % 16) return -1;
  return make_net(R).total;
}

size_t ls_lsnet_ws_bytes(const LsGridInfo& gi, int32_t n_tiles, int precision) {
  if (gi.R % 16) return 0;
  return ws_bytes(gi, n_tiles, precision);
}

int ls_lsnet_forward_impl(const float* w, int precision, int inputs, const float* x, const double* cz,
                          int32_t n_tiles, const LsGridInfo& gi, float* y_out, float* tex_out, void* ws,
                          size_t ws_bytes_given, hipStream_t st) {
  const int R = gi.R, res = gi.res, pad = gi.pad;
  if (R % 16) return LS_ERANGE;
  if (n_tiles == 0) return LS_OK;
  if (!ws || ws_bytes_given < ws_bytes(gi, n_tiles, precision)) return LS_EWORKSPACE;
  const Net net = make_net(R);
  const Derived d = derive(net, precision);
  const bool f32 = precision == LS_FP32;
  const int chunk = std::min<int>(n_tiles, f32 ? CHUNK_F32 : CHUNK_BF16);
  const Acts at = acts_per_tile(R, res, f32);
  LsArena ar{reinterpret_cast<char*>(ws), ws_bytes_given, 0};
  float* wf = ar.take<float>(d.n_f32);
  uint16_t* wb = ar.take<uint16_t>(d.n_bf16 > 0 ? d.n_bf16 : 1);
  float* act32 = f32 ? ar.take<float>(at.total * chunk) : nullptr;
  uint16_t* act16 = f32 ? nullptr : ar.take<uint16_t>(at.total * chunk);
  float* head = ar.take<float>((size_t)res * res * 4 * chunk);
  // derived weights
  {
    PrepArgs p;
    p.w = w;
    p.f32 = wf;
    p.bf16 = wb;
    p.L = net.L;
    p.inputs = inputs;
    p.nseg = d.nseg;
    for (int k = 0; k < NL; ++k) {
      p.woff[k] = net.woff[k];
      p.boff[k] = net.boff[k];
    }
    int64_t total = 0;
    for (int s = 0; s < d.nseg; ++s) {
      p.seg[s] = d.seg[s];
      total += d.seg[s].count;
    }
    LS_TRACE("lsnet_prep", st);
    hipLaunchKernelGGL(k_lsnet_prep, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, p);
    LS_LAUNCH_CHECK();
  }
  const int R2 = R / 2, R4 = R / 4, R8 = R / 8, R16 = R / 16;
  // windows of the final CNN's inputs: fin3 reads fin2 on the crop + 1,
  // fin2 reads fin1 on the crop + 2, fin1 reads the decoders on the crop + 3
  const Window w2 = crop_window(R, pad, res, 1), w1 = crop_window(R, pad, res, 2), wa = crop_window(R, pad, res, 3);
  const int64_t L = net.L;
  const double r_m = (double)gi.H * gi.scale_xy;
  for (int t0 = 0; t0 < n_tiles; t0 += chunk) {
    const int B = std::min(chunk, n_tiles - t0);
    const float* xc = x + (int64_t)t0 * R * R * 8;
    const SrcPart X = part_f32(xc, 8, R, 8, 0, false);
    if (f32) {
      float* A0 = act32;
      auto P = [&](int64_t off) { return A0 + off * B; };
      float *E1 = P(at.e1), *P1 = P(at.p1), *E2 = P(at.e2), *P2 = P(at.p2), *E3 = P(at.e3), *P3 = P(at.p3),
            *E4 = P(at.e4), *Fe = P(at.feat), *Z = P(at.z), *D = P(at.d), *Dd1 = P(at.dd1), *Dd2 = P(at.dd2),
            *Dd3 = P(at.dd3), *Aht = P(at.aht), *F1 = P(at.f1), *F2 = P(at.f2);
      // encoders
      LS_TRYN(conv32(src1(X), B, R, wf + d.enc1_t, wf + d.enc1_b, 64, 1, E1, 64, 0, 0, 0, R, st));
      LS_TRYN(ls_avgpool_f32(E1, P1, B, R, R, 64, st));
      for (int e = 0; e < 4; ++e) {
        const int l = L_ENC + 4 * e + 1;
        LS_TRYN(conv32(src1(part_f32(P1, 16, R2, 64, 16 * e, false)), B, R2, wf + d.conv_t[l], w + net.boff[l], 32,
                       1, E2, 128, 32 * e, 0, 0, R2, st));
      }
      LS_TRYN(ls_avgpool_f32(E2, P2, B, R2, R2, 128, st));
      for (int e = 0; e < 4; ++e) {
        const int l = L_ENC + 4 * e + 2;
        LS_TRYN(conv32(src1(part_f32(P2, 32, R4, 128, 32 * e, false)), B, R4, wf + d.conv_t[l], w + net.boff[l], 32,
                       1, E3, 128, 32 * e, 0, 0, R4, st));
      }
      LS_TRYN(ls_avgpool_f32(E3, P3, B, R4, R4, 128, st));
      for (int e = 0; e < 4; ++e) {
        const int l = L_ENC + 4 * e + 3;
        LS_TRYN(conv32(src1(part_f32(P3, 32, R8, 128, 32 * e, false)), B, R8, wf + d.conv_t[l], w + net.boff[l], 32,
                       1, E4, 128, 32 * e, 0, 0, R8, st));
      }
      LS_TRYN(ls_avgpool_f32(E4, Fe, B, R8, R8, 128, st));
      // merge
      LS_TRYN(fc_f32(Fe, wf + d.fc1_t, wf + d.fc1_b, Z, B, 512, (int)(4 * L), st));
      LS_TRYN(fc_f32(Z, wf + d.fc2_t, wf + d.fc2_b, D, B, (int)(2 * L), 512, st));
      // decoders (height: channel slice 0, texture: slice 1)
      for (int k = 0; k < 2; ++k) {
        const int l0 = k == 0 ? L_DECH : L_DECT;
        LS_TRYN(conv32(src1(part_f32(D, 32, R16, 64, 32 * k, true)), B, R8, wf + d.conv_t[l0], w + net.boff[l0], 32,
                       1, Dd1, 64, 32 * k, 0, 0, R8, st));
        LS_TRYN(conv32(src1(part_f32(Dd1, 32, R8, 64, 32 * k, true)), B, R4, wf + d.conv_t[l0 + 1],
                       w + net.boff[l0 + 1], 32, 1, Dd2, 64, 32 * k, 0, 0, R4, st));
        LS_TRYN(conv32(src1(part_f32(Dd2, 32, R4, 64, 32 * k, true)), B, R2, wf + d.conv_t[l0 + 2],
                       w + net.boff[l0 + 2], 16, 1, Dd3, 32, 16 * k, 0, 0, R2, st));
        LS_TRYN(conv32(src1(part_f32(Dd3, 16, R2, 32, 16 * k, true)), B, R, wf + d.conv_t[l0 + 3],
                       w + net.boff[l0 + 3], 16, 1, Aht, 32, 16 * k, wa.y0, wa.y0, wa.n, st));
      }
      // final CNN over [a_h, a_t, x], the last layer on the crop only (and
      // each earlier layer only where the next one reads it)
      ConvSrc s1;
      s1.a = window_part(part_f32(Aht, 32, wa.n, 32, 0, false), wa);
      s1.b = X;
      LS_TRYN(conv32(s1, B, R, wf + d.conv_t[L_FIN1], w + net.boff[L_FIN1], 32, 1, F1, 32, 0, w1.y0, w1.y0, w1.n, st));
      LS_TRYN(conv32(src1(window_part(part_f32(F1, 32, w1.n, 32, 0, false), w1)), B, R, wf + d.conv_t[L_FIN2],
                     w + net.boff[L_FIN2], 32, 1, F2, 32, 0, w2.y0, w2.y0, w2.n, st));
      LS_TRYN(conv32(src1(window_part(part_f32(F2, 32, w2.n, 32, 0, false), w2)), B, R, wf + d.conv_t[L_FIN3],
                     w + net.boff[L_FIN3], 4, 0, head, 4, 0, pad, pad, res, st));
    } else {
      uint16_t* A0 = act16;
      auto P = [&](int64_t off) { return A0 + off * B; };
      uint16_t *P1 = P(at.p1), *P2 = P(at.p2), *P3 = P(at.p3), *Fe = P(at.feat), *Z = P(at.z), *D = P(at.d),
               *Dd1 = P(at.dd1), *Dd2 = P(at.dd2), *Dd3 = P(at.dd3), *Aht = P(at.aht), *F1 = P(at.f1),
               *F2 = P(at.f2);
      // encoders: pooled outputs only
      LS_TRYN(conv16(src1(X), B, R, wb + d.enc1_p, 96, wf + d.enc1_b, 64, 1, nullptr, 64, 0, P1, 64, 0, nullptr, 0,
                     0, R, st));
      for (int e = 0; e < 4; ++e) {
        const int l = L_ENC + 4 * e + 1;
        LS_TRYN(conv16(src1(part_bf16(P1, 16, R2, 64, 16 * e, false)), B, R2, wb + d.conv_p[l], d.kpad[l],
                       w + net.boff[l], 32, 1, nullptr, 128, 0, P2, 128, 32 * e, nullptr, 0, 0, R2, st));
      }
      for (int e = 0; e < 4; ++e) {
        const int l = L_ENC + 4 * e + 2;
        LS_TRYN(conv16(src1(part_bf16(P2, 32, R4, 128, 32 * e, false)), B, R4, wb + d.conv_p[l], d.kpad[l],
                       w + net.boff[l], 32, 1, nullptr, 128, 0, P3, 128, 32 * e, nullptr, 0, 0, R4, st));
      }
      for (int e = 0; e < 4; ++e) {
        const int l = L_ENC + 4 * e + 3;
        LS_TRYN(conv16(src1(part_bf16(P3, 32, R8, 128, 32 * e, false)), B, R8, wb + d.conv_p[l], d.kpad[l],
                       w + net.boff[l], 32, 1, nullptr, 128, 0, Fe, 128, 32 * e, nullptr, 0, 0, R8, st));
      }
      LS_TRYN(fc_bf16(Fe, wb + d.fc1_p, wf + d.fc1_b, Z, B, 512, (int)(4 * L), st));
      LS_TRYN(fc_bf16(Z, wb + d.fc2_p, wf + d.fc2_b, D, B, (int)(2 * L), 512, st));
      for (int k = 0; k < 2; ++k) {
        const int l0 = k == 0 ? L_DECH : L_DECT;
        LS_TRYN(conv16(src1(part_bf16(D, 32, R16, 64, 32 * k, true)), B, R8, wb + d.conv_p[l0], d.kpad[l0],
                       w + net.boff[l0], 32, 1, Dd1, 64, 32 * k, nullptr, 0, 0, nullptr, 0, 0, R8, st));
        LS_TRYN(conv16(src1(part_bf16(Dd1, 32, R8, 64, 32 * k, true)), B, R4, wb + d.conv_p[l0 + 1],
                       d.kpad[l0 + 1], w + net.boff[l0 + 1], 32, 1, Dd2, 64, 32 * k, nullptr, 0, 0, nullptr, 0, 0,
                       R4, st));
        LS_TRYN(conv16(src1(part_bf16(Dd2, 32, R4, 64, 32 * k, true)), B, R2, wb + d.conv_p[l0 + 2],
                       d.kpad[l0 + 2], w + net.boff[l0 + 2], 16, 1, Dd3, 32, 16 * k, nullptr, 0, 0, nullptr, 0, 0,
                       R2, st));
        LS_TRYN(conv16(src1(part_bf16(Dd3, 16, R2, 32, 16 * k, true)), B, R, wb + d.conv_p[l0 + 3],
                       d.kpad[l0 + 3], w + net.boff[l0 + 3], 16, 1, Aht, 32, 16 * k, nullptr, 0, 0, nullptr, wa.y0,
                       wa.y0, wa.n, st));
      }
      ConvSrc s1;
      s1.a = window_part(part_bf16(Aht, 32, wa.n, 32, 0, false), wa);
      s1.b = X;
      LS_TRYN(conv16(s1, B, R, wb + d.conv_p[L_FIN1], d.kpad[L_FIN1], w + net.boff[L_FIN1], 32, 1, F1, 32, 0, nullptr,
                     0, 0, nullptr, w1.y0, w1.y0, w1.n, st));
      LS_TRYN(conv16(src1(window_part(part_bf16(F1, 32, w1.n, 32, 0, false), w1)), B, R, wb + d.conv_p[L_FIN2],
                     d.kpad[L_FIN2], w + net.boff[L_FIN2], 32, 1, F2, 32, 0, nullptr, 0, 0, nullptr, w2.y0, w2.y0,
                     w2.n, st));
      LS_TRYN(conv16(src1(window_part(part_bf16(F2, 32, w2.n, 32, 0, false), w2)), B, R, wb + d.conv_p[L_FIN3],
                     d.kpad[L_FIN3], w + net.boff[L_FIN3], 4, 0, nullptr, 4, 0, nullptr, 0, 0, head, pad, pad, res,
                     st));
    }
    {
      const int64_t ne = (int64_t)B * res * res;
      LS_TRACE("head_epilogue", st);
      hipLaunchKernelGGL(k_lsnet_epilogue, dim3((unsigned)((ne + 255) / 256)), dim3(256), 0, st, head, xc,
                         cz ? cz + t0 : nullptr, B, res, pad, r_m, inputs,
                         y_out ? y_out + (int64_t)t0 * res * res * 4 : nullptr,
                         tex_out ? tex_out + (int64_t)t0 * res * res * 4 : nullptr);
      LS_LAUNCH_CHECK();
    }
  }
  return LS_OK;
}
