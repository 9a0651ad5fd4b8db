// Internal interfaces of the refinement-network kernels.
#pragma once

#include "ls_common.hpp"

// One stored tensor seen as (part of) a conv input.
struct SrcPart {
  const float* f32;      // FP32 storage (FP32 path, and the network input x)
  const uint16_t* bf16;  // BF16 storage (BF16 path); exactly one of f32/bf16 is set
  const float* mask;     // FP32 backward: zero the value where mask <= 0 (same layout)
  int c;                 // channels taken from this part
  int h, w;              // stored spatial size
  int stride;            // channels per stored pixel
  int coff;              // first channel within the stored pixel
  int up;                // nearest x2 upsampling: stored at half resolution
  int oy, ox;            // embedding: stored (sy, sx) sits at input (sy + oy, sx + ox)
};

// Conv input: channels [0, a.c) from part a, [a.c, a.c + b.c) from part b.
struct ConvSrc {
  SrcPart a, b;
};

struct ConvArgs {
  ConvSrc src;
  int B, H, W;           // batch and input plane (zero padding outside)
  int y0, x0, Ho, Wo;    // output window inside the plane
  const float* wt;       // [9][cin][cout] weights of this layer
  const float* bias;     // [cout] or null
  int cout;
  int relu;
  float* out;            // [B][Ho][Wo][out_stride]
  int out_stride, out_coff;
  int cob_max;           // largest output-channel block per thread (32, 16, 8 or 4)
};

struct WgradArgs {
  ConvSrc src;
  int B, H, W;
  int y0, x0, Ho, Wo;
  int cout;
  const float* dA;          // gradient at the conv output, [B][Ho][Wo][d_stride]
  const float* mask;        // FP32 forward activation (ReLU mask) or null, same layout
  const uint16_t* g_bf16;   // instead of dA/mask: the masked gradient already rounded to BF16
  int d_stride;
  int round_in;             // round FP32-stored inputs to BF16 (BF16 path)
  float* partial;           // [nchunk][cout*9*cin + cout]
  int nchunk;
  int mfma;                 // BF16 gradient only: 1 the matrix-core im2col kernel, 2 the tile kernel
};

// Tiling choices per (layer, precision, pass), set by ls_set_conv_config.
int ls_conv_config_get(int layer, int precision, int pass);
// FP32 conv: config 0..3 -> channel block cap 32, 16, 8, 4
inline int ls_cob_for_config(int c) { return c <= 0 ? 32 : (c == 1 ? 16 : (c == 2 ? 8 : 4)); }
// weight gradient: config 0..2 -> pixel chunks 512, 256, 128 (vector FP32
// products); BF16 also 3..5 -> the same chunk counts on the matrix cores
inline int ls_wgrad_chunks_for_config(int c) {
  const int k = c < 0 ? 0 : c % 3;
  return k == 0 ? 512 : (k == 1 ? 256 : 128);
}

SrcPart src_plain(const float* p, int c, int h, int w, int stride, int coff, const float* mask);
SrcPart src_none();

int ls_conv_f32(const ConvArgs& a, hipStream_t st);
int ls_avgpool_f32(const float* in, float* out, int B, int H, int W, int C, hipStream_t st);
int ls_head_epilogue(const float* head, const float* x, const double* cz, int B, int res, int pad, double r_m,
                     float* y_out, float* tex_out, hipStream_t st);
int ls_prep_weights(const float* w, float* wt, float* wd, hipStream_t st);
int ls_wgrad_f32(const WgradArgs& a, float* grad_w_layer, hipStream_t st);
int ls_up_adjoint(const float* dhigh, int stride, float* dlow, int B, int h, int w, int c_low, hipStream_t st);
int ls_copy_channels(const float* src, int stride, int coff, float* dst, int C, int64_t npix, int acc, hipStream_t st);
// dst [B][H][H][C] += src, the window tensor [B][n][n][C] of the pixels [y0, y0 + n)^2
int ls_add_window(const float* src, int n, int y0, float* dst, int H, int B, int C, hipStream_t st);
int ls_pool_adjoint_add(const float* dlow, float* dhigh, int B, int H, int W, int C, hipStream_t st);
int ls_residual_adjoint(const float* dy, float* dx, int B, int res, int pad, hipStream_t st);
