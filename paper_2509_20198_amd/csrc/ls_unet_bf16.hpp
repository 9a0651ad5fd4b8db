// BF16 (matrix-core) path of the refinement network.
#pragma once

#include "ls_common.hpp"
#include "ls_unet.hpp"

// Packed BF16 weights: per layer [Npad][Kpad], Npad = cout rounded up to 16,
// Kpad = 9*cin rounded up to 32, k = tap*cin + ci, zero padding.
size_t ls_bf16_packed_offset(int layer);
size_t ls_bf16_packed_total();
int ls_bf16_kpad(int layer);

int ls_bf16_prep_weights(const uint16_t* w_bf16, uint16_t* packed, hipStream_t st);
// fuse: the activations are not kept (inference), so layer pairs may run
// fused without storing their first activation
int ls_bf16_forward(const float* w, const uint16_t* packed, const float* x, int B, const LsGridInfo& gi,
                    uint16_t* acts, float* head, bool fuse, hipStream_t st);
int ls_pack_bf16(const float* w, uint16_t* out, int64_t n, hipStream_t st);

// Backward helpers (BF16 operands, FP32 results).
size_t ls_bf16_dpacked_offset(int layer);
size_t ls_bf16_dpacked_total();
int ls_bf16_prep_dgrad_weights(const uint16_t* w_bf16, uint16_t* packed, hipStream_t st);
int ls_bf16_mask_round(const float* g, const uint16_t* act, uint16_t* out, int64_t n, hipStream_t st);
int ls_bf16_embed8(const float* g, uint16_t* out, int64_t npix, hipStream_t st);
// mask given: instead of FP32 `out`, write out_masked = BF16(dX where mask > 0, else 0)
int ls_bf16_dgrad(const ConvSrc& s, int B, int H, int layer, const uint16_t* dpacked, float* out, const uint16_t* mask,
                  uint16_t* out_masked, hipStream_t st);
// The input gradient with its channels split (LS_ENOTIMPL unless the
// persistent tile form runs): up_c > 0: channels [0, up_c) as the
// upsampling adjoint into up_out (FP32, half resolution), the others FP32
// into out (cin - up_c channels); else channels [0, split) masked by `mask`
// into out_masked (BF16, split channels), the others FP32 into out
// (cin - split channels; not computed when out is null).  n > 0 (up_c > 0
// only, y0 and n even): only the output window [y0, y0 + n)^2, out as
// [B][n][n] and up_out as [B][n/2][n/2] window tensors.
int ls_bf16_dgrad_split(const ConvSrc& s, int B, int H, int layer, const uint16_t* dpacked, float* out,
                        float* up_out, int up_c, const uint16_t* mask, uint16_t* out_masked, int split, hipStream_t st,
                        int y0 = 0, int n = 0);
// Windows of the full-resolution decoder level around the crop, where the
// head's output and its gradient reach (all clipped to the plane): the head
// input dA10 / A10 on the crop grown by one texel [h0, h0 + hn), dec1b's
// input dA9 / A9 by two [d0, d0 + dn).
struct Lvl1Win {
  int h0, hn, d0, dn;
};
inline Lvl1Win ls_lvl1_windows(int R, int pad, int res) {
  Lvl1Win w;
  w.h0 = pad - 1 > 0 ? pad - 1 : 0;
  const int h1 = pad + res + 1 < R ? pad + res + 1 : R;
  w.hn = h1 - w.h0;
  w.d0 = w.h0 - 1 > 0 ? w.h0 - 1 : 0;
  w.dn = (h1 + 1 < R ? h1 + 1 : R) - w.d0;
  return w;
}
// true when the BF16 forward that saves activations stores A9 and A10 as
// window tensors and the backward runs decoder level 1 on the windows: the
// input gradients of the head and dec1b use the persistent tile form
bool ls_bf16_lvl1_windowed();
// The input gradient on the output window [y0, y0 + n) x [x0, x0 + n) of
// the H x H plane: its first `split` channels masked by the activation
// `mask` into out_masked (BF16, [B][n][n][split]), the others FP32 into out2
// ([B][n][n][cin - split]) or not computed when out2 is null.  The mask is
// the window tensor [B][mask_n][mask_n][split] of the pixels [mask_o,
// mask_o + mask_n)^2, which must hold the output window.  Persistent tile
// form only (LS_ENOTIMPL otherwise).
int ls_bf16_dgrad_win(const ConvSrc& s, int B, int H, int layer, const uint16_t* dpacked, int y0, int x0, int n,
                      const uint16_t* mask, int mask_n, int mask_o, uint16_t* out_masked, int split, float* out2,
                      hipStream_t st);
int ls_bf16_mask_round_ex(const float* src, int stride, int coff, const uint16_t* act, const float* low, int B, int H,
                          int C, uint16_t* out, hipStream_t st, int sy0 = 0, int sn = 0);

// One 3x3 conv as 16 x 16 output tiles (LDS-staged input patch), the form
// every persistent BF16 conv launch takes.
struct ConvTileArgs {
  ConvSrc src;
  int B, H, W;           // input plane (zero padding outside)
  int y0, x0, Ho, Wo;    // output window inside the plane
  int tiles_x, tiles_y;  // output tiles per image
  const uint16_t* wp;    // packed weights [Npad][Kpad], k = tap*cin + ci
  int Kpad;
  const float* bias;
  int cout;
  int relu;
  uint16_t* out_bf16;    // [B][Ho][Wo][out_stride] at channel out_coff, or null
  float* out_f32;        // same layout, or null
  int out_stride, out_coff;
  uint16_t* pool_out;    // 2 x 2 average pool [B][Ho/2][Wo/2][pool_stride] at pool_coff, or null
  int pool_stride, pool_coff;
  const uint16_t* mask;  // BF16 output: zero where this activation (output layout) is not positive, or null
  // input-gradient splits (persistent form): channels below up_c summed
  // over 2 x 2 pixel blocks into up_out [B][Ho/2][Wo/2][up_c] (FP32), or
  // channels from split on written to out2_f32 [B][Ho][Wo][cout - split]
  float* up_out = nullptr;
  int up_c = 0;
  int split = 0;
  float* out2_f32 = nullptr;
  // a windowed output's mask read from a larger plane [B][mask_h][mask_w]
  // [out_stride], the window's pixel (0, 0) at (mask_y0, mask_x0); mask_w 0:
  // the mask has the output's layout (persistent form only)
  int mask_h = 0, mask_w = 0, mask_y0 = 0, mask_x0 = 0;
};

// Persistent pipelined BF16 conv (weights in LDS, next patch prefetched) on
// any ConvTileArgs whose input shape has a compiled form: nt 16-channel
// output tiles, part a with ca channels (nearest-upsampled if upa, FP32 if
// f32a), part b with cb channels (FP32 if f32b).  LS_ENOTIMPL otherwise.
int ls_bf16_conv_pipe(const ConvTileArgs& a, int nt, int ca, int cb, bool upa, bool f32a, bool f32b,
                      hipStream_t st, const char* trace = "conv_bf16");
