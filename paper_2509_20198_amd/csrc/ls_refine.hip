// Host orchestration of the refinement network: workspace layout, the
// forward layer sequence and the backward (adjoint) sequence.
#include <algorithm>

#include "ls_common.hpp"
#include "ls_unet.hpp"
#include "ls_unet_bf16.hpp"

namespace {

enum { E1A, E1B, E2A, E2B, BA, BB, D2A, D2B, D1A, D1B, HEAD };

constexpr int WG_MAX_CHUNKS = 512;
constexpr int64_t MAX_LAYER_PARAMS = 64 * 9 * 64 + 64;

// Activation layout (per tile, in elements): A1 A2 P1 A3 A4 P2 A5 A6 A7 A8 A9 A10
struct Acts {
  int64_t off[12];
  int64_t per_tile;
};

Acts act_layout(int R) {
  const int64_t f = (int64_t)R * R, h = f / 4, q = f / 16;
  const int64_t sz[12] = {16 * f, 16 * f, 16 * h, 32 * h, 32 * h, 32 * q, 64 * q, 64 * q, 32 * h, 32 * h, 16 * f, 16 * f};
  Acts a;
  int64_t o = 0;
  for (int i = 0; i < 12; ++i) {
    a.off[i] = o;
    o += sz[i];
  }
  a.per_tile = o;
  return a;
}

enum { iA1, iA2, iP1, iA3, iA4, iP2, iA5, iA6, iA7, iA8, iA9, iA10 };

struct RefineWs {
  float* wt;
  float* wd;
  uint16_t* wbt;   // BF16 [tap][cin][cout] copies (BF16 path)
  void* acts;      // activations when the caller keeps none
  float* head;     // [B][res][res][4]
  // backward
  float *dXC, *dA10, *dA9, *dU1, *dA8, *dA2, *dA7, *dU2, *dA6, *dA4, *dA5, *dP2, *dA3, *dP1, *dA1;
  float* partial;
  // BF16 backward: turned weights, masked BF16 gradient, padded head gradient
  uint16_t* wdb;
  uint16_t* gz;
  uint16_t* gz2;
  uint16_t* gy8;
  uint16_t* xb;  // the network input rounded to BF16 (read by the weight gradients of its two consumers)
};

size_t refine_layout(const LsGridInfo& gi, int32_t B, int precision, int backward, bool need_acts, void* base,
                     RefineWs* W) {
  LsArena A{reinterpret_cast<char*>(base), 0, 0};
  const int R = gi.R, res = gi.res;
  const int64_t f = (int64_t)R * R, h = f / 4, q = f / 16;
  const Acts al = act_layout(R);
  const size_t esz = precision == LS_BF16 ? 2 : 4;
  W->wt = A.take<float>(LS_NUM_PARAMS);
  W->wd = A.take<float>(LS_NUM_PARAMS);
  W->wbt = A.take<uint16_t>(ls_bf16_packed_total());
  W->acts = need_acts ? (void*)A.take<char>((size_t)al.per_tile * B * esz) : nullptr;
  W->head = A.take<float>((int64_t)B * res * res * 4);
  if (backward) {
    W->dXC = A.take<float>(B * 24 * f);
    W->dA10 = A.take<float>(B * 16 * f);
    W->dA9 = A.take<float>(B * 16 * f);
    W->dU1 = A.take<float>(B * 48 * f);
    W->dA8 = A.take<float>(B * 32 * h);
    W->dA2 = A.take<float>(B * 16 * f);
    W->dA7 = A.take<float>(B * 32 * h);
    W->dU2 = A.take<float>(B * 96 * h);
    W->dA6 = A.take<float>(B * 64 * q);
    W->dA4 = A.take<float>(B * 32 * h);
    W->dA5 = A.take<float>(B * 64 * q);
    W->dP2 = A.take<float>(B * 32 * q);
    W->dA3 = A.take<float>(B * 32 * h);
    W->dP1 = A.take<float>(B * 16 * h);
    W->dA1 = A.take<float>(B * 16 * f);
    W->partial = A.take<float>(WG_MAX_CHUNKS * MAX_LAYER_PARAMS);
    if (precision == LS_BF16) {
      W->wdb = A.take<uint16_t>(ls_bf16_dpacked_total());
      W->gz = A.take<uint16_t>(B * 16 * f);
      W->gz2 = A.take<uint16_t>(B * 16 * f);
      W->gy8 = A.take<uint16_t>((int64_t)B * res * res * 8);
      W->xb = A.take<uint16_t>(B * 8 * f);
    }
  }
  return A.used;
}

#define LS_TRY(expr)            \
  do {                          \
    int rc_ = (expr);           \
    if (rc_ != LS_OK) return rc_; \
  } while (0)

ConvArgs conv_args(const ConvSrc& s, int B, int H, const float* wt, const float* w, int l, float* out, int relu) {
  ConvArgs a;
  a.src = s;
  a.B = B;
  a.H = H;
  a.W = H;
  a.y0 = 0;
  a.x0 = 0;
  a.Ho = H;
  a.Wo = H;
  a.wt = wt + ls_layer_w_offset(l);
  a.bias = w ? w + ls_layer_b_offset(l) : nullptr;
  a.cout = LS_LAYERS[l].cout;
  a.relu = relu;
  a.out = out;
  a.out_stride = a.cout;
  a.out_coff = 0;
  a.cob_max = ls_cob_for_config(ls_conv_config_get(l, LS_FP32, 0));
  return a;
}

ConvSrc one(SrcPart a) {
  ConvSrc s;
  s.a = a;
  s.b = src_none();
  return s;
}

ConvSrc two(SrcPart a, SrcPart b) {
  ConvSrc s;
  s.a = a;
  s.b = b;
  return s;
}

SrcPart up(SrcPart p) {
  p.up = 1;
  return p;
}

// FP32 forward through all layers; acts points at the FP32 activation block.
int forward_f32(const float* w, const float* wt, const float* x, int B, const LsGridInfo& gi, float* acts, float* head,
                hipStream_t st) {
  const int R = gi.R, R2 = R / 2, R4 = R / 4;
  const Acts al = act_layout(R);
  auto A = [&](int i) { return acts + al.off[i] * B; };
  auto P = [&](int i, int c, int hw) { return src_plain(A(i), c, hw, hw, c, 0, nullptr); };
  const SrcPart X = src_plain(x, 8, R, R, 8, 0, nullptr);
  LS_TRY(ls_conv_f32(conv_args(one(X), B, R, wt, w, E1A, A(iA1), 1), st));
  LS_TRY(ls_conv_f32(conv_args(one(P(iA1, 16, R)), B, R, wt, w, E1B, A(iA2), 1), st));
  LS_TRY(ls_avgpool_f32(A(iA2), A(iP1), B, R, R, 16, st));
  LS_TRY(ls_conv_f32(conv_args(one(P(iP1, 16, R2)), B, R2, wt, w, E2A, A(iA3), 1), st));
  LS_TRY(ls_conv_f32(conv_args(one(P(iA3, 32, R2)), B, R2, wt, w, E2B, A(iA4), 1), st));
  LS_TRY(ls_avgpool_f32(A(iA4), A(iP2), B, R2, R2, 32, st));
  LS_TRY(ls_conv_f32(conv_args(one(P(iP2, 32, R4)), B, R4, wt, w, BA, A(iA5), 1), st));
  LS_TRY(ls_conv_f32(conv_args(one(P(iA5, 64, R4)), B, R4, wt, w, BB, A(iA6), 1), st));
  LS_TRY(ls_conv_f32(conv_args(two(up(P(iA6, 64, R4)), P(iA4, 32, R2)), B, R2, wt, w, D2A, A(iA7), 1), st));
  LS_TRY(ls_conv_f32(conv_args(one(P(iA7, 32, R2)), B, R2, wt, w, D2B, A(iA8), 1), st));
  LS_TRY(ls_conv_f32(conv_args(two(up(P(iA8, 32, R2)), P(iA2, 16, R)), B, R, wt, w, D1A, A(iA9), 1), st));
  LS_TRY(ls_conv_f32(conv_args(one(P(iA9, 16, R)), B, R, wt, w, D1B, A(iA10), 1), st));
  ConvArgs h = conv_args(two(P(iA10, 16, R), X), B, R, wt, w, HEAD, head, 0);
  h.y0 = gi.pad;
  h.x0 = gi.pad;
  h.Ho = gi.res;
  h.Wo = gi.res;
  LS_TRY(ls_conv_f32(h, st));
  return LS_OK;
}

int wgrad(const ConvSrc& s, int B, int H, int l, const float* dA, const float* mask, int d_stride, int y0, int x0,
          int Ho, int Wo, float* grad_w, float* partial, hipStream_t st) {
  WgradArgs a;
  a.src = s;
  a.B = B;
  a.H = H;
  a.W = H;
  a.y0 = y0;
  a.x0 = x0;
  a.Ho = Ho;
  a.Wo = Wo;
  a.cout = LS_LAYERS[l].cout;
  a.dA = dA;
  a.mask = mask;
  a.g_bf16 = nullptr;
  a.d_stride = d_stride;
  a.round_in = 0;
  a.partial = partial;
  a.mfma = 0;
  const int64_t npix = (int64_t)B * Ho * Wo;
  const int chunks = ls_wgrad_chunks_for_config(ls_conv_config_get(l, LS_FP32, 2));
  a.nchunk = (int)std::max<int64_t>(1, std::min<int64_t>(chunks, npix / 256));
  return ls_wgrad_f32(a, grad_w + ls_layer_w_offset(l), st);
}

// BF16 path: the gradient is the pre-masked BF16 tensor g (d_stride
// channels per pixel); FP32-stored inputs are rounded to BF16 on load.
int wgrad_bf16(const ConvSrc& s, int B, int H, int l, const uint16_t* g, int d_stride, int y0, int x0, int Ho, int Wo,
               float* grad_w, float* partial, hipStream_t st) {
  WgradArgs a;
  a.src = s;
  a.B = B;
  a.H = H;
  a.W = H;
  a.y0 = y0;
  a.x0 = x0;
  a.Ho = Ho;
  a.Wo = Wo;
  a.cout = LS_LAYERS[l].cout;
  a.dA = nullptr;
  a.mask = nullptr;
  a.g_bf16 = g;
  a.d_stride = d_stride;
  a.round_in = 1;
  a.partial = partial;
  // configs 0-2: vector units, 3-5: matrix cores on im2col slabs, 6-8:
  // matrix cores on 16 x 16 output tiles (up to 32 output channels; the
  // default where it applies)
  const int cfg = ls_conv_config_get(l, LS_BF16, 2);
  const bool tile_ok = a.cout <= 32;
  a.mfma = cfg < 0 ? (tile_ok ? 2 : 1) : (cfg >= 6 ? (tile_ok ? 2 : 1) : (cfg >= 3 ? 1 : 0));
  const int64_t npix = (int64_t)B * Ho * Wo;
  // default: 512 pixel chunks, 256 for layers with many weights on planes
  // below about 1.5 M pixels (measured on 256 tiles: there the partial sums,
  // 4 bytes per weight and chunk, cost more than the parallelism gains)
  const int64_t nw = (int64_t)a.cout * 9 * (s.a.c + s.b.c);
  const int chunks = cfg >= 0 ? ls_wgrad_chunks_for_config(cfg) : (npix < ((int64_t)3 << 19) && nw >= 6000 ? 256 : 512);
  a.nchunk = (int)std::max<int64_t>(1, std::min<int64_t>(chunks, npix / 256));
  return ls_wgrad_f32(a, grad_w + ls_layer_w_offset(l), st);
}

SrcPart bsrc(const uint16_t* p, int c, int hw) {
  SrcPart s = src_none();
  s.bf16 = p;
  s.c = c;
  s.h = hw;
  s.w = hw;
  s.stride = c;
  return s;
}

// dgrad of layer l: out = conv(dA masked by A, flipped/transposed weights)
int dgrad(const float* wd, int l, const float* dA, const float* mask, int B, int H, float* out, hipStream_t st) {
  const int cout = LS_LAYERS[l].cout, cin = LS_LAYERS[l].cin;
  ConvArgs a;
  a.src = one(src_plain(dA, cout, H, H, cout, 0, mask));
  a.B = B;
  a.H = H;
  a.W = H;
  a.y0 = 0;
  a.x0 = 0;
  a.Ho = H;
  a.Wo = H;
  a.wt = wd + ls_layer_w_offset(l);
  a.bias = nullptr;
  a.cout = cin;
  a.relu = 0;
  a.out = out;
  a.out_stride = cin;
  a.out_coff = 0;
  a.cob_max = ls_cob_for_config(ls_conv_config_get(l, LS_FP32, 1));
  return ls_conv_f32(a, st);
}

int backward_f32(const float* w, const float* wd, const float* x, const float* acts, const float* grad_y, int B,
                 const LsGridInfo& gi, float* grad_w, float* grad_x, const RefineWs& W, hipStream_t st) {
  const int R = gi.R, R2 = R / 2, R4 = R / 4, res = gi.res, pad = gi.pad;
  const int64_t f = (int64_t)R * R;
  const Acts al = act_layout(R);
  auto A = [&](int i) { return acts + al.off[i] * B; };
  auto P = [&](int i, int c, int hw) { return src_plain(A(i), c, hw, hw, c, 0, nullptr); };
  const SrcPart X = src_plain(x, 8, R, R, 8, 0, nullptr);
  // head: dXC = dgrad over the full plane of dY embedded at the crop
  {
    ConvArgs a;
    SrcPart g = src_plain(grad_y, 4, res, res, 4, 0, nullptr);
    g.oy = pad;
    g.ox = pad;
    a.src = one(g);
    a.B = B;
    a.H = R;
    a.W = R;
    a.y0 = 0;
    a.x0 = 0;
    a.Ho = R;
    a.Wo = R;
    a.wt = wd + ls_layer_w_offset(HEAD);
    a.bias = nullptr;
    a.cout = 24;
    a.relu = 0;
    a.out = W.dXC;
    a.out_stride = 24;
    a.out_coff = 0;
    a.cob_max = ls_cob_for_config(ls_conv_config_get(HEAD, LS_FP32, 1));
    LS_TRY(ls_conv_f32(a, st));
  }
  LS_TRY(wgrad(two(P(iA10, 16, R), X), B, R, HEAD, grad_y, nullptr, 4, pad, pad, res, res, grad_w, W.partial, st));
  LS_TRY(ls_copy_channels(W.dXC, 24, 0, W.dA10, 16, B * f, 0, st));
  // decoder level 1
  LS_TRY(wgrad(one(P(iA9, 16, R)), B, R, D1B, W.dA10, A(iA10), 16, 0, 0, R, R, grad_w, W.partial, st));
  LS_TRY(dgrad(wd, D1B, W.dA10, A(iA10), B, R, W.dA9, st));
  LS_TRY(wgrad(two(up(P(iA8, 32, R2)), P(iA2, 16, R)), B, R, D1A, W.dA9, A(iA9), 16, 0, 0, R, R, grad_w, W.partial, st));
  LS_TRY(dgrad(wd, D1A, W.dA9, A(iA9), B, R, W.dU1, st));
  LS_TRY(ls_up_adjoint(W.dU1, 48, W.dA8, B, R2, R2, 32, st));
  LS_TRY(ls_copy_channels(W.dU1, 48, 32, W.dA2, 16, B * f, 0, st));
  // decoder level 2
  LS_TRY(wgrad(one(P(iA7, 32, R2)), B, R2, D2B, W.dA8, A(iA8), 32, 0, 0, R2, R2, grad_w, W.partial, st));
  LS_TRY(dgrad(wd, D2B, W.dA8, A(iA8), B, R2, W.dA7, st));
  LS_TRY(wgrad(two(up(P(iA6, 64, R4)), P(iA4, 32, R2)), B, R2, D2A, W.dA7, A(iA7), 32, 0, 0, R2, R2, grad_w, W.partial,
               st));
  LS_TRY(dgrad(wd, D2A, W.dA7, A(iA7), B, R2, W.dU2, st));
  LS_TRY(ls_up_adjoint(W.dU2, 96, W.dA6, B, R4, R4, 64, st));
  LS_TRY(ls_copy_channels(W.dU2, 96, 64, W.dA4, 32, B * f / 4, 0, st));
  // bottleneck
  LS_TRY(wgrad(one(P(iA5, 64, R4)), B, R4, BB, W.dA6, A(iA6), 64, 0, 0, R4, R4, grad_w, W.partial, st));
  LS_TRY(dgrad(wd, BB, W.dA6, A(iA6), B, R4, W.dA5, st));
  LS_TRY(wgrad(one(P(iP2, 32, R4)), B, R4, BA, W.dA5, A(iA5), 64, 0, 0, R4, R4, grad_w, W.partial, st));
  LS_TRY(dgrad(wd, BA, W.dA5, A(iA5), B, R4, W.dP2, st));
  LS_TRY(ls_pool_adjoint_add(W.dP2, W.dA4, B, R2, R2, 32, st));
  // encoder level 2
  LS_TRY(wgrad(one(P(iA3, 32, R2)), B, R2, E2B, W.dA4, A(iA4), 32, 0, 0, R2, R2, grad_w, W.partial, st));
  LS_TRY(dgrad(wd, E2B, W.dA4, A(iA4), B, R2, W.dA3, st));
  LS_TRY(wgrad(one(P(iP1, 16, R2)), B, R2, E2A, W.dA3, A(iA3), 32, 0, 0, R2, R2, grad_w, W.partial, st));
  LS_TRY(dgrad(wd, E2A, W.dA3, A(iA3), B, R2, W.dP1, st));
  LS_TRY(ls_pool_adjoint_add(W.dP1, W.dA2, B, R, R, 16, st));
  // encoder level 1
  LS_TRY(wgrad(one(P(iA1, 16, R)), B, R, E1B, W.dA2, A(iA2), 16, 0, 0, R, R, grad_w, W.partial, st));
  LS_TRY(dgrad(wd, E1B, W.dA2, A(iA2), B, R, W.dA1, st));
  LS_TRY(wgrad(one(X), B, R, E1A, W.dA1, A(iA1), 16, 0, 0, R, R, grad_w, W.partial, st));
  if (grad_x) {
    // grad_x = dgrad(e1a) + head input part + residual
    LS_TRY(dgrad(wd, E1A, W.dA1, A(iA1), B, R, grad_x, st));
    LS_TRY(ls_copy_channels(W.dXC, 24, 16, grad_x, 8, B * f, 1, st));
    LS_TRY(ls_residual_adjoint(grad_y, grad_x, B, res, pad, st));
  }
  return LS_OK;
}

// BF16 backward: activations saved in BF16, every conv product (input and
// weight gradients on the matrix cores) takes BF16 operands with FP32
// accumulation.  The gradient at a layer's output is masked by its
// activation (ReLU') and rounded to BF16 once, as the operand of both
// products: where the layer above is a plain conv, by the epilogue of that
// layer's input-gradient conv; where it is a concatenation, an upsampling or
// a pool, by one pass that also reads the channel slice and adds the pool
// adjoint.  Gradients between those steps stay FP32.
int backward_bf16(const float* x, const uint16_t* acts, const float* grad_y, int B, const LsGridInfo& gi,
                  float* grad_w, float* grad_x, const RefineWs& W, hipStream_t st) {
  const int R = gi.R, R2 = R / 2, R4 = R / 4, res = gi.res, pad = gi.pad;
  const int64_t f = (int64_t)R * R;
  const Acts al = act_layout(R);
  auto A = [&](int i) { return acts + al.off[i] * B; };
  auto P = [&](int i, int c, int hw) { return bsrc(A(i), c, hw); };
  uint16_t* const g0 = W.gz;
  uint16_t* const g1 = W.gz2;
  auto wg = [&](int l, const uint16_t* g, const ConvSrc& in, int H) -> int {
    return wgrad_bf16(in, B, H, l, g, LS_LAYERS[l].cout, 0, 0, H, H, grad_w, W.partial, st);
  };
  // input gradient of layer l from its masked BF16 output gradient g: FP32
  // into dX, or masked by activation `act_below` into the BF16 buffer gb
  auto dg = [&](int l, const uint16_t* g, int H, float* dX, int act_below, uint16_t* gb) -> int {
    return ls_bf16_dgrad(one(bsrc(g, LS_LAYERS[l].cout, H)), B, H, l, W.wdb, dX,
                         act_below >= 0 ? A(act_below) : nullptr, gb, st);
  };
  // head: gradient embedded at the crop, padded to 8 channels.  Its input
  // gradient's first 16 channels (dA10) are masked and rounded in the
  // epilogue when the persistent form runs; the last 8 (the gradient of the
  // input skip) stay FP32, in dXC with xc_stride channels from xc_off.
  LS_TRY(ls_bf16_embed8(grad_y, W.gy8, (int64_t)B * res * res, st));
  // x in BF16 once (the rounding the weight-gradient staging would apply)
  {
    LS_TRACE("embed8", st);
    LS_TRY(ls_pack_bf16(x, W.xb, B * f * 8, st));
  }
  const SrcPart XB = bsrc(W.xb, 8, R);
  int xc_stride = 8, xc_off = 0;
  SrcPart u8 = P(iA8, 32, R2);
  u8.up = 1;
  SrcPart gy = bsrc(W.gy8, 8, res);
  gy.oy = pad;
  gy.ox = pad;
  // The gradients of decoder level 1 are computed only where they can be
  // nonzero: the head's output gradient lives on the crop, so dA10 on the
  // crop grown by one texel and dA9 by two (clipped to the plane), stored as
  // window tensors, with the ReLU masks A10 and A9 that the forward saved on
  // the same windows; their weight gradients sum over those windows only.
  const Lvl1Win lw = ls_lvl1_windows(R, pad, res);
  const int h0 = lw.h0, hn = lw.hn, d0 = lw.d0, dn = lw.dn, d1 = d0 + dn;
  SrcPart g1src = bsrc(g1, 16, R);
  const bool windowed = ls_bf16_lvl1_windowed();
  if (windowed) {
    SrcPart a9 = P(iA9, 16, dn), a10 = P(iA10, 16, hn);
    a9.oy = a9.ox = d0;
    a10.oy = a10.ox = h0;
    // dA10 and, for grad_x, the input skip's 8 channels (FP32 window tensor)
    int rc = ls_bf16_dgrad_win(one(gy), B, R, HEAD, W.wdb, h0, h0, hn, A(iA10), hn, h0, g0, 16,
                               grad_x ? W.dXC : nullptr, st);
    LS_TRY(rc);
    SrcPart g0w = bsrc(g0, 16, hn);
    g0w.oy = g0w.ox = h0;
    rc = ls_bf16_dgrad_win(one(g0w), B, R, D1B, W.wdb, d0, d0, dn, A(iA9), dn, d0, g1, 16, nullptr, st);
    LS_TRY(rc);
    LS_TRY(wgrad_bf16(two(a10, XB), B, R, HEAD, W.gy8, 8, pad, pad, res, res, grad_w, W.partial, st));
    LS_TRY(wgrad_bf16(one(a9), B, R, D1B, g0, 16, h0, h0, hn, hn, grad_w, W.partial, st));
    LS_TRY(wgrad_bf16(two(u8, P(iA2, 16, R)), B, R, D1A, g1, 16, d0, d0, dn, dn, grad_w, W.partial, st));
    g1src = bsrc(g1, 16, dn);
    g1src.oy = g1src.ox = d0;
  } else {
    // the last 8 channels only feed grad_x: without it, only dA10 is computed
    const int rc =
        ls_bf16_dgrad_split(one(gy), B, R, HEAD, W.wdb, grad_x ? W.dXC : nullptr, nullptr, 0, A(iA10), g0, 16, st);
    if (rc == LS_ENOTIMPL) {
      LS_TRY(ls_bf16_dgrad(one(gy), B, R, HEAD, W.wdb, W.dXC, nullptr, nullptr, st));
      // decoder level 1: dA10 is the first 16 of the head input's 24 channels
      LS_TRY(ls_bf16_mask_round_ex(W.dXC, 24, 0, A(iA10), nullptr, B, R, 16, g0, st));
      xc_stride = 24;
      xc_off = 16;
    } else {
      LS_TRY(rc);
    }
    LS_TRY(wgrad_bf16(two(P(iA10, 16, R), XB), B, R, HEAD, W.gy8, 8, pad, pad, res, res, grad_w, W.partial, st));
    LS_TRY(wg(D1B, g0, one(P(iA9, 16, R)), R));
    LS_TRY(dg(D1B, g0, R, nullptr, iA9, g1));
    LS_TRY(wg(D1A, g1, two(u8, P(iA2, 16, R)), R));
  }
  // dU1: the upsampled part's 32 channels go straight to their upsampling
  // adjoint dA8 when the persistent form runs, the skip part's 16 stay in
  // dU1 (u1_stride channels from u1_off)
  int u1_stride = 16, u1_off = 0;
  // with the windows, dU1 and its upsampling adjoint dA8 too are computed
  // only where dA9 reaches (window origin and size even for the 2 x 2 sums)
  int u0 = 0, un = 0;
  if (windowed) {
    u0 = std::max(0, d0 - 1) & ~1;
    un = std::min(R, (d1 + 2) & ~1) - u0;
  }
  {
    int rc = LS_ENOTIMPL;
    if (windowed) {
      rc = ls_bf16_dgrad_split(one(g1src), B, R, D1A, W.wdb, W.dU1, W.dA8, 32, nullptr, nullptr, 0, st, u0, un);
      if (rc == LS_ENOTIMPL) un = 0;
    }
    if (!windowed || rc == LS_ENOTIMPL)
      rc = ls_bf16_dgrad_split(one(g1src), B, R, D1A, W.wdb, W.dU1, W.dA8, 32, nullptr, nullptr, 0, st);
    if (rc == LS_ENOTIMPL) {
      LS_TRY(ls_bf16_dgrad(one(g1src), B, R, D1A, W.wdb, W.dU1, nullptr, nullptr, st));
      LS_TRY(ls_up_adjoint(W.dU1, 48, W.dA8, B, R2, R2, 32, st));
      u1_stride = 48;
      u1_off = 32;
    } else {
      LS_TRY(rc);
    }
  }
  // decoder level 2
  LS_TRY(ls_bf16_mask_round_ex(W.dA8, 32, 0, A(iA8), nullptr, B, R2, 32, g0, st, u0 / 2, un / 2));
  LS_TRY(wg(D2B, g0, one(P(iA7, 32, R2)), R2));
  LS_TRY(dg(D2B, g0, R2, nullptr, iA7, g1));
  SrcPart u6 = P(iA6, 64, R4);
  u6.up = 1;
  LS_TRY(wg(D2A, g1, two(u6, P(iA4, 32, R2)), R2));
  int u2_stride = 32, u2_off = 0;
  {
    const int rc = ls_bf16_dgrad_split(one(bsrc(g1, 32, R2)), B, R2, D2A, W.wdb, W.dU2, W.dA6, 64, nullptr, nullptr,
                                       0, st);
    if (rc == LS_ENOTIMPL) {
      LS_TRY(dg(D2A, g1, R2, W.dU2, -1, nullptr));
      LS_TRY(ls_up_adjoint(W.dU2, 96, W.dA6, B, R4, R4, 64, st));
      u2_stride = 96;
      u2_off = 64;
    } else {
      LS_TRY(rc);
    }
  }
  // bottleneck
  LS_TRY(ls_bf16_mask_round_ex(W.dA6, 64, 0, A(iA6), nullptr, B, R4, 64, g0, st));
  LS_TRY(wg(BB, g0, one(P(iA5, 64, R4)), R4));
  LS_TRY(dg(BB, g0, R4, nullptr, iA5, g1));
  LS_TRY(wg(BA, g1, one(P(iP2, 32, R4)), R4));
  LS_TRY(dg(BA, g1, R4, W.dP2, -1, nullptr));
  // encoder level 2: dA4 = skip slice of dU2 + pool adjoint of dP2
  LS_TRY(ls_bf16_mask_round_ex(W.dU2, u2_stride, u2_off, A(iA4), W.dP2, B, R2, 32, g0, st));
  LS_TRY(wg(E2B, g0, one(P(iA3, 32, R2)), R2));
  LS_TRY(dg(E2B, g0, R2, nullptr, iA3, g1));
  LS_TRY(wg(E2A, g1, one(P(iP1, 16, R2)), R2));
  LS_TRY(dg(E2A, g1, R2, W.dP1, -1, nullptr));
  // encoder level 1: dA2 = skip slice of dU1 + pool adjoint of dP1
  LS_TRY(ls_bf16_mask_round_ex(W.dU1, u1_stride, u1_off, A(iA2), W.dP1, B, R, 16, g0, st, u0, un));
  LS_TRY(wg(E1B, g0, one(P(iA1, 16, R)), R));
  LS_TRY(dg(E1B, g0, R, nullptr, iA1, g1));
  LS_TRY(wg(E1A, g1, one(XB), R));
  if (grad_x) {
    LS_TRY(dg(E1A, g1, R, grad_x, -1, nullptr));
    if (windowed)
      LS_TRY(ls_add_window(W.dXC, hn, h0, grad_x, R, B, 8, st));
    else
      LS_TRY(ls_copy_channels(W.dXC, xc_stride, xc_off, grad_x, 8, B * f, 1, st));
    LS_TRY(ls_residual_adjoint(grad_y, grad_x, B, res, pad, st));
  }
  return LS_OK;
}

}  // namespace

size_t ls_refine_act_bytes(const LsGridInfo& gi, int32_t n_tiles, int precision) {
  return (size_t)act_layout(gi.R).per_tile * n_tiles * (precision == LS_BF16 ? 2 : 4);
}

size_t ls_refine_ws_bytes(const LsGridInfo& gi, int32_t n_tiles, int precision, int backward) {
  RefineWs W;
  return refine_layout(gi, n_tiles, precision, backward, true, nullptr, &W);
}

int ls_refine_forward_impl(const float* w, const uint16_t* w_bf16, int precision, const float* x, const double* cz,
                           int32_t n_tiles, const LsGridInfo& gi, float* y_out, float* tex_out, void* act_save,
                           void* ws, size_t ws_bytes, hipStream_t st) {
  if (n_tiles <= 0) return LS_OK;
  RefineWs W;
  const size_t need = refine_layout(gi, n_tiles, precision, 0, act_save == nullptr, nullptr, &W);
  if (!ws || ws_bytes < need) return LS_EWORKSPACE;
  refine_layout(gi, n_tiles, precision, 0, act_save == nullptr, ws, &W);
  void* acts = act_save ? act_save : W.acts;
  const double r_m = (double)gi.H * gi.scale_xy;
  if (precision == LS_FP32) {
    LS_TRY(ls_prep_weights(w, W.wt, W.wd, st));
    LS_TRY(forward_f32(w, W.wt, x, n_tiles, gi, reinterpret_cast<float*>(acts), W.head, st));
  } else {
    LS_TRY(ls_bf16_prep_weights(w_bf16, W.wbt, st));
    LS_TRY(ls_bf16_forward(w, W.wbt, x, n_tiles, gi, reinterpret_cast<uint16_t*>(acts), W.head, act_save == nullptr,
                           st));
  }
  return ls_head_epilogue(W.head, x, cz, n_tiles, gi.res, gi.pad, r_m, y_out, tex_out, st);
}

int ls_refine_backward_impl(const float* w, const uint16_t* w_bf16, int precision, const float* x,
                            const void* act_save, const float* grad_y, int32_t n_tiles, const LsGridInfo& gi,
                            float* grad_w, float* grad_x, void* ws, size_t ws_bytes, hipStream_t st) {
  if (n_tiles <= 0) return ls_zero_f32(grad_w, LS_NUM_PARAMS, st);
  RefineWs W;
  const size_t need = refine_layout(gi, n_tiles, precision, 1, act_save == nullptr, nullptr, &W);
  if (!ws || ws_bytes < need) return LS_EWORKSPACE;
  refine_layout(gi, n_tiles, precision, 1, act_save == nullptr, ws, &W);
  if (precision == LS_FP32) {
    LS_TRY(ls_prep_weights(w, W.wt, W.wd, st));
    const float* acts = reinterpret_cast<const float*>(act_save);
    if (!acts) {
      LS_TRY(forward_f32(w, W.wt, x, n_tiles, gi, reinterpret_cast<float*>(W.acts), W.head, st));
      acts = reinterpret_cast<const float*>(W.acts);
    }
    return backward_f32(w, W.wd, x, acts, grad_y, n_tiles, gi, grad_w, grad_x, W, st);
  }
  LS_TRY(ls_bf16_prep_weights(w_bf16, W.wbt, st));
  LS_TRY(ls_bf16_prep_dgrad_weights(w_bf16, W.wdb, st));
  const uint16_t* acts = reinterpret_cast<const uint16_t*>(act_save);
  if (!acts) {
    LS_TRY(ls_bf16_forward(w, W.wbt, x, n_tiles, gi, reinterpret_cast<uint16_t*>(W.acts), W.head, false, st));
    acts = reinterpret_cast<const uint16_t*>(W.acts);
  }
  return backward_bf16(x, acts, grad_y, n_tiles, gi, grad_w, grad_x, W, st);
}
