// Internal helpers shared by the HIP translation units of liblidarscout.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lidarscout.h"

#define LS_HOST_CHECK(expr)                     \
  do {                                          \
    hipError_t e_ = (expr);                     \
    if (e_ != hipSuccess) {                     \
      ls_set_last_error(e_, #expr, __LINE__);   \
      return LS_EHIP;                           \
    }                                           \
  } while (0)

#define LS_LAUNCH_CHECK()                                      \
  do {                                                         \
    hipError_t e_ = hipGetLastError();                         \
    if (e_ != hipSuccess) {                                    \
      ls_set_last_error(e_, "kernel launch", __LINE__);        \
      return LS_EHIP;                                          \
    }                                                          \
  } while (0)

void ls_set_last_error(hipError_t e, const char* what, int line);
void ls_set_last_message(const char* what);

// Optional launch timing: when enabled with ls_trace_enable(), a scope
// records a start event on `st` at construction and a stop event at the end
// of the scope, so the pair brackets the kernels the scope enqueues.
struct LsTrace {
  LsTrace(const char* name, hipStream_t st);
  ~LsTrace();
  int slot;
  hipStream_t st;
};
#define LS_TRACE_CAT2(a, b) a##b
#define LS_TRACE_CAT(a, b) LS_TRACE_CAT2(a, b)
#define LS_TRACE(name, st) LsTrace LS_TRACE_CAT(ls_trace_, __LINE__)(name, st)

static inline hipStream_t ls_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

static inline size_t ls_align(size_t v, size_t a = 256) { return (v + a - 1) / a * a; }

// Bump allocator over the caller's workspace.
struct LsArena {
  char* base;
  size_t size;
  size_t used;
  template <class T>
  T* take(size_t count) {
    size_t off = ls_align(used);
    used = off + ls_align(count * sizeof(T));
    return base ? reinterpret_cast<T*>(base + off) : nullptr;
  }
};

// Derived grid quantities (host side).
struct LsGridInfo {
  int64_t ox, oy;
  int32_t S, res, pad, tx, ty;
  int32_t C;   // texel size (raw)
  int32_t R;   // padded grid side
  int32_t H;   // half window (raw)
  double scale_xy, scale_z, offset_z;
};

static inline int ls_grid_info(const ls_grid* g, LsGridInfo* gi) {
  if (!g) return LS_EINVAL;
  if (g->tile_size <= 0 || g->res <= 0 || g->pad < 0 || g->tiles_x <= 0 || g->tiles_y <= 0) return LS_ERANGE;
  if (g->tile_size % g->res) return LS_ERANGE;
  const int32_t C = g->tile_size / g->res;
  if (C % 2) return LS_ERANGE;
  const int64_t R = (int64_t)g->res + 2 * (int64_t)g->pad;
  if (R % 4 || R > 4096) return LS_ERANGE;
  const int64_t H = (int64_t)g->tile_size / 2 + (int64_t)g->pad * C;
  // tile-local coordinates below 2^18 keep every predicate exact: orientations
  // below 2^39 in double, in-circle terms below 2^79 in int128
  if (H > 262143) return LS_ERANGE;
  // origins within 2^40 raw units keep point-to-origin differences exact in double
  const int64_t lim = (int64_t)1 << 40;
  if (g->origin_x < -lim || g->origin_x > lim || g->origin_y < -lim || g->origin_y > lim) return LS_ERANGE;
  gi->ox = g->origin_x;
  gi->oy = g->origin_y;
  gi->S = g->tile_size;
  gi->res = g->res;
  gi->pad = g->pad;
  gi->tx = g->tiles_x;
  gi->ty = g->tiles_y;
  gi->C = C;
  gi->R = (int32_t)R;
  gi->H = (int32_t)H;
  gi->scale_xy = g->scale_xy;
  gi->scale_z = g->scale_z;
  gi->offset_z = g->offset_z;
  return LS_OK;
}

// Shared U-Net description (HIP side).
struct LsLayer {
  int cin, cout;
};
static constexpr int LS_NLAYER = 11;
static constexpr LsLayer LS_LAYERS[LS_NLAYER] = {{8, 16},  {16, 16}, {16, 32}, {32, 32}, {32, 64}, {64, 64},
                                                 {96, 32}, {32, 32}, {48, 16}, {16, 16}, {24, 4}};
static inline size_t ls_layer_w_offset(int l) {
  size_t off = 0;
  for (int k = 0; k < l; ++k) off += (size_t)LS_LAYERS[k].cout * 9 * LS_LAYERS[k].cin + LS_LAYERS[k].cout;
  return off;
}
static inline size_t ls_layer_b_offset(int l) {
  return ls_layer_w_offset(l) + (size_t)LS_LAYERS[l].cout * 9 * LS_LAYERS[l].cin;
}
static constexpr int LS_NUM_PARAMS = 119844;

// Entry points implemented in separate translation units.
int ls_refine_forward_impl(const float* w, const uint16_t* w_bf16, int precision, const float* x, const double* cz,
                           int32_t n_tiles, const LsGridInfo& gi, float* y_out, float* tex_out, void* act_save,
                           void* ws, size_t ws_bytes, hipStream_t st);
int ls_refine_backward_impl(const float* w, const uint16_t* w_bf16, int precision, const float* x,
                            const void* act_save, const float* grad_y, int32_t n_tiles, const LsGridInfo& gi,
                            float* grad_w, float* grad_x, void* ws, size_t ws_bytes, hipStream_t st);
size_t ls_refine_ws_bytes(const LsGridInfo& gi, int32_t n_tiles, int precision, int backward);
size_t ls_refine_act_bytes(const LsGridInfo& gi, int32_t n_tiles, int precision);
size_t ls_recon_ws_bytes(const LsGridInfo& gi, int32_t n_tiles, int64_t n);
int ls_recon_impl(const LsGridInfo& gi, const int32_t* x, const int32_t* y, const int32_t* z, const uint16_t* rgb,
                  int64_t n, const int32_t* tile_list, int32_t n_tiles, int32_t order, float* x_out, double* cz_out,
                  int32_t* bin_off, int32_t* bin_idx, int64_t bin_cap, int32_t* tile_status, void* ws,
                  size_t ws_bytes, hipStream_t st);
int ls_recon_noalloc_impl(const LsGridInfo& gi, const int32_t* x, const int32_t* y, const int32_t* z,
                          const uint16_t* rgb, int64_t n, const int32_t* tile_list, int32_t n_tiles, int32_t order,
                          float* x_out, double* cz_out, int32_t* bin_off, int32_t* bin_idx, int64_t bin_cap,
                          int32_t* tile_status, hipStream_t st);
int ls_splat_impl(const LsGridInfo& gi, const int32_t* x, const int32_t* y, const int32_t* z, const uint16_t* rgb,
                  int64_t n, const int32_t* tile_slot, int32_t n_slots, uint64_t* keys, float* tex_inout,
                  uint64_t* n_dropped, hipStream_t st);
int ls_resolve_impl(const LsGridInfo& gi, const uint64_t* keys, int32_t n_slots, float* tex_inout, hipStream_t st);
int ls_splat_mean_impl(const LsGridInfo& gi, const int32_t* x, const int32_t* y, const int32_t* z,
                       const uint16_t* rgb, int64_t n, const int32_t* tile_slot, int32_t n_slots, int64_t* acc,
                       uint64_t* n_dropped, hipStream_t st);
int ls_resolve_mean_impl(const LsGridInfo& gi, const int64_t* acc, int32_t n_slots, float* tex, hipStream_t st);
size_t ls_loss_ws_bytes();
int ls_target_loss_impl(const float* y, const float* t, const double* cz, int32_t n_tiles, const LsGridInfo& gi,
                        int kind, double* loss_out, float* grad, void* ws, size_t ws_bytes, hipStream_t st);
int ls_raster_impl(const ls_view& v, const int32_t* x, const int32_t* y, const int32_t* z, const uint16_t* rgb,
                   int64_t n, uint64_t* fb, uint64_t* n_drawn, hipStream_t st);
int ls_raster_resolve_impl(const uint64_t* fb, int64_t n_pixels, uint32_t* rgba, hipStream_t st);
int64_t ls_lsnet_params(int R);
size_t ls_lsnet_ws_bytes(const LsGridInfo& gi, int32_t n_tiles, int precision);
int ls_lsnet_forward_impl(const float* w, int precision, int inputs, const float* x, const double* cz,
                          int32_t n_tiles, const LsGridInfo& gi, float* y_out, float* tex_out, void* ws,
                          size_t ws_bytes, hipStream_t st);
int ls_zero_f32(float* p, int64_t n, hipStream_t st);
int ls_conv_num_configs_impl(int layer, int precision, int pass);
int ls_conv_config_get(int layer, int precision, int pass);
int ls_conv_config_set(int layer, int precision, int pass, int config);
