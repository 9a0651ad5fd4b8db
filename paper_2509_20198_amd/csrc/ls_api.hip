// C-ABI entry points of liblidarscout (declared in include/lidarscout.h):
// argument validation on the host, then the enqueue functions of the other
// translation units.
#include <stdio.h>
#include <string.h>

#include "ls_common.hpp"
#include "ls_unet_bf16.hpp"

namespace {

thread_local char g_last_error[256] = "";

__global__ void k_zero_f32(float* __restrict__ p, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0.f;
}

// per (layer, precision, pass) selected conv tiling; -1 = default
int g_conv_cfg[LS_NLAYER][2][3] = {};
bool g_conv_cfg_init = false;

void cfg_init() {
  if (g_conv_cfg_init) return;
  for (int l = 0; l < LS_NLAYER; ++l)
    for (int p = 0; p < 2; ++p)
      for (int q = 0; q < 3; ++q) g_conv_cfg[l][p][q] = -1;
  g_conv_cfg_init = true;
}

constexpr int TRACE_MAX = 16384;
bool g_trace_on = false;
bool g_trace_init = false;
int g_trace_n = 0;
hipEvent_t g_trace_ev[2 * TRACE_MAX];
const char* g_trace_name[TRACE_MAX];

}  // namespace

LsTrace::LsTrace(const char* name, hipStream_t s) : slot(-1), st(s) {
  if (!g_trace_on || g_trace_n >= TRACE_MAX) return;
  slot = g_trace_n++;
  g_trace_name[slot] = name;
  (void)hipEventRecord(g_trace_ev[2 * slot], st);
}

LsTrace::~LsTrace() {
  if (slot >= 0) (void)hipEventRecord(g_trace_ev[2 * slot + 1], st);
}

void ls_set_last_error(hipError_t e, const char* what, int line) {
  snprintf(g_last_error, sizeof(g_last_error), "%s (%d) at %s, line %d", hipGetErrorString(e), (int)e, what, line);
}

void ls_set_last_message(const char* what) { snprintf(g_last_error, sizeof(g_last_error), "%s", what); }

int ls_zero_f32(float* p, int64_t n, hipStream_t st) {
  if (n <= 0) return LS_OK;
  const int blocks = (int)((n + 255) / 256 < 4096 ? (n + 255) / 256 : 4096);
  hipLaunchKernelGGL(k_zero_f32, dim3(blocks), dim3(256), 0, st, p, n);
  LS_LAUNCH_CHECK();
  return LS_OK;
}

int ls_conv_num_configs_impl(int layer, int precision, int pass) {
  if (layer < 0 || layer >= LS_NLAYER || precision < 0 || precision > 1 || pass < 0 || pass > 2) return 0;
  // BF16 forward: 0 = direct operand fetch (4 pixel tiles per wave),
  //   1 = LDS-staged 16x16 tile, 2 = direct with 2 pixel tiles per wave,
  //   3 = LDS tile in persistent workgroups prefetching the next patch;
  //   enc1b and the head also 4 = fused with the layer before them when the
  //   activations are not kept (the head's default)
  // BF16 input gradient: 0 / 1 = direct with 4 / 2 pixel tiles per wave,
  //   2 = persistent LDS tile (the default)
  // FP32 conv (forward, input gradient): 0..3 = channel block cap 32, 16, 8, 4
  // weight gradient (both precisions): 0..2 = 512, 256, 128 pixel chunks;
  //   BF16 also 3..5 = the same on the matrix cores (im2col slabs) and
  //   6..8 = the same on the matrix cores by 16 x 16 output tiles
  if (pass == 2) return precision == LS_BF16 ? 9 : 3;
  if (precision == LS_BF16) return pass == 0 ? ((layer == 1 || layer == LS_NLAYER - 1) ? 5 : 4) : 3;
  return 4;
}
int ls_conv_config_get(int layer, int precision, int pass) {
  cfg_init();
  if (layer < 0 || layer >= LS_NLAYER || precision < 0 || precision > 1 || pass < 0 || pass > 2) return -1;
  return g_conv_cfg[layer][precision][pass];
}
int ls_conv_config_set(int layer, int precision, int pass, int config) {
  cfg_init();
  if (layer < 0 || layer >= LS_NLAYER || precision < 0 || precision > 1 || pass < 0 || pass > 2) return LS_ERANGE;
  if (config < -1 || config >= ls_conv_num_configs_impl(layer, precision, pass)) return LS_ERANGE;
  g_conv_cfg[layer][precision][pass] = config;
  return LS_OK;
}

extern "C" {

int ls_num_params(void) { return LS_NUM_PARAMS; }

const char* ls_version(void) { return "lidarscout-mi355x 0.1 (gfx950)"; }

const char* ls_last_error(void) { return g_last_error; }

const char* ls_status_string(int status) {
  switch (status) {
    case LS_OK: return "ok";
    case LS_EINVAL: return "invalid argument (null pointer or size)";
    case LS_ERANGE: return "grid or option out of the supported range";
    case LS_EHIP: return "HIP runtime error (see ls_last_error)";
    case LS_ENOTIMPL: return "not implemented";
    case LS_EWORKSPACE: return "workspace smaller than ls_workspace_bytes()";
    case LS_ECAP: return "output capacity too small";
    case LS_ESCRATCH: return "input larger than the fixed scratch of this entry point";
    default: return "unknown status";
  }
}

size_t ls_workspace_bytes(int op, const ls_grid* g, int32_t n_tiles, int64_t n_points, int precision) {
  LsGridInfo gi;
  if (ls_grid_info(g, &gi) != LS_OK || n_tiles < 0 || n_points < 0) return 0;
  switch (op) {
    case LS_OP_RECON: return ls_recon_ws_bytes(gi, n_tiles, n_points);
    case LS_OP_REFINE: return ls_refine_ws_bytes(gi, n_tiles, precision, 0);
    case LS_OP_BACKWARD: return ls_refine_ws_bytes(gi, n_tiles, precision, 1);
    case LS_OP_LOSS: return ls_loss_ws_bytes();
    case LS_OP_REFINE_LSNET:
      return (precision == LS_FP32 || precision == LS_BF16) ? ls_lsnet_ws_bytes(gi, n_tiles, precision) : 0;
    default: return 0;
  }
}

size_t ls_act_bytes(const ls_grid* g, int32_t n_tiles, int precision) {
  LsGridInfo gi;
  if (ls_grid_info(g, &gi) != LS_OK || n_tiles < 0) return 0;
  return ls_refine_act_bytes(gi, n_tiles, precision);
}

int ls_recon_tiles(const ls_grid* g, const int32_t* x, const int32_t* y, const int32_t* z, const uint16_t* rgb,
                   int64_t n, const int32_t* tile_list, int32_t n_tiles, int32_t order, float* x_out, double* cz_out,
                   int32_t* bin_off, int32_t* bin_idx, int64_t bin_cap, int32_t* tile_status, void* ws,
                   size_t ws_bytes, void* stream) {
  LsGridInfo gi;
  const int rc = ls_grid_info(g, &gi);
  if (rc != LS_OK) return rc;
  if (order != LS_ORDER_LIST && order != LS_ORDER_LONGEST_FIRST) return LS_ERANGE;
  if (n < 0 || n_tiles < 0 || n > 0x7fffffffLL) return LS_EINVAL;
  if (n > 0 && (!x || !y || !z || !rgb)) return LS_EINVAL;
  if (n_tiles > 0 && (!tile_list || !x_out || !cz_out || !tile_status)) return LS_EINVAL;
  if ((bin_off == nullptr) != (bin_idx == nullptr)) return LS_EINVAL;
  if (bin_idx && bin_cap < 0) return LS_EINVAL;
  if ((int64_t)gi.tx * gi.ty > 0x7fffffffLL) return LS_ERANGE;
  return ls_recon_impl(gi, x, y, z, rgb, n, tile_list, n_tiles, order, x_out, cz_out, bin_off, bin_idx, bin_cap,
                       tile_status, ws, ws_bytes, ls_stream(stream));
}

int ls_recon_tiles_noalloc(const ls_grid* g, const int32_t* x, const int32_t* y, const int32_t* z,
                           const uint16_t* rgb, int64_t n, const int32_t* tile_list, int32_t n_tiles, int32_t order,
                           float* x_out, double* cz_out, int32_t* bin_off, int32_t* bin_idx, int64_t bin_cap,
                           int32_t* tile_status, void* stream) {
  LsGridInfo gi;
  const int rc = ls_grid_info(g, &gi);
  if (rc != LS_OK) return rc;
  if (order != LS_ORDER_LIST && order != LS_ORDER_LONGEST_FIRST) return LS_ERANGE;
  if (n < 0 || n_tiles < 0 || n > 0x7fffffffLL) return LS_EINVAL;
  if (n > 0 && (!x || !y || !z || !rgb)) return LS_EINVAL;
  if (n_tiles > 0 && (!tile_list || !x_out || !cz_out || !tile_status)) return LS_EINVAL;
  if ((bin_off == nullptr) != (bin_idx == nullptr)) return LS_EINVAL;
  if (bin_idx && bin_cap < 0) return LS_EINVAL;
  if ((int64_t)gi.tx * gi.ty > 0x7fffffffLL) return LS_ERANGE;
  return ls_recon_noalloc_impl(gi, x, y, z, rgb, n, tile_list, n_tiles, order, x_out, cz_out, bin_off, bin_idx,
                               bin_cap, tile_status, ls_stream(stream));
}

int ls_refine_tiles(const float* w, const uint16_t* w_bf16, int precision, const float* x, const double* cz,
                    int32_t n_tiles, const ls_grid* g, float* y_out, float* tex_out, void* act_save, void* ws,
                    size_t ws_bytes, void* stream) {
  LsGridInfo gi;
  const int rc = ls_grid_info(g, &gi);
  if (rc != LS_OK) return rc;
  if (precision != LS_FP32 && precision != LS_BF16) return LS_ERANGE;
  if (n_tiles < 0) return LS_EINVAL;
  if (n_tiles > 0 && (!w || !x)) return LS_EINVAL;
  if (precision == LS_BF16 && !w_bf16) return LS_EINVAL;
  if (tex_out && !cz) return LS_EINVAL;
  return ls_refine_forward_impl(w, w_bf16, precision, x, cz, n_tiles, gi, y_out, tex_out, act_save, ws, ws_bytes,
                                ls_stream(stream));
}

int64_t ls_lsnet_num_params(const ls_grid* g) {
  LsGridInfo gi;
  if (ls_grid_info(g, &gi) != LS_OK) return -1;
  return ls_lsnet_params(gi.R);
}

int ls_lsnet_refine_tiles(const float* w, int precision, int32_t inputs, const float* x, const double* cz,
                          int32_t n_tiles, const ls_grid* g, float* y_out, float* tex_out, void* ws, size_t ws_bytes,
                          void* stream) {
  LsGridInfo gi;
  const int rc = ls_grid_info(g, &gi);
  if (rc != LS_OK) return rc;
  if (gi.R % 16) return LS_ERANGE;
  if (precision != LS_FP32 && precision != LS_BF16) return LS_ERANGE;
  if (inputs < 1 || inputs > LS_IN_ALL) return LS_ERANGE;
  if (n_tiles < 0) return LS_EINVAL;
  if (n_tiles > 0 && (!w || !x)) return LS_EINVAL;
  if (tex_out && !cz) return LS_EINVAL;
  return ls_lsnet_forward_impl(w, precision, inputs, x, cz, n_tiles, gi, y_out, tex_out, ws, ws_bytes,
                               ls_stream(stream));
}

int ls_refine_backward(const float* w, const uint16_t* w_bf16, int precision, const float* x,
                       const void* act_save, const float* grad_y, int32_t n_tiles, const ls_grid* g, float* grad_w,
                       float* grad_x, void* ws, size_t ws_bytes, void* stream) {
  LsGridInfo gi;
  const int rc = ls_grid_info(g, &gi);
  if (rc != LS_OK) return rc;
  if (precision != LS_FP32 && precision != LS_BF16) return LS_ERANGE;
  if (n_tiles < 0 || !grad_w) return LS_EINVAL;
  if (n_tiles > 0 && (!w || !x || !grad_y)) return LS_EINVAL;
  if (precision == LS_BF16 && !w_bf16) return LS_EINVAL;
  return ls_refine_backward_impl(w, w_bf16, precision, x, act_save, grad_y, n_tiles, gi, grad_w, grad_x, ws,
                                 ws_bytes, ls_stream(stream));
}

int ls_splat_points(const ls_grid* g, const int32_t* x, const int32_t* y, const int32_t* z, const uint16_t* rgb,
                    int64_t n, const int32_t* tile_slot, int32_t n_slots, uint64_t* keys, float* tex_inout,
                    uint64_t* n_dropped, void* stream) {
  LsGridInfo gi;
  const int rc = ls_grid_info(g, &gi);
  if (rc != LS_OK) return rc;
  if (n < 0 || n_slots < 0) return LS_EINVAL;
  if (n > 0 && (!x || !y || !z || !rgb || !tile_slot || !keys || !n_dropped)) return LS_EINVAL;
  if (tex_inout && !keys) return LS_EINVAL;
  return ls_splat_impl(gi, x, y, z, rgb, n, tile_slot, n_slots, keys, tex_inout, n_dropped, ls_stream(stream));
}

int ls_resolve_keys(const ls_grid* g, const uint64_t* keys, int32_t n_slots, float* tex_inout, void* stream) {
  LsGridInfo gi;
  const int rc = ls_grid_info(g, &gi);
  if (rc != LS_OK) return rc;
  if (n_slots < 0 || (n_slots > 0 && (!keys || !tex_inout))) return LS_EINVAL;
  return ls_resolve_impl(gi, keys, n_slots, tex_inout, ls_stream(stream));
}

int ls_splat_mean(const ls_grid* g, const int32_t* x, const int32_t* y, const int32_t* z, const uint16_t* rgb,
                  int64_t n, const int32_t* tile_slot, int32_t n_slots, int64_t* acc, uint64_t* n_dropped,
                  void* stream) {
  LsGridInfo gi;
  const int rc = ls_grid_info(g, &gi);
  if (rc != LS_OK) return rc;
  if (n < 0 || n_slots < 0) return LS_EINVAL;
  if (n > 0 && (!x || !y || !z || !rgb || !tile_slot || !acc || !n_dropped)) return LS_EINVAL;
  return ls_splat_mean_impl(gi, x, y, z, rgb, n, tile_slot, n_slots, acc, n_dropped, ls_stream(stream));
}

int ls_resolve_mean(const ls_grid* g, const int64_t* acc, int32_t n_slots, float* tex, void* stream) {
  LsGridInfo gi;
  const int rc = ls_grid_info(g, &gi);
  if (rc != LS_OK) return rc;
  if (n_slots < 0 || (n_slots > 0 && (!acc || !tex))) return LS_EINVAL;
  return ls_resolve_mean_impl(gi, acc, n_slots, tex, ls_stream(stream));
}

int ls_target_loss(const float* y, const float* t, const double* cz, int32_t n_tiles, const ls_grid* g, int kind,
                   double* loss_out, float* grad, void* ws, size_t ws_bytes, void* stream) {
  LsGridInfo gi;
  const int rc = ls_grid_info(g, &gi);
  if (rc != LS_OK) return rc;
  if (kind != LS_LOSS_CLIPPED_MSE && kind != LS_LOSS_L1) return LS_ERANGE;
  if (n_tiles < 0 || !loss_out) return LS_EINVAL;
  if (n_tiles > 0 && (!y || !t || !cz)) return LS_EINVAL;
  return ls_target_loss_impl(y, t, cz, n_tiles, gi, kind, loss_out, grad, ws, ws_bytes, ls_stream(stream));
}

int ls_raster_points(const ls_view* v, const int32_t* x, const int32_t* y, const int32_t* z, const uint16_t* rgb,
                     int64_t n, uint64_t* fb, uint64_t* n_drawn, void* stream) {
  if (!v || n < 0) return LS_EINVAL;
  if (v->width < 1 || v->height < 1 || v->width > 32768 || v->height > 32768) return LS_ERANGE;
  if (n > 0 && (!x || !y || !z || !rgb || !fb)) return LS_EINVAL;
  return ls_raster_impl(*v, x, y, z, rgb, n, fb, n_drawn, ls_stream(stream));
}

int ls_raster_resolve(const uint64_t* fb, int64_t n_pixels, uint32_t* rgba, void* stream) {
  if (n_pixels < 0 || (n_pixels > 0 && (!fb || !rgba))) return LS_EINVAL;
  return ls_raster_resolve_impl(fb, n_pixels, rgba, ls_stream(stream));
}

int ls_pack_weights_bf16(const float* w, uint16_t* w_bf16, void* stream) {
  if (!w || !w_bf16) return LS_EINVAL;
  return ls_pack_bf16(w, w_bf16, LS_NUM_PARAMS, ls_stream(stream));
}

int ls_trace_enable(int on) {
  if (on && !g_trace_init) {
    for (int i = 0; i < 2 * TRACE_MAX; ++i) LS_HOST_CHECK(hipEventCreate(&g_trace_ev[i]));
    g_trace_init = true;
  }
  g_trace_on = on != 0;
  g_trace_n = 0;
  return LS_OK;
}

int ls_trace_count(void) { return g_trace_n; }

int ls_trace_record(int i, const char** name, float* ms) {
  if (i < 0 || i >= g_trace_n || !name || !ms) return LS_EINVAL;
  LS_HOST_CHECK(hipEventSynchronize(g_trace_ev[2 * i + 1]));
  LS_HOST_CHECK(hipEventElapsedTime(ms, g_trace_ev[2 * i], g_trace_ev[2 * i + 1]));
  *name = g_trace_name[i];
  return LS_OK;
}

int ls_conv_num_configs(int layer, int precision, int pass) { return ls_conv_num_configs_impl(layer, precision, pass); }
int ls_set_conv_config(int layer, int precision, int pass, int config) {
  return ls_conv_config_set(layer, precision, pass, config);
}
int ls_get_conv_config(int layer, int precision, int pass) { return ls_conv_config_get(layer, precision, pass); }

}  // extern "C"
