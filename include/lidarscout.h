/* lidarscout.h - C-ABI of the MI355X (gfx950) per-tile heightmap library.
 *
 * The library implements the data-parallel hot path of LidarScout (Erler,
 * Herzberger, Wimmer, Schuetz, HPG 2025): sparse "chunk points" are binned
 * into fixed patches ("tiles" here) with a padding ring, interpolated into
 * nearest-neighbour and Delaunay-linear height + colour maps (Section 3.3,
 * Algorithm 1), normalised (Section 3.4), refined by a small convolutional
 * network (Section 3.4), and full-resolution points are later splatted into
 * the heightmap textures with packed 64-bit keys (Sections 3.5 and 3.6).
 *
 * Conventions for every entry point:
 *  - Pointers are DEVICE pointers (memory of the current HIP device) unless
 *    the comment says (host).  The caller owns every buffer; the library
 *    never allocates device memory inside these calls.  Scratch memory is a
 *    caller-provided workspace of at least ls_workspace_bytes() bytes.
 *  - Work is enqueued asynchronously on `stream` (a hipStream_t passed as
 *    void*; NULL = the default stream).  No call synchronises the host, so
 *    every call can be captured into a HIP graph.
 *  - Return value: LS_OK (0) or a negative ls_status for argument errors,
 *    detected on the host before anything is enqueued.  Errors that depend
 *    on data are reported per tile in tile_status (bit flags ls_tile_flag)
 *    and never abort a call.
 *  - Coordinates are LAS raw integers: metres = raw * scale (+ offset for z).
 *  - Layouts are row-major; images are NHWC: [tile][row][col][channel], row
 *    index along +y, column index along +x.
 */
#ifndef LIDARSCOUT_H
#define LIDARSCOUT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Region and tiling, passed by (host) pointer.
 * Tile (tx, ty) covers [origin + t*tile_size, origin + (t+1)*tile_size) on
 * each axis.  Its output grid has res x res texels of cell = tile_size/res
 * raw units (640 m / 64 = 10 m in the paper, Section 3.1).  Its network
 * input is the padded grid of R = res + 2*pad texels per side (96 with the
 * paper's 16-texel ring, Section 3.3), covering the window
 * [c - H, c + H) with c the tile centre and H = tile_size/2 + pad*cell.
 * Requirements: tile_size % res == 0, cell even, R % 4 == 0, pad >= 0,
 * 1 <= res, H <= 262143 raw units (2^18 - 1: with 1 cm units, cells up to
 * 40 m at res 64 with the 16-texel ring), |origin_x|, |origin_y| <= 2^40. */
typedef struct ls_grid {
  int64_t origin_x, origin_y;
  int32_t tile_size;
  int32_t res, pad;
  int32_t tiles_x, tiles_y;
  double scale_xy, scale_z, offset_z;
} ls_grid;

typedef enum ls_status {
  LS_OK = 0,
  LS_EINVAL = -1,     /* null pointer or inconsistent size */
  LS_ERANGE = -2,     /* grid parameters out of the supported range */
  LS_EHIP = -3,       /* HIP runtime error (see ls_last_error) */
  LS_ENOTIMPL = -4,   /* option not implemented */
  LS_EWORKSPACE = -5, /* workspace smaller than ls_workspace_bytes() */
  LS_ECAP = -6,       /* a caller-sized output cannot hold the result */
  LS_ESCRATCH = -7    /* input larger than a fixed-size scratch entry point accepts */
} ls_status;

/* per-tile status flags written by ls_recon_tiles */
typedef enum ls_tile_flag {
  LS_TILE_EMPTY = 1,      /* no point in the window: all outputs 0, cz = 0 */
  LS_TILE_NN_ONLY = 2,    /* < 3 distinct points or all collinear: linear = NN */
  LS_TILE_CAP = 4,        /* bin_cap too small; bin_off[n_tiles] holds the need */
  LS_TILE_DEGENERATE = 8, /* triangulation safeguard hit (never expected) */
  LS_TILE_BADID = 16      /* tile id outside the region or listed twice */
} ls_tile_flag;

typedef enum ls_precision { LS_FP32 = 0, LS_BF16 = 1 } ls_precision;

/* Order in which ls_recon_tiles takes its tiles from the work queue.
 *  LS_ORDER_LIST: the order of tile_list, e.g. by distance to the viewer, so
 *    that construction is prioritised towards the viewpoint (Section 1 and
 *    the Section 4.1 discussion of Table 2: nearby heightmaps first).
 *  LS_ORDER_LONGEST_FIRST: descending window point count (in steps of 4
 *    points), so the last tiles to start are short and the workgroups finish
 *    together; for throughput on a batch with no priority.
 * Results per output slot do not depend on the order. */
typedef enum ls_order { LS_ORDER_LIST = 0, LS_ORDER_LONGEST_FIRST = 1 } ls_order;

typedef enum ls_op {
  LS_OP_RECON = 0,
  LS_OP_REFINE = 1,
  LS_OP_BACKWARD = 2,
  LS_OP_SPLAT = 3,
  LS_OP_LOSS = 4,
  LS_OP_REFINE_LSNET = 5
} ls_op;

/* Number of network parameters (119,844 for the 3-level U-Net).
 * Flat FP32 layout, layers in order enc1a 8->16, enc1b 16->16, enc2a 16->32,
 * enc2b 32->32, bot_a 32->64, bot_b 64->64, dec2a 96->32, dec2b 32->32,
 * dec1a 48->16, dec1b 16->16, head 24->4; per layer W[Cout][3][3][Cin]
 * followed by b[Cout]. */
int ls_num_params(void);

/* Bytes of caller workspace needed by `op` for n_tiles tiles and n_points
 * input points (recon: sparse points; splat: unused, returns 0).  Depends
 * only on the sizes, never on the data. */
size_t ls_workspace_bytes(int op, const ls_grid* g, int32_t n_tiles, int64_t n_points, int precision);

/* Bytes of the activation buffer ls_refine_tiles can save for
 * ls_refine_backward (FP32 or BF16 activations, per `precision`). */
size_t ls_act_bytes(const ls_grid* g, int32_t n_tiles, int precision);

/* Tile binning + Algorithm 1 + normalisation (Sections 3.3-3.4).
 *  x, y, z [n] int32 raw; rgb [n][3] uint16 (16-bit LAS colour).
 *  tile_list [n_tiles]: linear tile ids ty*tiles_x + tx, distinct.  Output
 *    slot k belongs to tile_list[k].
 *  order: ls_order; LS_ORDER_LIST processes the tiles in tile_list order
 *    (workgroups take them from a queue in that order), LS_ORDER_LONGEST_FIRST
 *    by descending window point count.  Other values: LS_ERANGE.
 *  x_out [n_tiles][R][R][8] FP32: channel 0 (h_lin - cz)/r, 1 (h_nn - cz)/r,
 *    2-4 linear RGB/65535, 5-7 nearest RGB/65535, with r = H*scale_xy
 *    metres and h in metres.
 *  cz_out [n_tiles] FP64: the linear height (metres) at texel (R/2, R/2).
 *  bin_off [n_tiles+1], bin_idx [bin_cap] (both nullable together): if
 *    given, receive the CSR of point indices in each tile's window in
 *    ascending index order; if bin_cap is too small every tile gets
 *    LS_TILE_CAP and bin_off[n_tiles] the required size.
 *  tile_status [n_tiles]: ls_tile_flag bits.
 *  ws: workspace of ls_workspace_bytes(LS_OP_RECON, g, n_tiles, n, 0).
 * Points outside every listed window are ignored.  Nearest-neighbour ties
 * go to the smallest (d^2, y, x); duplicate positions keep the largest
 * (z, R, G, B).  Linear values cover exactly the closed convex hull. */
int ls_recon_tiles(const ls_grid* g, const int32_t* x, const int32_t* y, const int32_t* z, const uint16_t* rgb,
                   int64_t n, const int32_t* tile_list, int32_t n_tiles, int32_t order, float* x_out, double* cz_out,
                   int32_t* bin_off, int32_t* bin_idx, int64_t bin_cap, int32_t* tile_status, void* ws,
                   size_t ws_bytes, void* stream);

/* Allocation-free ls_recon_tiles, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Same arguments, results and errors as ls_recon_tiles,
 * without the workspace: the library uses a fixed array of
 * LS_RECON_SCRATCH_BYTES in device memory instead, which every device the
 * call runs on holds until the process ends.  The call allocates nothing.
 * Limit: LS_ESCRATCH (nothing enqueued) when the inputs need more than the
 * array with a single persistent workgroup (per point of n about 600 bytes,
 * per tile of the region 4 bytes, per listed tile 20 bytes, plus 12*R*R
 * bytes per workgroup: about 80,000 points with the 96 x 96 grid); inputs
 * that fit run on as many workgroups as the array holds (fewer than
 * ls_recon_tiles uses when the points fill most of it, so slower).
 * Every call on one GPU shares its array and leaves its contents behind;
 * calls that overlap on one GPU (other streams, other threads) race on it,
 * so serialise them. */
#define LS_RECON_SCRATCH_BYTES ((size_t)48 << 20)
int ls_recon_tiles_noalloc(const ls_grid* g, const int32_t* x, const int32_t* y, const int32_t* z,
                           const uint16_t* rgb, int64_t n, const int32_t* tile_list, int32_t n_tiles, int32_t order,
                           float* x_out, double* cz_out, int32_t* bin_off, int32_t* bin_idx, int64_t bin_cap,
                           int32_t* tile_status, void* stream);

/* Refinement network forward (Section 3.4) on a batch of tiles.
 *  w [num_params] FP32; w_bf16 [num_params] BF16 bit patterns (required
 *    for LS_BF16, from ls_pack_weights_bf16; ignored for LS_FP32).
 *  x [n_tiles][R][R][8] FP32 (from ls_recon_tiles); cz [n_tiles] FP64.
 *  y_out [n_tiles][res][res][4] FP32 normalised (h, r, g, b); nullable.
 *  tex_out [n_tiles][res][res][4] FP32 texture: h = cz + r*y_h metres,
 *    rgb = clamp(y_rgb, 0, 1); nullable (cz may then be NULL).
 *  act_save: nullable; if given (ls_act_bytes bytes) the activations the
 *    backward needs are kept there.
 *  LS_FP32: FP32 operands and accumulation.  LS_BF16: BF16 operands on
 *  the matrix cores, FP32 accumulation, FP32 bias/residual/denormalise.
 *  ws: ls_workspace_bytes(LS_OP_REFINE, g, n_tiles, 0, precision). */
int ls_refine_tiles(const float* w, const uint16_t* w_bf16, int precision, const float* x, const double* cz,
                    int32_t n_tiles, const ls_grid* g, float* y_out, float* tex_out, void* act_save, void* ws,
                    size_t ws_bytes, void* stream);

/* The paper's own refinement network (Section 3.4, architecture paragraph):
 * every input (h_lin, h_nn, rgb_lin, rgb_nn) has its own encoder of four
 * conv3x3 + ReLU + 2x2 average-pool layers (c -> 16 -> 32 -> 32 -> 32); two
 * fully connected layers merge the height features [F_hlin, F_hnn] and the
 * colour features [F_rgblin, F_rgbnn] into 256 values each (ReLU); two more
 * (ReLU) map the 512 merged values to the R/16 x R/16 x 32 inputs of a
 * height decoder and a texture decoder, each four times nearest x2
 * upsampling + conv3x3 + ReLU (32 -> 32 -> 32 -> 16 -> 16); the original
 * inputs are concatenated with both decoder outputs (40 channels) and a
 * final CNN (conv3x3 40 -> 32 ReLU, 32 -> 32 ReLU, 32 -> 4) is evaluated on
 * the centre res x res crop and added to the crop of the linear input, as
 * ls_refine_tiles does.  The layer sizes are this library's reading of the
 * paper's description (its figure is missing): 2,528,708 parameters at
 * R = 96 ("about 2.5 M").  Requires R % 16 == 0.
 * Flat FP32 weights, layers in the order enc_hlin1..4, enc_hnn1..4,
 * enc_rgblin1..4, enc_rgbnn1..4, fc1_h (2L -> 256), fc1_c (2L -> 256),
 * fc2_h (512 -> L), fc2_t (512 -> L), dec_h1..4, dec_t1..4, fin1, fin2, fin3
 * with L = (R/16)^2 * 32; conv layers W[Cout][3][3][Cin] then b[Cout];
 * fully connected W[N][K] then b[N], K indexing the concatenated input, the
 * feature images flattened in (row, column, channel) order and the FC2
 * outputs read as (row, column, channel) images.
 * Returns the parameter count, or -1 for an invalid grid or R % 16 != 0. */
int64_t ls_lsnet_num_params(const ls_grid* g);

/* Inputs of the paper's network, as bits of `inputs` (Section 4.3 ablation:
 * variants that see only some of the reconstructed maps).  An absent input
 * reads as zero everywhere (its encoder then yields a constant feature
 * vector, which the FC layers absorb into their biases, and its skip
 * channels contribute nothing), and an absent linear input also drops out
 * of the residual: y = f3 + crop(x_lin if present).  HM only = h_lin | h_nn
 * (its colour output is unused), NN only = h_nn | rgb_nn, Lin only = h_lin |
 * rgb_lin. */
typedef enum ls_inputs {
  LS_IN_HLIN = 1,
  LS_IN_HNN = 2,
  LS_IN_RGBLIN = 4,
  LS_IN_RGBNN = 8,
  LS_IN_ALL = 15,
  LS_IN_HM_ONLY = LS_IN_HLIN | LS_IN_HNN,
  LS_IN_NN_ONLY = LS_IN_HNN | LS_IN_RGBNN,
  LS_IN_LIN_ONLY = LS_IN_HLIN | LS_IN_RGBLIN
} ls_inputs;

/* Forward of that network on a batch: same x, cz, y_out, tex_out as
 * ls_refine_tiles; `inputs` selects the inputs the network sees (ls_inputs
 * bits, LS_IN_ALL for the full network).  LS_FP32: FP32 operands and
 * accumulation; LS_BF16: the
 * FP32 weights rounded to BF16 (nearest even) inside the call, BF16
 * operands on the matrix cores with FP32 accumulation, every stored hidden
 * activation BF16, the final layer, residual and denormalisation FP32.
 *  ws: ls_workspace_bytes(LS_OP_REFINE_LSNET, g, n_tiles, 0, precision)
 *    bytes (bounded: the batch is processed in chunks).
 * Errors: LS_ERANGE for R % 16 != 0, another precision or inputs outside
 * [1, LS_IN_ALL]; LS_EINVAL for null w or x (n_tiles > 0), or tex_out
 * without cz; LS_EWORKSPACE. */
int ls_lsnet_refine_tiles(const float* w, int precision, int32_t inputs, const float* x, const double* cz,
                          int32_t n_tiles, const ls_grid* g, float* y_out, float* tex_out, void* ws, size_t ws_bytes,
                          void* stream);

/* Refinement network backward, for training the network (Section 3.4,
 * training paragraph: the network is fitted to ground-truth heightmaps with a
 * loss on its normalised output; any loss can be used, the caller supplies
 * its gradient).  Given dL/dy [n_tiles][res][res][4] for the normalised
 * output, writes grad_w [num_params] (overwritten, summed over the batch) and,
 * if non-null, grad_x [n_tiles][R][R][8].  act_save: the buffer filled by
 * ls_refine_tiles with the same inputs and precision, or NULL to recompute
 * the forward inside (activation recomputation).  LS_BF16: the decoder's
 * full-resolution level and its gradients are computed only near the crop,
 * where the head reads them (same values; the weight gradient's FP32
 * partial sums are grouped differently from a whole-plane computation).
 * Errors: LS_EINVAL for a null grad_w or (n_tiles > 0) null w, x or grad_y,
 * or a null w_bf16 with LS_BF16; LS_ERANGE for another precision;
 * LS_EWORKSPACE for a short workspace.
 *  ws: ls_workspace_bytes(LS_OP_BACKWARD, g, n_tiles, 0, precision). */
int ls_refine_backward(const float* w, const uint16_t* w_bf16, int precision, const float* x,
                       const void* act_save, const float* grad_y, int32_t n_tiles, const ls_grid* g, float* grad_w,
                       float* grad_x, void* ws, size_t ws_bytes, void* stream);

/* Full-resolution splat (Sections 3.5-3.6): every point with texel
 * gx = floor((x - origin_x)/cell), gy likewise, inside the region and in a
 * tile whose tile_slot[ty*tiles_x + tx] >= 0, raises
 *   keys[slot][gy % res][gx % res] = max(old, key),
 *   key = ((uint32)z ^ 0x80000000) << 32 | R>>8 << 24 | G>>8 << 16 | B>>8 << 8 | 0xFF,
 * i.e. the texel keeps its highest point (ties: larger packed colour).
 * keys [n_slots][res][res] accumulate across calls (caller zeroes them
 * once).  *n_dropped (device, uint64) is incremented by the number of
 * points outside the region or in unmapped tiles.  tex_inout (nullable,
 * [n_slots][res][res][4] FP32): afterwards every texel whose key is
 * non-zero is overwritten with h = (float)(z*scale_z + offset_z) (double
 * multiply then add, correctly rounded) and byte/255 colours; other texels
 * keep their value.  Any point order is accepted; Morton-ordered input
 * (50,000-point chunks of Section 3.1) is the fast case. */
int ls_splat_points(const ls_grid* g, const int32_t* x, const int32_t* y, const int32_t* z, const uint16_t* rgb,
                    int64_t n, const int32_t* tile_slot, int32_t n_slots, uint64_t* keys, float* tex_inout,
                    uint64_t* n_dropped, void* stream);

/* Resolve only (the second half of ls_splat_points). */
int ls_resolve_keys(const ls_grid* g, const uint64_t* keys, int32_t n_slots, float* tex_inout, void* stream);

/* Ground-truth accumulation for training (Section 3.4, training data: each
 * ground-truth heightmap and texture is the per-texel average of all points
 * that fall on the texel).  Every point with texel gx = floor((x -
 * origin_x)/cell), gy likewise, inside the region and in a tile whose
 * tile_slot[ty*tiles_x + tx] >= 0, adds
 *   acc[slot][gy % res][gx % res] += (z, R, G, B, 1)
 * with z the raw int32 height and R, G, B the 16-bit colours.  acc
 * [n_slots][res][res][5] int64 (sum z, sum R, sum G, sum B, count)
 * accumulates across calls (the caller zeroes it once); integer sums, so
 * the result is exact for any point order.  *n_dropped (device, uint64) is
 * incremented by the points outside the region or in unmapped tiles.
 * Errors: LS_EINVAL for n > 0 with a null array; LS_ERANGE for a grid whose
 * texel extent times the cell exceeds 2^31. */
int ls_splat_mean(const ls_grid* g, const int32_t* x, const int32_t* y, const int32_t* z, const uint16_t* rgb,
                  int64_t n, const int32_t* tile_slot, int32_t n_slots, int64_t* acc, uint64_t* n_dropped,
                  void* stream);

/* Mean texture from ls_splat_mean sums: tex [n_slots][res][res][4] FP32 =
 * (mean z * scale_z + offset_z metres, mean R/65535, mean G/65535, mean
 * B/65535), each mean a double division rounded once to FP32 after the
 * scale (multiply, then add, no contraction); texels with count 0 are NaN in
 * all four channels (gaps, masked out of the loss). */
int ls_resolve_mean(const ls_grid* g, const int64_t* acc, int32_t n_slots, float* tex, void* stream);

/* Loss kinds of ls_target_loss. */
typedef enum ls_loss {
  LS_LOSS_CLIPPED_MSE = 0, /* Section 3.4 training: squared error clipped to [0, 1], NaN targets masked */
  LS_LOSS_L1 = 1           /* mean absolute error */
} ls_loss;

/* Training loss of the normalised network output against a target texture
 * (Section 3.4, training: a mean squared error in which elements with a NaN
 * ground truth are ignored, the errors clipped to [0, 1], the height and
 * texture losses averaged).
 *  y [n_tiles][res][res][4] FP32: network output (h, r, g, b), normalised.
 *  t [n_tiles][res][res][4] FP32: target texture, height in metres, colour
 *    in [0, 1], NaN = no ground truth; its height is normalised like the
 *    input, (t_h - cz[tile]) / r with r = H*scale_xy.
 *  cz [n_tiles] FP64 (from ls_recon_tiles).
 *  Per element d = y - target (double): LS_LOSS_CLIPPED_MSE e = min(d^2, 1),
 *  gradient d/N where d^2 <= 1, else 0; LS_LOSS_L1 e = |d|, gradient
 *  sign(d)/(2N) (sign(0) = 0).  N = n_tiles*res*res for heights and three
 *  times that for colours; L_h = sum e_h / N_h, L_rgb = sum e_rgb / N_rgb,
 *  L = (L_h + L_rgb) / 2.  NaN targets give e = 0 and gradient 0.
 *  loss_out [3] FP64 (device): L, L_h, L_rgb; the sums are reduced in a
 *    fixed order (deterministic).
 *  grad (nullable) [n_tiles][res][res][4] FP32: dL/dy, rounded once.
 *  ws: ls_workspace_bytes(LS_OP_LOSS, ...) bytes.
 * Errors: LS_EINVAL for null y, t, cz or loss_out; LS_ERANGE for another
 * kind; LS_EWORKSPACE for a short workspace. */
int ls_target_loss(const float* y, const float* t, const double* cz, int32_t n_tiles, const ls_grid* g, int kind,
                   double* loss_out, float* grad, void* ws, size_t ws_bytes, void* stream);

/* View of the point rasteriser (host). */
typedef struct ls_view {
  double m[16];                /* view-projection, row-major: clip = m * (X, Y, Z, 1) */
  int64_t origin_x, origin_y;  /* raw units; X = (x - origin_x)*scale_xy, Y likewise (metres) */
  double scale_xy, scale_z, offset_z; /* Z = z*scale_z + offset_z (metres) */
  int32_t width, height;       /* frame buffer size in pixels */
} ls_view;

/* Point rasteriser (Section 3.6, points: depth and colour packed into one
 * 64-bit integer per point, the nearest kept per pixel by a 64-bit atomic
 * minimum, then a resolve pass).  Per point, in double precision without
 * contraction: clip rows c_r = ((m[4r]*X + m[4r+1]*Y) + m[4r+2]*Z) + m[4r+3];
 * drawn iff w = c_3 > 0 and ndc = (c_0/w, c_1/w) in [-1, 1)^2; pixel column
 * floor(((ndc_x + 1)*0.5)*width), row likewise (row 0 at ndc_y = -1);
 *   key = bits((float)w) << 32 | 0xFF << 24 | B8 << 16 | G8 << 8 | R8
 * (C8 = C16 >> 8), fb[row][col] = min(fb, key).
 *  fb [height][width] uint64, in/out: the caller fills it with all ones
 *    (empty) and it accumulates across calls; bit-exact for any order.
 *  n_drawn (nullable, device uint64): incremented by the points drawn.
 * Errors: LS_EINVAL for a null view, or n > 0 with a null array or fb;
 * LS_ERANGE for width or height outside [1, 32768]. */
int ls_raster_points(const ls_view* v, const int32_t* x, const int32_t* y, const int32_t* z, const uint16_t* rgb,
                     int64_t n, uint64_t* fb, uint64_t* n_drawn, void* stream);

/* Resolve of the rasteriser: rgba[i] = low 32 bits of fb[i] (R8 | G8 << 8 |
 * B8 << 16 | 0xFF << 24), 0 for an empty pixel (all ones). */
int ls_raster_resolve(const uint64_t* fb, int64_t n_pixels, uint32_t* rgba, void* stream);

/* FP32 -> BF16 (round to nearest even) weight copy for LS_BF16. */
int ls_pack_weights_bf16(const float* w, uint16_t* w_bf16, void* stream);

/* Conv tiling selection used by the autotuner: config index per
 * (layer 0..10, precision, pass 0=forward 1=dgrad 2=wgrad); -1 = default.
 * ls_conv_num_configs reports how many configs a (layer, precision, pass)
 * accepts.  Host-side state, applies to later calls in this process. */
int ls_conv_num_configs(int layer, int precision, int pass);
int ls_set_conv_config(int layer, int precision, int pass, int config);
int ls_get_conv_config(int layer, int precision, int pass);

/* Launch timing for measurement (not part of the method).  When enabled,
 * every kernel group the library enqueues is bracketed by a pair of HIP
 * events recorded on its stream (up to 16384 groups; the count restarts at
 * each ls_trace_enable call).  ls_trace_record(i) waits for group i and
 * returns its kernel-group name (static host string) and elapsed ms.  Leave
 * disabled (the default) when capturing HIP graphs. */
int ls_trace_enable(int on);
int ls_trace_count(void);
int ls_trace_record(int i, const char** name, float* ms);

const char* ls_status_string(int status);
/* Text of the last LS_EHIP error on this thread (host string). */
const char* ls_last_error(void);
const char* ls_version(void);

#ifdef __cplusplus
}
#endif
#endif /* LIDARSCOUT_H */
