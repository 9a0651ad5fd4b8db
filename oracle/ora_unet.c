/* FP64 oracle: refinement network forward and backward.
 * TEST INFRASTRUCTURE ONLY (see ora.h).
 *
 * The paper refines the interpolated maps with a CNN whose inputs are the
 * linear and NN height maps and textures on the padded 96x96 grid and whose
 * output is the centre 64x64 height + RGB (Section 3.4).  Its exact layer
 * list is not recoverable (the architecture figure is missing), so the
 * network here is a small 3-level U-Net with the paper's input-skip head:
 *
 *   A1 = relu(conv(X, enc1a))        8->16   @R      A2 = relu(conv(A1, enc1b)) 16->16
 *   P1 = avgpool2(A2)                                  @R/2
 *   A3 = relu(conv(P1, enc2a))      16->32             A4 = relu(conv(A3, enc2b)) 32->32
 *   P2 = avgpool2(A4)                                  @R/4
 *   A5 = relu(conv(P2, bot_a))      32->64             A6 = relu(conv(A5, bot_b)) 64->64
 *   U2 = [up2(A6), A4]              96 ch @R/2
 *   A7 = relu(conv(U2, dec2a))      96->32             A8 = relu(conv(A7, dec2b)) 32->32
 *   U1 = [up2(A8), A2]              48 ch @R
 *   A9 = relu(conv(U1, dec1a))      48->16             A10 = relu(conv(A9, dec1b)) 16->16
 *   Hd = conv([A10, X], head)       24->4, no ReLU, only on the centre res x res crop
 *   Y  = crop(X[..., {0, 2, 3, 4}]) + Hd
 *
 * Every conv is 3x3, stride 1, zero padding at the R x R (or pooled) border.
 * Weights: per layer W[Cout][3][3][Cin] then b[Cout], layers in the order
 * above (119,844 values).  Images are HWC (channel fastest).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct { int cin, cout; } ora_layer;
static const ora_layer LAYERS[11] = {{8, 16},  {16, 16}, {16, 32}, {32, 32}, {32, 64}, {64, 64},
                                     {96, 32}, {32, 32}, {48, 16}, {16, 16}, {24, 4}};
enum { E1A, E1B, E2A, E2B, BA, BB, D2A, D2B, D1A, D1B, HEAD, NLAYER };

static size_t layer_offset(int l) {
  size_t off = 0;
  for (int k = 0; k < l; ++k) off += (size_t)LAYERS[k].cout * 9 * LAYERS[k].cin + LAYERS[k].cout;
  return off;
}

int64_t ora_unet_num_params(void) { return (int64_t)layer_offset(NLAYER); }

/* out[y][x][co] = b[co] + sum_{ky,kx,ci} w[co][ky][kx][ci] * in[y+ky-1][x+kx-1][ci],
 * for rows [y0, y1) and columns [x0, x1) of an H x W image; out is indexed
 * relative to (y0, x0) with row width (x1 - x0). */
static void conv3x3(const double* in, int H, int W, int cin, const double* w, const double* b, int cout,
                    double* out, int relu, int y0, int y1, int x0, int x1) {
  const int ow = x1 - x0;
  for (int y = y0; y < y1; ++y)
    for (int x = x0; x < x1; ++x)
      for (int co = 0; co < cout; ++co) {
        double s = b[co];
        for (int ky = 0; ky < 3; ++ky) {
          const int yy = y + ky - 1;
          if (yy < 0 || yy >= H) continue;
          for (int kx = 0; kx < 3; ++kx) {
            const int xx = x + kx - 1;
            if (xx < 0 || xx >= W) continue;
            const double* wp = w + (((size_t)co * 3 + ky) * 3 + kx) * cin;
            const double* ip = in + ((size_t)yy * W + xx) * cin;
            for (int ci = 0; ci < cin; ++ci) s += wp[ci] * ip[ci];
          }
        }
        out[((size_t)(y - y0) * ow + (x - x0)) * cout + co] = (relu && s < 0.0) ? 0.0 : s;
      }
}

/* Adjoint of conv3x3 for the same window: given dout (already multiplied by
 * the ReLU mask), accumulate dw, db and (if din) din. */
static void conv3x3_adj(const double* in, int H, int W, int cin, const double* w, int cout, const double* dout,
                        double* dw, double* db, double* din, int y0, int y1, int x0, int x1) {
  const int ow = x1 - x0;
  for (int y = y0; y < y1; ++y)
    for (int x = x0; x < x1; ++x)
      for (int co = 0; co < cout; ++co) {
        const double gv = dout[((size_t)(y - y0) * ow + (x - x0)) * cout + co];
        if (gv == 0.0) continue;
        db[co] += gv;
        for (int ky = 0; ky < 3; ++ky) {
          const int yy = y + ky - 1;
          if (yy < 0 || yy >= H) continue;
          for (int kx = 0; kx < 3; ++kx) {
            const int xx = x + kx - 1;
            if (xx < 0 || xx >= W) continue;
            const size_t wo = (((size_t)co * 3 + ky) * 3 + kx) * cin;
            const size_t io = ((size_t)yy * W + xx) * cin;
            for (int ci = 0; ci < cin; ++ci) {
              dw[wo + ci] += gv * in[io + ci];
              if (din) din[io + ci] += gv * w[wo + ci];
            }
          }
        }
      }
}

static void avgpool2(const double* in, int H, int W, int c, double* out) {
  for (int y = 0; y < H / 2; ++y)
    for (int x = 0; x < W / 2; ++x)
      for (int k = 0; k < c; ++k) {
        const double s = in[((size_t)(2 * y) * W + 2 * x) * c + k] + in[((size_t)(2 * y) * W + 2 * x + 1) * c + k] +
                         in[((size_t)(2 * y + 1) * W + 2 * x) * c + k] +
                         in[((size_t)(2 * y + 1) * W + 2 * x + 1) * c + k];
        out[((size_t)y * (W / 2) + x) * c + k] = 0.25 * s;
      }
}

static void avgpool2_adj(const double* dout, int H, int W, int c, double* din) {
  for (int y = 0; y < H; ++y)
    for (int x = 0; x < W; ++x)
      for (int k = 0; k < c; ++k) din[((size_t)y * W + x) * c + k] += 0.25 * dout[((size_t)(y / 2) * (W / 2) + x / 2) * c + k];
}

/* dst[y][x][0:c1] = up2(a)[y][x], dst[y][x][c1:c1+c2] = b[y][x]; dst is H x W */
static void up_concat(const double* a, int c1, const double* b, int c2, int H, int W, double* dst) {
  const int c = c1 + c2;
  for (int y = 0; y < H; ++y)
    for (int x = 0; x < W; ++x) {
      double* d = dst + ((size_t)y * W + x) * c;
      const double* pa = a + ((size_t)(y / 2) * (W / 2) + x / 2) * c1;
      const double* pb = b + ((size_t)y * W + x) * c2;
      for (int k = 0; k < c1; ++k) d[k] = pa[k];
      for (int k = 0; k < c2; ++k) d[c1 + k] = pb[k];
    }
}

static void up_concat_adj(const double* dd, int c1, int c2, int H, int W, double* da, double* db) {
  const int c = c1 + c2;
  for (int y = 0; y < H; ++y)
    for (int x = 0; x < W; ++x) {
      const double* d = dd + ((size_t)y * W + x) * c;
      double* pa = da + ((size_t)(y / 2) * (W / 2) + x / 2) * c1;
      double* pb = db + ((size_t)y * W + x) * c2;
      for (int k = 0; k < c1; ++k) pa[k] += d[k];
      for (int k = 0; k < c2; ++k) pb[k] += d[c1 + k];
    }
}

static void relu_mask(double* g, const double* act, size_t n) {
  for (size_t i = 0; i < n; ++i)
    if (!(act[i] > 0.0)) g[i] = 0.0;
}

typedef struct {
  double *A[11]; /* A[1..10] used */
  double *P1, *P2, *U2, *U1, *XC;
} ora_acts;

static void acts_alloc(ora_acts* a, int R) {
  const size_t f = (size_t)R * R, h = f / 4, q = f / 16;
  memset(a, 0, sizeof(*a));
  a->A[1] = malloc(sizeof(double) * f * 16); a->A[2] = malloc(sizeof(double) * f * 16);
  a->P1 = malloc(sizeof(double) * h * 16);
  a->A[3] = malloc(sizeof(double) * h * 32); a->A[4] = malloc(sizeof(double) * h * 32);
  a->P2 = malloc(sizeof(double) * q * 32);
  a->A[5] = malloc(sizeof(double) * q * 64); a->A[6] = malloc(sizeof(double) * q * 64);
  a->U2 = malloc(sizeof(double) * h * 96);
  a->A[7] = malloc(sizeof(double) * h * 32); a->A[8] = malloc(sizeof(double) * h * 32);
  a->U1 = malloc(sizeof(double) * f * 48);
  a->A[9] = malloc(sizeof(double) * f * 16); a->A[10] = malloc(sizeof(double) * f * 16);
  a->XC = malloc(sizeof(double) * f * 24);
}

static void acts_free(ora_acts* a) {
  for (int k = 1; k <= 10; ++k) free(a->A[k]);
  free(a->P1); free(a->P2); free(a->U2); free(a->U1); free(a->XC);
}

/* forward of one tile: x [R][R][8] -> y [res][res][4] (normalised units) */
static void forward_tile(const double* w, const double* x, int res, int pad, ora_acts* a, double* y) {
  const int R = res + 2 * pad, R2 = R / 2, R4 = R / 4;
  const double* W[NLAYER];
  const double* B[NLAYER];
  for (int l = 0; l < NLAYER; ++l) {
    W[l] = w + layer_offset(l);
    B[l] = W[l] + (size_t)LAYERS[l].cout * 9 * LAYERS[l].cin;
  }
  conv3x3(x, R, R, 8, W[E1A], B[E1A], 16, a->A[1], 1, 0, R, 0, R);
  conv3x3(a->A[1], R, R, 16, W[E1B], B[E1B], 16, a->A[2], 1, 0, R, 0, R);
  avgpool2(a->A[2], R, R, 16, a->P1);
  conv3x3(a->P1, R2, R2, 16, W[E2A], B[E2A], 32, a->A[3], 1, 0, R2, 0, R2);
  conv3x3(a->A[3], R2, R2, 32, W[E2B], B[E2B], 32, a->A[4], 1, 0, R2, 0, R2);
  avgpool2(a->A[4], R2, R2, 32, a->P2);
  conv3x3(a->P2, R4, R4, 32, W[BA], B[BA], 64, a->A[5], 1, 0, R4, 0, R4);
  conv3x3(a->A[5], R4, R4, 64, W[BB], B[BB], 64, a->A[6], 1, 0, R4, 0, R4);
  up_concat(a->A[6], 64, a->A[4], 32, R2, R2, a->U2);
  conv3x3(a->U2, R2, R2, 96, W[D2A], B[D2A], 32, a->A[7], 1, 0, R2, 0, R2);
  conv3x3(a->A[7], R2, R2, 32, W[D2B], B[D2B], 32, a->A[8], 1, 0, R2, 0, R2);
  up_concat(a->A[8], 32, a->A[2], 16, R, R, a->U1);
  conv3x3(a->U1, R, R, 48, W[D1A], B[D1A], 16, a->A[9], 1, 0, R, 0, R);
  conv3x3(a->A[9], R, R, 16, W[D1B], B[D1B], 16, a->A[10], 1, 0, R, 0, R);
  for (size_t p = 0; p < (size_t)R * R; ++p) {
    for (int k = 0; k < 16; ++k) a->XC[p * 24 + k] = a->A[10][p * 16 + k];
    for (int k = 0; k < 8; ++k) a->XC[p * 24 + 16 + k] = x[p * 8 + k];
  }
  conv3x3(a->XC, R, R, 24, W[HEAD], B[HEAD], 4, y, 0, pad, pad + res, pad, pad + res);
  static const int SEL[4] = {0, 2, 3, 4};
  for (int i = 0; i < res; ++i)
    for (int j = 0; j < res; ++j)
      for (int k = 0; k < 4; ++k)
        y[((size_t)i * res + j) * 4 + k] += x[((size_t)(i + pad) * R + (j + pad)) * 8 + SEL[k]];
}

/* Batch forward.  x: [n][R][R][8]; y: [n][res][res][4]. */
int ora_unet_forward(const double* w, const double* x, int n, int res, int pad, double* y, int nthreads) {
  const int R = res + 2 * pad;
  if (R % 4) return -1;
#pragma omp parallel num_threads(nthreads > 0 ? nthreads : 1)
  {
    ora_acts a;
    acts_alloc(&a, R);
#pragma omp for schedule(static)
    for (int t = 0; t < n; ++t)
      forward_tile(w, x + (size_t)t * R * R * 8, res, pad, &a, y + (size_t)t * res * res * 4);
    acts_free(&a);
  }
  return 0;
}

/* Backward of one tile given dY [res][res][4]: accumulates gw, writes gx
 * [R][R][8] if non-null. */
static void backward_tile(const double* w, const double* x, const double* dy, int res, int pad, ora_acts* a,
                          double* gw, double* gx, double* ybuf) {
  const int R = res + 2 * pad, R2 = R / 2, R4 = R / 4;
  const size_t f = (size_t)R * R, h = f / 4, q = f / 16;
  forward_tile(w, x, res, pad, a, ybuf);
  const double* W[NLAYER];
  double* GW[NLAYER];
  double* GB[NLAYER];
  for (int l = 0; l < NLAYER; ++l) {
    W[l] = w + layer_offset(l);
    GW[l] = gw + layer_offset(l);
    GB[l] = GW[l] + (size_t)LAYERS[l].cout * 9 * LAYERS[l].cin;
  }
  double* dXC = calloc(f * 24, sizeof(double));
  double* dA10 = calloc(f * 16, sizeof(double));
  double* dA9 = calloc(f * 16, sizeof(double));
  double* dU1 = calloc(f * 48, sizeof(double));
  double* dA8 = calloc(h * 32, sizeof(double));
  double* dA2 = calloc(f * 16, sizeof(double));
  double* dA7 = calloc(h * 32, sizeof(double));
  double* dU2 = calloc(h * 96, sizeof(double));
  double* dA6 = calloc(q * 64, sizeof(double));
  double* dA4 = calloc(h * 32, sizeof(double));
  double* dA5 = calloc(q * 64, sizeof(double));
  double* dP2 = calloc(q * 32, sizeof(double));
  double* dA3 = calloc(h * 32, sizeof(double));
  double* dP1 = calloc(h * 16, sizeof(double));
  double* dA1 = calloc(f * 16, sizeof(double));
  double* dX = calloc(f * 8, sizeof(double));
  /* head (no ReLU), crop window only */
  conv3x3_adj(a->XC, R, R, 24, W[HEAD], 4, dy, GW[HEAD], GB[HEAD], dXC, pad, pad + res, pad, pad + res);
  for (size_t p = 0; p < f; ++p) {
    for (int k = 0; k < 16; ++k) dA10[p * 16 + k] = dXC[p * 24 + k];
    for (int k = 0; k < 8; ++k) dX[p * 8 + k] = dXC[p * 24 + 16 + k];
  }
  /* residual: Y = crop(X sel) + head */
  static const int SEL[4] = {0, 2, 3, 4};
  for (int i = 0; i < res; ++i)
    for (int j = 0; j < res; ++j)
      for (int k = 0; k < 4; ++k)
        dX[((size_t)(i + pad) * R + (j + pad)) * 8 + SEL[k]] += dy[((size_t)i * res + j) * 4 + k];
  relu_mask(dA10, a->A[10], f * 16);
  conv3x3_adj(a->A[9], R, R, 16, W[D1B], 16, dA10, GW[D1B], GB[D1B], dA9, 0, R, 0, R);
  relu_mask(dA9, a->A[9], f * 16);
  conv3x3_adj(a->U1, R, R, 48, W[D1A], 16, dA9, GW[D1A], GB[D1A], dU1, 0, R, 0, R);
  up_concat_adj(dU1, 32, 16, R, R, dA8, dA2);
  relu_mask(dA8, a->A[8], h * 32);
  conv3x3_adj(a->A[7], R2, R2, 32, W[D2B], 32, dA8, GW[D2B], GB[D2B], dA7, 0, R2, 0, R2);
  relu_mask(dA7, a->A[7], h * 32);
  conv3x3_adj(a->U2, R2, R2, 96, W[D2A], 32, dA7, GW[D2A], GB[D2A], dU2, 0, R2, 0, R2);
  up_concat_adj(dU2, 64, 32, R2, R2, dA6, dA4);
  relu_mask(dA6, a->A[6], q * 64);
  conv3x3_adj(a->A[5], R4, R4, 64, W[BB], 64, dA6, GW[BB], GB[BB], dA5, 0, R4, 0, R4);
  relu_mask(dA5, a->A[5], q * 64);
  conv3x3_adj(a->P2, R4, R4, 32, W[BA], 64, dA5, GW[BA], GB[BA], dP2, 0, R4, 0, R4);
  avgpool2_adj(dP2, R2, R2, 32, dA4);
  relu_mask(dA4, a->A[4], h * 32);
  conv3x3_adj(a->A[3], R2, R2, 32, W[E2B], 32, dA4, GW[E2B], GB[E2B], dA3, 0, R2, 0, R2);
  relu_mask(dA3, a->A[3], h * 32);
  conv3x3_adj(a->P1, R2, R2, 16, W[E2A], 32, dA3, GW[E2A], GB[E2A], dP1, 0, R2, 0, R2);
  avgpool2_adj(dP1, R, R, 16, dA2);
  relu_mask(dA2, a->A[2], f * 16);
  conv3x3_adj(a->A[1], R, R, 16, W[E1B], 16, dA2, GW[E1B], GB[E1B], dA1, 0, R, 0, R);
  relu_mask(dA1, a->A[1], f * 16);
  conv3x3_adj(x, R, R, 8, W[E1A], 16, dA1, GW[E1A], GB[E1A], dX, 0, R, 0, R);
  if (gx) memcpy(gx, dX, sizeof(double) * f * 8);
  free(dXC); free(dA10); free(dA9); free(dU1); free(dA8); free(dA2); free(dA7); free(dU2);
  free(dA6); free(dA4); free(dA5); free(dP2); free(dA3); free(dP1); free(dA1); free(dX);
}

/* Batch backward.  gw [num_params] is overwritten with the sum over tiles;
 * gx [n][R][R][8] is optional.  The sum over tiles is taken in tile order
 * from per-tile gradients, so the result does not depend on nthreads. */
int ora_unet_backward(const double* w, const double* x, const double* dy, int n, int res, int pad, double* gw,
                      double* gx, int nthreads) {
  const int R = res + 2 * pad;
  if (R % 4) return -1;
  const size_t P = layer_offset(NLAYER);
  double* per = calloc((size_t)n * P, sizeof(double));
#pragma omp parallel num_threads(nthreads > 0 ? nthreads : 1)
  {
    ora_acts a;
    acts_alloc(&a, R);
    double* ybuf = malloc(sizeof(double) * (size_t)res * res * 4);
#pragma omp for schedule(dynamic, 1)
    for (int t = 0; t < n; ++t)
      backward_tile(w, x + (size_t)t * R * R * 8, dy + (size_t)t * res * res * 4, res, pad, &a, per + (size_t)t * P,
                    gx ? gx + (size_t)t * R * R * 8 : NULL, ybuf);
    free(ybuf);
    acts_free(&a);
  }
  for (size_t k = 0; k < P; ++k) {
    double s = 0.0;
    for (int t = 0; t < n; ++t) s += per[(size_t)t * P + k];
    gw[k] = s;
  }
  free(per);
  return 0;
}
