/* FP64 oracle: the paper's refinement network (Section 3.4, architecture
 * paragraph).  TEST INFRASTRUCTURE ONLY (see ora.h).
 *
 * The paper states the structure but its figure is missing: every input is
 * encoded by its own convolution layers, the feature vectors are merged by
 * separate fully connected layers in two steps, two separate CNNs decode the
 * merged vector to a heightmap and a texture, one skip connection
 * concatenates the original inputs with the decoder outputs, another CNN
 * reduces that to the output channels, and the centre res x res region is
 * kept; about 2.5 M parameters.  The layer sizes below are this build's
 * reading of it (2,528,708 parameters at R = 96):
 *
 *   inputs  I0 = h_lin (x channel 0), I1 = h_nn (1), I2 = rgb_lin (2-4),
 *           I3 = rgb_nn (5-7); c_i = 1, 1, 3, 3
 *   encoder i: four times  e = avgpool2(relu(conv3x3(e)))   c_i->16->32->32->32,
 *           R -> R/16; F_i = e flattened (row, column, channel), L = (R/16)^2 * 32
 *   FC1     z_h = relu(W1h [F_0, F_1] + b)   2L -> 256
 *           z_c = relu(W1c [F_2, F_3] + b)   2L -> 256
 *   FC2     d_h = relu(W2h [z_h, z_c] + b)   512 -> L   (an R/16 x R/16 x 32 image)
 *           d_t = relu(W2t [z_h, z_c] + b)   512 -> L
 *   decoder k (h, t): four times  a = relu(conv3x3(up2(a)))   32->32->32->16->16, R/16 -> R
 *   final   S = [a_h, a_t, X] (40 channels at R)
 *           f1 = relu(conv3x3(S)) 40->32, f2 = relu(conv3x3(f1)) 32->32,
 *           f3 = conv3x3(f2) 32->4, no ReLU, on the centre res x res crop
 *   output  Y = crop(X[..., {0, 2, 3, 4}]) + f3
 *
 * conv3x3: stride 1, zero padding; up2: nearest neighbour x2; avgpool2: mean
 * of 2 x 2.  Weights, in the order above: conv W[Cout][3][3][Cin] then
 * b[Cout]; fully connected W[N][K] then b[N] (K index = position in the
 * concatenated input).  Images are HWC.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct { int kind, cin, cout; } pn_layer; /* kind 0 conv3x3, 1 fully connected */

enum { PN_ENC = 0, PN_FC1H = 16, PN_FC1C, PN_FC2H, PN_FC2T, PN_DECH, PN_DECT = PN_DECH + 4, PN_F1 = PN_DECT + 4,
       PN_F2, PN_F3, PN_NL };

static void pn_layers(int R, pn_layer* L) {
  const int cin0[4] = {1, 1, 3, 3};
  const int F = (R / 16) * (R / 16) * 32;
  for (int i = 0; i < 4; ++i) {
    const int c[5] = {cin0[i], 16, 32, 32, 32};
    for (int k = 0; k < 4; ++k) L[4 * i + k] = (pn_layer){0, c[k], c[k + 1]};
  }
  L[PN_FC1H] = (pn_layer){1, 2 * F, 256};
  L[PN_FC1C] = (pn_layer){1, 2 * F, 256};
  L[PN_FC2H] = (pn_layer){1, 512, F};
  L[PN_FC2T] = (pn_layer){1, 512, F};
  const int d[5] = {32, 32, 32, 16, 16};
  for (int k = 0; k < 4; ++k) {
    L[PN_DECH + k] = (pn_layer){0, d[k], d[k + 1]};
    L[PN_DECT + k] = (pn_layer){0, d[k], d[k + 1]};
  }
  L[PN_F1] = (pn_layer){0, 40, 32};
  L[PN_F2] = (pn_layer){0, 32, 32};
  L[PN_F3] = (pn_layer){0, 32, 4};
}

static size_t pn_size(const pn_layer* l) {
  return l->kind == 0 ? (size_t)l->cout * 9 * l->cin + l->cout : (size_t)l->cout * l->cin + l->cout;
}

int64_t ora_pnet_num_params(int R) {
  if (R <= 0 || R % 16) return -1;
  pn_layer L[PN_NL];
  pn_layers(R, L);
  size_t n = 0;
  for (int k = 0; k < PN_NL; ++k) n += pn_size(&L[k]);
  return (int64_t)n;
}

/* out[y][x][co] = b[co] + sum w[co][ky][kx][ci] * in[y+ky-1][x+kx-1][ci]
 * over an H x W image whose pixels hold `stride` channels of which channels
 * [coff, coff + cin) are read; rows [y0, y1), columns [x0, x1). */
static void conv(const double* in, int H, int W, int stride, int coff, int cin, const double* w, const double* b,
                 int cout, double* out, int relu, int y0, int y1, int x0, int x1) {
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
            const double* ip = in + ((size_t)yy * W + xx) * stride + coff;
            for (int ci = 0; ci < cin; ++ci) s += wp[ci] * ip[ci];
          }
        }
        out[((size_t)(y - y0) * ow + (x - x0)) * cout + co] = (relu && s < 0.0) ? 0.0 : s;
      }
}

static void pool(const double* in, int H, int W, int c, double* out) {
  for (int y = 0; y < H / 2; ++y)
    for (int x = 0; x < W / 2; ++x)
      for (int k = 0; k < c; ++k) {
        const double s = in[((size_t)(2 * y) * W + 2 * x) * c + k] + in[((size_t)(2 * y) * W + 2 * x + 1) * c + k] +
                         in[((size_t)(2 * y + 1) * W + 2 * x) * c + k] +
                         in[((size_t)(2 * y + 1) * W + 2 * x + 1) * c + k];
        out[((size_t)y * (W / 2) + x) * c + k] = 0.25 * s;
      }
}

static void up2(const double* in, int h, int w, int c, double* out) {
  for (int y = 0; y < 2 * h; ++y)
    for (int x = 0; x < 2 * w; ++x)
      memcpy(out + ((size_t)y * 2 * w + x) * c, in + ((size_t)(y / 2) * w + x / 2) * c, sizeof(double) * c);
}

/* out[n] = relu?(b[n] + sum_k W[n][k] * in[k]), in = [a (ka values), b (kb values)] */
static void fc(const double* a, int ka, const double* bv, int kb, const double* w, const double* bias, int N,
               double* out, int relu) {
  const int K = ka + kb;
  for (int n = 0; n < N; ++n) {
    double s = bias[n];
    const double* wr = w + (size_t)n * K;
    for (int k = 0; k < ka; ++k) s += wr[k] * a[k];
    for (int k = 0; k < kb; ++k) s += wr[ka + k] * bv[k];
    out[n] = (relu && s < 0.0) ? 0.0 : s;
  }
}

static void forward_tile(const double* w, const double* x, int res, int pad, double* y) {
  const int R = res + 2 * pad;
  pn_layer L[PN_NL];
  pn_layers(R, L);
  const double* wl[PN_NL];
  {
    size_t off = 0;
    for (int k = 0; k < PN_NL; ++k) {
      wl[k] = w + off;
      off += pn_size(&L[k]);
    }
  }
#define WB(k) wl[k], wl[k] + (size_t)L[k].cout * (L[k].kind == 0 ? 9 * L[k].cin : L[k].cin)
  const int F = (R / 16) * (R / 16) * 32;
  const size_t big = (size_t)R * R * 40;
  double* t0 = malloc(sizeof(double) * big);
  double* t1 = malloc(sizeof(double) * big);
  double* feat[4];
  const int coff0[4] = {0, 1, 2, 5};
  for (int i = 0; i < 4; ++i) {
    feat[i] = malloc(sizeof(double) * F);
    /* encoder i: conv at h, then pool to h / 2 */
    int h = R;
    const double* src = x;
    int stride = 8, coff = coff0[i];
    for (int k = 0; k < 4; ++k) {
      const pn_layer* l = &L[4 * i + k];
      conv(src, h, h, stride, coff, l->cin, WB(4 * i + k), l->cout, t0, 1, 0, h, 0, h);
      pool(t0, h, h, l->cout, k == 3 ? feat[i] : t1);
      h /= 2;
      src = t1;
      stride = l->cout;
      coff = 0;
    }
  }
  double zh[256], zc[256], zz[512];
  fc(feat[0], F, feat[1], F, WB(PN_FC1H), 256, zh, 1);
  fc(feat[2], F, feat[3], F, WB(PN_FC1C), 256, zc, 1);
  memcpy(zz, zh, sizeof zh);
  memcpy(zz + 256, zc, sizeof zc);
  double* S = malloc(sizeof(double) * (size_t)R * R * 40);
  double* d = malloc(sizeof(double) * F);
  for (int k = 0; k < 2; ++k) {
    fc(zz, 512, NULL, 0, WB(k == 0 ? PN_FC2H : PN_FC2T), F, d, 1);
    /* decoder: up, conv; R/16 -> R */
    int h = R / 16;
    memcpy(t1, d, sizeof(double) * F);
    for (int j = 0; j < 4; ++j) {
      const int li = (k == 0 ? PN_DECH : PN_DECT) + j;
      up2(t1, h, h, L[li].cin, t0);
      h *= 2;
      conv(t0, h, h, L[li].cin, 0, L[li].cin, WB(li), L[li].cout, t1, 1, 0, h, 0, h);
    }
    /* a_k (16 channels at R) into channels [16 k, 16 k + 16) of S */
    for (size_t p = 0; p < (size_t)R * R; ++p) memcpy(S + p * 40 + 16 * k, t1 + p * 16, sizeof(double) * 16);
  }
  for (size_t p = 0; p < (size_t)R * R; ++p) memcpy(S + p * 40 + 32, x + p * 8, sizeof(double) * 8);
  conv(S, R, R, 40, 0, 40, WB(PN_F1), 32, t0, 1, 0, R, 0, R);
  conv(t0, R, R, 32, 0, 32, WB(PN_F2), 32, t1, 1, 0, R, 0, R);
  double* f3 = malloc(sizeof(double) * (size_t)res * res * 4);
  conv(t1, R, R, 32, 0, 32, WB(PN_F3), 4, f3, 0, pad, pad + res, pad, pad + res);
  const int ch[4] = {0, 2, 3, 4};
  for (int i = 0; i < res; ++i)
    for (int j = 0; j < res; ++j)
      for (int c = 0; c < 4; ++c)
        y[((size_t)i * res + j) * 4 + c] = x[((size_t)(i + pad) * R + (j + pad)) * 8 + ch[c]] + f3[((size_t)i * res + j) * 4 + c];
#undef WB
  for (int i = 0; i < 4; ++i) free(feat[i]);
  free(t0);
  free(t1);
  free(S);
  free(d);
  free(f3);
}

/* y [n][res][res][4] from x [n][R][R][8]; returns -1 when R is not a
 * multiple of 16. */
int ora_pnet_forward(const double* w, const double* x, int n, int res, int pad, double* y, int nthreads) {
  const int R = res + 2 * pad;
  if (R <= 0 || R % 16) return -1;
#pragma omp parallel for num_threads(nthreads > 0 ? nthreads : 1) schedule(dynamic, 1)
  for (int t = 0; t < n; ++t)
    forward_tile(w, x + (size_t)t * R * R * 8, res, pad, y + (size_t)t * res * res * 4);
  return 0;
}
