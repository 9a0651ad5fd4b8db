/* FP64 oracle: ground-truth heightmaps as per-texel means of all points, and
 * the training losses on the network's normalised output.  TEST
 * INFRASTRUCTURE ONLY (see ora.h).
 *
 * Section 3.4 (training data) builds each ground-truth heightmap and texture
 * by averaging every point that falls on a texel; texels without points are
 * gaps (NaN).  Section 3.4 (training) fits the network with a mean squared
 * error in which elements whose ground truth is NaN contribute zero, the
 * height and texture losses are clipped to [0, 1] and the two are averaged.
 * Readings taken here: the clip applies to every loss element (the squared
 * error of one texel channel), and the means run over all elements of the
 * crop, gaps included (their elements are zero).  The configured L1 loss
 * (half the mean absolute height error plus half the mean absolute colour
 * error, sign(0) = 0) is the second loss kind.
 */
#include <math.h>
#include <stdint.h>

static int64_t floordiv(int64_t a, int64_t b) {
  int64_t q = a / b;
  if ((a % b != 0) && ((a < 0) != (b < 0))) q -= 1;
  return q;
}

/* acc: [n_slots][res][res][5] = (sum z raw, sum R16, sum G16, sum B16,
 * count), accumulated (the caller zeroes it once).  Points are taken one by
 * one in input order; returns the number dropped (outside the region or in a
 * tile whose slot is negative). */
int64_t ora_splat_mean(int64_t ox, int64_t oy, int32_t tile_size, int32_t res, int32_t tiles_x, int32_t tiles_y,
                       const int32_t* x, const int32_t* y, const int32_t* z, const uint16_t* rgb, int64_t n,
                       const int32_t* tile_slot, int64_t* acc) {
  const int64_t C = tile_size / res;
  int64_t dropped = 0;
  for (int64_t i = 0; i < n; ++i) {
    const int64_t gx = floordiv((int64_t)x[i] - ox, C), gy = floordiv((int64_t)y[i] - oy, C);
    if (gx < 0 || gy < 0 || gx >= (int64_t)tiles_x * res || gy >= (int64_t)tiles_y * res) {
      ++dropped;
      continue;
    }
    const int32_t s = tile_slot[(gy / res) * tiles_x + gx / res];
    if (s < 0) {
      ++dropped;
      continue;
    }
    int64_t* a = acc + 5 * (((int64_t)s * res + gy % res) * res + gx % res);
    a[0] += z[i];
    a[1] += rgb[3 * i];
    a[2] += rgb[3 * i + 1];
    a[3] += rgb[3 * i + 2];
    a[4] += 1;
  }
  return dropped;
}

/* tex: [n_cells][4] = (mean height in metres, mean colour in [0, 1]); a texel
 * with no point is NaN in all four channels.  Height: the mean of the raw
 * heights (double division) times scale_z plus offset_z (double multiply,
 * double add, no contraction), rounded to float.  Colour: the mean of the
 * 16-bit values divided by 65535 in double, rounded to float. */
void ora_resolve_mean(const int64_t* acc, int64_t n_cells, double scale_z, double offset_z, float* tex) {
  for (int64_t i = 0; i < n_cells; ++i) {
    const int64_t* a = acc + 5 * i;
    if (a[4] == 0) {
      for (int c = 0; c < 4; ++c) tex[4 * i + c] = NAN;
      continue;
    }
    const double cnt = (double)a[4];
    double h = (double)a[0] / cnt;
    h = h * scale_z;
    h = h + offset_z;
    tex[4 * i] = (float)h;
    for (int c = 1; c < 4; ++c) {
      const double m = (double)a[c] / cnt;
      tex[4 * i + c] = (float)(m / 65535.0);
    }
  }
}

/* Loss of the normalised network output y [n][res][res][4] (h, r, g, b)
 * against a target texture t [n][res][res][4] (height in metres, colour in
 * [0, 1], NaN = no ground truth), both FP32 as stored.  The target height is
 * normalised like the input: (t_h - cz[tile]) / r_m.
 *   kind 0, clipped MSE:  e = min(d^2, 1),  dL/dy = d / N  where d^2 <= 1, else 0
 *   kind 1, L1:           e = |d|,          dL/dy = sign(d) / (2 N)
 * with d = y - t; L_h = sum e over heights / N_h, L_rgb = sum e over colours /
 * N_rgb, N_h = n*res*res, N_rgb = 3*N_h, L = (L_h + L_rgb) / 2 (for kind 0 the
 * gradient d/N is 0.5 * 2d/N).  Elements with a NaN target give e = 0 and a
 * zero gradient.  out[0..2] = L, L_h, L_rgb; grad (nullable) [n][res][res][4]. */
int ora_target_loss(const float* yv, const float* tv, const double* cz, int32_t n, int32_t res, double r_m,
                    int kind, double* out, double* grad) {
  if (kind != 0 && kind != 1) return -1;
  const int64_t px = (int64_t)res * res;
  const double Nh = (double)n * (double)px, Nc = 3.0 * Nh;
  double sh = 0.0, sc = 0.0;
  for (int32_t t = 0; t < n; ++t)
    for (int64_t p = 0; p < px; ++p)
      for (int c = 0; c < 4; ++c) {
        const int64_t k = ((int64_t)t * px + p) * 4 + c;
        const double N = c == 0 ? Nh : Nc;
        double g = 0.0, e = 0.0;
        if (!isnan(tv[k])) {
          const double target = c == 0 ? ((double)tv[k] - cz[t]) / r_m : (double)tv[k];
          const double d = (double)yv[k] - target;
          if (kind == 0) {
            const double sq = d * d;
            if (sq <= 1.0) {
              e = sq;
              g = d / N;
            } else {
              e = 1.0;
            }
          } else {
            e = fabs(d);
            g = (d > 0.0 ? 1.0 : (d < 0.0 ? -1.0 : 0.0)) / (2.0 * N);
          }
        }
        if (c == 0)
          sh += e;
        else
          sc += e;
        if (grad) grad[k] = g;
      }
  out[1] = sh / Nh;
  out[2] = sc / Nc;
  out[0] = 0.5 * (out[1] + out[2]);
  return 0;
}
