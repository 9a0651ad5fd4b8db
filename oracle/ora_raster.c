/* FP64 oracle: point rasteriser with packed 64-bit depth-and-colour keys and
 * a resolve pass.  TEST INFRASTRUCTURE ONLY (see ora.h).
 *
 * Section 3.6 (rendering, points): every point is projected to the screen,
 * its depth and colour are packed into one 64-bit integer and each pixel
 * keeps the smallest (the nearest point) with a 64-bit atomic minimum; a
 * screen-space resolve pass then takes the colour from the low bits.
 *
 * Definitions used here (the paper gives the technique, not the maths):
 *  world position, metres, relative to the camera origin (ox, oy):
 *    X = (x - ox) * sx,  Y = (y - oy) * sx,  Z = z * sz + oz
 *  clip = M * (X, Y, Z, 1), M row-major 4 x 4, each row summed left to
 *    right (((m0 X + m1 Y) + m2 Z) + m3), double precision, no contraction;
 *  a point is drawn iff w > 0 and both ndc = clip / w lie in [-1, 1);
 *  pixel column floor(((ndc_x + 1) * 0.5) * width), row likewise with
 *    height (row 0 at ndc_y = -1);
 *  key = bits(float(w)) << 32 | 0xFF << 24 | B8 << 16 | G8 << 8 | R8, with
 *    C8 = C16 >> 8 (positive floats order like their bit patterns, so the
 *    smallest key is the nearest point; ties go to the smaller colour word);
 *  an empty pixel holds all ones; the resolve writes the low 32 bits (RGBA8,
 *    alpha 255) of every other pixel and 0 for the empty ones.
 * Points are taken one by one, in input order.
 */
#include <math.h>
#include <stdint.h>
#include <string.h>

/* Returns the number of points drawn (inside the view). */
int64_t ora_raster(const double* M, int64_t ox, int64_t oy, double sx, double sz, double oz, int32_t width,
                   int32_t height, const int32_t* x, const int32_t* y, const int32_t* z, const uint16_t* rgb,
                   int64_t n, uint64_t* fb) {
  int64_t drawn = 0;
  for (int64_t i = 0; i < n; ++i) {
    const double X = (double)((int64_t)x[i] - ox) * sx;
    const double Y = (double)((int64_t)y[i] - oy) * sx;
    double Z = (double)z[i] * sz;
    Z = Z + oz;
    double c[4];
    for (int r = 0; r < 4; ++r) {
      double a = M[4 * r] * X;
      a = a + M[4 * r + 1] * Y;
      a = a + M[4 * r + 2] * Z;
      a = a + M[4 * r + 3];
      c[r] = a;
    }
    const double w = c[3];
    if (!(w > 0.0)) continue;
    const double nx = c[0] / w, ny = c[1] / w;
    if (!(nx >= -1.0 && nx < 1.0 && ny >= -1.0 && ny < 1.0)) continue;
    const int64_t px = (int64_t)floor(((nx + 1.0) * 0.5) * (double)width);
    const int64_t py = (int64_t)floor(((ny + 1.0) * 0.5) * (double)height);
    if (px < 0 || px >= width || py < 0 || py >= height) continue;
    const float d = (float)w;
    uint32_t db;
    memcpy(&db, &d, 4);
    const uint64_t col = (uint64_t)0xFF << 24 | (uint64_t)(rgb[3 * i + 2] >> 8) << 16 |
                         (uint64_t)(rgb[3 * i + 1] >> 8) << 8 | (uint64_t)(rgb[3 * i] >> 8);
    const uint64_t key = ((uint64_t)db << 32) | col;
    uint64_t* p = fb + py * (int64_t)width + px;
    if (key < *p) *p = key;
    ++drawn;
  }
  return drawn;
}

void ora_raster_resolve(const uint64_t* fb, int64_t n_pixels, uint32_t* rgba) {
  for (int64_t i = 0; i < n_pixels; ++i) rgba[i] = fb[i] == UINT64_MAX ? 0u : (uint32_t)(fb[i] & 0xFFFFFFFFu);
}
