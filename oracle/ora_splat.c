/* FP64 oracle: full-resolution splat into the heightmap textures and the
 * resolve pass.  TEST INFRASTRUCTURE ONLY (see ora.h).
 *
 * Section 3.5 keeps some of the unloaded full-resolution detail by updating
 * the heightmap textures; Section 3.6 encodes depth and colour in one 64-bit
 * word reduced with an atomic and decoded by a resolve pass.  The update
 * operator is not named; it is read here as the per-texel maximum height:
 *   key = ((z as uint32) ^ 0x80000000) << 32 | R8 << 24 | G8 << 16 | B8 << 8 | 0xFF
 * (R8 = R16 >> 8), so a larger key means a higher point, ties going to the
 * larger packed colour; 0 means "no point".  The oracle takes the points one
 * by one, in input order, and keeps the maximum per texel.
 */
#include <stdint.h>

static int64_t floordiv(int64_t a, int64_t b) {
  int64_t q = a / b;
  if ((a % b != 0) && ((a < 0) != (b < 0))) q -= 1;
  return q;
}

/* keys: [n_slots][res][res] (row = y).  Returns the number of dropped points
 * (outside the region or in a tile whose slot is negative). */
int64_t ora_splat(int64_t ox, int64_t oy, int32_t tile_size, int32_t res, int32_t tiles_x, int32_t tiles_y,
                  const int32_t* x, const int32_t* y, const int32_t* z, const uint16_t* rgb, int64_t n,
                  const int32_t* tile_slot, uint64_t* keys) {
  const int64_t C = tile_size / res;
  int64_t dropped = 0;
  for (int64_t i = 0; i < n; ++i) {
    const int64_t gx = floordiv((int64_t)x[i] - ox, C), gy = floordiv((int64_t)y[i] - oy, C);
    if (gx < 0 || gy < 0 || gx >= (int64_t)tiles_x * res || gy >= (int64_t)tiles_y * res) { ++dropped; continue; }
    const int64_t tx = gx / res, ty = gy / res;
    const int32_t s = tile_slot[ty * tiles_x + tx];
    if (s < 0) { ++dropped; continue; }
    const uint64_t hi = (uint64_t)((uint32_t)z[i] ^ 0x80000000u);
    const uint64_t key = (hi << 32) | ((uint64_t)(rgb[3 * i] >> 8) << 24) | ((uint64_t)(rgb[3 * i + 1] >> 8) << 16) |
                         ((uint64_t)(rgb[3 * i + 2] >> 8) << 8) | 0xFFu;
    const int64_t cell = ((int64_t)s * res + (gy % res)) * res + (gx % res);
    if (key > keys[cell]) keys[cell] = key;
  }
  return dropped;
}

/* tex: [n_cells][4] = (h metres, r, g, b in [0,1]); texels whose key is 0
 * keep their value.  h = (float)(z * scale_z + offset_z) with a double
 * multiply and a double add (built without contraction); colour = byte / 255. */
void ora_resolve(const uint64_t* keys, int64_t n_cells, double scale_z, double offset_z, float* tex) {
  for (int64_t i = 0; i < n_cells; ++i) {
    const uint64_t k = keys[i];
    if (k == 0) continue;
    const int32_t zr = (int32_t)((uint32_t)(k >> 32) ^ 0x80000000u);
    double h = (double)zr * scale_z;
    h = h + offset_z;
    tex[4 * i] = (float)h;
    tex[4 * i + 1] = (float)((k >> 24) & 0xFF) / 255.0f;
    tex[4 * i + 2] = (float)((k >> 16) & 0xFF) / 255.0f;
    tex[4 * i + 3] = (float)((k >> 8) & 0xFF) / 255.0f;
  }
}
