/* FP64 CPU oracle for LidarScout's per-tile heightmap hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this code.  It shares no code,
 * header, table or constant with the HIP library: the geometry, network and
 * splat are written again here from the paper's definitions, in the plainest
 * form, so that the GPU path can be checked against it.
 *
 * Units: x, y, z are LAS raw integers (1 raw = scale metres).  Tile-local
 * coordinates u = x - cx, v = y - cy are exact int64.  Heights in metres
 * are z * scale_z + offset_z in double precision.
 */
#ifndef LIDARSCOUT_ORACLE_H
#define LIDARSCOUT_ORACLE_H
#include <stdint.h>

#define ORA_OK 0
#define ORA_EMPTY 1
#define ORA_NN_ONLY 2

typedef struct {
  int64_t origin_x, origin_y;
  int32_t tile_size, res, pad, tiles_x, tiles_y;
  double scale_xy, scale_z, offset_z;
} ora_grid;

/* one tile-local sparse point */
typedef struct {
  int64_t u, v;
  int32_t z;
  int32_t rgb[3];
} ora_pt;

#endif
