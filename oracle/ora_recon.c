/* FP64 oracle: tile binning, canonicalisation, nearest-neighbour and
 * Delaunay-linear interpolation, normalisation (LidarScout, Sections 3.3-3.4,
 * Algorithm 1).  TEST INFRASTRUCTURE ONLY (see ora.h).
 *
 * Readings of the paper taken here:
 *  - a tile's sparse input is every point in its padded window
 *    [c - H, c + H)^2, H = tile/2 + pad * cell (the grid-based structure of
 *    Section 3.3 hands each patch its nearby chunk points);
 *  - grid sample j of row i sits at the texel centre
 *    (-H + cell/2 + j*cell, -H + cell/2 + i*cell), rows along +y (Algorithm 1
 *    grid G, at the 10 m/texel spacing of Section 3.1);
 *  - the corner padding points of Algorithm 1 are taken at infinity, so
 *    linear interpolation covers exactly the closed convex hull and every
 *    other texel takes the nearest point (Algorithm 1 "outside convex hull");
 *  - duplicate (u, v) keep the lexicographically largest (z, R, G, B);
 *  - nearest-neighbour ties go to the smallest (d^2, v, u);
 *  - c_z is the linear height at texel (R/2, R/2) and r is the padded half
 *    side H in metres (Section 3.4 normalisation).
 */
#include "ora.h"

#include <stdlib.h>
#include <string.h>

typedef __int128 i128;

static int64_t floordiv(int64_t a, int64_t b) {
  int64_t q = a / b;
  if ((a % b != 0) && ((a < 0) != (b < 0))) q -= 1;
  return q;
}

static int64_t half_window(const ora_grid* g) {
  return (int64_t)g->tile_size / 2 + (int64_t)g->pad * (g->tile_size / g->res);
}

/* ------------------------------------------------------------------------ */
/* Binning: bin k lists, in ascending input order, every point inside the
 * padded window of tile tile_list[k].  Returns the total entry count; fills
 * bin_idx only when it fits in cap.                                         */
int64_t ora_bin(const ora_grid* g, const int32_t* x, const int32_t* y, int64_t n,
                const int32_t* tile_list, int32_t n_tiles, int64_t* bin_off,
                int32_t* bin_idx, int64_t cap) {
  const int64_t S = g->tile_size, H = half_window(g);
  const int64_t nt = (int64_t)g->tiles_x * g->tiles_y;
  int32_t* slot = (int32_t*)malloc(sizeof(int32_t) * (size_t)nt);
  int64_t* fill = (int64_t*)calloc((size_t)n_tiles + 1, sizeof(int64_t));
  for (int64_t t = 0; t < nt; ++t) slot[t] = -1;
  for (int32_t k = 0; k < n_tiles; ++k)
    if (tile_list[k] >= 0 && tile_list[k] < nt && slot[tile_list[k]] < 0) slot[tile_list[k]] = k;
  /* windows reach at most K tiles beyond the tile that holds the point */
  const int64_t K = 1 + H / S;
  for (int pass = 0; pass < 2; ++pass) {
    if (pass == 1) {
      int64_t run = 0;
      for (int32_t k = 0; k < n_tiles; ++k) {
        int64_t c = fill[k];
        bin_off[k] = run;
        fill[k] = run;
        run += c;
      }
      bin_off[n_tiles] = run;
      if (run > cap) break;
    }
    for (int64_t i = 0; i < n; ++i) {
      const int64_t px = x[i], py = y[i];
      const int64_t tx0 = floordiv(px - g->origin_x, S), ty0 = floordiv(py - g->origin_y, S);
      for (int64_t ty = ty0 - K; ty <= ty0 + K; ++ty) {
        if (ty < 0 || ty >= g->tiles_y) continue;
        const int64_t cy = g->origin_y + ty * S + S / 2;
        if (!(cy - H <= py && py < cy + H)) continue;
        for (int64_t tx = tx0 - K; tx <= tx0 + K; ++tx) {
          if (tx < 0 || tx >= g->tiles_x) continue;
          const int64_t cx = g->origin_x + tx * S + S / 2;
          if (!(cx - H <= px && px < cx + H)) continue;
          const int32_t s = slot[ty * g->tiles_x + tx];
          if (s < 0) continue;
          if (pass == 0) fill[s] += 1;
          else bin_idx[fill[s]++] = (int32_t)i;
        }
      }
    }
  }
  int64_t total = bin_off[n_tiles];
  if (n_tiles == 0) total = 0;
  free(slot);
  free(fill);
  return total;
}

/* ------------------------------------------------------------------------ */
/* Canonicalisation: sort by (v, u), keep one point per (u, v): the one with
 * the largest (z, R, G, B).  Returns the number of unique points.           */
static int cmp_pt(const void* A, const void* B) {
  const ora_pt* a = (const ora_pt*)A;
  const ora_pt* b = (const ora_pt*)B;
  if (a->v != b->v) return a->v < b->v ? -1 : 1;
  if (a->u != b->u) return a->u < b->u ? -1 : 1;
  if (a->z != b->z) return a->z > b->z ? -1 : 1; /* larger first */
  for (int c = 0; c < 3; ++c)
    if (a->rgb[c] != b->rgb[c]) return a->rgb[c] > b->rgb[c] ? -1 : 1;
  return 0;
}

int ora_canon(ora_pt* p, int m) {
  if (m <= 0) return 0;
  qsort(p, (size_t)m, sizeof(ora_pt), cmp_pt);
  int w = 1;
  for (int i = 1; i < m; ++i)
    if (p[i].u != p[w - 1].u || p[i].v != p[w - 1].v) p[w++] = p[i];
  return w;
}

/* ------------------------------------------------------------------------ */
/* exact predicates */
static int64_t orient(const ora_pt* a, const ora_pt* b, int64_t qx, int64_t qy) {
  return (b->u - a->u) * (qy - a->v) - (b->v - a->v) * (qx - a->u);
}

/* > 0 iff d lies strictly inside the circle through a, b, c (a, b, c CCW) */
static int incircle(const ora_pt* a, const ora_pt* b, const ora_pt* c, const ora_pt* d) {
  const int64_t adx = a->u - d->u, ady = a->v - d->v;
  const int64_t bdx = b->u - d->u, bdy = b->v - d->v;
  const int64_t cdx = c->u - d->u, cdy = c->v - d->v;
  const i128 al = (i128)adx * adx + (i128)ady * ady;
  const i128 bl = (i128)bdx * bdx + (i128)bdy * bdy;
  const i128 cl = (i128)cdx * cdx + (i128)cdy * cdy;
  const i128 det = al * (i128)(bdx * cdy - cdx * bdy) + bl * (i128)(cdx * ady - adx * cdy) +
                   cl * (i128)(adx * bdy - bdx * ady);
  return (det > 0) - (det < 0);
}

/* ------------------------------------------------------------------------ */
/* Nearest point to (qx, qy): smallest (d^2, v, u).  Brute force.            */
int ora_nearest(const ora_pt* p, int m, int64_t qx, int64_t qy) {
  int best = -1;
  int64_t bd = 0;
  for (int i = 0; i < m; ++i) {
    const int64_t dx = p[i].u - qx, dy = p[i].v - qy;
    const int64_t d = dx * dx + dy * dy;
    if (best < 0 || d < bd || (d == bd && (p[i].v < p[best].v || (p[i].v == p[best].v && p[i].u < p[best].u)))) {
      best = i;
      bd = d;
    }
  }
  return best;
}

/* ------------------------------------------------------------------------ */
/* Delaunay triangulation by Bowyer-Watson insertion.  The unbounded side is
 * handled with a ghost vertex: ghost triangle (a, b, G) stands for hull edge
 * a->b with the outside on its left, and "contains" a point strictly left of
 * a->b or strictly inside the segment ab.  Each insertion removes every
 * triangle whose (open) circumdisk holds the new point and re-triangulates
 * the cavity from it.  Points are inserted in a seeded random order.
 * Output: CCW real triangles as index triples; returns their count, 0 if
 * the points are fewer than 3 or all collinear, -1 if cap is too small.     */
#define GHOST (-1)
typedef struct { int v[3]; int alive; } ora_tri;

static int tri_contains(const ora_pt* p, const ora_tri* t, int q) {
  if (t->v[2] != GHOST) return incircle(&p[t->v[0]], &p[t->v[1]], &p[t->v[2]], &p[q]) > 0;
  const ora_pt* a = &p[t->v[0]];
  const ora_pt* b = &p[t->v[1]];
  const int64_t o = orient(a, b, p[q].u, p[q].v);
  if (o > 0) return 1;
  if (o < 0) return 0;
  /* collinear: inside the open segment? */
  const int64_t d1 = (p[q].u - a->u) * (b->u - a->u) + (p[q].v - a->v) * (b->v - a->v);
  const int64_t d2 = (p[q].u - b->u) * (a->u - b->u) + (p[q].v - b->v) * (a->v - b->v);
  return d1 > 0 && d2 > 0;
}

static uint64_t xorshift(uint64_t* s) {
  uint64_t x = *s;
  x ^= x << 13;
  x ^= x >> 7;
  x ^= x << 17;
  *s = x;
  return x;
}

int ora_delaunay(const ora_pt* p, int m, uint64_t seed, int32_t* tri_out, int cap) {
  if (m < 3) return 0;
  int i2 = -1;
  for (int k = 2; k < m; ++k)
    if (orient(&p[0], &p[1], p[k].u, p[k].v) != 0) { i2 = k; break; }
  if (i2 < 0) return 0;

  int ntri_cap = 4 * m + 16;
  ora_tri* T = (ora_tri*)malloc(sizeof(ora_tri) * (size_t)ntri_cap);
  int nt = 0;
  int a = 0, b = 1, c = i2;
  if (orient(&p[a], &p[b], p[c].u, p[c].v) < 0) { int t = a; a = b; b = t; }
  ora_tri t0 = {{a, b, c}, 1}, g0 = {{b, a, GHOST}, 1}, g1 = {{c, b, GHOST}, 1}, g2 = {{a, c, GHOST}, 1};
  T[nt++] = t0; T[nt++] = g0; T[nt++] = g1; T[nt++] = g2;

  /* insertion order: the remaining points, shuffled */
  int* order = (int*)malloc(sizeof(int) * (size_t)m);
  int no = 0;
  for (int k = 0; k < m; ++k)
    if (k != 0 && k != 1 && k != i2) order[no++] = k;
  uint64_t s = seed * 2654435761u + 0x9E3779B97F4A7C15ull;
  if (s == 0) s = 1;
  for (int k = no - 1; k > 0; --k) {
    int j = (int)(xorshift(&s) % (uint64_t)(k + 1));
    int t = order[k]; order[k] = order[j]; order[j] = t;
  }

  int* cav = (int*)malloc(sizeof(int) * (size_t)ntri_cap);
  int* bnd = (int*)malloc(sizeof(int) * 2 * (size_t)ntri_cap);
  for (int oi = 0; oi < no; ++oi) {
    const int q = order[oi];
    int nc = 0;
    for (int t = 0; t < nt; ++t)
      if (T[t].alive && tri_contains(p, &T[t], q)) cav[nc++] = t;
    /* boundary: directed cavity edges whose reverse is not a cavity edge */
    int nb = 0;
    for (int i = 0; i < nc; ++i) {
      const int* tv = T[cav[i]].v;
      for (int e = 0; e < 3; ++e) {
        const int e0 = tv[e], e1 = tv[(e + 1) % 3];
        int shared = 0;
        for (int j = 0; j < nc && !shared; ++j) {
          if (j == i) continue;
          const int* uv = T[cav[j]].v;
          for (int f = 0; f < 3; ++f)
            if (uv[f] == e1 && uv[(f + 1) % 3] == e0) { shared = 1; break; }
        }
        if (!shared) { bnd[2 * nb] = e0; bnd[2 * nb + 1] = e1; ++nb; }
      }
    }
    for (int i = 0; i < nc; ++i) T[cav[i]].alive = 0;
    /* compact when needed */
    if (nt + nb > ntri_cap) {
      int w = 0;
      for (int t = 0; t < nt; ++t)
        if (T[t].alive) T[w++] = T[t];
      nt = w;
      if (nt + nb > ntri_cap) {
        ntri_cap = 2 * (nt + nb);
        T = (ora_tri*)realloc(T, sizeof(ora_tri) * (size_t)ntri_cap);
        cav = (int*)realloc(cav, sizeof(int) * (size_t)ntri_cap);
        bnd = (int*)realloc(bnd, sizeof(int) * 2 * (size_t)ntri_cap);
      }
    }
    for (int i = 0; i < nb; ++i) {
      const int e0 = bnd[2 * i], e1 = bnd[2 * i + 1];
      ora_tri nw;
      nw.alive = 1;
      if (e0 == GHOST) { nw.v[0] = e1; nw.v[1] = q; nw.v[2] = GHOST; }
      else if (e1 == GHOST) { nw.v[0] = q; nw.v[1] = e0; nw.v[2] = GHOST; }
      else { nw.v[0] = e0; nw.v[1] = e1; nw.v[2] = q; }
      T[nt++] = nw;
    }
  }
  int out = 0;
  for (int t = 0; t < nt; ++t) {
    if (!T[t].alive || T[t].v[2] == GHOST) continue;
    if (out < cap) {
      tri_out[3 * out] = T[t].v[0];
      tri_out[3 * out + 1] = T[t].v[1];
      tri_out[3 * out + 2] = T[t].v[2];
    }
    ++out;
  }
  free(T); free(order); free(cav); free(bnd);
  return out <= cap ? out : -1;
}

/* ------------------------------------------------------------------------ */
/* One tile, Algorithm 1 + normalisation.  pts: the tile's points (raw, in any
 * order; canonicalised in place).  Outputs (all optional except xout/cz):
 *   xout[R][R][8]: [(h_lin-cz)/r, (h_nn-cz)/r, rgb_lin/65535, rgb_nn/65535]
 *   hm_nn, hm_lin [R][R] in metres; nn_idx [R][R] (canonical index, -1 if
 *   empty); inside [R][R] (1 where linear interpolation applied).
 * Returns the tile status (ORA_OK / ORA_EMPTY / ORA_NN_ONLY).               */
int ora_recon_tile(const ora_grid* g, ora_pt* pts, int m_raw, uint64_t seed, double* xout, double* cz_out,
                   double* hm_nn, double* hm_lin, int32_t* nn_idx, int8_t* inside, int32_t* n_unique) {
  const int R = g->res + 2 * g->pad;
  const int64_t C = g->tile_size / g->res;
  const int64_t H = half_window(g);
  const double r_m = (double)H * g->scale_xy;
  const int m = ora_canon(pts, m_raw);
  if (n_unique) *n_unique = m;
  const size_t NT = (size_t)R * R;
  double* lin = (double*)malloc(sizeof(double) * NT * 4);
  double* nnv = (double*)malloc(sizeof(double) * NT * 4);
  int8_t* ins = (int8_t*)calloc(NT, 1);
  int status = ORA_OK;
  if (m == 0) {
    memset(xout, 0, sizeof(double) * NT * 8);
    *cz_out = 0.0;
    if (hm_nn) memset(hm_nn, 0, sizeof(double) * NT);
    if (hm_lin) memset(hm_lin, 0, sizeof(double) * NT);
    if (nn_idx) for (size_t k = 0; k < NT; ++k) nn_idx[k] = -1;
    if (inside) memset(inside, 0, NT);
    free(lin); free(nnv); free(ins);
    return ORA_EMPTY;
  }
  /* NN interpolation for every texel (Algorithm 1, "NN Interpolation") */
  for (int i = 0; i < R; ++i)
    for (int j = 0; j < R; ++j) {
      const int64_t qx = -H + C / 2 + (int64_t)j * C, qy = -H + C / 2 + (int64_t)i * C;
      const int k = ora_nearest(pts, m, qx, qy);
      const size_t t = (size_t)i * R + j;
      nnv[4 * t] = (double)pts[k].z * g->scale_z + g->offset_z;
      for (int c = 0; c < 3; ++c) nnv[4 * t + 1 + c] = (double)pts[k].rgb[c];
      if (nn_idx) nn_idx[t] = k;
    }
  /* Delaunay triangulation and linear interpolation inside the hull */
  int32_t* tri = (int32_t*)malloc(sizeof(int32_t) * 3 * (size_t)(2 * m + 8));
  const int ntri = ora_delaunay(pts, m, seed, tri, 2 * m + 8);
  if (ntri <= 0) status = ORA_NN_ONLY;
  int64_t* bb = (int64_t*)malloc(sizeof(int64_t) * 4 * (size_t)(ntri > 0 ? ntri : 1));
  for (int t = 0; t < ntri; ++t) {
    int64_t x0 = pts[tri[3 * t]].u, x1 = x0, y0 = pts[tri[3 * t]].v, y1 = y0;
    for (int e = 1; e < 3; ++e) {
      const ora_pt* q = &pts[tri[3 * t + e]];
      if (q->u < x0) x0 = q->u;
      if (q->u > x1) x1 = q->u;
      if (q->v < y0) y0 = q->v;
      if (q->v > y1) y1 = q->v;
    }
    bb[4 * t] = x0; bb[4 * t + 1] = x1; bb[4 * t + 2] = y0; bb[4 * t + 3] = y1;
  }
  for (int i = 0; i < R; ++i)
    for (int j = 0; j < R; ++j) {
      const int64_t qx = -H + C / 2 + (int64_t)j * C, qy = -H + C / 2 + (int64_t)i * C;
      const size_t tt = (size_t)i * R + j;
      int found = -1;
      for (int t = 0; t < ntri && found < 0; ++t) {
        if (qx < bb[4 * t] || qx > bb[4 * t + 1] || qy < bb[4 * t + 2] || qy > bb[4 * t + 3]) continue;
        const ora_pt* a = &pts[tri[3 * t]];
        const ora_pt* b = &pts[tri[3 * t + 1]];
        const ora_pt* c = &pts[tri[3 * t + 2]];
        if (orient(a, b, qx, qy) >= 0 && orient(b, c, qx, qy) >= 0 && orient(c, a, qx, qy) >= 0) found = t;
      }
      if (found >= 0) {
        const ora_pt* a = &pts[tri[3 * found]];
        const ora_pt* b = &pts[tri[3 * found + 1]];
        const ora_pt* c = &pts[tri[3 * found + 2]];
        const double area = (double)orient(a, b, c->u, c->v);
        const double la = (double)orient(b, c, qx, qy) / area;
        const double lb = (double)orient(c, a, qx, qy) / area;
        const double lc = (double)orient(a, b, qx, qy) / area;
        const double za = (double)a->z * g->scale_z + g->offset_z;
        const double zb = (double)b->z * g->scale_z + g->offset_z;
        const double zc = (double)c->z * g->scale_z + g->offset_z;
        lin[4 * tt] = la * za + lb * zb + lc * zc;
        for (int k = 0; k < 3; ++k)
          lin[4 * tt + 1 + k] = la * (double)a->rgb[k] + lb * (double)b->rgb[k] + lc * (double)c->rgb[k];
        ins[tt] = 1;
      } else {
        for (int k = 0; k < 4; ++k) lin[4 * tt + k] = nnv[4 * tt + k];
      }
    }
  /* normalisation (Section 3.4) */
  const double cz = lin[4 * ((size_t)(R / 2) * R + R / 2)];
  *cz_out = cz;
  for (size_t t = 0; t < NT; ++t) {
    xout[8 * t + 0] = (lin[4 * t] - cz) / r_m;
    xout[8 * t + 1] = (nnv[4 * t] - cz) / r_m;
    for (int k = 0; k < 3; ++k) {
      xout[8 * t + 2 + k] = lin[4 * t + 1 + k] / 65535.0;
      xout[8 * t + 5 + k] = nnv[4 * t + 1 + k] / 65535.0;
    }
    if (hm_nn) hm_nn[t] = nnv[4 * t];
    if (hm_lin) hm_lin[t] = lin[4 * t];
    if (inside) inside[t] = ins[t];
  }
  free(lin); free(nnv); free(ins); free(tri); free(bb);
  return status;
}

/* ------------------------------------------------------------------------ */
/* Whole batch: bin, then reconstruct every listed tile.  x_out is
 * [n_tiles][R][R][8], cz [n_tiles], status [n_tiles].                       */
int ora_recon_tiles(const ora_grid* g, const int32_t* x, const int32_t* y, const int32_t* z,
                    const uint16_t* rgb, int64_t n, const int32_t* tile_list, int32_t n_tiles,
                    double* x_out, double* cz, int32_t* status, int nthreads) {
  int64_t* off = (int64_t*)malloc(sizeof(int64_t) * ((size_t)n_tiles + 1));
  const int64_t total = ora_bin(g, x, y, n, tile_list, n_tiles, off, NULL, 0);
  int32_t* idx = (int32_t*)malloc(sizeof(int32_t) * (size_t)(total > 0 ? total : 1));
  ora_bin(g, x, y, n, tile_list, n_tiles, off, idx, total);
  const int R = g->res + 2 * g->pad;
  const int64_t S = g->tile_size;
  (void)nthreads;
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads > 0 ? nthreads : 1)
  for (int32_t k = 0; k < n_tiles; ++k) {
    const int32_t t = tile_list[k];
    const int64_t cx = g->origin_x + (int64_t)(t % g->tiles_x) * S + S / 2;
    const int64_t cy = g->origin_y + (int64_t)(t / g->tiles_x) * S + S / 2;
    const int m = (int)(off[k + 1] - off[k]);
    ora_pt* p = (ora_pt*)malloc(sizeof(ora_pt) * (size_t)(m > 0 ? m : 1));
    for (int i = 0; i < m; ++i) {
      const int32_t s = idx[off[k] + i];
      p[i].u = (int64_t)x[s] - cx;
      p[i].v = (int64_t)y[s] - cy;
      p[i].z = z[s];
      for (int c = 0; c < 3; ++c) p[i].rgb[c] = rgb[3 * (int64_t)s + c];
    }
    status[k] = ora_recon_tile(g, p, m, (uint64_t)k + 1, x_out + (size_t)k * R * R * 8, &cz[k], NULL, NULL,
                               NULL, NULL, NULL);
    free(p);
  }
  free(off);
  free(idx);
  return 0;
}
