// Tile binning and per-tile interpolated heightmaps (LidarScout Section 3.3,
// Algorithm 1; normalisation of Section 3.4) for gfx950.
//
// Pipeline of ls_recon_tiles, all on one stream, no host round trip:
//   1. k_init / k_tile_pos: map linear tile id -> output slot.
//   2. k_bin_count, k_bin_scan, k_bin_scatter: CSR of the points in every
//      listed tile's padded window [c - H, c + H)^2 (a point sits in 1, 2 or
//      4 windows with the paper's 16-texel ring).
//   3. k_bin_sort (only when the caller asks for the CSR): ascending order.
//   4. k_recon: persistent, one workgroup per tile popped from a queue that
//      holds the tiles in the caller's list order (viewpoint priority) or by
//      descending window point count (longest first, so the last tiles to
//      start are short and the workgroups finish together).  Phases,
//      separated by barriers:
//        a. gather the tile's points to tile-local coordinates and bucket
//           them into a G x G grid over the window (LDS counting sort);
//        b. sort each bucket by (v, u) and drop duplicate positions,
//           keeping the largest (z, R, G, B) -> canonical points;
//        c. face map reset;
//        d. Delaunay triangulation: every point computes its own star by
//           gift-wrapping (first point hit by a circle growing from a
//           Delaunay edge), with exact orientation and in-circle tests and a
//           symbolic perturbation of the lifted heights (lower canonical
//           index = larger perturbation) that makes the triangulation unique
//           when points are cocircular.  A triangle is rasterised by its
//           lowest-index vertex into a per-texel face map (top-left rule),
//           hull edges by one endpoint, so every texel of the closed convex
//           hull gets a containing triangle.  Waves whose walks are done go
//           on to the nearest point of every texel centre (exact distances,
//           ties by (d^2, v, u)) by scans over the buckets;
//        e. c_z from the centre texel, then per texel: barycentric height and
//           colour inside the hull, nearest point outside it (the paper's
//           corner padding points taken at infinity), normalised and written
//           as one NHWC row of 8 FP32 channels.
#include <algorithm>
#include <mutex>

#include "ls_common.hpp"

namespace {

constexpr int RB = 512;                  // threads per recon workgroup
constexpr int LDS_INTS = 16000;          // 62.5 KiB of LDS per recon workgroup
constexpr int MAXG = 88;                 // max buckets per side
constexpr int MAXB = MAXG * MAXG;        // max buckets
static_assert(2 * (MAXB + 1) <= LDS_INTS, "bucket offsets must fit twice in the recon LDS");
constexpr int STAR_MAX_STEPS = 1024;     // safeguard on one point's star walk
constexpr uint64_t FACE_NONE = ~0ull;
constexpr int SUCC_K = 8;                // cached star successors per point
constexpr uint64_t SUCC_EMPTY = ~0ull;
constexpr int SEARCH_MAX_HITS = 8;       // a wave searches once at most this many lanes can step from the lists
constexpr int SORT_LDS = 16384;          // bin segments up to this size sort in LDS

struct BinParams {
  int64_t ox, oy;
  double invS;  // 1 / S
  int32_t S, H, tiles_x, tiles_y, K;
  int32_t n_tiles;
  int64_t n;
  const int32_t* x;
  const int32_t* y;
  const int32_t* tile_pos;
  int32_t* counts;
  int32_t* fill;
  int32_t* bin_off;
  int32_t* bin_idx;
  int64_t cap;
  int32_t* flags;  // [0]: cap overflow
  int32_t* order;  // recon processing order (tile slots)
  int32_t order_mode;  // LS_ORDER_LIST or LS_ORDER_LONGEST_FIRST
};

// floor(a / S) for |a| < 2^53: the double quotient is within one of it
// (a is exact in double), then an exact integer correction.
__device__ __forceinline__ int64_t floordiv_s(int64_t a, int32_t S, double invS) {
  int64_t q = (int64_t)floor((double)a * invS);
  if (q * S > a)
    --q;
  else if ((q + 1) * S <= a)
    ++q;
  return q;
}

// Visit every listed tile whose padded window contains point i.
template <class F>
__device__ __forceinline__ void for_each_window(const BinParams& p, int64_t i, F&& f) {
  const int64_t px = p.x[i], py = p.y[i];
  const int64_t tx0 = floordiv_s(px - p.ox, p.S, p.invS), ty0 = floordiv_s(py - p.oy, p.S, p.invS);
  for (int64_t ty = ty0 - p.K; ty <= ty0 + p.K; ++ty) {
    if (ty < 0 || ty >= p.tiles_y) continue;
    const int64_t cy = p.oy + ty * p.S + p.S / 2;
    if (py < cy - p.H || py >= cy + p.H) continue;
    for (int64_t tx = tx0 - p.K; tx <= tx0 + p.K; ++tx) {
      if (tx < 0 || tx >= p.tiles_x) continue;
      const int64_t cx = p.ox + tx * p.S + p.S / 2;
      if (px < cx - p.H || px >= cx + p.H) continue;
      const int32_t s = p.tile_pos[ty * p.tiles_x + tx];
      if (s >= 0) f(s);
    }
  }
}

__global__ void k_fill_i32(int32_t* __restrict__ a, int64_t n, int32_t v) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    a[i] = v;
}

__global__ void k_tile_pos(const int32_t* __restrict__ tile_list, int32_t n_tiles, int64_t n_all,
                           int32_t* __restrict__ tile_pos, int32_t* __restrict__ status) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n_tiles) return;
  const int32_t t = tile_list[k];
  if (t < 0 || t >= n_all) {
    status[k] = LS_TILE_BADID;
    return;
  }
  // lowest slot wins for a tile listed twice; the others are flagged
  atomicMin(&tile_pos[t], k);
}

__global__ void k_tile_dup(const int32_t* __restrict__ tile_list, int32_t n_tiles, int64_t n_all,
                           const int32_t* __restrict__ tile_pos, int32_t* __restrict__ status) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n_tiles) return;
  const int32_t t = tile_list[k];
  if (t >= 0 && t < n_all && tile_pos[t] != k) status[k] = LS_TILE_BADID;
}

__global__ void k_tile_pos_fix(int32_t* __restrict__ tile_pos, int64_t n_all) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n_all; i += (int64_t)gridDim.x * blockDim.x)
    if (tile_pos[i] == 0x7fffffff) tile_pos[i] = -1;
}

__global__ void k_bin_count(BinParams p) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < p.n; i += (int64_t)gridDim.x * blockDim.x)
    for_each_window(p, i, [&](int32_t s) { atomicAdd(&p.counts[s], 1); });
}

// Workgroup-private tile histograms: each workgroup bins a contiguous chunk
// of points into an LDS histogram and adds it to the global counts with one
// atomic per tile it touched (instead of one global atomic per membership on
// a few hot counters).
constexpr int BIN_THREADS = 1024;
constexpr int BIN_LDS_TILES = 8192;

__global__ void __launch_bounds__(BIN_THREADS) k_bin_count_lds(BinParams p, int64_t per_block) {
  __shared__ int s_cnt[BIN_LDS_TILES];
  for (int t = threadIdx.x; t < p.n_tiles; t += BIN_THREADS) s_cnt[t] = 0;
  __syncthreads();
  const int64_t i0 = blockIdx.x * per_block, i1 = min(p.n, i0 + per_block);
  for (int64_t i = i0 + threadIdx.x; i < i1; i += BIN_THREADS)
    for_each_window(p, i, [&](int32_t s) { atomicAdd(&s_cnt[s], 1); });
  __syncthreads();
  for (int t = threadIdx.x; t < p.n_tiles; t += BIN_THREADS)
    if (s_cnt[t]) atomicAdd(&p.counts[t], s_cnt[t]);
}

// Scatter with the same chunks: local counts, one global reservation per
// touched tile, then positions from LDS cursors.  Within a tile the order of
// workgroups (and of lanes) is arbitrary; the per-tile sort restores
// ascending order when the caller asks for the CSR.
__global__ void __launch_bounds__(BIN_THREADS) k_bin_scatter_lds(BinParams p, int64_t per_block) {
  __shared__ int s_cnt[BIN_LDS_TILES];
  for (int t = threadIdx.x; t < p.n_tiles; t += BIN_THREADS) s_cnt[t] = 0;
  __syncthreads();
  const int64_t i0 = blockIdx.x * per_block, i1 = min(p.n, i0 + per_block);
  for (int64_t i = i0 + threadIdx.x; i < i1; i += BIN_THREADS)
    for_each_window(p, i, [&](int32_t s) { atomicAdd(&s_cnt[s], 1); });
  __syncthreads();
  for (int t = threadIdx.x; t < p.n_tiles; t += BIN_THREADS) {
    const int c = s_cnt[t];
    if (c) s_cnt[t] = p.bin_off[t] + atomicAdd(&p.fill[t], c);
  }
  __syncthreads();
  for (int64_t i = i0 + threadIdx.x; i < i1; i += BIN_THREADS)
    for_each_window(p, i, [&](int32_t s) {
      const int32_t pos = atomicAdd(&s_cnt[s], 1);
      if (pos < p.cap) p.bin_idx[pos] = (int32_t)i;
    });
}

constexpr int ORDER_KEYS = 4096;

// Descending window count, in steps of 4 points, as an ascending key.
__device__ __forceinline__ int order_key(int32_t count) {
  return ORDER_KEYS - 1 - min(max(count, 0) >> 2, ORDER_KEYS - 1);
}

// Single-workgroup exclusive scan of counts -> bin_off (n_tiles + 1 entries),
// then the recon processing order: the caller's list order, or a counting
// sort of the tile slots by order_key (slots with equal keys in any order;
// the results do not depend on the order).
__global__ void __launch_bounds__(1024) k_bin_scan(BinParams p) {
  __shared__ int64_t s_part[1024];
  __shared__ int64_t s_carry;
  __shared__ int s_hist[ORDER_KEYS];
  const int tid = threadIdx.x;
  if (tid == 0) s_carry = 0;
  __syncthreads();
  for (int64_t base = 0; base < p.n_tiles; base += 1024) {
    const int64_t i = base + tid;
    const int64_t v = i < p.n_tiles ? p.counts[i] : 0;
    s_part[tid] = v;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {
      const int64_t t = tid >= o ? s_part[tid - o] : 0;
      __syncthreads();
      s_part[tid] += t;
      __syncthreads();
    }
    const int64_t excl = s_carry + s_part[tid] - v;
    if (i < p.n_tiles) p.bin_off[i] = (int32_t)(excl < 0x7fffffff ? excl : 0x7fffffff);
    __syncthreads();
    if (tid == 1023) s_carry += s_part[1023];
    __syncthreads();
  }
  if (tid == 0) {
    const int64_t total = s_carry;
    p.bin_off[p.n_tiles] = (int32_t)(total < 0x7fffffff ? total : 0x7fffffff);
    p.flags[0] = total > p.cap ? 1 : 0;
  }
  if (p.order_mode == LS_ORDER_LIST) {
    for (int i = tid; i < p.n_tiles; i += 1024) p.order[i] = i;
    return;
  }
  constexpr int PER = ORDER_KEYS / 1024;
  for (int b = tid; b < ORDER_KEYS; b += 1024) s_hist[b] = 0;
  __syncthreads();
  for (int i = tid; i < p.n_tiles; i += 1024) atomicAdd(&s_hist[order_key(p.counts[i])], 1);
  __syncthreads();
  int run = 0;
  for (int j = 0; j < PER; ++j) run += s_hist[tid * PER + j];
  s_part[tid] = run;
  __syncthreads();
  for (int o = 1; o < 1024; o <<= 1) {
    const int64_t t = tid >= o ? s_part[tid - o] : 0;
    __syncthreads();
    s_part[tid] += t;
    __syncthreads();
  }
  int excl = (int)(s_part[tid] - run);
  for (int j = 0; j < PER; ++j) {
    const int c = s_hist[tid * PER + j];
    s_hist[tid * PER + j] = excl;
    excl += c;
  }
  __syncthreads();
  for (int i = tid; i < p.n_tiles; i += 1024) p.order[atomicAdd(&s_hist[order_key(p.counts[i])], 1)] = i;
}

__global__ void k_bin_scatter(BinParams p) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < p.n; i += (int64_t)gridDim.x * blockDim.x)
    for_each_window(p, i, [&](int32_t s) {
      const int32_t r = atomicAdd(&p.fill[s], 1);
      const int64_t pos = (int64_t)p.bin_off[s] + r;
      if (pos < p.cap) p.bin_idx[pos] = (int32_t)i;
    });
}

// In-place ascending bitonic sort of one bin segment; segments longer than
// SORT_LDS use `spill` (2 entries per bin entry, so the power-of-two
// padding always fits).
__global__ void __launch_bounds__(RB) k_bin_sort(const int32_t* __restrict__ bin_off, int32_t n_tiles,
                                                 int32_t* __restrict__ bin_idx, int32_t* __restrict__ spill,
                                                 const int32_t* __restrict__ flags) {
  __shared__ int32_t s_buf[SORT_LDS];
  if (flags[0]) return;
  for (int k = blockIdx.x; k < n_tiles; k += gridDim.x) {
    const int32_t off = __builtin_amdgcn_readfirstlane(bin_off[k]);
    const int32_t cnt = __builtin_amdgcn_readfirstlane(bin_off[k + 1]) - off;
    if (cnt <= 1) continue;  // uniform: k comes from blockIdx, the counts are readfirstlane'd
    int n2 = 1;
    while (n2 < cnt) n2 <<= 1;
    int32_t* buf = n2 <= SORT_LDS ? s_buf : spill + 2 * (int64_t)off;
    for (int i = threadIdx.x; i < n2; i += RB) buf[i] = i < cnt ? bin_idx[off + i] : 0x7fffffff;
    __syncthreads();
    for (int kk = 2; kk <= n2; kk <<= 1)
      for (int j = kk >> 1; j > 0; j >>= 1) {
        for (int i = threadIdx.x; i < n2; i += RB) {
          const int l = i ^ j;
          if (l > i) {
            const int32_t a = buf[i], b = buf[l];
            const bool asc = (i & kk) == 0;
            if ((a > b) == asc) {
              buf[i] = b;
              buf[l] = a;
            }
          }
        }
        __syncthreads();
      }
    for (int i = threadIdx.x; i < cnt; i += RB) bin_idx[off + i] = buf[i];
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// per-tile reconstruction
// ---------------------------------------------------------------------------
struct ReconParams {
  int64_t ox, oy;
  int32_t S, tiles_x, C, R, H;
  double scale_z, offset_z, inv_r;
  int32_t n_tiles;
  const int32_t* x;
  const int32_t* y;
  const int32_t* z;
  const uint16_t* rgb;
  const int32_t* tile_list;
  const int32_t* bin_off;
  const int32_t* bin_idx;
  const int32_t* flags;
  // per bin entry scratch: staging (reused for the canonical heights and
  // colours), sorted copies, canonical coordinates
  int32_t* su;
  int32_t* sv;
  int32_t* sz;
  uint64_t* srgb;  // R | G << 16 | B << 32
  int32_t* sslot;
  int32_t* tu;
  int32_t* tv;
  int32_t* tz;
  uint64_t* trgb;
  int2* cuv;
  uint64_t* tris;  // 2 entries per bin entry: large triangles of a tile, rasterised after its stars
  uint64_t* succ;  // SUCC_K entries per bin entry: known star successors (key << 32 | third vertex)
  int32_t* succ_n;  // per bin entry: successor entries claimed
  // per workgroup scratch
  uint64_t* facemap;  // [gridDim][R*R]
  int32_t* nnidx;     // [gridDim][R*R]
  int32_t* queue;
  const int32_t* order;  // queue position -> tile slot
  float* x_out;
  double* cz_out;
  int32_t* status;
};

// Pointers into LDS typed as such, so that reads through them are LDS reads
// (a generic pointer that may point to LDS or to global memory compiles to
// flat loads, which wait on both the LDS and the vector-memory counters).
typedef const __attribute__((address_space(3))) int32_t* LdsI32;
typedef const __attribute__((address_space(3))) uint64_t* LdsU64;
// Point coordinates (u, v) as one 8-byte read, from LDS or global memory.
struct UvLds {
  LdsU64 p;
  __device__ __forceinline__ int2 operator[](int i) const {
    const uint64_t w = p[i];
    return make_int2((int)(uint32_t)w, (int)(uint32_t)(w >> 32));
  }
};
struct UvGlobal {
  const int2* p;
  __device__ __forceinline__ int2 operator[](int i) const { return p[i]; }
};

// A tile's canonical points: coordinates through UVP (UvLds when the
// tile's points are staged in LDS, else UvGlobal).
template <class UVP>
struct TileT {
  UVP uv;       // canonical coordinates
  LdsI32 boff;  // G*G + 1 canonical bucket offsets
  int G, H, W2;
  double bw;  // bucket width in raw units
};

// floor(w * G / W2) for 0 <= w < W2 <= 2^19 and G <= 88 (all products below
// 2^26, so the float estimate of a quotient below 88 is off by far less
// than one): a float reciprocal estimate, then an exact integer correction
// by at most one.
__device__ __forceinline__ int bucket_1d(int w, int G, int W2) {
  const int num = w * G;
  int q = (int)((float)num * __builtin_amdgcn_rcpf((float)W2));
  if (q * W2 > num)
    --q;
  else if ((q + 1) * W2 <= num)
    ++q;
  return q;
}

__device__ __forceinline__ double orient_d(double ax, double ay, double bx, double by, double px, double py) {
  // exact: |differences| < 2^19, products < 2^38, result < 2^39
  return (bx - ax) * (py - ay) - (by - ay) * (px - ax);
}

__device__ __forceinline__ int sgn_d(double v) { return (v > 0.0) - (v < 0.0); }

// Exact sign of the in-circle determinant in int128 (|terms| < 2^79), then
// the symbolic perturbation for exactly cocircular points.  Kept out of line:
// the floating-point filter below settles nearly every call.
__device__ __noinline__ int incircle_exact(int a, int b, int c, int d, int2 pa, int2 pb, int2 pc, int2 pd) {
  const int64_t adx = pa.x - pd.x, ady = pa.y - pd.y;
  const int64_t bdx = pb.x - pd.x, bdy = pb.y - pd.y;
  const int64_t cdx = pc.x - pd.x, cdy = pc.y - pd.y;
  const __int128 e = (__int128)(adx * adx + ady * ady) * (__int128)(bdx * cdy - cdx * bdy) +
                     (__int128)(bdx * bdx + bdy * bdy) * (__int128)(cdx * ady - adx * cdy) +
                     (__int128)(cdx * cdx + cdy * cdy) * (__int128)(adx * bdy - bdx * ady);
  if (e > 0) return 1;
  if (e < 0) return -1;
  int w = a;
  if (b < w) w = b;
  if (c < w) w = c;
  if (d < w) w = d;
  if (w == d) return -1;
  if (w == a) return sgn_d(orient_d(pb.x, pb.y, pc.x, pc.y, pd.x, pd.y));
  if (w == b) return sgn_d(orient_d(pc.x, pc.y, pa.x, pa.y, pd.x, pd.y));
  return sgn_d(orient_d(pa.x, pa.y, pb.x, pb.y, pd.x, pd.y));
}

// Sign of the in-circle determinant of d against CCW (a, b, c): > 0 when d
// is strictly inside.  Floating-point filter first, exact int128 otherwise,
// then the symbolic perturbation for exactly cocircular points.
__device__ __forceinline__ int incircle_sos(int a, int b, int c, int d, int2 pa, int2 pb, int2 pc, int2 pd) {
  const double fadx = (double)(pa.x - pd.x), fady = (double)(pa.y - pd.y);
  const double fbdx = (double)(pb.x - pd.x), fbdy = (double)(pb.y - pd.y);
  const double fcdx = (double)(pc.x - pd.x), fcdy = (double)(pc.y - pd.y);
  const double al = fadx * fadx + fady * fady;
  const double bl = fbdx * fbdx + fbdy * fbdy;
  const double cl = fcdx * fcdx + fcdy * fcdy;
  const double bc = fbdx * fcdy - fcdx * fbdy;
  const double ca = fcdx * fady - fadx * fcdy;
  const double ab = fadx * fbdy - fbdx * fady;
  const double t1 = al * bc, t2 = bl * ca, t3 = cl * ab;
  const double det = t1 + t2 + t3;
  const double perm = fabs(t1) + fabs(t2) + fabs(t3);
  if (fabs(det) > 8.8817841970012523e-16 * perm) return sgn_d(det);  // 8 * 2^-53
  return incircle_exact(a, b, c, d, pa, pb, pc, pd);
}

template <class TT>
__device__ __forceinline__ bool ring_covers_grid(const TT& T, int bx0, int by0, int r) {
  return bx0 - r <= 0 && by0 - r <= 0 && bx0 + r >= T.G - 1 && by0 + r >= T.G - 1;
}

// Nearest canonical point to (qx, qy), ties by smallest (d^2, v, u); skips
// point `skip`.  Returns -1 if no point.  Chebyshev rings of buckets around
// q's bucket; once a candidate exists, buckets farther from q than it are
// skipped, and the search stops when the candidate is closer than the
// nearest side of the square visited so far.
template <class TT>
__device__ int ring_nearest(const TT& T, int qx, int qy, int skip) {
  const int G = T.G;
  const int bx0 = bucket_1d(qx + T.H, G, T.W2), by0 = bucket_1d(qy + T.H, G, T.W2);
  const double fx = qx + T.H, fy = qy + T.H;  // grid-local
  int best = -1;
  double bd = 0.0;  // squared distance, exact in double (below 2^40)
  int bu = 0, bv = 0;
  for (int r = 0;; ++r) {
    const int ylo = by0 - r, yhi = by0 + r, xlo = bx0 - r, xhi = bx0 + r;
    for (int by = max(ylo, 0); by <= min(yhi, G - 1); ++by) {
      const bool full = (by == ylo || by == yhi);
      const int step = full ? 1 : (xhi - xlo);
      for (int bx = xlo; bx <= xhi; bx += (step > 0 ? step : 1)) {
        if (bx < 0 || bx >= G) continue;
        if (best >= 0) {
          // distance from q to the bucket rectangle, rounded outwards
          const double x0 = floor(bx * T.bw) - 1.0, x1 = ceil((bx + 1) * T.bw) + 1.0;
          const double y0 = floor(by * T.bw) - 1.0, y1 = ceil((by + 1) * T.bw) + 1.0;
          const double dx = fmax(fmax(x0 - fx, fx - x1), 0.0), dy = fmax(fmax(y0 - fy, fy - y1), 0.0);
          if (dx * dx + dy * dy > bd) continue;
        }
        const int b = by * G + bx;
        const int e = T.boff[b + 1];
        for (int p = T.boff[b]; p < e; ++p) {
          if (p == skip) continue;
          const int2 q = T.uv[p];
          const double dx = q.x - qx, dy = q.y - qy;
          const double d = fma(dx, dx, dy * dy);
          if (best < 0 || d < bd || (d == bd && (q.y < bv || (q.y == bv && q.x < bu)))) {
            best = p;
            bd = d;
            bu = q.x;
            bv = q.y;
          }
        }
      }
    }
    if (best >= 0) {
      // distance from q to the outside of the square of buckets visited
      const double L = fmin(fmin(fx - floor((bx0 - r) * T.bw), ceil((bx0 + r + 1) * T.bw) - fx),
                            fmin(fy - floor((by0 - r) * T.bw), ceil((by0 + r + 1) * T.bw) - fy)) -
                       1.0;
      if (L > 0.0 && bd < L * L) break;
    }
    if (ring_covers_grid(T, bx0, by0, r)) break;
  }
  return best;
}

// Nearest points of an 8 x 8 block of texels, one texel per lane of a wave
// (lane = 8 * row + column): every lane scans the same candidate list, the
// points of the buckets under the block widened by one bucket on each side,
// so the loops are uniform and each point is read once per wave (an LDS
// broadcast).  A texel keeps the scan's answer when its best squared
// distance is below the squared distance to every side of the scanned
// bucket rectangle that faces more buckets (sides rounded inwards by one raw
// unit).  While some lane of the wave cannot prove its answer (sparse parts
// of the window), the rectangle grows by one bucket ring, scanned the same
// way, up to two rings; a lane still unproven then falls back to
// ring_nearest.  Same order on (d^2, v, u), so the result equals
// ring_nearest's.
template <class TT>
__device__ int nearest_block(const TT& T, int q0, int C, int R, int bi, int bj, int lane, int& qx, int& qy) {
  const int G = T.G;
  const int i = bi * 8 + (lane >> 3), j = bj * 8 + (lane & 7);
  const bool in_grid = i < R && j < R;
  qx = q0 + j * C;
  qy = q0 + i * C;
  const int i1 = min(bi * 8 + 7, R - 1), j1 = min(bj * 8 + 7, R - 1);
  int bx0 = max(bucket_1d(q0 + bj * 8 * C + T.H, G, T.W2) - 1, 0);
  int bx1 = min(bucket_1d(q0 + j1 * C + T.H, G, T.W2) + 1, G - 1);
  int by0 = max(bucket_1d(q0 + bi * 8 * C + T.H, G, T.W2) - 1, 0);
  int by1 = min(bucket_1d(q0 + i1 * C + T.H, G, T.W2) + 1, G - 1);
  int best = -1, bu = 0, bv = 0;
  double bd = 0.0;  // squared distance, exact in double (below 2^40)
  // buckets xlo..xhi of rows ylo..yhi (those of a row are contiguous)
  auto scan = [&](int ylo, int yhi, int xlo, int xhi) {
    if (xlo > xhi) return;
    for (int by = ylo; by <= yhi; ++by) {
      const int e = T.boff[by * G + xhi + 1];
      for (int p = T.boff[by * G + xlo]; p < e; ++p) {
        const int2 q = T.uv[p];
        const double dx = q.x - qx, dy = q.y - qy;
        const double d = fma(dx, dx, dy * dy);
        if (best < 0 || d < bd || (d == bd && (q.y < bv || (q.y == bv && q.x < bu)))) {
          best = p;
          bd = d;
          bu = q.x;
          bv = q.y;
        }
      }
    }
  };
  scan(by0, by1, bx0, bx1);
  const double fx = qx + T.H, fy = qy + T.H;  // grid-local
  bool proven = false;
  for (int ring = 0;; ++ring) {
    // distance from q to the unscanned buckets
    double L = 1e300;
    if (bx0 > 0) L = fmin(L, fx - (ceil(bx0 * T.bw) + 1.0));
    if (bx1 < G - 1) L = fmin(L, (floor((bx1 + 1) * T.bw) - 1.0) - fx);
    if (by0 > 0) L = fmin(L, fy - (ceil(by0 * T.bw) + 1.0));
    if (by1 < G - 1) L = fmin(L, (floor((by1 + 1) * T.bw) - 1.0) - fy);
    proven = best >= 0 && (L >= 1e300 || (L > 0.0 && bd < L * L));
    if (ring == 2 || __ballot(in_grid && !proven) == 0) break;
    const int nx0 = max(bx0 - 1, 0), nx1 = min(bx1 + 1, G - 1), ny0 = max(by0 - 1, 0), ny1 = min(by1 + 1, G - 1);
    scan(ny0, by0 - 1, nx0, nx1);      // new rows below
    scan(by1 + 1, ny1, nx0, nx1);      // new rows above
    scan(by0, by1, nx0, bx0 - 1);      // new columns on the left
    scan(by0, by1, bx1 + 1, nx1);      // new columns on the right
    bx0 = nx0;
    bx1 = nx1;
    by0 = ny0;
    by1 = ny1;
  }
  if (proven) return best;
  return ring_nearest(T, qx, qy, -1);
}

// Bucket index range of the tile-local box [x0, x1] x [y0, y1] widened by
// `slack` raw units, clamped to the grid.
struct BucketBox {
  int x0, x1, y0, y1;
};
template <class TT>
__device__ __forceinline__ int bucket_clamped(const TT& T, double w) {
  const double c = fmin(fmax(w, (double)-T.H), (double)(T.H - 1));
  return bucket_1d((int)c + T.H, T.G, T.W2);
}
template <class TT>
__device__ __forceinline__ BucketBox bucket_box(const TT& T, double x0, double x1, double y0, double y1,
                                                double slack) {
  BucketBox r;
  r.x0 = bucket_clamped(T, floor(x0 - slack));
  r.x1 = bucket_clamped(T, ceil(x1 + slack));
  r.y0 = bucket_clamped(T, floor(y0 - slack));
  r.y1 = bucket_clamped(T, ceil(y1 + slack));
  return r;
}

// The third vertex of the Delaunay triangle on the left of edge a->b: the
// first point met by a circle through a and b whose centre moves left.
// Returns -1 if no point lies strictly left of a->b (a->b is a hull edge).
// Buckets are visited in Chebyshev rings around the midpoint, each ring
// clipped to the bounding box of the region a better point could still lie
// in: the window on the left of the line and, once a candidate exists, the
// part of its circumcircle on that side (for a centre on the right this is
// the thin cap between the chord and the parallel tangent).  Inside the box,
// buckets entirely right of the line or outside the circle are skipped.
template <class TT>
__device__ int third_left(const TT& T, int a, int b) {
  const int2 A = T.uv[a], B = T.uv[b];
  const int ax = A.x, ay = A.y, bx = B.x, by = B.y;
  const int mx = (ax + bx) >> 1, my = (ay + by) >> 1;
  const int bx0 = bucket_1d(mx + T.H, T.G, T.W2), by0 = bucket_1d(my + T.H, T.G, T.W2);
  const double fbx = bx - ax, fby = by - ay;
  const double bl = fbx * fbx + fby * fby;
  // window [-H, H-1]^2 clipped to the closed left half-plane (corners on
  // the line included, crossings rounded outwards by the slack below)
  double hx0 = 1e300, hx1 = -1e300, hy0 = 1e300, hy1 = -1e300;
  bool any_left = false;
  {
    const double lo = -T.H, hi = T.H - 1;
    const double px[4] = {lo, hi, hi, lo}, py[4] = {lo, lo, hi, hi};
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int j = (i + 1) & 3;
      const double oi = orient_d(ax, ay, bx, by, px[i], py[i]), oj = orient_d(ax, ay, bx, by, px[j], py[j]);
      any_left |= oi > 0.0;
      if (oi >= 0.0) {
        hx0 = fmin(hx0, px[i]);
        hx1 = fmax(hx1, px[i]);
        hy0 = fmin(hy0, py[i]);
        hy1 = fmax(hy1, py[i]);
      }
      if ((oi > 0.0 && oj < 0.0) || (oi < 0.0 && oj > 0.0)) {
        // crossing point in float (error far below the slack added below)
        const double t = (double)((float)oi * __builtin_amdgcn_rcpf((float)(oi - oj)));
        const double qx = px[i] + t * (px[j] - px[i]), qy = py[i] + t * (py[j] - py[i]);
        hx0 = fmin(hx0, qx);
        hx1 = fmax(hx1, qx);
        hy0 = fmin(hy0, qy);
        hy1 = fmax(hy1, qy);
      }
    }
  }
  if (!any_left) return -1;
  const BucketBox half = bucket_box(T, hx0, hx1, hy0, hy1, 2.0);
  BucketBox bb = half;
  int rmax = max(max(bx0 - bb.x0, bb.x1 - bx0), max(by0 - bb.y0, bb.y1 - by0));
  int best = -1;
  int2 C = make_int2(0, 0);
  // Circle through a, b and the best point as of the last geometry update.
  // Circles through a and b are nested on the left of the line (a point
  // inside one lies inside every circle whose centre is farther left), and
  // every improvement moves the centre right, so the possibly stale circle
  // stays a conservative filter; the exact in-circle test decides.
  double ocx = 0.0, ocy = 0.0;
  double lim2 = 0.0;  // squared reach of that circle, with margin
  bool have_circle = false, dirty = false;
  // orient(a, b, .) is linear with gradient (-fby, fbx): over a rectangle it
  // peaks at the corner these signs pick
  const bool hi_x = fby <= 0.0, hi_y = fbx >= 0.0;
  const double inv_ll = 1.0 / sqrt(bl);
  auto update_circle = [&]() {
    // circumcircle of (a, b, best) relative to a
    const double cx = C.x - ax, cy = C.y - ay;
    const double cl = cx * cx + cy * cy;
    const double iD = 0.5 / (fbx * cy - fby * cx);
    const double ox = (cy * bl - fby * cl) * iD, oy = (fbx * cl - cx * bl) * iD;
    const double rho = sqrt(ox * ox + oy * oy);
    ocx = ox + ax;
    ocy = oy + ay;
    {
      const double lim = rho * (1.0 + 1e-9) + 2.0;
      lim2 = lim * lim;
    }
    // signed distance of the centre from the line, > 0 on the left
    const double dc = (fbx * oy - fby * ox) * inv_ll;
    double cx0, cx1, cy0, cy1;
    if (dc <= 0.0) {
      // sagitta rho - |dc| = (|ab|/2)^2 / (rho + |dc|), free of cancellation
      const double h = bl / (4.0 * (rho - dc)) * (1.0 + 1e-9);
      const double nx = -fby * inv_ll * h, ny = fbx * inv_ll * h;
      cx0 = fmin(fmin(ax, bx), fmin(ax + nx, bx + nx));
      cx1 = fmax(fmax(ax, bx), fmax(ax + nx, bx + nx));
      cy0 = fmin(fmin(ay, by), fmin(ay + ny, by + ny));
      cy1 = fmax(fmax(ay, by), fmax(ay + ny, by + ny));
    } else {
      cx0 = ocx - rho;
      cx1 = ocx + rho;
      cy0 = ocy - rho;
      cy1 = ocy + rho;
    }
    const BucketBox cb = bucket_box(T, cx0, cx1, cy0, cy1, 2.0 + rho * 1e-9);
    bb.x0 = max(half.x0, cb.x0);
    bb.x1 = min(half.x1, cb.x1);
    bb.y0 = max(half.y0, cb.y0);
    bb.y1 = min(half.y1, cb.y1);
    rmax = max(max(bx0 - bb.x0, bb.x1 - bx0), max(by0 - bb.y0, bb.y1 - by0));
    have_circle = true;
    dirty = false;
  };
  auto visit = [&](int qx, int qy) {
    // bucket rectangle in tile-local coordinates, rounded outwards to integers
    const double x0 = floor(qx * T.bw) - T.H - 1.0, x1 = ceil((qx + 1) * T.bw) - T.H + 1.0;
    const double y0 = floor(qy * T.bw) - T.H - 1.0, y1 = ceil((qy + 1) * T.bw) - T.H + 1.0;
    if (orient_d(ax, ay, bx, by, hi_x ? x1 : x0, hi_y ? y1 : y0) <= 0.0) return;
    if (have_circle) {
      const double dx = fmax(fmax(x0 - ocx, ocx - x1), 0.0), dy = fmax(fmax(y0 - ocy, ocy - y1), 0.0);
      if (dx * dx + dy * dy > lim2) return;
    }
    const int bi = qy * T.G + qx;
    const int e = T.boff[bi + 1];
    for (int p = T.boff[bi]; p < e; ++p) {
      if (p == a || p == b) continue;
      const int2 P = T.uv[p];
      if (orient_d(ax, ay, bx, by, P.x, P.y) <= 0.0) continue;
      if (best >= 0) {
        // clearly outside the circle: no need for the exact test (the margin
        // covers the rounding of the centre and radius)
        if (have_circle) {
          const double ex = P.x - ocx, ey = P.y - ocy;
          if (ex * ex + ey * ey > lim2) continue;
        }
        if (incircle_sos(a, b, best, p, A, B, C, P) <= 0) continue;
      }
      best = p;
      C = P;
      dirty = true;
    }
  };
  for (int r = 0; r <= rmax; ++r) {
    // the cells of ring r inside the box, enumerated by one index so the
    // bucket visit is instantiated once: bottom row, side cells of the
    // middle rows, top row
    const BucketBox q = bb;
    const int ylo = by0 - r, yhi = by0 + r, xlo = bx0 - r, xhi = bx0 + r;
    const int X0 = max(xlo, q.x0), X1 = min(xhi, q.x1);
    const int nrow = X1 >= X0 ? X1 - X0 + 1 : 0;
    const int nA = (ylo >= q.y0 && ylo <= q.y1) ? nrow : 0;
    const int nC = (r > 0 && yhi >= q.y0 && yhi <= q.y1) ? nrow : 0;
    const int ym0 = max(ylo + 1, q.y0), ym1 = min(yhi - 1, q.y1);
    const bool sL = xlo >= q.x0 && xlo <= q.x1, sR = xhi >= q.x0 && xhi <= q.x1;
    const int k = (int)sL + (int)sR;
    const int nB = ym1 >= ym0 ? (ym1 - ym0 + 1) * k : 0;
    const int total = nA + nB + nC;
    for (int t = 0; t < total; ++t) {
      int cx, cy;
      if (t < nA) {
        cy = ylo;
        cx = X0 + t;
      } else if (t < nA + nB) {
        const int u = t - nA;
        cy = ym0 + (k == 2 ? (u >> 1) : u);
        cx = (k == 2) ? ((u & 1) ? xhi : xlo) : (sL ? xlo : xhi);
      } else {
        cy = yhi;
        cx = X0 + (t - nA - nB);
      }
      visit(cx, cy);
    }
    if (dirty) update_circle();
  }
  return best;
}

__device__ __forceinline__ uint64_t face_key(int a, int b, int c) {
  // rotate so the lowest index comes first (keeps CCW order)
  if (b < a && b < c) {
    const int t = a;
    a = b;
    b = c;
    c = t;
  } else if (c < a && c < b) {
    const int t = c;
    c = b;
    b = a;
    a = t;
  }
  return ((uint64_t)a << 42) | ((uint64_t)b << 21) | (uint64_t)c;
}

// Top-left ownership of an edge P->Q for points exactly on it: equivalent to
// testing the point nudged by an infinitesimal (-1, -delta).
__device__ __forceinline__ bool edge_owned(int px, int py, int qx, int qy) {
  const int dy = qy - py, dx = qx - px;
  return dy > 0 || (dy == 0 && dx < 0);
}

__device__ __forceinline__ int floor_div_i(int a, int b) {
  int q = a / b;
  if ((a % b != 0) && ((a < 0) != (b < 0))) --q;
  return q;
}

// texel index range covering [lo, hi] in tile-local raw coordinates
__device__ __forceinline__ void texel_range(int lo, int hi, int H, int C, int R, int& j0, int& j1) {
  const int q0 = -H + C / 2;
  j0 = -floor_div_i(q0 - lo, C);  // ceil((lo - q0) / C)
  j1 = floor_div_i(hi - q0, C);
  if (j0 < 0) j0 = 0;
  if (j1 > R - 1) j1 = R - 1;
}

__device__ __forceinline__ bool tri_inside(int ax, int ay, int bx, int by, int cx, int cy, bool oa, bool ob, bool oc,
                                           double qx, double qy) {
  const double e0 = orient_d(bx, by, cx, cy, qx, qy);
  if (e0 < 0.0 || (e0 == 0.0 && !oa)) return false;
  const double e1 = orient_d(cx, cy, ax, ay, qx, qy);
  if (e1 < 0.0 || (e1 == 0.0 && !ob)) return false;
  const double e2 = orient_d(ax, ay, bx, by, qx, qy);
  return !(e2 < 0.0 || (e2 == 0.0 && !oc));
}

// Narrow [lo, hi] to the x-interval of {q : orient(P, Q, q) >= 0} on the
// horizontal line y = qy (approximate; the caller settles the ends exactly).
__device__ __forceinline__ void edge_clip(int px, int py, int qx, int qy, double y, double& lo, double& hi) {
  const double dy = qy - py;
  const double k = (double)(qx - px) * (y - py);  // orient = k - dy * (x - px)
  if (dy > 0.0)
    hi = fmin(hi, px + k / dy);
  else if (dy < 0.0)
    lo = fmax(lo, px + k / dy);
  else if (k < 0.0) {
    lo = 1.0;
    hi = 0.0;
  }
}

// Write `key` into every texel whose centre lies in CCW triangle (a, b, c)
// under the top-left rule.  Row by row: the span from the three edges is
// widened by one texel, its two ends are settled with the exact test, and
// the texels between them are filled without further tests (a triangle's
// row section is an interval).
template <class TT>
__device__ void raster_triangle(const TT& T, int a, int b, int c, int C, int R, uint64_t* __restrict__ fm) {
  const int2 A = T.uv[a], B = T.uv[b], Cc = T.uv[c];
  const int ax = A.x, ay = A.y, bx = B.x, by = B.y, cx = Cc.x, cy = Cc.y;
  int i0, i1, j0, j1;
  texel_range(min(ax, min(bx, cx)), max(ax, max(bx, cx)), T.H, C, R, j0, j1);
  texel_range(min(ay, min(by, cy)), max(ay, max(by, cy)), T.H, C, R, i0, i1);
  const bool oa = edge_owned(bx, by, cx, cy), ob = edge_owned(cx, cy, ax, ay), oc = edge_owned(ax, ay, bx, by);
  const uint64_t key = face_key(a, b, c);
  const int q0 = -T.H + C / 2;
  const double invC = 1.0 / C;
  for (int i = i0; i <= i1; ++i) {
    const double qy = q0 + i * C;
    double lo = -1e300, hi = 1e300;
    edge_clip(bx, by, cx, cy, qy, lo, hi);
    edge_clip(cx, cy, ax, ay, qy, lo, hi);
    edge_clip(ax, ay, bx, by, qy, lo, hi);
    if (!(lo <= hi + 2.0 * C)) continue;
    int jl = max(j0, (int)floor((fmax(lo, -3.0 * T.H) - q0) * invC) - 1);
    int jr = min(j1, (int)ceil((fmin(hi, 3.0 * T.H) - q0) * invC) + 1);
    while (jl <= jr && !tri_inside(ax, ay, bx, by, cx, cy, oa, ob, oc, q0 + jl * C, qy)) ++jl;
    while (jr >= jl && !tri_inside(ax, ay, bx, by, cx, cy, oa, ob, oc, q0 + jr * C, qy)) --jr;
    uint64_t* __restrict__ row = fm + i * R;
    for (int j = jl; j <= jr; ++j) row[j] = key;
  }
}

// Texel bounding box of triangle (a, b, c); false when it holds no texel.
template <class TT>
__device__ __forceinline__ bool tri_texel_box(const TT& T, int a, int b, int c, int C, int R, int& i0, int& i1,
                                              int& j0, int& j1) {
  const int2 A = T.uv[a], B = T.uv[b], Cc = T.uv[c];
  texel_range(min(A.x, min(B.x, Cc.x)), max(A.x, max(B.x, Cc.x)), T.H, C, R, j0, j1);
  texel_range(min(A.y, min(B.y, Cc.y)), max(A.y, max(B.y, Cc.y)), T.H, C, R, i0, i1);
  return i0 <= i1 && j0 <= j1;
}

// Triangles are rasterised after the star phase by groups of RASTER_LANES
// lanes (one lane per texel of the box), not by the lane that finds them, so
// rasterisation neither holds up the lanes of a wave that walk their stars
// nor diverges with the box sizes.
constexpr int RASTER_LANES = 8;

// raster_triangle's result, computed by the RASTER_LANES lanes of a group:
// every texel of the box gets the exact top-left test.
template <class TT>
__device__ void raster_triangle_group(const TT& T, uint64_t key, int C, int R, uint64_t* __restrict__ fm, int lane) {
  const int a = (int)(key >> 42), b = (int)((key >> 21) & 0x1FFFFF), c = (int)(key & 0x1FFFFF);
  int i0, i1, j0, j1;
  if (!tri_texel_box(T, a, b, c, C, R, i0, i1, j0, j1)) return;
  const int2 A = T.uv[a], B = T.uv[b], Cc = T.uv[c];
  const int ax = A.x, ay = A.y, bx = B.x, by = B.y, cx = Cc.x, cy = Cc.y;
  const bool oa = edge_owned(bx, by, cx, cy), ob = edge_owned(cx, cy, ax, ay), oc = edge_owned(ax, ay, bx, by);
  const int q0 = -T.H + C / 2;
  const int w = j1 - j0 + 1, n = (i1 - i0 + 1) * w;
  const float rw = __builtin_amdgcn_rcpf((float)w);
  for (int e = lane; e < n; e += RASTER_LANES) {
    // e / w from a float estimate (e < 2^14), corrected exactly
    int di = (int)((float)e * rw);
    if (di * w > e)
      --di;
    else if ((di + 1) * w <= e)
      ++di;
    const int i = i0 + di, j = j0 + (e - di * w);
    if (tri_inside(ax, ay, bx, by, cx, cy, oa, ob, oc, q0 + j * C, q0 + i * C)) fm[i * R + j] = key;
  }
}

// Texels lying exactly on hull edge a->b get the triangle next to it.  Per
// texel row the line crosses at most one texel centre, found exactly in
// integers.
template <class TT>
__device__ void raster_hull_edge(const TT& T, int a, int b, uint64_t key, int C, int R, uint64_t* __restrict__ fm) {
  const int2 A = T.uv[a], B = T.uv[b];
  const int ax = A.x, ay = A.y, bx = B.x, by = B.y;
  int i0, i1, j0, j1;
  texel_range(min(ax, bx), max(ax, bx), T.H, C, R, j0, j1);
  texel_range(min(ay, by), max(ay, by), T.H, C, R, i0, i1);
  const int q0 = -T.H + C / 2;
  const int64_t dx = bx - ax, dy = by - ay;
  if (dy == 0) {
    // the edge lies on a texel row only if ay is a row centre (then i0 == i1)
    if (i0 > i1 || q0 + i0 * C != ay) return;
    for (int j = j0; j <= j1; ++j) fm[i0 * R + j] = key;
    return;
  }
  // x = ax + dx * (y - ay) / dy must be an integer texel centre; every
  // quantity is an integer below 2^39, so the double quotient, its rounding
  // and the check of the product are exact
  const double fdx = (double)dx, fdy = (double)dy;
  for (int i = i0; i <= i1; ++i) {
    const double num = fdx * (double)(q0 + i * C - ay);
    const double xr = rint(num / fdy);
    if (xr * fdy != num) continue;
    const int xo = ax + (int)xr - q0;
    if (xo % C) continue;
    const int j = xo / C;
    if (j >= j0 && j <= j1) fm[i * R + j] = key;
  }
}

__device__ int block_scan_excl(int* s, int n, int* s_tmp) {
  const int tid = threadIdx.x;
  const int per = (n + RB - 1) / RB;
  const int beg = min(n, tid * per), end = min(n, beg + per);
  int sum = 0;
  for (int i = beg; i < end; ++i) sum += s[i];
  const int lane = tid & 63, wid = tid >> 6;
  int v = sum;
  for (int o = 1; o < 64; o <<= 1) {
    const int t = __shfl_up(v, o, 64);
    if (lane >= o) v += t;
  }
  if (lane == 63) s_tmp[wid] = v;
  __syncthreads();
  if (tid == 0) {
    int run = 0;
    for (int w = 0; w < RB / 64; ++w) {
      const int t = s_tmp[w];
      s_tmp[w] = run;
      run += t;
    }
    s_tmp[RB / 64] = run;
  }
  __syncthreads();
  int excl = v - sum + s_tmp[wid];
  for (int i = beg; i < end; ++i) {
    const int t = s[i];
    s[i] = excl;
    excl += t;
  }
  const int total = s_tmp[RB / 64];
  __syncthreads();
  return total;
}

__device__ __forceinline__ bool pt_less(int u0, int v0, int z0, uint64_t c0, int u1, int v1, int z1, uint64_t c1) {
  // order by (v, u) ascending, then (z, R, G, B) descending
  if (v0 != v1) return v0 < v1;
  if (u0 != u1) return u0 < u1;
  if (z0 != z1) return z0 > z1;
  const uint64_t k0 = ((c0 & 0xFFFF) << 32) | (((c0 >> 16) & 0xFFFF) << 16) | ((c0 >> 32) & 0xFFFF);
  const uint64_t k1 = ((c1 & 0xFFFF) << 32) | (((c1 >> 16) & 0xFFFF) << 16) | ((c1 >> 32) & 0xFFFF);
  return k0 > k1;
}

__device__ __forceinline__ void write_zero_tile(const ReconParams& P, int k) {
  const int64_t n8 = (int64_t)P.R * P.R * 2;
  float4* o = reinterpret_cast<float4*>(P.x_out + (int64_t)k * P.R * P.R * 8);
  for (int64_t i = threadIdx.x; i < n8; i += RB) o[i] = make_float4(0.f, 0.f, 0.f, 0.f);
}

// Four waves per SIMD (128 VGPRs) so two 512-lane workgroups share a CU: the
// searches are latency-bound (LDS reads, dependent FP64 chains), and the
// second workgroup hides more of it than the few spills this costs.
__global__ void __launch_bounds__(RB, 4) k_recon(ReconParams P) {
  // region 0 holds the raw bucket offsets while bucketing, then the
  // canonical coordinates; the canonical bucket offsets sit at the end
  __shared__ __align__(16) int s_mem[LDS_INTS];
  __shared__ int s_tmp[RB / 64 + 1];
  __shared__ int s_hdr[5];  // tile index, flags, bin offset, bin count, tile id
  __shared__ int s_flags;
  __shared__ int s_ntri;
  __shared__ int s_next;
  __shared__ int s_nnblk;
  __shared__ double s_cz;
  const int tid = threadIdx.x;
  const int R = P.R, C = P.C, H = P.H, W2 = 2 * P.H;
  const int RR = R * R;
  uint64_t* __restrict__ fm = P.facemap + (int64_t)blockIdx.x * RR;
  int32_t* __restrict__ nn = P.nnidx + (int64_t)blockIdx.x * RR;
  const bool cap_overflow = P.flags[0] != 0;
  // Control flow below depends only on values that thread 0 fetches and
  // broadcasts through LDS, read back with readfirstlane so the compiler
  // sees them as uniform: every barrier then stays in uniform control flow
  // and the loop has a single back edge (an earlier form with a `continue`
  // let the compiler re-enter the barriers without the queue fetch).
  for (;;) {
    if (tid == 0) {
      const int q = atomicAdd(P.queue, 1);
      const int kk = q < P.n_tiles ? P.order[q] : q;
      s_hdr[0] = kk;
      if (kk < P.n_tiles) {
        int f = cap_overflow ? LS_TILE_CAP : 0;
        f |= P.status[kk] & LS_TILE_BADID;
        const int32_t o = P.bin_off[kk];
        s_hdr[1] = f;
        s_hdr[2] = o;
        s_hdr[3] = (f & (LS_TILE_CAP | LS_TILE_BADID)) ? 0 : P.bin_off[kk + 1] - o;
        s_hdr[4] = P.tile_list[kk];
      }
    }
    __syncthreads();
    const int k = __builtin_amdgcn_readfirstlane(s_hdr[0]);
    if (k >= P.n_tiles) break;
    const int flags = __builtin_amdgcn_readfirstlane(s_hdr[1]);
    const int32_t off = __builtin_amdgcn_readfirstlane(s_hdr[2]);
    const int32_t cnt = __builtin_amdgcn_readfirstlane(s_hdr[3]);
    const int32_t t = __builtin_amdgcn_readfirstlane(s_hdr[4]);
    if (cnt == 0) {
      write_zero_tile(P, k);
      if (tid == 0) {
        P.cz_out[k] = 0.0;
        P.status[k] = flags | LS_TILE_EMPTY;
      }
    } else {
      const int64_t cx = P.ox + (int64_t)(t % P.tiles_x) * P.S + P.S / 2;
      const int64_t cy = P.oy + (int64_t)(t / P.tiles_x) * P.S + P.S / 2;
      int G = 1;
      {
        const int want = (int)sqrtf((float)cnt * 0.5f);
        G = want < 1 ? 1 : (want > MAXG ? MAXG : want);
      }
      const int NB = G * G;
      int* s_b = s_mem;
      int* s_k = s_mem + LDS_INTS - (NB + 1);
      const bool uv_lds = 2 * cnt <= LDS_INTS - (NB + 1);
      // ---- a. gather + bucket histogram
      for (int b = tid; b <= NB; b += RB) s_b[b] = 0;
      if (tid == 0) {
        s_flags = 0;
        s_ntri = 0;
        s_next = 0;
        s_nnblk = 0;
      }
      __syncthreads();
      for (int e = tid; e < cnt; e += RB) {
        const int32_t gi = P.bin_idx[off + e];
        const int u = (int)((int64_t)P.x[gi] - cx), v = (int)((int64_t)P.y[gi] - cy);
        P.su[off + e] = u;
        P.sv[off + e] = v;
        P.sz[off + e] = P.z[gi];
        const uint16_t* c3 = P.rgb + 3 * (int64_t)gi;
        P.srgb[off + e] = (uint64_t)c3[0] | ((uint64_t)c3[1] << 16) | ((uint64_t)c3[2] << 32);
        const int b = bucket_1d(v + H, G, W2) * G + bucket_1d(u + H, G, W2);
        P.sslot[off + e] = atomicAdd(&s_b[b], 1);
      }
      __syncthreads();
      block_scan_excl(s_b, NB + 1, s_tmp);
      // Scatter into bucket order, sort every bucket by (v, u) with the
      // largest (z, R, G, B) first, drop repeated positions and write the
      // canonical points.  The sorted copies live in the free middle of the
      // LDS (between the bucket counts and the kept counts) when the window
      // fits, else in global memory at the window's offset.
      auto bucket_sort = [&](int* __restrict__ tu, int* __restrict__ tv, int* __restrict__ tz,
                             uint64_t* __restrict__ tc, int base) -> int {
        for (int e = tid; e < cnt; e += RB) {
          const int u = P.su[off + e], v = P.sv[off + e];
          const int b = bucket_1d(v + H, G, W2) * G + bucket_1d(u + H, G, W2);
          const int pos = base + s_b[b] + P.sslot[off + e];
          tu[pos] = u;
          tv[pos] = v;
          tz[pos] = P.sz[off + e];
          tc[pos] = P.srgb[off + e];
        }
        __syncthreads();
        // ---- b. per-bucket sort + dedupe
        if (tid == 0) s_k[NB] = 0;
        for (int b = tid; b < NB; b += RB) {
          const int lo = base + s_b[b], hi = base + s_b[b + 1];
          for (int i = lo + 1; i < hi; ++i) {
            const int u = tu[i], v = tv[i], zz = tz[i];
            const uint64_t c = tc[i];
            int j = i - 1;
            while (j >= lo && pt_less(u, v, zz, c, tu[j], tv[j], tz[j], tc[j])) {
              tu[j + 1] = tu[j];
              tv[j + 1] = tv[j];
              tz[j + 1] = tz[j];
              tc[j + 1] = tc[j];
              --j;
            }
            tu[j + 1] = u;
            tv[j + 1] = v;
            tz[j + 1] = zz;
            tc[j + 1] = c;
          }
          int kept = 0;
          for (int i = lo; i < hi; ++i)
            if (i == lo || tu[i] != tu[i - 1] || tv[i] != tv[i - 1]) ++kept;
          s_k[b] = kept;
        }
        __syncthreads();
        const int mm = __builtin_amdgcn_readfirstlane(block_scan_excl(s_k, NB + 1, s_tmp));
        for (int b = tid; b < NB; b += RB) {
          const int lo = base + s_b[b], hi = base + s_b[b + 1];
          int w = off + s_k[b];
          for (int i = lo; i < hi; ++i)
            if (i == lo || tu[i] != tu[i - 1] || tv[i] != tv[i - 1]) {
              P.cuv[w] = make_int2(tu[i], tv[i]);
              P.sz[w] = tz[i];
              P.srgb[w] = tc[i];
              ++w;
            }
        }
        __syncthreads();
        return mm;
      };
      // sorted copies in LDS: colours (8-byte aligned) then u, v, z
      const int a0 = (NB + 2) & ~1;
      const bool sort_lds = a0 + 5 * cnt <= LDS_INTS - (NB + 1);
      int m;
      if (sort_lds)
        m = bucket_sort(s_mem + a0 + 2 * cnt, s_mem + a0 + 3 * cnt, s_mem + a0 + 4 * cnt,
                        reinterpret_cast<uint64_t*>(s_mem + a0), 0);
      else
        m = bucket_sort(P.tu, P.tv, P.tz, P.trgb, off);
      // canonical coordinates in LDS when they fit, and behind them the
      // colours and heights read per texel by the output pass
      int2* s_uv = reinterpret_cast<int2*>(s_mem);
      uint64_t* s_c = reinterpret_cast<uint64_t*>(s_mem + 2 * m);
      int32_t* s_z = s_mem + 4 * m;
      const bool attr_lds = uv_lds && 5 * m <= LDS_INTS - (NB + 1);
      if (uv_lds)
        for (int p = tid; p < m; p += RB) {
          s_uv[p] = P.cuv[off + p];
          if (attr_lds) {
            s_c[p] = P.srgb[off + p];
            s_z[p] = P.sz[off + p];
          }
        }
      __syncthreads();
      // Phases c-e once per pointer kind: LDS pointers when the points and
      // their attributes are staged in LDS, global ones otherwise.
      double cz = 0.0;
      bool has_dt = false;
      auto phases = [&](auto uvp, auto Tz, auto Tc) {
      TileT<decltype(uvp)> T;
      T.uv = uvp;
      T.boff = (LdsI32)s_k;
      T.G = G;
      T.H = H;
      T.W2 = W2;
      T.bw = (double)W2 / G;
      // ---- c. face map reset (the nearest points follow the stars)
      const int q0 = -H + C / 2;
      for (int tt = tid; tt < RR; tt += RB) fm[tt] = FACE_NONE;
      // collinearity check
      bool noncol = false;
      if (m >= 3) {
        const int2 p0 = T.uv[0], p1 = T.uv[1];
        for (int p = tid; p < m; p += RB) {
          const int2 q = T.uv[p];
          if (orient_d(p0.x, p0.y, p1.x, p1.y, q.x, q.y) != 0.0) noncol = true;
        }
      }
      // face keys pack three point indices in 21 bits each
      has_dt = (__builtin_amdgcn_readfirstlane(__syncthreads_or(noncol)) != 0) && m < (1 << 21);
      if (m >= (1 << 21) && tid == 0) atomicOr(&s_flags, LS_TILE_DEGENERATE);
      // ---- d. Delaunay stars, rasterised into the face map
      uint64_t* __restrict__ tris = P.tris + 2 * (int64_t)off;
      // a triangle that covers a texel centre is queued for the group pass
      // below (or rasterised at once if the queue, sized for the 2m - 5
      // triangles of a triangulation, is full)
      auto emit = [&](int p, int q, int r) {
        int i0, i1, j0, j1;
        if (!tri_texel_box(T, p, q, r, C, R, i0, i1, j0, j1)) return;
        const int slot = atomicAdd(&s_ntri, 1);
        if (slot < 2 * cnt) {
          tris[slot] = face_key(p, q, r);
          return;
        }
        raster_triangle(T, p, q, r, C, R, fm);
      };
      if (has_dt) {
        // nearest neighbour of every point: the first edge of its star;
        // successor lists cleared
        int32_t* __restrict__ nb0 = P.sslot + off;
        uint64_t* __restrict__ succ = P.succ + (int64_t)off * SUCC_K;
        int32_t* __restrict__ succ_n = P.succ_n + off;
        for (int a = tid; a < m; a += RB) {
          nb0[a] = ring_nearest(T, T.uv[a].x, T.uv[a].y, a);
          succ_n[a] = 0;
          ulonglong2* s2 = reinterpret_cast<ulonglong2*>(succ + (int64_t)a * SUCC_K);
#pragma unroll
          for (int j = 0; j < SUCC_K / 2; ++j) s2[j] = make_ulonglong2(SUCC_EMPTY, SUCC_EMPTY);
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __syncthreads();
        // Every triangle lies in the stars of its three vertices.  A search
        // that finds triangle (p, q, c) left of p->q also answers the
        // searches left of q->c (third vertex p) and c->p (third vertex q);
        // it records them in the successor lists of q and c, keyed by the
        // edge's second vertex.  The search is exact, so a recorded answer
        // is the answer the search would give.
        auto succ_find = [&](int p, int q) -> int {
          const uint64_t* l = succ + (int64_t)p * SUCC_K;
          uint64_t v[SUCC_K];
#pragma unroll
          for (int j = 0; j < SUCC_K; ++j) v[j] = __hip_atomic_load(l + j, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
          int c = -1;
#pragma unroll
          for (int j = 0; j < SUCC_K; ++j)
            if (v[j] != SUCC_EMPTY && (int)(v[j] >> 32) == q) c = (int)(uint32_t)v[j];
          return c;
        };
        auto succ_put = [&](int p, int q, int c) {
          const int j = __hip_atomic_fetch_add(succ_n + p, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
          if (j < SUCC_K)
            __hip_atomic_store(succ + (int64_t)p * SUCC_K + j, ((uint64_t)(uint32_t)q << 32) | (uint32_t)c,
                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        };
        // Each lane walks one star at a time and takes the next point from a
        // shared counter as soon as its star is done, so the lanes of a wave
        // are not held at star boundaries.  The walk turns counter-clockwise
        // from the nearest neighbour b0; if it meets the hull it resumes
        // clockwise from b0.  Steps whose answer is already recorded are
        // taken at once; a wave searches only when few of its lanes can
        // step from the lists, and then all its waiting lanes search
        // together.
        int a = atomicAdd(&s_next, 1);
        int b0 = 0, b = 0, steps = 0, prev_b = -1, hull_b = -1;
        bool back = false, first = true;
        uint64_t hull_key = FACE_NONE;
        auto start = [&]() {
          b0 = nb0[a];
          b = b0;
          steps = 0;
          prev_b = -1;  // second vertex of the last counter-clockwise triangle
          hull_b = -1;
          back = false;
          first = true;
          hull_key = FACE_NONE;
        };
        if (a < m) start();
        // one step with c the third vertex left of the current edge (-1: none)
        auto advance = [&](int c) {
          // forward: triangle (a, b, c) left of a->b; backward: (b, a, c)
          const int p = back ? b : a, q = back ? a : b;
          bool done = false;
          if (c < 0) {
            if (back) {
              done = true;
            } else {
              hull_b = b;
              if (prev_b >= 0) hull_key = face_key(a, prev_b, b);
              back = true;
              b = b0;
            }
          } else {
            if (back && first && hull_key == FACE_NONE) hull_key = face_key(p, q, c);
            if (back) first = false;
            if (a < b && a < c) emit(p, q, c);
            prev_b = b;
            b = c;
            if (!back && b == b0) done = true;
          }
          if (!done && ++steps >= STAR_MAX_STEPS) {
            atomicOr(&s_flags, LS_TILE_DEGENERATE);
            done = true;
          }
          if (done) {
            if (hull_b >= 0 && hull_key != FACE_NONE) raster_hull_edge(T, a, hull_b, hull_key, C, R, fm);
            a = atomicAdd(&s_next, 1);
            if (a < m) start();
          }
        };
        for (;;) {
          const bool live = a < m;
          if (__ballot(live) == 0) break;
          const int p = back ? b : a, q = back ? a : b;
          int c = live ? succ_find(p, q) : -1;
          const bool hit = c >= 0;
          bool step = hit;
          if (__popcll(__ballot(hit)) <= SEARCH_MAX_HITS && live && !hit) {
            c = third_left(T, p, q);
            if (c >= 0) {
              succ_put(q, c, p);
              succ_put(c, p, q);
            }
            step = true;
          }
          if (step) advance(c);
        }
      }
      // nearest point per texel: 8 x 8 texel blocks taken from a shared
      // counter by each wave once its star walks are done, so the waves
      // that finish early fill the tail of the star phase
      {
        const int nbs = (R + 7) / 8, lane = tid & 63;
        for (;;) {
          int blk = 0;
          if (lane == 0) blk = atomicAdd(&s_nnblk, 1);
          blk = __builtin_amdgcn_readfirstlane(__shfl(blk, 0));
          if (blk >= nbs * nbs) break;
          const int bi = blk / nbs, bj = blk - bi * nbs;
          int qx, qy;
          const int b = nearest_block(T, q0, C, R, bi, bj, lane, qx, qy);
          const int i = bi * 8 + (lane >> 3), j = bj * 8 + (lane & 7);
          if (i < R && j < R) nn[i * R + j] = b;
        }
      }
      __syncthreads();
      {
        const int ntri = min(__builtin_amdgcn_readfirstlane(s_ntri), 2 * cnt);
        for (int t = tid / RASTER_LANES; t < ntri; t += RB / RASTER_LANES)
          raster_triangle_group(T, tris[t], C, R, fm, tid % RASTER_LANES);
      }
      __syncthreads();
      // ---- e. interpolation, normalisation, output
      auto lin_value = [&](int tt, double* out4) {
        const int i = tt / R, j = tt - i * R;
        const uint64_t f = fm[tt];
        if (f == FACE_NONE) {
          const int p = nn[tt];
          out4[0] = (double)Tz[p] * P.scale_z + P.offset_z;
          const uint64_t c = Tc[p];
          out4[1] = (double)(c & 0xFFFF);
          out4[2] = (double)((c >> 16) & 0xFFFF);
          out4[3] = (double)((c >> 32) & 0xFFFF);
          return;
        }
        const int a = (int)(f >> 42), b = (int)((f >> 21) & 0x1FFFFF), c = (int)(f & 0x1FFFFF);
        const int2 A = T.uv[a], B = T.uv[b], Cc = T.uv[c];
        const double qx = q0 + j * C, qy = q0 + i * C;
        const double ob = orient_d(Cc.x, Cc.y, A.x, A.y, qx, qy);
        const double oc = orient_d(A.x, A.y, B.x, B.y, qx, qy);
        const double O = orient_d(A.x, A.y, B.x, B.y, Cc.x, Cc.y);
        const double lb = ob / O, lc = oc / O;
        const double za = Tz[a], zb = Tz[b], zc = Tz[c];
        const double h = za + lb * (zb - za) + lc * (zc - za);
        out4[0] = h * P.scale_z + P.offset_z;
        const uint64_t ca = Tc[a], cb = Tc[b], cc = Tc[c];
        for (int ch = 0; ch < 3; ++ch) {
          const double va = (double)((ca >> (16 * ch)) & 0xFFFF), vb = (double)((cb >> (16 * ch)) & 0xFFFF),
                       vc = (double)((cc >> (16 * ch)) & 0xFFFF);
          out4[1 + ch] = va + lb * (vb - va) + lc * (vc - va);
        }
      };
      if (tid == 0) {
        double v4[4];
        lin_value((R / 2) * R + R / 2, v4);
        s_cz = v4[0];
      }
      __syncthreads();
      cz = s_cz;
      float4* __restrict__ out = reinterpret_cast<float4*>(P.x_out + (int64_t)k * RR * 8);
      for (int tt = tid; tt < RR; tt += RB) {
        double lv[4];
        lin_value(tt, lv);
        const int p = nn[tt];
        const double hn = (double)Tz[p] * P.scale_z + P.offset_z;
        const uint64_t c = Tc[p];
        const double k65 = 1.0 / 65535.0;
        out[2 * tt] = make_float4((float)((lv[0] - cz) * P.inv_r), (float)((hn - cz) * P.inv_r), (float)(lv[1] * k65),
                                  (float)(lv[2] * k65));
        out[2 * tt + 1] = make_float4((float)(lv[3] * k65), (float)((double)(c & 0xFFFF) * k65),
                                      (float)((double)((c >> 16) & 0xFFFF) * k65),
                                      (float)((double)((c >> 32) & 0xFFFF) * k65));
      }
      };
      if (attr_lds)
        phases(UvLds{(LdsU64)s_uv}, (LdsI32)s_z, (LdsU64)s_c);
      else
        phases(UvGlobal{P.cuv + off}, (const int32_t*)(P.sz + off), (const uint64_t*)(P.srgb + off));
    if (tid == 0) {
      P.cz_out[k] = cz;
      int st = flags | s_flags;
      if (!has_dt) st |= LS_TILE_NN_ONLY;
      P.status[k] = st;
    }
    }
    __syncthreads();
  }
}

int g_num_cu = 0;

int num_cus() {
  if (g_num_cu <= 0) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 256;
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || v <= 0) v = 256;
    g_num_cu = v;
  }
  return g_num_cu;
}

struct ReconLayout {
  int32_t* tile_pos;
  int32_t* counts;
  int32_t* fill;
  int32_t* flags;
  int32_t* queue;
  int32_t* order;
  int32_t* bin_off;
  int32_t* bin_idx;
  int32_t* sort_scratch;
  int32_t *su, *sv, *sz, *sslot, *tu, *tv, *tz;
  uint64_t *srgb, *trgb;
  int2* cuv;
  uint64_t* tris;
  uint64_t* succ;
  int32_t* succ_n;
  uint64_t* facemap;
  int32_t* nnidx;
  int n_wg;
  int64_t entries;
};

int64_t max_multiplicity(const LsGridInfo& gi) {
  const int64_t per = (2 * (int64_t)gi.H) / gi.S + 1;
  return per * per;
}

int recon_wg_count(int32_t n_tiles) {
  const int want = 2 * num_cus();
  return n_tiles < want ? (n_tiles > 0 ? n_tiles : 1) : want;
}

// Workspace layout for n_tiles tiles, n points and nwg recon workgroups.
size_t recon_layout(const LsGridInfo& gi, int32_t n_tiles, int64_t n, void* base, ReconLayout* L, int nwg) {
  LsArena A{reinterpret_cast<char*>(base), 0, 0};
  const int64_t nall = (int64_t)gi.tx * gi.ty;
  const int64_t E = n * max_multiplicity(gi) + 1;
  const int64_t RR = (int64_t)gi.R * gi.R;
  L->tile_pos = A.take<int32_t>(nall);
  L->counts = A.take<int32_t>(n_tiles + 1);
  L->fill = A.take<int32_t>(n_tiles + 1);
  L->flags = A.take<int32_t>(4);
  L->queue = L->flags + 1;
  L->order = A.take<int32_t>(n_tiles);
  L->bin_off = A.take<int32_t>(n_tiles + 1);
  L->bin_idx = A.take<int32_t>(E);
  L->sort_scratch = A.take<int32_t>(2 * E);
  L->su = A.take<int32_t>(E);
  L->sv = A.take<int32_t>(E);
  L->sz = A.take<int32_t>(E);
  L->sslot = A.take<int32_t>(E);
  L->tu = A.take<int32_t>(E);
  L->tv = A.take<int32_t>(E);
  L->tz = A.take<int32_t>(E);
  L->srgb = A.take<uint64_t>(E);
  L->trgb = A.take<uint64_t>(E);
  L->cuv = A.take<int2>(E);
  L->tris = A.take<uint64_t>(2 * E);
  L->succ = A.take<uint64_t>(SUCC_K * E);
  L->succ_n = A.take<int32_t>(E);
  L->facemap = A.take<uint64_t>(RR * nwg);
  L->nnidx = A.take<int32_t>(RR * nwg);
  L->n_wg = nwg;
  L->entries = E;
  return A.used;
}

// Enqueue the whole recon pipeline with its workspace at `ws` laid out for
// nwg recon workgroups (the caller has checked that it is large enough).
int recon_enqueue(const LsGridInfo& gi, const int32_t* x, const int32_t* y, const int32_t* z, const uint16_t* rgb,
                  int64_t n, const int32_t* tile_list, int32_t n_tiles, int32_t order, float* x_out, double* cz_out,
                  int32_t* bin_off, int32_t* bin_idx, int64_t bin_cap, int32_t* tile_status, void* ws, int nwg,
                  hipStream_t st) {
  ReconLayout L;
  recon_layout(gi, n_tiles, n, ws, &L, nwg);
  const bool user_csr = bin_off && bin_idx;
  int32_t* boff = user_csr ? bin_off : L.bin_off;
  int32_t* bidx = user_csr ? bin_idx : L.bin_idx;
  const int64_t cap = user_csr ? bin_cap : L.entries;
  const int64_t nall = (int64_t)gi.tx * gi.ty;

  const int T = 256;
  LS_TRACE("recon_all", st);
  auto blocks = [&](int64_t cnt) { return (int)std::min<int64_t>((cnt + T - 1) / T, 65535); };
  hipLaunchKernelGGL(k_fill_i32, dim3(blocks(nall)), dim3(T), 0, st, L.tile_pos, nall, 0x7fffffff);
  hipLaunchKernelGGL(k_fill_i32, dim3(blocks(n_tiles + 1)), dim3(T), 0, st, L.counts, (int64_t)n_tiles + 1, 0);
  hipLaunchKernelGGL(k_fill_i32, dim3(blocks(n_tiles + 1)), dim3(T), 0, st, L.fill, (int64_t)n_tiles + 1, 0);
  hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(T), 0, st, L.flags, (int64_t)4, 0);
  hipLaunchKernelGGL(k_fill_i32, dim3(blocks(n_tiles)), dim3(T), 0, st, tile_status, (int64_t)n_tiles, 0);
  hipLaunchKernelGGL(k_tile_pos, dim3(blocks(n_tiles)), dim3(T), 0, st, tile_list, n_tiles, nall, L.tile_pos,
                     tile_status);
  hipLaunchKernelGGL(k_tile_dup, dim3(blocks(n_tiles)), dim3(T), 0, st, tile_list, n_tiles, nall, L.tile_pos,
                     tile_status);
  hipLaunchKernelGGL(k_tile_pos_fix, dim3(blocks(nall)), dim3(T), 0, st, L.tile_pos, nall);
  LS_LAUNCH_CHECK();

  BinParams bp;
  bp.ox = gi.ox;
  bp.oy = gi.oy;
  bp.invS = 1.0 / gi.S;
  bp.S = gi.S;
  bp.H = gi.H;
  bp.tiles_x = gi.tx;
  bp.tiles_y = gi.ty;
  bp.K = 1 + gi.H / gi.S;
  bp.n_tiles = n_tiles;
  bp.n = n;
  bp.x = x;
  bp.y = y;
  bp.tile_pos = L.tile_pos;
  bp.counts = L.counts;
  bp.fill = L.fill;
  bp.bin_off = boff;
  bp.bin_idx = bidx;
  bp.cap = cap;
  bp.flags = L.flags;
  bp.order = L.order;
  bp.order_mode = order;
  const int pb = (int)std::min<int64_t>((n + T - 1) / T, 8192);
  // workgroup-private histograms when the tile list fits in LDS
  const bool lds_bins = n_tiles <= BIN_LDS_TILES;
  const int64_t chunk = 4096;
  const int nchunks = (int)std::max<int64_t>(1, (n + chunk - 1) / chunk);
  {
    LS_TRACE("bin_count", st);
    if (n > 0) {
      if (lds_bins)
        hipLaunchKernelGGL(k_bin_count_lds, dim3(nchunks), dim3(BIN_THREADS), 0, st, bp, chunk);
      else
        hipLaunchKernelGGL(k_bin_count, dim3(pb > 0 ? pb : 1), dim3(T), 0, st, bp);
    }
  }
  {
    LS_TRACE("bin_scan", st);
    hipLaunchKernelGGL(k_bin_scan, dim3(1), dim3(1024), 0, st, bp);
  }
  {
    LS_TRACE("bin_scatter", st);
    if (n > 0) {
      if (lds_bins)
        hipLaunchKernelGGL(k_bin_scatter_lds, dim3(nchunks), dim3(BIN_THREADS), 0, st, bp, chunk);
      else
        hipLaunchKernelGGL(k_bin_scatter, dim3(pb > 0 ? pb : 1), dim3(T), 0, st, bp);
    }
  }
  if (user_csr)
    hipLaunchKernelGGL(k_bin_sort, dim3(std::min(n_tiles, 4 * num_cus())), dim3(RB), 0, st, boff, n_tiles, bidx,
                       L.sort_scratch, L.flags);
  LS_LAUNCH_CHECK();

  ReconParams rp;
  rp.ox = gi.ox;
  rp.oy = gi.oy;
  rp.S = gi.S;
  rp.tiles_x = gi.tx;
  rp.C = gi.C;
  rp.R = gi.R;
  rp.H = gi.H;
  rp.scale_z = gi.scale_z;
  rp.offset_z = gi.offset_z;
  rp.inv_r = 1.0 / ((double)gi.H * gi.scale_xy);
  rp.n_tiles = n_tiles;
  rp.x = x;
  rp.y = y;
  rp.z = z;
  rp.rgb = rgb;
  rp.tile_list = tile_list;
  rp.bin_off = boff;
  rp.bin_idx = bidx;
  rp.flags = L.flags;
  rp.su = L.su;
  rp.sv = L.sv;
  rp.sz = L.sz;
  rp.srgb = L.srgb;
  rp.sslot = L.sslot;
  rp.tu = L.tu;
  rp.tv = L.tv;
  rp.tz = L.tz;
  rp.trgb = L.trgb;
  rp.cuv = L.cuv;
  rp.tris = L.tris;
  rp.succ = L.succ;
  rp.succ_n = L.succ_n;
  rp.facemap = L.facemap;
  rp.nnidx = L.nnidx;
  rp.queue = L.queue;
  rp.order = L.order;
  rp.x_out = x_out;
  rp.cz_out = cz_out;
  rp.status = tile_status;
  {
    LS_TRACE("recon_tile", st);
    hipLaunchKernelGGL(k_recon, dim3(L.n_wg), dim3(RB), 0, st, rp);
  }
  LS_LAUNCH_CHECK();
  return LS_OK;
}

}  // namespace

size_t ls_recon_ws_bytes(const LsGridInfo& gi, int32_t n_tiles, int64_t n) {
  ReconLayout L;
  return recon_layout(gi, n_tiles, n, nullptr, &L, recon_wg_count(n_tiles));
}

// ---------------------------------------------------------------------------
// Allocation-free variant: the workspace is a fixed array in device memory.
// Host code never passes the array's name to a kernel (in host code it is a
// stand-in, not a device address); it takes the address that
// hipGetSymbolAddress returns on each device, once per device.
// ---------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[LS_RECON_SCRATCH_BYTES];

namespace {

constexpr int SCRATCH_MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[SCRATCH_MAX_DEVICES] = {};

// Device address of `scratch` on the current device (looked up on the first
// call on that device, with the device current).
int scratch_address(void** out) {
  int dev = -1;
  LS_HOST_CHECK(hipGetDevice(&dev));
  if (dev < 0 || dev >= SCRATCH_MAX_DEVICES) {
    ls_set_last_message("device ordinal beyond the scratch table");
    return LS_EHIP;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      ls_set_last_error(e != hipSuccess ? e : hipErrorInvalidSymbol, "hipGetSymbolAddress(scratch)", __LINE__);
      return LS_EHIP;
    }
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return LS_OK;
}

}  // namespace

int ls_recon_noalloc_impl(const LsGridInfo& gi, const int32_t* x, const int32_t* y, const int32_t* z,
                          const uint16_t* rgb, int64_t n, const int32_t* tile_list, int32_t n_tiles, int32_t order,
                          float* x_out, double* cz_out, int32_t* bin_off, int32_t* bin_idx, int64_t bin_cap,
                          int32_t* tile_status, hipStream_t st) {
  if (n_tiles <= 0) return LS_OK;
  ReconLayout L;
  const size_t cap = LS_RECON_SCRATCH_BYTES;
  const size_t one = recon_layout(gi, n_tiles, n, nullptr, &L, 1);
  if (one > cap) return LS_ESCRATCH;
  // as many persistent workgroups as the scratch holds (their face and
  // nearest-point maps are the only part that grows with the count)
  int nwg = recon_wg_count(n_tiles);
  if (nwg > 1) {
    const size_t per_wg = recon_layout(gi, n_tiles, n, nullptr, &L, 2) - one;
    const int64_t fit = 1 + (int64_t)((cap - one) / (per_wg ? per_wg : 1));
    if (fit < nwg) nwg = (int)fit;
    while (nwg > 1 && recon_layout(gi, n_tiles, n, nullptr, &L, nwg) > cap) --nwg;
  }
  void* ws = nullptr;
  const int rc = scratch_address(&ws);
  if (rc != LS_OK) return rc;
  return recon_enqueue(gi, x, y, z, rgb, n, tile_list, n_tiles, order, x_out, cz_out, bin_off, bin_idx, bin_cap,
                       tile_status, ws, nwg, st);
}

int ls_recon_impl(const LsGridInfo& gi, const int32_t* x, const int32_t* y, const int32_t* z, const uint16_t* rgb,
                  int64_t n, const int32_t* tile_list, int32_t n_tiles, int32_t order, float* x_out, double* cz_out,
                  int32_t* bin_off, int32_t* bin_idx, int64_t bin_cap, int32_t* tile_status, void* ws,
                  size_t ws_bytes, hipStream_t st) {
  if (n_tiles <= 0) return LS_OK;
  ReconLayout L;
  const int nwg = recon_wg_count(n_tiles);
  const size_t need = recon_layout(gi, n_tiles, n, nullptr, &L, nwg);
  if (ws_bytes < need || !ws) return LS_EWORKSPACE;
  return recon_enqueue(gi, x, y, z, rgb, n, tile_list, n_tiles, order, x_out, cz_out, bin_off, bin_idx, bin_cap,
                       tile_status, ws, nwg, st);
}
