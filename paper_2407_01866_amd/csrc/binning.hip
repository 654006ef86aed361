// Footprint bound and tile binning (Image-GS Sec. 3.2): per-Gaussian preprocessing, exact
// circle/tile hit counting, pair emission and per-tile ranges over the sorted pair list.
#include "common.hpp"

#include <algorithm>

namespace igs {
namespace {

constexpr int kThreads = 256;

__global__ void fill_u32_kernel(uint32_t *__restrict__ p, int64_t count, uint32_t value) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; i < count; i += stride) p[i] = value;
}

__global__ void fill_f32_kernel(float *__restrict__ p, int64_t count, float value) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; i < count; i += stride) p[i] = value;
}

// Closed tile rectangle [x0, x1] x [y0, y1] (clipped to the image) against the circle of radius
// r = 3 max(s1, s2) about mu, evaluated in double with every product and sum rounded on its own
// so that the decision is reproducible bit for bit.  Tangency counts as a hit.
__device__ __forceinline__ bool circle_meets_tile(double mx, double my, double r2, int tx, int ty,
                                                  int H, int W) {
#pragma clang fp contract(off)
  double x0 = (double)(tx * kTile), y0 = (double)(ty * kTile);
  double x1 = (double)min(tx * kTile + kTile, W), y1 = (double)min(ty * kTile + kTile, H);
  double cx = mx < x0 ? x0 : (mx > x1 ? x1 : mx);
  double cy = my < y0 ? y0 : (my > y1 ? y1 : my);
  double dx = mx - cx;
  double dy = my - cy;
  double d2 = dx * dx + dy * dy;
  return d2 <= r2;
}

struct TileBox {
  int tx0, tx1, ty0, ty1;  // inclusive; empty when tx0 > tx1
  double mx, my, r2;
};

// Candidate tile range of one Gaussian: every tile whose rectangle can meet the circle.  The test
// above passes only tiles within r (1 + 2^-51) of mu along each axis (its squares and sum are
// rounded), and mu -+ r is evaluated to within a few ulps of its magnitude, so the range is taken
// over mu -+ (r + m) with a margin m = 1e-9 (1 + |mu| + r), far above both: a superset of the
// hits, each of which is then tested exactly.
__device__ __forceinline__ TileBox tile_box(float fmx, float fmy, float fs1, float fs2,
                                            int tiles_x, int tiles_y) {
#pragma clang fp contract(off)
  TileBox b;
  b.mx = (double)fmx;
  b.my = (double)fmy;
  double r = 3.0 * (double)(fs1 > fs2 ? fs1 : fs2);
  b.r2 = r * r;
  if (!(isfinite(b.mx) && isfinite(b.my) && isfinite(r))) {
    b.tx0 = b.ty0 = 1;
    b.tx1 = b.ty1 = 0;
    return b;
  }
  const double mgx = 1e-9 * (1.0 + fabs(b.mx) + r), mgy = 1e-9 * (1.0 + fabs(b.my) + r);
  double lo_x = floor((b.mx - r - mgx) / kTile), hi_x = floor((b.mx + r + mgx) / kTile);
  double lo_y = floor((b.my - r - mgy) / kTile), hi_y = floor((b.my + r + mgy) / kTile);
  lo_x = fmax(lo_x, 0.0);
  lo_y = fmax(lo_y, 0.0);
  hi_x = fmin(hi_x, (double)(tiles_x - 1));
  hi_y = fmin(hi_y, (double)(tiles_y - 1));
  if (lo_x > hi_x || lo_y > hi_y) {
    b.tx0 = b.ty0 = 1;
    b.tx1 = b.ty1 = 0;
    return b;
  }
  b.tx0 = (int)lo_x;
  b.tx1 = (int)hi_x;
  b.ty0 = (int)lo_y;
  b.ty1 = (int)hi_y;
  return b;
}

// The hits of tile row ty among the columns [tx0, tx1].  Along a row the test above depends on the
// column only through |dx|, the distance from mu_x to the tile's x-range, and passes for all |dx|
// up to a threshold (the rounded square and sum are monotone), while |dx| grows with the distance
// from the column nearest mu_x.  So the hits are one run [L, R] about that column: its ends are
// found by the exact test at an estimate (mu_x -+ the chord's half width) and at its neighbours.
// Returns R - L + 1, or 0 when the row has no hit.
__device__ __forceinline__ int row_run(double mx, double my, double r2, int ty, int tx0, int tx1,
                                       int H, int W, int &L) {
#pragma clang fp contract(off)
  const double y0 = (double)(ty * kTile), y1 = (double)min(ty * kTile + kTile, H);
  const double cy = my < y0 ? y0 : (my > y1 ? y1 : my);
  const double dy = my - cy;
  const double dy2 = dy * dy;
  // circle_meets_tile for the row's tiles: the same roundings, the row's dy^2 formed once
  auto hit = [&](int tx) {
    const double x0 = (double)(tx * kTile), x1 = (double)min(tx * kTile + kTile, W);
    const double cx = mx < x0 ? x0 : (mx > x1 ? x1 : mx);
    const double dx = mx - cx;
    return dx * dx + dy2 <= r2;
  };
  const int c = (int)fmin(fmax(floor(mx * (1.0 / kTile)), (double)tx0), (double)tx1);
  L = c;
  if (!hit(c)) return 0;
  // run ends estimated in float (the exact tests below settle them)
  const float hw = sqrtf(fmaxf((float)(r2 - dy2), 0.f)), mxf = (float)mx;
  int R = (int)fminf(fmaxf(floorf((mxf + hw) * (1.f / kTile)), (float)c), (float)tx1);
  int Lx = (int)fmaxf(fminf(floorf((mxf - hw) * (1.f / kTile)), (float)c), (float)tx0);
  while (R < tx1 && hit(R + 1)) ++R;
  while (R > c && !hit(R)) --R;
  while (Lx > tx0 && hit(Lx - 1)) --Lx;
  while (Lx < c && !hit(Lx)) ++Lx;
  L = Lx;
  return R - Lx + 1;
}

// Gaussians whose candidate tile box has more than this many tiles are enumerated by their
// whole wave, one box row per lane (row_run), instead of by their own lanes, so one very large
// Gaussian does not serialize the kernel.
constexpr int kCoopTiles = 64;
// Smaller boxes are enumerated by a quad of consecutive lanes per Gaussian (lane q of the quad
// tests tiles q, q + 4, ... in row-major order), which gives the kernels four times the waves.
constexpr int kQuad = 4;
constexpr int kQuadGauss = kThreads / kQuad;  // Gaussians per workgroup

// A box of at most kCoopTiles tiles as recorded by the preprocess kernel for the emit kernel:
// origin (12 bits each; tile coordinates are below 4096) and width - 1 (6 bits), with the hit
// pattern in a 64-bit mask (bit t = tile t of the box in row-major order).  kBoxCoop marks a box
// the emit kernel enumerates again itself (larger boxes, which walk rows).
constexpr uint32_t kBoxCoop = 0xFFFFFFFFu;
__device__ __forceinline__ uint32_t pack_box(int tx0, int ty0, int w) {
  return (uint32_t)tx0 | ((uint32_t)ty0 << 12) | ((uint32_t)(w - 1) << 24);
}

// Advances (x, y) by k positions in row-major order over rows of width w >= 1.
__device__ __forceinline__ void rowmajor_step(int &x, int &y, int k, int w) {
  x += k;
  while (x >= w) {
    x -= w;
    ++y;
  }
}

struct CoopBox {  // the candidate box of one Gaussian, broadcast from its lane
  double mx, my, r2;
  int tx0, ty0, w, area, H, W;
};

__device__ __forceinline__ double bcast_f64(double v, int src) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), src);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), src);
  return __hiloint2double(hi, lo);
}

__device__ __forceinline__ CoopBox coop_box(const TileBox &b, const ImageDesc &im, int src) {
  CoopBox c;
  c.mx = bcast_f64(b.mx, src);
  c.my = bcast_f64(b.my, src);
  c.r2 = bcast_f64(b.r2, src);
  c.tx0 = __builtin_amdgcn_readlane(b.tx0, src);
  c.ty0 = __builtin_amdgcn_readlane(b.ty0, src);
  c.w = __builtin_amdgcn_readlane(b.tx1 - b.tx0 + 1, src);
  c.area = c.w * __builtin_amdgcn_readlane(b.ty1 - b.ty0 + 1, src);
  c.H = __builtin_amdgcn_readlane(im.H, src);
  c.W = __builtin_amdgcn_readlane(im.W, src);
  return c;
}

__device__ __forceinline__ int box_area(const TileBox &b) {
  return b.tx0 > b.tx1 ? 0 : (b.tx1 - b.tx0 + 1) * (b.ty1 - b.ty0 + 1);
}

// Per Gaussian: rotation/inverse-scale coefficients (A, B; C, D) with e = (A dx + B dy,
// C dx + D dy) = diag(1/s1, 1/s2) R(theta)^T (x - mu), so that q = |e|^2 (Eq. 1-2); kept in
// float for ranking and in double for the blend weights; plus the exact tile-hit count, its
// exclusive prefix within the workgroup's Gaussians (offsets, finished by the emit kernel) and
// the workgroup's total (block_tot).  The kernel also zeroes the render's status block and
// zero_words words (the tile ranges, when the sort does not write them all), which the later
// binning kernels fill in; it is launched with at least one workgroup even for N = 0.
__global__ __launch_bounds__(kThreads) void preprocess_kernel(
    const float *__restrict__ params, int N, Images imgs, float4 *__restrict__ g32a,
    float2 *__restrict__ g32b, double4 *__restrict__ g64, uint32_t *__restrict__ counts,
    int64_t *__restrict__ offsets, uint32_t *__restrict__ block_tot,
    uint64_t *__restrict__ hit_mask, uint32_t *__restrict__ hit_box, int64_t *__restrict__ status,
    uint32_t *__restrict__ zero_words, int64_t nzero) {
  __shared__ uint32_t s_wtot[kThreads / 64];
  {
    const int64_t g = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (g < 8) status[g] = 0;
    for (int64_t k = g; k < nzero; k += (int64_t)gridDim.x * kThreads) zero_words[k] = 0u;
  }
  if (N <= 0) return;
  const int i = blockIdx.x * kQuadGauss + (int)(threadIdx.x / kQuad);
  const int q = threadIdx.x & (kQuad - 1);
  const bool valid = i < N;
  const int lane = threadIdx.x & 63;
  const int ii = valid ? i : N - 1;  // lanes past N mirror the last Gaussian and write nothing
  const ImageDesc im = imgs.by_gauss(ii);
  float mx = params[ii], my = params[(size_t)N + ii], th = params[2 * (size_t)N + ii];
  float s1 = params[3 * (size_t)N + ii], s2 = params[4 * (size_t)N + ii];
  TileBox b = tile_box(mx, my, s1, s2, im.tiles_x, im.tiles_y);
  const int area = valid ? box_area(b) : 0;
  if (valid && q == 0) {  // (before the tile loops, so that little stays live across them)
    double sn, cs;
    sincos((double)th, &sn, &cs);
    double u1 = 1.0 / (double)s1, u2 = 1.0 / (double)s2;
    double A = u1 * cs, B = u1 * sn, C = -u2 * sn, D = u2 * cs;
    g64[i] = make_double4(A, B, C, D);
    g32a[i] = make_float4(mx, my, (float)A, (float)B);
    g32b[i] = make_float2((float)C, (float)D);
  }
  uint32_t c = 0;
  uint64_t hm = 0;  // hit pattern of a small box
  if (area > 0 && area <= kCoopTiles) {  // (a non-empty box has width >= 1)
    const int w = b.tx1 - b.tx0 + 1;
    int x = 0, y = 0;
    rowmajor_step(x, y, q, w);
    for (int t = q; t < area; t += kQuad) {
      if (circle_meets_tile(b.mx, b.my, b.r2, b.tx0 + x, b.ty0 + y, im.H, im.W)) {
        ++c;
        hm |= 1ull << t;
      }
      rowmajor_step(x, y, kQuad, w);
    }
  }
  c += __shfl_xor(c, 1, 64);  // the quad's total and pattern, in every lane of the quad
  c += __shfl_xor(c, 2, 64);
  hm |= __shfl_xor(hm, 1, 64);
  hm |= __shfl_xor(hm, 2, 64);
  if (valid && q == 0) {
    hit_box[i] = area > kCoopTiles ? kBoxCoop
                                   : (area > 0 ? pack_box(b.tx0, b.ty0, b.tx1 - b.tx0 + 1) : 0u);
    hit_mask[i] = hm;
  }
  uint64_t big = __ballot(area > kCoopTiles && q == 0);
  while (big) {
    const int src = __ffsll((unsigned long long)big) - 1;
    big &= big - 1;
    const CoopBox cb = coop_box(b, im, src);
    const int rows = cb.area / cb.w;
    uint32_t hits = 0;
    for (int r0 = 0; r0 < rows; r0 += 64) {
      int L;
      if (r0 + lane < rows)
        hits += (uint32_t)row_run(cb.mx, cb.my, cb.r2, cb.ty0 + r0 + lane, cb.tx0,
                                  cb.tx0 + cb.w - 1, cb.H, cb.W, L);
    }
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) hits += __shfl_xor(hits, d, 64);
    if (lane == src) c = hits;
  }
  // exclusive prefix of the workgroup's counts (one per quad, from its first lane)
  const uint32_t v = (valid && q == 0) ? c : 0u;
  uint32_t inc = v;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint32_t t = __shfl_up(inc, d, 64);
    if (lane >= d) inc += t;
  }
  if (lane == 63) s_wtot[threadIdx.x >> 6] = inc;
  __syncthreads();
  uint32_t woff = 0, tot = 0;
#pragma unroll
  for (int k = 0; k < kThreads / 64; ++k) {
    woff += k < (int)(threadIdx.x >> 6) ? s_wtot[k] : 0u;
    tot += s_wtot[k];
  }
  if (valid && q == 0) {
    counts[i] = c;
    offsets[i] = (int64_t)(woff + inc - v);
  }
  if (threadIdx.x == 0) block_tot[blockIdx.x] = tot;
}

// Writes the tile key of every tile the Gaussian hits at emit index u (from the Gaussian's scanned
// offset on), and records the Gaussian of each emit index (in the key's bits from gid_shift on
// when gid_shift > 0, else in pair_gid[u]); the pair list is thereby in ascending
// Gaussian index, which the stable sort keeps within each tile, and the pairs of Gaussian i are
// the emit indices [offsets[i], offsets[i] + counts[i]), in row-major tile order.  Nothing is
// written past the capacity.
// offsets arrives as prefixes within each preprocess workgroup (the emit kernel's workgroups take
// the same Gaussians), whose totals are block_tot; the block adds the sum of the earlier blocks'
// totals (integers: exact in any order), writes the finished offsets back, and the last
// Gaussian's thread writes the pair total and the overflow flag.
__global__ __launch_bounds__(kThreads) void emit_kernel(
    const float *__restrict__ params, int N, Images imgs, const uint32_t *__restrict__ counts,
    int64_t *__restrict__ offsets, const uint32_t *__restrict__ block_tot, int64_t cap,
    int64_t *__restrict__ status, uint32_t *__restrict__ keys, uint32_t *__restrict__ pair_gid,
    int gid_shift, const uint64_t *__restrict__ hit_mask, const uint32_t *__restrict__ hit_box) {
  __shared__ int64_t s_wave[kThreads / 64];
  __shared__ int64_t s_prefix;
  const int i = blockIdx.x * kQuadGauss + (int)(threadIdx.x / kQuad);
  const int q = threadIdx.x & (kQuad - 1);
  const int lane = threadIdx.x & 63;
  {
    int64_t part = 0;
    for (int r = threadIdx.x; r < (int)blockIdx.x; r += kThreads) part += block_tot[r];
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) part += __shfl_down(part, d, 64);
    if (lane == 0) s_wave[threadIdx.x >> 6] = part;
    __syncthreads();
    if (threadIdx.x == 0) {
      int64_t t = 0;
      for (int k = 0; k < kThreads / 64; ++k) t += s_wave[k];
      s_prefix = t;
    }
    __syncthreads();
  }
  const int ii = i < N ? i : N - 1;
  const uint32_t c = i < N ? counts[ii] : 0u;
  // the quad's first lane reads and rewrites the offset; the others take it by shuffle
  int64_t o = (i < N && q == 0) ? offsets[i] + s_prefix : 0;
  o = __shfl(o, lane & ~(kQuad - 1), 64);
  if (i < N && q == 0) offsets[i] = o;
  if (i == N - 1 && q == 0) {
    const int64_t P = o + (int64_t)c;
    status[kStatPairs] = P;
    status[kStatOverflow] = P > cap ? 1 : 0;
    status[kStatSkip] = P > cap ? 1 : 0;
  }
  const bool active = c != 0 && o + (int64_t)c <= cap;
  const ImageDesc im = imgs.by_gauss(ii);
  const uint32_t bx = active ? hit_box[ii] : 0u;
  const bool coop = active && bx == kBoxCoop;
  if (active && !coop) {
    // a small box's hits from the pattern the preprocess kernel recorded: lane q of the quad
    // writes the hits of ranks q, q + 4, ... (the pattern's set bits, in row-major order)
    const int tx0 = (int)(bx & 0xFFFu), ty0 = (int)((bx >> 12) & 0xFFFu), w = (int)(bx >> 24) + 1;
    const uint32_t inv = (65536u + (uint32_t)w - 1u) / (uint32_t)w;  // (t inv) >> 16 = t / w
    uint64_t m = hit_mask[ii];                                          // for t < 64, w <= 64
    for (int k = 0; k < q; ++k) m &= m - 1;
    for (uint32_t rank = (uint32_t)q; m != 0 && rank < c; rank += kQuad) {
      const int t = __ffsll((unsigned long long)m) - 1;
      const int ty = (int)(((uint32_t)t * inv) >> 16), tx = t - ty * w;
      const int64_t u = IGS_IDX(o + rank, cap, kSiteEmit);
      const uint32_t tile = (uint32_t)(im.tile_off + (ty0 + ty) * im.tiles_x + tx0 + tx);
      if (gid_shift) {
        keys[u] = tile | ((uint32_t)i << gid_shift);
      } else {
        keys[u] = tile;
        pair_gid[u] = (uint32_t)i;
      }
#pragma unroll
      for (int k = 0; k < kQuad; ++k) m &= m - 1;
    }
  }
  TileBox b{};
  if (coop) {
    const float mx = params[ii], my = params[(size_t)N + ii];
    const float s1 = params[3 * (size_t)N + ii], s2 = params[4 * (size_t)N + ii];
    b = tile_box(mx, my, s1, s2, im.tiles_x, im.tiles_y);
  }
  uint64_t big = __ballot(coop && q == 0);
  while (big) {
    const int src = __ffsll((unsigned long long)big) - 1;
    big &= big - 1;
    const CoopBox cb = coop_box(b, im, src);
    const int64_t so = __builtin_amdgcn_readlane((int)(o & 0xFFFFFFFF), src) & 0xFFFFFFFFll;
    const int64_t sbase = so | ((int64_t)__builtin_amdgcn_readlane((int)(o >> 32), src) << 32);
    const uint32_t sc = (uint32_t)__builtin_amdgcn_readlane((int)c, src);
    const int tiles_x = __builtin_amdgcn_readlane(im.tiles_x, src);
    const int tile_off = __builtin_amdgcn_readlane(im.tile_off, src);
    const uint32_t gid = (uint32_t)__builtin_amdgcn_readlane(i, src);
    // 64 box rows at a time: each lane finds its row's run, a scan over the lanes places the
    // runs in row order, then the wave writes the runs one row after another, lanes along the run
    const int rows = cb.area / cb.w;
    uint32_t k = 0;  // hits written so far (uniform)
    for (int r0 = 0; r0 < rows; r0 += 64) {
      int L = 0;
      const uint32_t cnt = r0 + lane < rows
                               ? (uint32_t)row_run(cb.mx, cb.my, cb.r2, cb.ty0 + r0 + lane, cb.tx0,
                                                   cb.tx0 + cb.w - 1, cb.H, cb.W, L)
                               : 0u;
      uint32_t inc = cnt;
#pragma unroll
      for (int d = 1; d < 64; d <<= 1) {
        const uint32_t t = __shfl_up(inc, d, 64);
        if (lane >= d) inc += t;
      }
      const uint32_t start = k + inc - cnt;
      uint64_t live = __ballot(cnt > 0);
      while (live) {
        const int rl = __ffsll((unsigned long long)live) - 1;
        live &= live - 1;
        const uint32_t rc = (uint32_t)__builtin_amdgcn_readlane((int)cnt, rl);
        const uint32_t rs = (uint32_t)__builtin_amdgcn_readlane((int)start, rl);
        const int rL = __builtin_amdgcn_readlane(L, rl);
        const uint32_t row_key = (uint32_t)(tile_off + (cb.ty0 + r0 + rl) * tiles_x + rL);
        for (uint32_t j = lane; j < rc; j += 64) {
          const uint32_t rank = rs + j;
          if (rank < sc) {
            const int64_t u = IGS_IDX(sbase + rank, cap, kSiteEmit);
            const uint32_t tile = row_key + j;
            if (gid_shift) {
              keys[u] = tile | (gid << gid_shift);
            } else {
              keys[u] = tile;
              pair_gid[u] = gid;
            }
          }
        }
      }
      k += (uint32_t)__builtin_amdgcn_readlane((int)inc, 63);
    }
  }
}

// After the sort: the Gaussian of every sorted pair (from its emit index) and [start, end) of
// every tile in the sorted list (ranges zeroed beforehand), in one pass.
__global__ __launch_bounds__(kThreads) void resolve_ranges_kernel(
    const uint32_t *__restrict__ src, const uint32_t *__restrict__ pair_gid,
    const uint32_t *__restrict__ keys, const int64_t *__restrict__ status, int64_t cap,
    uint32_t *__restrict__ vals, int2 *__restrict__ ranges) {
  int64_t P = status[kStatOverflow] ? 0 : status[kStatPairs];
  if (P > cap) P = 0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < P; p += stride) {
    vals[p] = pair_gid[IGS_IDX(src[p], cap, kSiteResolve)];
    const uint32_t k = keys[p];
    if (p == 0 || keys[p - 1] != k) ranges[k].x = (int)p;
    if (p == P - 1 || keys[p + 1] != k) ranges[k].y = (int)(p + 1);
  }
}

// Per-render statistics from the tile ranges: the largest |S_j|, whether any exceeds the 16-bit
// slot range (which also marks the gradient as unusable when the render saves 16-bit slots for a
// separate adjoint: slots16), E_fwd = sum_j |S_j| times the tile's pixel count and E_bwd = sum_j min(K, |S_j|)
// times the tile's pixel count.  Every block reduces its tiles and adds them with 64-bit integer
// atomics (exact and order independent) into the status block, zeroed beforehand.
constexpr int kStatThreads = 256;
__global__ __launch_bounds__(kStatThreads) void tile_stats_kernel(const int2 *__restrict__ ranges,
                                                                  int T, Images imgs, int K,
                                                                  int slots16,
                                                                  int64_t *__restrict__ status) {
  __shared__ unsigned long long s_max[kStatThreads / 64], s_ef[kStatThreads / 64],
      s_eb[kStatThreads / 64];
  unsigned long long mx = 0, ef = 0, eb = 0;
  const int t = blockIdx.x * kStatThreads + threadIdx.x;
  if (t < T) {
    const int2 r = ranges[t];
    const unsigned long long c = (unsigned long long)(r.y - r.x);
    const ImageDesc im = imgs.by_tile(t);
    const int lt = t - im.tile_off;
    const int tx = lt % im.tiles_x, ty = lt / im.tiles_x;
    const unsigned long long npx =
        (unsigned long long)min(im.W - tx * kTile, kTile) * min(im.H - ty * kTile, kTile);
    mx = c;
    ef = c * npx;
    eb = (c < (unsigned long long)K ? c : (unsigned long long)K) * npx;
  }
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) {
    const unsigned long long omx = __shfl_down(mx, d, 64);
    mx = omx > mx ? omx : mx;
    ef += __shfl_down(ef, d, 64);
    eb += __shfl_down(eb, d, 64);
  }
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) {
    s_max[w] = mx;
    s_ef[w] = ef;
    s_eb[w] = eb;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int k = 1; k < kStatThreads / 64; ++k) {
      mx = s_max[k] > mx ? s_max[k] : mx;
      ef += s_ef[k];
      eb += s_eb[k];
    }
    unsigned long long *st = reinterpret_cast<unsigned long long *>(status);
    atomicMax(&st[kStatMaxList], mx);
    if (mx > 0xFFFF) {
      atomicMax(&st[kStatSlotOverflow], 1ull);
      if (slots16) atomicMax(&st[kStatSkip], 1ull);
    }
    atomicAdd(&st[kStatEvalsFwd], ef);
    atomicAdd(&st[kStatEvalsBwd], eb);
  }
}

// Lanes of the wave whose digit d (its low `bits` bits) equals the calling lane's, among the valid
// lanes: one ballot per bit.
__device__ __forceinline__ uint64_t match_digit(uint32_t d, int bits, bool valid) {
  uint64_t peers = __ballot(valid);
  for (int b = 0; b < bits; ++b) {
    const bool bit = (d >> b) & 1u;
    const uint64_t m = __ballot(bit);
    peers &= bit ? m : ~m;
  }
  return peers;
}

// Second stage of the pair sort.  The pairs arrive partitioned stably by the top hb bits of the
// tile key (from emit order, so each group's pairs are in ascending emit index); workgroup g owns
// group g, the tiles [g 2^lb, (g + 1) 2^lb), and its segment [s0, s1) of the partitioned list.
// Each wave takes a contiguous share of the segment, in whole rounds of 64 pairs, and counts it
// per tile (lanes with equal tiles found by match_digit; the lowest of them adds their number to
// the wave's own counter).  The counts give every tile's range and statistics and, scanned
// tile-major over the waves, where each wave's pairs of each tile start.  Each wave then scatters
// its share in order with no further synchronization, since only it touches its own positions.
// Result: tile-major order with each tile's pairs in ascending emit index, the same as a stable
// sort of the whole list by tile.  The first IT rounds of a share stay in registers between the
// two passes, with their ranks; longer shares are read again.  A segment of at most kGroupStage
// pairs is scattered into LDS and written out contiguously (coalesced stores rather than one
// memory request per pair); a longer one is scattered to memory directly.
constexpr int kGroupStage = 12288;
template <int NT, int IT>
__global__ __launch_bounds__(NT) void group_sort_kernel(
    const uint32_t *__restrict__ keys, const uint32_t *__restrict__ emit_idx,
    const uint32_t *__restrict__ hist_off, const uint32_t *__restrict__ run_sums, int nruns,
    int64_t nblocks, int64_t cap, int lb, int gid_shift, const uint32_t *__restrict__ pair_gid,
    Images imgs, int T, int K, const int64_t *__restrict__ status,
    unsigned long long *__restrict__ part, uint32_t *__restrict__ src, uint32_t *__restrict__ vals,
    int2 *__restrict__ ranges) {
  constexpr int kW = NT / 64;
  static_assert(NT >= 256, "one thread per tile of a group");
  __shared__ uint32_t wcnt[kW][256];  // per-wave counts, then the wave's next position per tile
  __shared__ uint32_t tcnt[256], tstart[256];
  __shared__ int64_t s_pre[kW][2];
  __shared__ unsigned long long s_st[kW][3];
  __shared__ uint32_t stage[2][kGroupStage];  // sorted emit indices and Gaussians of the segment
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int g = blockIdx.x;
  const int R = 1 << lb;
  const uint32_t mask = (uint32_t)R - 1;
  int64_t P = status[kStatOverflow] ? 0 : status[kStatPairs];
  if (P > cap) P = 0;
  // the segment: the partition's digit offsets at (g, block 0) and (g + 1, block 0)
  const int64_t h0 = (int64_t)g * nblocks, h1 = h0 + nblocks;
  const bool last = g + 1 == (int)gridDim.x;
  const uint32_t o0 = hist_off[h0];
  const uint32_t o1 = last ? 0u : hist_off[h1];
  for (int i = tid; i < kW * 256; i += NT) (&wcnt[0][0])[i] = 0u;
  int64_t a0 = 0, a1 = 0;
  if (run_sums) {
    const int64_t r0 = h0 / kScanBlockItems, r1 = h1 / kScanBlockItems;
    for (int r = tid; r < nruns; r += NT) {
      const int64_t v = run_sums[r];
      a0 += r < r0 ? v : 0;
      a1 += r < r1 ? v : 0;
    }
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
      a0 += __shfl_down(a0, d, 64);
      a1 += __shfl_down(a1, d, 64);
    }
    if (lane == 0) {
      s_pre[w][0] = a0;
      s_pre[w][1] = a1;
    }
  }
  __syncthreads();
  if (run_sums) {
    a0 = a1 = 0;
#pragma unroll
    for (int k = 0; k < kW; ++k) {
      a0 += s_pre[k][0];
      a1 += s_pre[k][1];
    }
  }
  const int64_t s0 = (int64_t)o0 + a0;
  const int64_t s1 = last ? P : (int64_t)o1 + a1;
  // this wave's share [b0, b1)
  const int64_t share = ((s1 - s0 + kW - 1) / kW + 63) & ~(int64_t)63;
  const int64_t b0 = min(s0 + (int64_t)w * share, s1), b1 = min(b0 + share, s1);
  const int rounds = (int)((b1 - b0 + 63) >> 6);
  const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  // pass 1: per-wave counts per tile
  uint32_t kk[IT], vv[IT], rk[IT];
#pragma unroll
  for (int r = 0; r < IT; ++r) {
    const int64_t i = b0 + (int64_t)r * 64 + lane;
    kk[r] = i < b1 ? keys[i] : 0u;
    vv[r] = i < b1 ? emit_idx[i] : 0u;
    rk[r] = 0u;
  }
#pragma unroll
  for (int r = 0; r < IT; ++r) {
    if (r >= rounds) break;  // uniform over the wave
    const bool valid = b0 + (int64_t)r * 64 + lane < b1;
    const uint32_t d = kk[r] & mask;
    const uint64_t peers = match_digit(d, lb, valid);
    const uint32_t rank = (uint32_t)__popcll(peers & lt_mask), c = (uint32_t)__popcll(peers);
    rk[r] = rank | (c << 8);
    if (valid && rank == 0) wcnt[w][d] += c;
  }
  for (int r = IT; r < rounds; ++r) {
    const int64_t i = b0 + (int64_t)r * 64 + lane;
    const bool valid = i < b1;
    const uint32_t d = (valid ? keys[i] : 0u) & mask;
    const uint64_t peers = match_digit(d, lb, valid);
    if (valid && __popcll(peers & lt_mask) == 0) wcnt[w][d] += (uint32_t)__popcll(peers);
  }
  __syncthreads();
  // tile totals; tile starts (exclusive scan, four tiles per lane of the first wave)
  if (tid < R) {
    uint32_t t = 0;
#pragma unroll
    for (int k = 0; k < kW; ++k) t += wcnt[k][tid];
    tcnt[tid] = t;
  }
  __syncthreads();
  if (w == 0) {
    uint32_t c[4], sum = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int d = lane * 4 + j;
      c[j] = d < R ? tcnt[d] : 0u;
      sum += c[j];
    }
    uint32_t inc = sum;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const uint32_t o = __shfl_up(inc, d, 64);
      if (lane >= d) inc += o;
    }
    uint32_t run = (uint32_t)s0 + inc - sum;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int d = lane * 4 + j;
      if (d < R) tstart[d] = run;
      run += c[j];
    }
  }
  __syncthreads();
  // every wave's first position per tile; ranges and statistics of the group's tiles
  {
    unsigned long long mx = 0, ef = 0, eb = 0;
    if (tid < R) {
      const uint32_t st = tstart[tid];
      uint32_t run = st;
#pragma unroll
      for (int k = 0; k < kW; ++k) {
        const uint32_t c = wcnt[k][tid];
        wcnt[k][tid] = run;
        run += c;
      }
      const int t = g * R + tid;
      const uint32_t c = tcnt[tid];
      if (t < T) {
        ranges[t] = c ? make_int2((int)st, (int)(st + c)) : make_int2(0, 0);
        if (c) {
          const ImageDesc im = imgs.by_tile(t);
          const int lt = t - im.tile_off;
          const int tx = lt % im.tiles_x, ty = lt / im.tiles_x;
          const unsigned long long npx =
              (unsigned long long)min(im.W - tx * kTile, kTile) * min(im.H - ty * kTile, kTile);
          mx = c;
          ef = c * npx;
          eb = (c < (uint32_t)K ? c : (uint32_t)K) * npx;
        }
      }
    }
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
      const unsigned long long omx = __shfl_down(mx, d, 64);
      mx = omx > mx ? omx : mx;
      ef += __shfl_down(ef, d, 64);
      eb += __shfl_down(eb, d, 64);
    }
    if (lane == 0) {
      s_st[w][0] = mx;
      s_st[w][1] = ef;
      s_st[w][2] = eb;
    }
  }
  __syncthreads();
  if (tid == 0) {  // the group's share of the statistics, summed by group_stats_kernel
    unsigned long long mx = 0, ef = 0, eb = 0;
#pragma unroll
    for (int k = 0; k < kW; ++k) {
      mx = s_st[k][0] > mx ? s_st[k][0] : mx;
      ef += s_st[k][1];
      eb += s_st[k][2];
    }
    part[3 * g] = mx;
    part[3 * g + 1] = ef;
    part[3 * g + 2] = eb;
  }
  // pass 2: each wave scatters its share in order (a lane reads its tile's next position, the
  // lowest lane of the tile then advances it past the round's pairs of that tile)
  const int64_t n = s1 - s0;
  const bool staged = n <= kGroupStage;  // uniform over the workgroup
  auto place = [&](uint32_t base, uint32_t rank, uint32_t e, uint32_t gid) {
    if (staged) {
      const int64_t j = IGS_IDX((int64_t)base + rank - s0, n, kSiteSortScatter);
      stage[0][j] = e;
      stage[1][j] = gid;
    } else {
      const int64_t pos = IGS_IDX((int64_t)base + rank, cap, kSiteSortScatter);
      src[pos] = e;
      vals[pos] = gid;
    }
  };
#pragma unroll
  for (int r = 0; r < IT; ++r) {
    if (r >= rounds) break;  // uniform over the wave
    const bool valid = b0 + (int64_t)r * 64 + lane < b1;
    if (valid) {
      const uint32_t d = kk[r] & mask, rank = rk[r] & 0xFFu;
      const uint32_t base = wcnt[w][d];
      place(base, rank, vv[r],
            gid_shift ? kk[r] >> gid_shift : pair_gid[IGS_IDX((int64_t)vv[r], cap, kSiteResolve)]);
      if (rank == 0) wcnt[w][d] = base + (rk[r] >> 8);
    }
  }
  for (int r = IT; r < rounds; ++r) {
    const int64_t i = b0 + (int64_t)r * 64 + lane;
    const bool valid = i < b1;
    const uint32_t key = valid ? keys[i] : 0u;
    const uint32_t d = key & mask;
    const uint64_t peers = match_digit(d, lb, valid);
    if (valid) {
      const uint32_t rank = (uint32_t)__popcll(peers & lt_mask);
      const uint32_t base = wcnt[w][d];
      const uint32_t e = emit_idx[i];
      place(base, rank, e,
            gid_shift ? key >> gid_shift : pair_gid[IGS_IDX((int64_t)e, cap, kSiteResolve)]);
      if (rank == 0) wcnt[w][d] = base + (uint32_t)__popcll(peers);
    }
  }
  if (staged) {
    __syncthreads();
    for (int j = tid; j < (int)n; j += NT) {
      src[s0 + j] = stage[0][j];
      vals[s0 + j] = stage[1][j];
    }
  }
}

// The tile statistics from the groups' shares, when no later kernel of the call sums them.
__global__ __launch_bounds__(256) void group_stats_kernel(const unsigned long long *__restrict__ part,
                                                          int G, int slots16,
                                                          int64_t *__restrict__ status) {
  sum_group_stats(part, G, slots16, status);
}

__global__ __launch_bounds__(kThreads) void tile_order_keys_kernel(const int2 *__restrict__ ranges,
                                                                   int T, uint32_t *__restrict__ keys,
                                                                   uint32_t *__restrict__ vals,
                                                                   int64_t *__restrict__ count) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t == 0) count[0] = T;
  if (t >= T) return;
  const int2 r = ranges[t];
  const int c = min(r.y - r.x, 0xFFFF);
  keys[t] = (uint32_t)(0xFFFF - c);
  vals[t] = (uint32_t)t;
}

inline int grid_for(int64_t count, int threads, int max_blocks = 65536) {
  int64_t b = (count + threads - 1) / threads;
  if (b < 1) b = 1;
  if (b > max_blocks) b = max_blocks;
  return (int)b;
}

}  // namespace

hipError_t launch_fill_u32(uint32_t *p, int64_t count, uint32_t value, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  fill_u32_kernel<<<grid_for(count, kThreads, 4096), kThreads, 0, s>>>(p, count, value);
  return hipGetLastError();
}

hipError_t launch_fill_f32(float *p, int64_t count, float value, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  fill_f32_kernel<<<grid_for(count, kThreads, 4096), kThreads, 0, s>>>(p, count, value);
  return hipGetLastError();
}

int gauss_blocks(int N) { return (N + kQuadGauss - 1) / kQuadGauss; }

hipError_t launch_preprocess(const float *params, int N, const Images &imgs, float4 *g32a,
                             float2 *g32b, double4 *g64, uint32_t *counts, int64_t *offsets,
                             uint32_t *block_tot, uint64_t *hit_mask, uint32_t *hit_box,
                             int64_t *status, int2 *ranges, int T, hipStream_t s) {
  const int grid = std::max(gauss_blocks(N), 1);
  preprocess_kernel<<<grid, kThreads, 0, s>>>(params, N, imgs, g32a, g32b, g64, counts, offsets,
                                              block_tot, hit_mask, hit_box, status,
                                              reinterpret_cast<uint32_t *>(ranges),
                                              2 * (int64_t)T);
  return hipGetLastError();
}

hipError_t launch_offsets_emit(const float *params, int N, const Images &imgs,
                               const uint32_t *counts, int64_t *offsets, int64_t cap,
                               int64_t *status, uint32_t *keys, uint32_t *pair_gid,
                               int gid_shift, const uint32_t *block_tot,
                               const uint64_t *hit_mask, const uint32_t *hit_box, hipStream_t s) {
  if (N <= 0) return hipSuccess;  // the status block already holds 0 pairs, no overflow
  emit_kernel<<<gauss_blocks(N), kThreads, 0, s>>>(params, N, imgs, counts, offsets, block_tot,
                                                   cap, status, keys, pair_gid, gid_shift,
                                                   hit_mask, hit_box);
  return hipGetLastError();
}

constexpr int kGroupThreads = 1024;
constexpr int kGroupItems = 8;

hipError_t launch_group_sort(const uint32_t *keys, const uint32_t *emit_idx,
                             const PartitionOffsets &po, int64_t cap, int hb, int lb,
                             int gid_shift, const uint32_t *pair_gid, const Images &imgs, int T,
                             int K, bool slots16, int64_t *status, uint64_t *group_part,
                             uint32_t *src, uint32_t *vals, int2 *ranges, bool stats_kernel,
                             hipStream_t s) {
  if (lb < 0 || lb > 8 || hb < 1 || hb > 8) return hipErrorInvalidValue;
  unsigned long long *part = reinterpret_cast<unsigned long long *>(group_part);
  group_sort_kernel<kGroupThreads, kGroupItems><<<1u << hb, kGroupThreads, 0, s>>>(
      keys, emit_idx, po.hist_off, po.run_sums, po.nruns, po.nblocks, cap, lb, gid_shift,
      pair_gid, imgs, T, K, status, part, src, vals, ranges);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (!stats_kernel) return hipSuccess;
  group_stats_kernel<<<1, 256, 0, s>>>(part, 1 << hb, slots16 ? 1 : 0, status);
  return hipGetLastError();
}

hipError_t launch_resolve_ranges(const uint32_t *src, const uint32_t *pair_gid,
                                const uint32_t *keys, const int64_t *status, int64_t cap,
                                uint32_t *vals, int2 *ranges, hipStream_t s) {
  resolve_ranges_kernel<<<grid_for(cap, kThreads, 8192), kThreads, 0, s>>>(src, pair_gid, keys,
                                                                           status, cap, vals,
                                                                           ranges);
  return hipGetLastError();
}

hipError_t launch_tile_order_keys(const int2 *ranges, int T, uint32_t *keys, uint32_t *vals,
                                  int64_t *count, hipStream_t s) {
  tile_order_keys_kernel<<<(T + kThreads - 1) / kThreads, kThreads, 0, s>>>(ranges, T, keys, vals,
                                                                            count);
  return hipGetLastError();
}

hipError_t launch_tile_stats(const int2 *ranges, int T, const Images &imgs, int K, bool slots16,
                             int64_t *status, hipStream_t s) {
  if (T <= 0) return hipSuccess;
  tile_stats_kernel<<<(T + kStatThreads - 1) / kStatThreads, kStatThreads, 0, s>>>(
      ranges, T, imgs, K, slots16 ? 1 : 0, status);
  return hipGetLastError();
}

}  // namespace igs
