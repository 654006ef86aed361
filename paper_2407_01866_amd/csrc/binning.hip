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

// Candidate tile range of one Gaussian: every tile whose rectangle can meet the circle, widened
// by one tile on each side so that rounding of mu +- r never drops a tangent tile.
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
  double lo_x = floor((b.mx - r) / kTile) - 1.0, hi_x = floor((b.mx + r) / kTile) + 1.0;
  double lo_y = floor((b.my - r) / kTile) - 1.0, hi_y = floor((b.my + r) / kTile) + 1.0;
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

// Gaussians whose candidate tile box has more than this many tiles are enumerated by their
// whole wave (lane t tests tiles t, t + 64, ... of the box, in the box's row-major order) instead
// of by their own lane, so one very large Gaussian does not serialize the kernel.
constexpr int kCoopTiles = 64;
// Smaller boxes are enumerated by a quad of consecutive lanes per Gaussian (lane q of the quad
// tests tiles q, q + 4, ... in row-major order), which gives the kernels four times the waves.
constexpr int kQuad = 4;
constexpr int kQuadGauss = kThreads / kQuad;  // Gaussians per workgroup

// Advances (x, y) by k positions in row-major order over rows of width w >= 1.
__device__ __forceinline__ void rowmajor_step(int &x, int &y, int k, int w) {
  x += k;
  while (x >= w) {
    x -= w;
    ++y;
  }
}

// The bits of a wave ballot that belong to the calling lane's quad.
__device__ __forceinline__ uint32_t quad_bits(uint64_t m, int lane) {
  return (uint32_t)(m >> (lane & ~(kQuad - 1))) & ((1u << kQuad) - 1u);
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
// float for ranking and in double for the blend weights; plus the exact tile-hit count.  The
// kernel also zeroes the render's status block and the tile ranges (zero_words words), which
// the later binning kernels fill in; it is launched with at least one workgroup even for N = 0.
__global__ __launch_bounds__(kThreads) void preprocess_kernel(
    const float *__restrict__ params, int N, Images imgs, float4 *__restrict__ g32a,
    float2 *__restrict__ g32b, double4 *__restrict__ g64, uint32_t *__restrict__ counts,
    int64_t *__restrict__ status, uint32_t *__restrict__ zero_words, int64_t nzero) {
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
  uint32_t c = 0;
  if (area > 0 && area <= kCoopTiles) {  // (a non-empty box has width >= 1)
    const int w = b.tx1 - b.tx0 + 1;
    int x = 0, y = 0;
    rowmajor_step(x, y, q, w);
    for (int t = q; t < area; t += kQuad) {
      c += circle_meets_tile(b.mx, b.my, b.r2, b.tx0 + x, b.ty0 + y, im.H, im.W);
      rowmajor_step(x, y, kQuad, w);
    }
  }
  c += __shfl_xor(c, 1, 64);  // the quad's total, in every lane of the quad
  c += __shfl_xor(c, 2, 64);
  uint64_t big = __ballot(area > kCoopTiles && q == 0);
  while (big) {
    const int src = __ffsll((unsigned long long)big) - 1;
    big &= big - 1;
    const CoopBox cb = coop_box(b, im, src);
    uint32_t hits = 0;
    for (int t0 = 0; t0 < cb.area; t0 += 64) {
      const int t = t0 + lane;
      const bool hit = t < cb.area && circle_meets_tile(cb.mx, cb.my, cb.r2, cb.tx0 + t % cb.w,
                                                        cb.ty0 + t / cb.w, cb.H, cb.W);
      hits += (uint32_t)__popcll(__ballot(hit));
    }
    if (lane == src) c = hits;
  }
  if (!valid || q != 0) return;
  double sn, cs;
  sincos((double)th, &sn, &cs);
  double u1 = 1.0 / (double)s1, u2 = 1.0 / (double)s2;
  double A = u1 * cs, B = u1 * sn, C = -u2 * sn, D = u2 * cs;
  g64[i] = make_double4(A, B, C, D);
  g32a[i] = make_float4(mx, my, (float)A, (float)B);
  g32b[i] = make_float2((float)C, (float)D);
  counts[i] = c;
}

// Writes the tile key of every tile the Gaussian hits at emit index u (from the Gaussian's scanned
// offset on), and records the Gaussian of each emit index; the pair list is thereby in ascending
// Gaussian index, which the stable sort keeps within each tile, and the pairs of Gaussian i are
// the emit indices [offsets[i], offsets[i] + counts[i]), in row-major tile order.  Nothing is
// written past the capacity.
// offsets arrives as the scan's per-run prefixes (runs of kScanBlockItems counts, whose totals are
// run_sums); a block's Gaussians lie in one run, so the block adds the sum of the earlier runs'
// totals (integers: exact in any order), writes the finished offsets back, and the last Gaussian's
// thread writes the pair total and the overflow flag.
static_assert(kScanBlockItems % kQuadGauss == 0, "an emit block must not straddle two scan runs");
__global__ __launch_bounds__(kThreads) void emit_kernel(
    const float *__restrict__ params, int N, Images imgs, const uint32_t *__restrict__ counts,
    int64_t *__restrict__ offsets, const int64_t *__restrict__ run_sums, int64_t cap,
    int64_t *__restrict__ status, uint32_t *__restrict__ keys, uint32_t *__restrict__ pair_gid) {
  __shared__ int64_t s_wave[kThreads / 64];
  __shared__ int64_t s_prefix;
  const int i = blockIdx.x * kQuadGauss + (int)(threadIdx.x / kQuad);
  const int q = threadIdx.x & (kQuad - 1);
  const int lane = threadIdx.x & 63;
  {
    const int run = (int)(((int64_t)blockIdx.x * kQuadGauss) / kScanBlockItems);
    int64_t part = 0;
    for (int r = threadIdx.x; r < run; r += kThreads) part += run_sums[r];
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
  float mx = params[ii], my = params[(size_t)N + ii];
  float s1 = params[3 * (size_t)N + ii], s2 = params[4 * (size_t)N + ii];
  TileBox b = tile_box(mx, my, s1, s2, im.tiles_x, im.tiles_y);
  const int area = active ? box_area(b) : 0;
  if (area > 0 && area <= kCoopTiles) {  // (a non-empty box has width >= 1)
    // the quad walks the box in row-major order, four tiles per step; a hit's rank is the quad's
    // hits so far plus those of its lower lanes in this step
    const int w = b.tx1 - b.tx0 + 1;
    int x = 0, y = 0;
    rowmajor_step(x, y, q, w);
    uint32_t k = 0;
    for (int t0 = 0; t0 < area; t0 += kQuad) {  // uniform over the quad
      const int t = t0 + q;
      const int tx = b.tx0 + x, ty = b.ty0 + y;
      rowmajor_step(x, y, kQuad, w);
      const bool hit = t < area && circle_meets_tile(b.mx, b.my, b.r2, tx, ty, im.H, im.W);
      const uint32_t qm = quad_bits(__ballot(hit), lane);
      const uint32_t rank = k + (uint32_t)__popc(qm & ((1u << q) - 1u));
      if (hit && rank < c) {
        const int64_t u = IGS_IDX(o + rank, cap, kSiteEmit);
        keys[u] = (uint32_t)(im.tile_off + ty * im.tiles_x + tx);
        pair_gid[u] = (uint32_t)i;
      }
      k += (uint32_t)__popc(qm);
    }
  }
  uint64_t big = __ballot(area > kCoopTiles && q == 0);
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
    uint32_t k = 0;  // hits written so far (uniform)
    for (int t0 = 0; t0 < cb.area; t0 += 64) {
      const int t = t0 + lane;
      const int tx = cb.tx0 + t % cb.w, ty = cb.ty0 + t / cb.w;
      const bool hit = t < cb.area && circle_meets_tile(cb.mx, cb.my, cb.r2, tx, ty, cb.H, cb.W);
      const uint64_t m = __ballot(hit);
      const uint32_t rank = k + (uint32_t)__popcll(m & ((1ull << lane) - 1ull));
      if (hit && rank < sc) {
        const int64_t u = IGS_IDX(sbase + rank, cap, kSiteEmit);
        keys[u] = (uint32_t)(tile_off + ty * tiles_x + tx);
        pair_gid[u] = gid;
      }
      k += (uint32_t)__popcll(m);
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

hipError_t launch_preprocess(const float *params, int N, const Images &imgs, float4 *g32a,
                             float2 *g32b, double4 *g64, uint32_t *counts, int64_t *status,
                             int2 *ranges, int T, hipStream_t s) {
  const int grid = std::max((N + kQuadGauss - 1) / kQuadGauss, 1);
  preprocess_kernel<<<grid, kThreads, 0, s>>>(params, N, imgs, g32a, g32b, g64, counts, status,
                                              reinterpret_cast<uint32_t *>(ranges),
                                              2 * (int64_t)T);
  return hipGetLastError();
}

hipError_t launch_offsets_emit(const float *params, int N, const Images &imgs,
                               const uint32_t *counts, int64_t *offsets, int64_t cap,
                               int64_t *status, uint32_t *keys, uint32_t *pair_gid,
                               int64_t *scan_tmp, hipStream_t s) {
  if (N <= 0) return hipSuccess;  // the status block already holds 0 pairs, no overflow
  hipError_t e = scan_u32_to_i64_blocks(counts, offsets, N, scan_tmp, s);
  if (e != hipSuccess) return e;
  emit_kernel<<<(N + kQuadGauss - 1) / kQuadGauss, kThreads, 0, s>>>(
      params, N, imgs, counts, offsets, scan_tmp, cap, status, keys, pair_gid);
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
