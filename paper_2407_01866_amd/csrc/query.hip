// Decoding side of the representation (Image-GS Sec. 1, Sec. 3.2, Sec. 4.1):
//
// * random access: the colour of the representation at arbitrary points of the image plane, each
//   evaluated on its own with the renderer's rule (the point's tile j, every member of S_j ranked
//   by q at the point, the top K blended by Eq. 5), using the tile lists of a binning pass.  The
//   ranking and the blend are the forward rasterizer's operations, so at a pixel centre a query
//   returns exactly the rendered pixel;
// * storage in float16 (Sec. 4.1: the trained attributes are quantized to float16): conversion
//   of the fitter's parameters (normalized mean, rotation, inverse scales, colour) to float16
//   with round-to-nearest-even, and decoding of a prefix of a stored set, its first N_prefix
//   Gaussians, into the renderer's float32 units.  Gaussians added by the error-guided schedule
//   are appended, so every prefix boundary of the schedule is a level of detail.
#include "raster_common.hpp"

#include <hip/hip_fp16.h>

#include <algorithm>

namespace igs {
namespace {

constexpr int kQueryThreads = 256;

// Sort keys of the points: the tile of each point (T for a point outside the image); the sort
// takes the point's index as the value, so that it groups the points by tile in input order.
__global__ __launch_bounds__(kQueryThreads) void query_keys_kernel(
    const float *__restrict__ pts, int M, int H, int W, int tiles_x, int tiles_y,
    uint32_t *__restrict__ keys, int64_t *__restrict__ count) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0) count[0] = M;
  if (i >= M) return;
  const float2 pt = reinterpret_cast<const float2 *>(pts)[i];
  const float fx = pt.x, fy = pt.y;
  const bool inside = fx >= 0.f && fx < (float)W && fy >= 0.f && fy < (float)H;
  keys[i] = inside ? (uint32_t)(min((int)fy / kTile, tiles_y - 1) * tiles_x +
                                min((int)fx / kTile, tiles_x - 1))
                   : (uint32_t)(tiles_x * tiles_y);
}

// One thread per point, in the order `order` gives (points grouped by tile, so that the lanes of
// a wave walk the same hit set and load the same candidates), or in input order when order is
// null.  With an order, each XCD takes a contiguous run of the sorted points (the workgroup ids
// it receives are mapped as the raster kernels map tiles), so the Gaussians of neighbouring
// tiles stay in that XCD's L2.  Points outside [0, W) x [0, H) (or not finite) decode to 0.
// NC >= n: the colours are accumulated in registers and each point's n results are written
// together.  A tile of at most qstage(NC) members has its members' colours staged in the wave's
// LDS rows while its candidates are loaded, so the blend reads them there instead of gathering
// n scattered parameters per winner.  REC: every Gaussian's data is read from one record of
// query_rec_stride(n) floats (query_records_kernel) instead of from the three geometry arrays and
// n parameter rows, so a member touches one or two cache lines instead of up to n + 3.
__host__ __device__ constexpr int qstage(int nc) { return nc <= 16 ? 128 : 64; }
// Record of one Gaussian for the point queries: float4 (mu_x, mu_y, A, B) at 0, float2 (C, D) at
// 4, double4 (A, B, C, D) at 8, the n colours from 16; 128 bytes for n <= 16.
__host__ __device__ constexpr int query_rec_stride(int n) { return n <= 16 ? 32 : 48; }

// One float4 of a record per thread, so that a wave's stores are contiguous: slot 0 the ranking
// geometry, 1 (C, D), 2-3 the blend geometry, then the colours four at a time (zero past n).
__global__ __launch_bounds__(256) void query_records_kernel(
    const float4 *__restrict__ g32a, const float2 *__restrict__ g32b,
    const double4 *__restrict__ g64, const float *__restrict__ params, int N, int n,
    float *__restrict__ rec) {
  const int slots = query_rec_stride(n) / 4;
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t i = j / slots;
  const int sl = (int)(j - i * slots);
  if (i >= N) return;
  float4 v;
  if (sl == 0) {
    v = g32a[i];
  } else if (sl == 1) {
    const float2 b = g32b[i];
    v = make_float4(b.x, b.y, 0.f, 0.f);
  } else if (sl < 4) {
    const double2 d = reinterpret_cast<const double2 *>(g64 + i)[sl - 2];
    __builtin_memcpy(&v, &d, sizeof(v));
  } else {
    const int c0 = 4 * (sl - 4);
    float c[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) c[u] = c0 + u < n ? params[(size_t)(5 + c0 + u) * N + i] : 0.f;
    v = make_float4(c[0], c[1], c[2], c[3]);
  }
  reinterpret_cast<float4 *>(rec)[j] = v;
}

template <int NC>
__host__ __device__ constexpr size_t query_lds_bytes() {
  return (size_t)(kQueryThreads / 64) * qstage(NC) * NC * sizeof(float);
}

template <int NC, int KT, bool REC>
__global__ __launch_bounds__(kQueryThreads) void query_kernel(
    const float *__restrict__ params, int N, int n, int H, int W, int K, int tiles_x,
    int tiles_y, const int2 *__restrict__ ranges, const uint32_t *__restrict__ vals,
    const float4 *__restrict__ g32a, const float2 *__restrict__ g32b,
    const double4 *__restrict__ g64, const float *__restrict__ rec, const float *__restrict__ pts,
    int M, const uint32_t *__restrict__ order, float *__restrict__ out) {
  constexpr int QS = qstage(NC);
  constexpr int RS = query_rec_stride(NC);
  extern __shared__ __align__(16) unsigned char qsm[];
  float *__restrict__ scol = reinterpret_cast<float *>(qsm) + (threadIdx.x >> 6) * QS * NC;
  const int blk = order ? xcd_tile(blockIdx.x, gridDim.x) : blockIdx.x;
  const int t = blk * blockDim.x + threadIdx.x;
  const bool valid = t < M;  // lanes past the end stay for the wave-wide broadcasts
  const int i = valid ? (order ? (int)order[t] : t) : 0;
  const float2 pt = valid ? reinterpret_cast<const float2 *>(pts)[i] : make_float2(-1.f, -1.f);
  const float fx = pt.x, fy = pt.y;
  const bool inside = fx >= 0.f && fx < (float)W && fy >= 0.f && fy < (float)H;
  int tile = -1, start = 0, cnt = 0;
  if (inside) {
    tile = min((int)fy / kTile, tiles_y - 1) * tiles_x + min((int)fx / kTile, tiles_x - 1);
    const int2 rg = ranges[tile];
    start = rg.x;
    cnt = rg.y - rg.x;
  }
  double tk[KT];
#pragma unroll
  for (int k = 0; k < KT; ++k) tk[k] = kKeyEmpty;
  // one pass per distinct tile among the wave's lanes (one or two once the points are grouped):
  // the wave loads that tile's candidates 64 at a time, one per lane, and broadcasts each to
  // every lane with readlane; the lanes of that tile rank it.  Each lane also bounds its
  // candidate's q from below over the whole tile (every point of the tile lies in it), and the
  // wave visits the 64 in ascending buckets of that bound, skipping a candidate whose bound
  // exceeds the largest K-th key of the tile's lanes (it cannot enter any of their lists) and
  // stopping once a bucket's floor does; the lists are those of ranking every candidate.
  const int lane = threadIdx.x & 63;
  float res[NC];  // the point's colour (0 outside the image)
#pragma unroll
  for (int ch = 0; ch < NC; ++ch) res[ch] = 0.f;
  uint64_t todo = __ballot(tile >= 0);
  while (todo) {
    const int tc = __builtin_amdgcn_readlane(tile, __ffsll((unsigned long long)todo) - 1);
    const int2 rg = ranges[tc];
    const int ustart = __builtin_amdgcn_readfirstlane(rg.x);
    const int ucnt = __builtin_amdgcn_readfirstlane(rg.y - rg.x);
    const bool mine = tile == tc;
    const float rx0 = (float)((tc % tiles_x) * kTile), ry0 = (float)((tc / tiles_x) * kTile);
    for (int b0 = 0; b0 < ucnt; b0 += 64) {
      const int nb = min(64, ucnt - b0);
      float4 a = make_float4(0.f, 0.f, 0.f, 0.f);
      float2 b = make_float2(0.f, 0.f);
      float lb = 0.f;
      if (lane < nb) {
        const uint32_t gid = vals[ustart + b0 + lane];
        if (REC) {
          const float *__restrict__ r = rec + (size_t)gid * RS;
          a = *reinterpret_cast<const float4 *>(r);
          b = *reinterpret_cast<const float2 *>(r + 4);
          if (ucnt <= QS) {
#pragma unroll
            for (int ch = 0; ch < NC; ++ch)
              if (ch < n) scol[(b0 + lane) * NC + ch] = r[16 + ch];
          }
        } else {
          a = g32a[gid];
          b = g32b[gid];
          if (ucnt <= QS) {
#pragma unroll
            for (int ch = 0; ch < NC; ++ch)
              if (ch < n) scol[(b0 + lane) * NC + ch] = params[(size_t)(5 + ch) * N + gid];
          }
        }
        const float A = a.z, B = a.w, C = b.x, D = b.y;
        const float p11 = fmaf(A, A, C * C), p12 = fmaf(A, B, C * D), p22 = fmaf(B, B, D * D);
        const float r1 = fmaf(A, A, B * B), r2 = fmaf(C, C, D * D);  // 1/s_1^2, 1/s_2^2
        const float kappa =
            sqrtf(fmaxf(r1, r2) * __builtin_amdgcn_rcpf(fminf(r1, r2))) * 1.001f;
        const float i11 = __builtin_amdgcn_rcpf(p11), i22 = __builtin_amdgcn_rcpf(p22);
        const float dxa = rx0 - a.x, dxb = (rx0 + (float)kTile) - a.x;
        const float dya = ry0 - a.y, dyb = (ry0 + (float)kTile) - a.y;
        lb = safe_lb(rect_min_q(A, B, C, D, i11, p12, -p12 * dxa * i22, -p12 * dxb * i22, dxa,
                                dxb, dya, dyb),
                     kappa);
      }
      const int bk = lb_bucket(lb);
      const uint64_t live = nb == 64 ? ~0ull : ((1ull << nb) - 1ull);
      for (int bb = 0; bb < kBuckets; ++bb) {
        uint64_t set = __ballot(bk == bb) & live;
        if (!set) continue;
        // the largest K-th key among the tile's lanes (the lists only shrink: a stale value is
        // safe); every bound in this bucket and the later ones is at least its floor
        float q_tau = __uint_as_float(
            wave_max_u32(mine ? (uint32_t)__double2hiint(tk[KT - 1]) : 0u) - kKeyBias);
        if (bucket_floor(bb) > q_tau) break;
        for (int v = 0; set; ++v) {
          const int k = __ffsll((unsigned long long)set) - 1;
          set &= set - 1;
          if ((v & 7) == 7)
            q_tau = __uint_as_float(
                wave_max_u32(mine ? (uint32_t)__double2hiint(tk[KT - 1]) : 0u) - kKeyBias);
          if (__int_as_float(__builtin_amdgcn_readlane(__float_as_int(lb), k)) > q_tau) continue;
          const float mx = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(a.x), k));
          const float my = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(a.y), k));
          const float A = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(a.z), k));
          const float B = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(a.w), k));
          const float C = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(b.x), k));
          const float D = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(b.y), k));
          const double key = rank_key(quad_q32(A, B, C, D, fx - mx, fy - my), b0 + k);
          if (mine && key < tk[KT - 1]) topk_insert<KT>(tk, key);
        }
      }
    }
    // the blend of the tile's lanes: the winners re-evaluated in double, weights relative to the
    // best, colours summed in rank order (from the staged rows when the tile has them)
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    if (mine) {
      const int keff = min(K, cnt);
      float w[KT];
      uint32_t src[KT];
      int slot[KT];
      float Z = 0.f, shift = 0.f;
#pragma unroll
      for (int k = 0; k < KT; ++k) {
        w[k] = 0.f;
        src[k] = 0;
        slot[k] = 0;
        if (k < keff && key_valid(tk[k])) {
          slot[k] = key_slot(tk[k]);
          const uint32_t gid = vals[start + slot[k]];
          const double4 c = REC ? *reinterpret_cast<const double4 *>(rec + (size_t)gid * RS + 8)
                                : g64[gid];
          const float4 ga = REC ? *reinterpret_cast<const float4 *>(rec + (size_t)gid * RS)
                                : g32a[gid];
          double e1, e2;
          const double q = quad_form64(fx, fy, ga.x, ga.y, c.x, c.y, c.z, c.w, e1, e2);
          if (k == 0) shift = (float)q;
          w[k] = blend_weight(q, shift);
          Z += w[k];
          src[k] = gid;
        }
      }
      const float invZ = Z > 0.f ? 1.0f / Z : 0.0f;
      float acc[NC];
#pragma unroll
      for (int ch = 0; ch < NC; ++ch) acc[ch] = 0.f;
      // LDS and global colour reads stay in separate loops (a read through a pointer that may
      // address either miscompiles for gfx950)
      if (ucnt <= QS) {
#pragma unroll
        for (int k = 0; k < KT; ++k) {
          if (k < keff && key_valid(tk[k])) {
#pragma unroll
            for (int ch = 0; ch < NC; ++ch)
              if (ch < n) acc[ch] = fmaf(w[k], scol[slot[k] * NC + ch], acc[ch]);
          }
        }
      } else {
#pragma unroll
        for (int k = 0; k < KT; ++k) {
          if (k < keff && key_valid(tk[k])) {
#pragma unroll
            for (int ch = 0; ch < NC; ++ch)
              if (ch < n)
                acc[ch] = fmaf(w[k],
                               REC ? rec[(size_t)src[k] * RS + 16 + ch]
                                   : params[(size_t)(5 + ch) * N + src[k]],
                               acc[ch]);
          }
        }
      }
#pragma unroll
      for (int ch = 0; ch < NC; ++ch) res[ch] = acc[ch] * invZ;
    }
    // the staged rows are read before the next tile's are written
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    todo &= ~__ballot(mine);
  }
  if (!valid) return;
  float *__restrict__ o = out + (size_t)i * n;
#pragma unroll
  for (int ch = 0; ch < NC; ++ch)
    if (ch < n) o[ch] = res[ch];
}
__global__ __launch_bounds__(256) void to_fp16_kernel(const float *__restrict__ src, int64_t count,
                                                      uint16_t *__restrict__ dst) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = __half_as_ushort(__float2half_rn(src[i]));
}

// Stored float16 fitter parameters [5+n][N_src] -> float32 renderer parameters [5+n][N_prefix]
// of the first N_prefix Gaussians: mean x W and x H, rotation, scale = 1 / inverse scale, colour
// (the conversions igs_adam_step applies after each update).
__global__ __launch_bounds__(256) void decode_fp16_kernel(const uint16_t *__restrict__ src,
                                                          int N_src, int N_prefix, float W,
                                                          float H, float *__restrict__ dst) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const int r = blockIdx.y;
  if (j >= N_prefix) return;
  const float p = __half2float(__ushort_as_half(src[(size_t)r * N_src + j]));
  float v = p;
  if (r == 0) v = p * W;
  else if (r == 1) v = p * H;
  else if (r == 3 || r == 4) v = 1.0f / p;
  dst[(size_t)r * N_prefix + j] = v;
}

}  // namespace

namespace {
template <int NC>
hipError_t launch_query_nc(const float *params, int N, int n, int H, int W, int K, int tiles_x,
                           int tiles_y, const int2 *ranges, const uint32_t *vals,
                           const float4 *g32a, const float2 *g32b, const double4 *g64,
                           const float *rec, const float *points, int M, const uint32_t *order,
                           float *out, int grid, hipStream_t s) {
  switch (pick_kt(K)) {
#define IGS_QUERY_CASE(KT)                                                                     \
  case KT:                                                                                     \
    if (rec)                                                                                   \
      query_kernel<NC, KT, true><<<grid, kQueryThreads, query_lds_bytes<NC>(), s>>>(          \
          params, N, n, H, W, K, tiles_x, tiles_y, ranges, vals, g32a, g32b, g64, rec, points, \
          M, order, out);                                                                      \
    else                                                                                       \
      query_kernel<NC, KT, false><<<grid, kQueryThreads, query_lds_bytes<NC>(), s>>>(         \
          params, N, n, H, W, K, tiles_x, tiles_y, ranges, vals, g32a, g32b, g64, rec, points, \
          M, order, out);                                                                      \
    break;
    IGS_FOR_EACH_KT(IGS_QUERY_CASE)
#undef IGS_QUERY_CASE
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

struct QueryWs {
  size_t keys, vals, keys_alt, vals_alt, hist, hist_off, scan_tmp, count, rec, total;
  int key_bits, passes, digit_bits;
  int64_t nblocks;
};

QueryWs query_ws(int64_t M, int N, int n, int H, int W) {
  const int64_t T = (int64_t)((W + kTile - 1) / kTile) * ((H + kTile - 1) / kTile);
  QueryWs L{};
  L.key_bits = 1;
  while ((int64_t)1 << L.key_bits <= T) ++L.key_bits;  // keys 0..T
  L.passes = (L.key_bits + 7) / 8;
  L.digit_bits = (L.key_bits + L.passes - 1) / L.passes;
  L.nblocks = (std::max<int64_t>(M, 1) + kSortTileItems - 1) / kSortTileItems;
  const size_t arr = align_up((size_t)std::max<int64_t>(M, 1) * sizeof(uint32_t));
  const int64_t hist_elems = ((int64_t)1 << L.digit_bits) * L.nblocks;
  size_t o = 0;
  L.keys = o;
  o += arr;
  L.vals = o;
  o += arr;
  L.keys_alt = o;
  o += arr;
  L.vals_alt = o;
  o += arr;
  L.hist = o;
  o += align_up((size_t)hist_elems * sizeof(uint32_t));
  L.hist_off = o;
  o += align_up((size_t)hist_elems * sizeof(uint32_t));
  L.scan_tmp = o;
  o += align_up(scan_temp_elems(hist_elems) * sizeof(uint32_t));
  L.count = o;
  o += align_up(sizeof(int64_t));
  L.rec = o;
  o += align_up((size_t)std::max(N, 0) * query_rec_stride(n) * sizeof(float));
  L.total = o;
  return L;
}
}  // namespace

size_t query_workspace_bytes(int64_t M, int N, int n, int H, int W) {
  return query_ws(M, N, n, H, W).total;
}

hipError_t launch_query(const float *params, int N, int n, int H, int W, int K,
                        const int2 *ranges, const uint32_t *vals, const float4 *g32a,
                        const float2 *g32b, const double4 *g64, const float *points, int M,
                        float *out, void *ws, hipStream_t s) {
  if (M <= 0) return hipSuccess;
  const int tiles_x = (W + kTile - 1) / kTile, tiles_y = (H + kTile - 1) / kTile;
  const int grid = (M + kQueryThreads - 1) / kQueryThreads;
  const uint32_t *order = nullptr;
  const float *rec = nullptr;
  if (ws) {
    const QueryWs L = query_ws(M, N, n, H, W);
    char *b = static_cast<char *>(ws);
    uint32_t *keys = reinterpret_cast<uint32_t *>(b + L.keys);
    uint32_t *vs = reinterpret_cast<uint32_t *>(b + L.vals);
    uint32_t *keys_alt = reinterpret_cast<uint32_t *>(b + L.keys_alt);
    uint32_t *vals_alt = reinterpret_cast<uint32_t *>(b + L.vals_alt);
    int64_t *count = reinterpret_cast<int64_t *>(b + L.count);
    const bool alt = sort_starts_in_alt(L.passes);
    query_keys_kernel<<<grid, kQueryThreads, 0, s>>>(points, M, H, W, tiles_x, tiles_y,
                                                     alt ? keys_alt : keys, count);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = radix_sort_pairs(keys, vs, keys_alt, vals_alt, count, M, L.key_bits, L.passes,
                         L.digit_bits, reinterpret_cast<uint32_t *>(b + L.hist),
                         reinterpret_cast<uint32_t *>(b + L.hist_off),
                         reinterpret_cast<uint32_t *>(b + L.scan_tmp), s, false, true);
    if (e != hipSuccess) return e;
    order = vs;
    if (N > 0) {
      float *r = reinterpret_cast<float *>(b + L.rec);
      const int64_t nv = (int64_t)N * (query_rec_stride(n) / 4);
      query_records_kernel<<<(unsigned)((nv + 255) / 256), 256, 0, s>>>(g32a, g32b, g64, params,
                                                                         N, n, r);
      e = hipGetLastError();
      if (e != hipSuccess) return e;
      rec = r;
    }
  }
  if (n <= 4) return launch_query_nc<4>(params, N, n, H, W, K, tiles_x, tiles_y, ranges, vals,
                                         g32a, g32b, g64, rec, points, M, order, out, grid, s);
  if (n <= 9) return launch_query_nc<9>(params, N, n, H, W, K, tiles_x, tiles_y, ranges, vals,
                                         g32a, g32b, g64, rec, points, M, order, out, grid, s);
  if (n <= 16) return launch_query_nc<16>(params, N, n, H, W, K, tiles_x, tiles_y, ranges, vals,
                                           g32a, g32b, g64, rec, points, M, order, out, grid, s);
  return launch_query_nc<32>(params, N, n, H, W, K, tiles_x, tiles_y, ranges, vals, g32a, g32b,
                             g64, rec, points, M, order, out, grid, s);
}

hipError_t launch_to_fp16(const float *src, int64_t count, uint16_t *dst, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  const int grid = (int)std::min<int64_t>((count + 255) / 256, 4096);
  to_fp16_kernel<<<grid, 256, 0, s>>>(src, count, dst);
  return hipGetLastError();
}

hipError_t launch_decode_fp16(const uint16_t *src, int N_src, int n, int N_prefix, int H, int W,
                              float *dst, hipStream_t s) {
  if (N_prefix <= 0) return hipSuccess;
  const dim3 grid((N_prefix + 255) / 256, 5 + n);
  decode_fp16_kernel<<<grid, 256, 0, s>>>(src, N_src, N_prefix, (float)W, (float)H, dst);
  return hipGetLastError();
}

}  // namespace igs
