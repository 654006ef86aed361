// Device helpers shared by the forward and adjoint rasterizers.  Both must evaluate the blend
// weights with exactly the same operations so that the adjoint sees the forward's weights.
#pragma once

#include "common.hpp"

namespace igs {

// Mahalanobis form q = |e|^2 (Eq. 1-2) in double, e = (A dx + B dy, C dx + D dy), for a pixel
// centre (fx, fy) and mean (mx, my).  Explicit fma keeps the rounding identical everywhere.
__device__ __forceinline__ double quad_form64(float fx, float fy, float mx, float my, double A,
                                              double B, double C, double D, double &e1,
                                              double &e2) {
  double dx = (double)fx - (double)mx;
  double dy = (double)fy - (double)my;
  e1 = fma(A, dx, B * dy);
  e2 = fma(C, dx, D * dy);
  return fma(e1, e1, e2 * e2);
}

// Ranking key of a candidate at a pixel: the pair (q, slot), slot = its position in S_j, packed
// as the bit pattern of a positive double (high word = float bits of q plus one exponent step,
// low word = slot), so comparing keys compares (q, slot) lexicographically.  q is clamped below
// 1e38, so a non-finite value can only rank last.  kKeyEmpty (+inf) marks an unused list entry.
constexpr uint32_t kKeyBias = 0x00800000u;
constexpr float kQMax = 1e38f;

__device__ __forceinline__ double rank_key(float q, int slot) {
  return __hiloint2double((int)(__float_as_uint(fminf(q, kQMax)) + kKeyBias), slot);
}
__device__ __forceinline__ int key_slot(double k) { return __double2loint(k); }
__device__ __forceinline__ bool key_valid(double k) {
  return (uint32_t)__double2hiint(k) < 0x7F000000u;  // not the +inf sentinel
}
#define kKeyEmpty __longlong_as_double(0x7FF0000000000000ll)

// q = (A dx + B dy)^2 + (C dx + D dy)^2 in float32, as the ranking evaluates it.
__device__ __forceinline__ float quad_q32(float A, float B, float C, float D, float dx, float dy) {
  const float e1 = fmaf(A, dx, B * dy), e2 = fmaf(C, dx, D * dy);
  return fmaf(e1, e1, e2 * e2);
}

// Sorted insertion into a register-resident ascending top-KT list of keys: entry k becomes
// min(old k, max(key, old k-1)), one max and one min per entry with no chain between entries.
template <int KT>
__device__ __forceinline__ void topk_insert(double (&tk)[KT], double key) {
#pragma unroll
  for (int k = KT - 1; k > 0; --k) tk[k] = __builtin_fmin(tk[k], __builtin_fmax(key, tk[k - 1]));
  tk[0] = __builtin_fmin(tk[0], key);
}

// Blend weight exp(-(q - shift)/2) (Eq. 5 scaled by exp(shift/2), which cancels in the ratio),
// as 2^((q - shift) * (-log2(e) / 2)): one multiply and the hardware base-2 exponential.
__device__ __forceinline__ float blend_weight(double q, float shift) {
  return __builtin_amdgcn_exp2f((float)(q - (double)shift) * -0.72134752044448170f);
}

// Candidate culling (the forward rasterizer and the point queries): a lower bound of q over a
// rectangle of evaluation points, and 16 coarse buckets of such bounds for a counting-sort order.
constexpr int kBuckets = 16;

// Minimum of q over the rectangle [dxa, dxb] x [dya, dyb] of offsets from the mean: 0 if the
// rectangle holds the mean, else the least of the four edge minima, each the 1-D minimum of the
// quadratic along the edge (at -p12 dx / p22, resp. -p12 dy / p11) clamped to the edge.  tya, tyb
// are the unclamped minimizers along the edges x = dxa and x = dxb.  In float32 with the same
// factored expression as the ranking, so its error is that of the ranking's q; an inexact
// minimizer changes an edge minimum only in second order.
__device__ __forceinline__ float rect_min_q(float A, float B, float C, float D, float i11,
                                            float p12, float tya, float tyb, float dxa, float dxb,
                                            float dya, float dyb) {
  if (dxa <= 0.f && dxb >= 0.f && dya <= 0.f && dyb >= 0.f) return 0.f;
  float best = quad_q32(A, B, C, D, dxa, fminf(fmaxf(tya, dya), dyb));
  best = fminf(best, quad_q32(A, B, C, D, dxb, fminf(fmaxf(tyb, dya), dyb)));
  best = fminf(best, quad_q32(A, B, C, D, fminf(fmaxf(-p12 * dya * i11, dxa), dxb), dya));
  best = fminf(best, quad_q32(A, B, C, D, fminf(fmaxf(-p12 * dyb * i11, dxa), dxb), dyb));
  return best;
}

// A lower bound of the float32 q that the ranking evaluates at any point of the rectangle: the minimum over the rectangle, itself evaluated in float32 (relative error below
// 16 ulp(1) times the condition number kappa = s_max/s_min, like the ranking's q), shrunk by
// 64 ulp(1) times kappa.  0 (never skip) when the margin reaches 1 or the input is not finite;
// capped at 1e37 so that a lane with fewer than K keys (sentinel threshold) never skips.
__device__ __forceinline__ float safe_lb(float m, float kappa) {
  const float f = 1.0f - 64.0f * 5.9604644775390625e-8f * kappa;
  const float v = m * f;
  if (!(f > 0.f) || !(v >= 0.f)) return 0.f;
  return fminf(v, 1e37f);
}

// Bucket of a lower bound: 0 for 0, 1 for (0, 1/4), then one per octave from 1/4 up to >= 2048.
__device__ __forceinline__ int lb_bucket(float lb) {
  if (!(lb > 0.f)) return 0;
  const int e = (int)((__float_as_uint(lb) >> 23) & 0xFF) - 127;  // floor(log2 lb) for normals
  return 1 + min(max(e + 3, 0), kBuckets - 2);
}
// Smallest value any bound in bucket b can have.
__device__ __forceinline__ float bucket_floor(int b) {
  return b <= 1 ? 0.f : __uint_as_float((uint32_t)(127 + b - 4) << 23);  // 2^(b-4)
}

// Maximum over the 64 lanes of a wave, with DPP row shifts and row broadcasts (no LDS); every
// lane of a row sees the partial maxima of lower lanes, lane 63 the total, which is returned to
// all lanes as a scalar.
__device__ __forceinline__ uint32_t wave_max_u32(uint32_t v) {
  v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xF, 0xF, false));  // shr 1
  v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xF, 0xF, false));  // shr 2
  v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xF, 0xF, false));  // shr 4
  v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xF, 0xF, false));  // shr 8
  v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xA, 0xF, false));  // bcast 15
  v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xC, 0xF, false));  // bcast 31
  return (uint32_t)__builtin_amdgcn_readlane((int)v, 63);
}

// The mean absolute and mean squared differences of one image from its per-tile loss sums
// (sum |d|, sum d^2), in a fixed order: thread t of a kLossThreads block adds tiles t, t + 256,
// ... (eight loads in flight, added in tile order), then a shuffle tree per wave and the waves in
// order.  Every thread of the block calls it (it synchronizes the block); thread 0 writes
// out[0..1].  Shared by the forward's loss pass and the single-pass fit's gradient reduction, so
// both give the same loss bit for bit.
constexpr int kLossThreads = 256;
__device__ __forceinline__ void tile_loss_final(const double2 *__restrict__ part,
                                                const ImageDesc &im, int n, double *out,
                                                double *sh) {
  const int T = im.tiles_x * im.tiles_y;
  double a = 0.0, b = 0.0;
  int t = threadIdx.x;
  for (; t + 7 * kLossThreads < T; t += 8 * kLossThreads) {
    double2 v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = part[im.tile_off + t + u * kLossThreads];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      a += v[u].x;
      b += v[u].y;
    }
  }
  for (; t < T; t += kLossThreads) {
    const double2 v = part[im.tile_off + t];
    a += v.x;
    b += v.y;
  }
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) {
    a += __shfl_down(a, d, 64);
    b += __shfl_down(b, d, 64);
  }
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) {
    sh[2 * w] = a;
    sh[2 * w + 1] = b;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double sa = 0.0, sb = 0.0;
    for (int k = 0; k < kLossThreads / 64; ++k) {
      sa += sh[2 * k];
      sb += sh[2 * k + 1];
    }
    const double inv = 1.0 / ((double)n * (double)im.H * (double)im.W);
    out[0] = sa * inv;
    out[1] = sb * inv;
  }
}

// Kernel variants by top-K capacity: the smallest KT >= K is used (the first K entries of a
// sorted top-KT list are the top-K).
#define IGS_FOR_EACH_KT(X) X(1) X(2) X(4) X(8) X(10) X(16) X(32)

inline int pick_kt(int K) {
  const int kts[] = {1, 2, 4, 8, 10, 16, 32};
  for (int kt : kts)
    if (K <= kt) return kt;
  return -1;
}

// XCD-aware tile order.  Workgroup ids are dealt round-robin to the 8 XCDs, so map the ids an
// XCD receives (bid = x, x+8, x+16, ...) onto one contiguous run of tiles: neighbouring tiles
// share Gaussians, which then stay in that XCD's L2.  A bijection on [0, T): XCD x receives
// q + (x < r) ids (T = 8q + r) and its run starts at x*q + min(x, r).
__device__ __forceinline__ int xcd_tile(int bid, int T) {
  constexpr int kXcd = 8;
  const int q = T / kXcd, r = T % kXcd;
  const int x = bid % kXcd, k = bid / kXcd;
  return x * q + min(x, r) + k;
}

// Tile scheduling of the raster kernels.  Queue index idx names tile xcd_tile(idx, T) (or
// tile_order[idx]).  One workgroup per tile: workgroup b takes index b.  Persistent: a grid of
// resident workgroups, a multiple of 8, where workgroup b (on XCD b % 8 under the round-robin
// dispatch) pulls k = counters[b % 8]++ and takes index 8k + b % 8, i.e. the indices the
// one-per-tile launch would send to the same XCD, in the same order, until they run out.  The
// counters are zeroed before every persistent launch.
struct TileQueue {
  int *counters;  // [8], zero at launch (persistent only)
  int persistent;
};

// Advances to the workgroup's next queue index; false when there is none.  Every thread of the
// workgroup must call it (it synchronizes the workgroup in the persistent mode).
__device__ __forceinline__ bool next_tile_index(const TileQueue &q, int T, bool first, int &idx) {
  __shared__ int s_next;
  if (!q.persistent) {
    idx = blockIdx.x;
    return first && idx < T;
  }
  __syncthreads();  // every thread has read the previous index
  if (threadIdx.x == 0) {
    const int x = blockIdx.x & 7;
    s_next = atomicAdd(&q.counters[x], 1) * 8 + x;
  }
  __syncthreads();
  idx = s_next;
  return idx < T;
}

}  // namespace igs
