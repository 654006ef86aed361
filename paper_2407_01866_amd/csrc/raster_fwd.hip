// Forward rasterizer (Image-GS Sec. 3.2, Eq. 5): one workgroup per 16 x 16 tile, one lane per
// pixel.  The tile's hit set S_j is staged through LDS in batches of 256 Gaussians; every lane
// ranks every member by its float32 Mahalanobis form q and keeps a register-resident sorted top-K
// of (q, slot), slot being the member's position in S_j, so that equal q rank the lower Gaussian
// index first.  The K winners are then re-evaluated in double so that the normalized blend weights
// exp(-(q_i - q_min)/2) carry no float32 cancellation error.
//
// Ranking key: the pair (q, slot) packed as the bit pattern of a positive double, high word =
// float bits of q plus one exponent step (keeps the double normal when q = 0), low word = slot.
// For non-negative floats the bit pattern orders like the value, and so does a positive double's,
// so comparing the doubles compares (q, slot) lexicographically; every position of the sorted
// insertion is then one v_max_f64 and one v_min_f64 (full rate on this GPU), and the result does not
// depend on the order in which candidates arrive.  This file is built with -fno-honor-nans so the
// min/max are not wrapped in NaN-quieting instructions; q is clamped below 1e38 before packing so a
// non-finite value can only rank last.
//
// Candidate order and wave-level culling.  Because the keys are unique, any processing order gives
// the same lists, so each batch is visited in ascending order of a lower bound of q over the tile
// (16 coarse buckets of a counting sort).  Each wave (16 x 4 pixels) also has, per candidate, a
// lower bound of the float32 q over its own pixel rectangle, shrunk by a margin that covers float32
// evaluation error; a candidate whose bound exceeds the largest K-th key of the wave's lanes cannot
// enter any of their lists and is skipped by the whole wave, and once the bucket floor exceeds it
// the wave stops.  Winners come early in this order, so most of the tail is skipped.
#include "raster_common.hpp"

namespace igs {
namespace {

// Candidates staged in LDS per batch: 192 keeps the kernel's LDS (124 B per candidate for n = 9)
// small enough for six workgroups per CU, the occupancy its registers allow.
constexpr int kFwdBatch = 192;
// LDS bytes before the colour rows: per candidate 48 B of ranking data in visiting order and 40 B
// of blend geometry in slot order, then the bucket counters.
constexpr unsigned kFwdLdsFixed = 88 * kFwdBatch + 2 * 16 * 4;
constexpr int kBuckets = 16;
constexpr int kWaves = kRasterThreads / 64;  // each wave covers 4 rows of the tile

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

// A lower bound of the float32 q that the ranking evaluates at any pixel centre of the
// rectangle: the minimum over the rectangle, itself evaluated in float32 (relative error below
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

// Fused L1 epilogue (L1 = true): besides the image, each pixel compares its colour with the
// target, d = c_r - c_t per channel (in double, exact), and keeps what the adjoint of the mean
// absolute error needs: the sign of every d as a 2-bit code (01 = +, 11 = -, 00 = 0) and
// g . c_r with g = sign(d) / (n H W), evaluated exactly as the adjoint would evaluate it from an
// explicit gradient image.  The tile's sums of |d| and d^2 go to loss_part[tile].
struct L1Out {
  const float *target;  // [n][H][W] per image, concatenated like the images
  float2 *rec;          // per pixel: (g . c_r, sign codes)
  double2 *part;        // per tile: (sum |d|, sum d^2)
};

__device__ __forceinline__ double2 block_sum2(double a, double b, double *sh,
                                              int nwaves = kRasterThreads / 64) {
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
  double2 t = make_double2(0.0, 0.0);
  if (threadIdx.x == 0)
    for (int k = 0; k < nwaves; ++k) {
      t.x += sh[2 * k];
      t.y += sh[2 * k + 1];
    }
  return t;  // valid in thread 0
}

// Register budget: six waves per SIMD (<= 80 VGPRs) for lists of up to 10 keys; five with the
// fused L1 epilogue at 8 and 10 keys, where 80 registers would spill.
__host__ __device__ constexpr int fwd_min_waves(int kt, bool l1, bool p) {
  return kt <= 10 ? ((p && kt >= 8) ? 5 : 6) : (kt <= 16 ? 4 : 2);
}

// P: persistent scheduling (a compile-time choice so that the one-workgroup-per-tile kernel keeps
// the register budget of straight-line code).
template <int KT, bool L1, bool P>
__global__ __launch_bounds__(kRasterThreads)
__attribute__((amdgpu_waves_per_eu(fwd_min_waves(KT, L1, P)))) void raster_fwd_kernel(
    const int2 *__restrict__ ranges, const uint32_t *__restrict__ vals,
    const float4 *__restrict__ g32a, const float2 *__restrict__ g32b,
    const double4 *__restrict__ g64, const float *__restrict__ params, int N, int n, int K, int T,
    Images imgs, const int *__restrict__ tile_order, float *__restrict__ image_all,
    uint16_t *__restrict__ slots_all, float2 *__restrict__ aux_all, L1Out l1, TileQueue queue,
    int cull) {
  extern __shared__ __align__(16) unsigned char smem[];
  // ranking data in visiting order (position m of the batch's candidate order)
  float4 *s_pgeo = reinterpret_cast<float4 *>(smem);                  // mu_x, mu_y, A, B
  float4 *s_pcd = reinterpret_cast<float4 *>(smem + 16 * kFwdBatch);     // C, D, slot, bucket floor
  float *s_plbw = reinterpret_cast<float *>(smem + 32 * kFwdBatch);      // [kWaves][kFwdBatch] bounds
  // blend data in slot order (position j in S_j minus the batch base)
  float2 *s_mu = reinterpret_cast<float2 *>(smem + 48 * kFwdBatch);      // mu_x, mu_y
  double *s64 = reinterpret_cast<double *>(smem + 56 * kFwdBatch);       // [kFwdBatch][4] A,B,C,D
  int *s_bcnt = reinterpret_cast<int *>(smem + 88 * kFwdBatch);          // [kBuckets] counters
  int *s_bstart = s_bcnt + kBuckets;                                  // [kBuckets] starts
  float *s_col = reinterpret_cast<float *>(smem + kFwdLdsFixed);      // [kFwdBatch][n]
  const int ncp = n;

  const int tid = threadIdx.x;
  int idx = 0;
  if (!P) queue.persistent = 0;
  for (bool first = true; next_tile_index(queue, T, first, idx); first = false) {
  const int tile = __builtin_amdgcn_readfirstlane(tile_order ? tile_order[idx] : xcd_tile(idx, T));
  const ImageDesc im = imgs.by_tile(tile);
  const int W = im.W, H = im.H;
  const int64_t HW = (int64_t)H * W;
  float *__restrict__ image = image_all + (int64_t)n * im.pix_off;
  uint16_t *__restrict__ slots = slots_all + (int64_t)K * im.pix_off;
  float2 *__restrict__ aux = aux_all + im.pix_off;
  const int lt = tile - im.tile_off;
  const int tx = lt % im.tiles_x, ty = lt / im.tiles_x;
  const int px = tx * kTile + (tid & (kTile - 1)), py = ty * kTile + tid / kTile;
  const bool inside = px < W && py < H;
  const float fx = (float)px + 0.5f, fy = (float)py + 0.5f;
  const int2 rg = ranges[tile];
  // uniform over the workgroup; readfirstlane keeps the loop bounds in scalar registers
  const int start = __builtin_amdgcn_readfirstlane(rg.x);
  const int cnt = __builtin_amdgcn_readfirstlane(rg.y - rg.x);
  const bool single = cnt <= kFwdBatch;  // whole S_j stays resident for the blend

  double tk[KT];
#pragma unroll
  for (int k = 0; k < KT; ++k) tk[k] = kKeyEmpty;

  const int wave = tid >> 6;
  if (tid < kBuckets) s_bcnt[tid] = 0;
  for (int base = 0; base < cnt; base += kFwdBatch) {
    const int nb = min(kFwdBatch, cnt - base);
    __syncthreads();
    int bucket = 0, brank = 0;
    float4 a = make_float4(0.f, 0.f, 0.f, 0.f);
    float2 b = make_float2(0.f, 0.f);
    float lbw[kWaves];
    if (tid < nb) {
      const uint32_t gid = vals[start + base + tid];
      a = g32a[gid];
      b = g32b[gid];
      if (single) {
        s_mu[tid] = make_float2(a.x, a.y);
        const double4 c = g64[gid];
        s64[4 * tid + 0] = c.x;
        s64[4 * tid + 1] = c.y;
        s64[4 * tid + 2] = c.z;
        s64[4 * tid + 3] = c.w;
        for (int ch = 0; ch < n; ++ch) s_col[tid * ncp + ch] = params[(size_t)(5 + ch) * N + gid];
      }
      // lower bounds of q over each wave's pixel-centre rectangle (16 x 4 centres); without
      // culling every bound is 0 (nothing is skipped) and the order is the slot order
      float tile_lb = 0.f;
#pragma unroll
      for (int w = 0; w < kWaves; ++w) lbw[w] = 0.f;
      if (cull) {
      const float A = a.z, B = a.w, C = b.x, D = b.y;
      const float p11 = fmaf(A, A, C * C), p12 = fmaf(A, B, C * D), p22 = fmaf(B, B, D * D);
      const float r1 = fmaf(A, A, B * B), r2 = fmaf(C, C, D * D);  // 1/s_1^2, 1/s_2^2
      const float kappa = sqrtf(fmaxf(r1, r2) / fminf(r1, r2)) * 1.001f;
      const float i11 = 1.0f / p11, i22 = 1.0f / p22;
      const float dxa = ((float)(tx * kTile) + 0.5f) - a.x;
      const float dxb = ((float)(tx * kTile + kTile - 1) + 0.5f) - a.x;
      const float tya = -p12 * dxa * i22, tyb = -p12 * dxb * i22;
      tile_lb = 3.0e38f;
#pragma unroll
      for (int w = 0; w < kWaves; ++w) {
        const float dya = ((float)(ty * kTile + 4 * w) + 0.5f) - a.y;
        const float dyb = ((float)(ty * kTile + 4 * w + 3) + 0.5f) - a.y;
        lbw[w] = safe_lb(rect_min_q(A, B, C, D, i11, p12, tya, tyb, dxa, dxb, dya, dyb), kappa);
        tile_lb = fminf(tile_lb, lbw[w]);
      }
      }
      bucket = lb_bucket(tile_lb);
      brank = atomicAdd(&s_bcnt[bucket], 1);
    }
    __syncthreads();
    if (tid < 64) {  // bucket starts: exclusive scan of the counters (one wave)
      const int c = tid < kBuckets ? s_bcnt[tid] : 0;
      int inc = c;
#pragma unroll
      for (int d = 1; d < kBuckets; d <<= 1) {
        const int o = __shfl_up(inc, d, 64);
        if (tid >= d) inc += o;
      }
      if (tid < kBuckets) s_bstart[tid] = inc - c;
    }
    __syncthreads();
    if (tid < nb) {  // scatter the ranking data into visiting order
      const int pos = s_bstart[bucket] + brank;
      s_pgeo[pos] = a;
      s_pcd[pos] = make_float4(b.x, b.y, __int_as_float(base + tid), bucket_floor(bucket));
#pragma unroll
      for (int w = 0; w < kWaves; ++w) s_plbw[w * kFwdBatch + pos] = lbw[w];
    }
    if (tid < kBuckets) s_bcnt[tid] = 0;  // ready for the next batch
    __syncthreads();
    // four positions per step; the skip decisions are wave-uniform (scalar branches)
    for (int m = 0; m < nb; m += 4) {
      // the largest K-th key of the wave (the lists only shrink, so a stale value is safe)
      const uint32_t th = wave_max_u32((uint32_t)__double2hiint(tk[KT - 1]));
      const float q_tau = __uint_as_float(th - kKeyBias);
      // every later candidate's bound is at least the floor of this position's bucket
      if (__int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(s_pcd[m].w))) > q_tau)
        break;
      const float4 lb4 = *reinterpret_cast<const float4 *>(&s_plbw[wave * kFwdBatch + m]);
      const float lbu[4] = {lb4.x, lb4.y, lb4.z, lb4.w};
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        if (m + u >= nb) break;
        if (__int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(lbu[u]))) > q_tau)
          continue;
        const float4 g = s_pgeo[m + u];
        const float4 cd = s_pcd[m + u];
        const float dx = fx - g.x, dy = fy - g.y;
        const float e1 = fmaf(g.z, dx, g.w * dy);
        const float e2 = fmaf(cd.x, dx, cd.y * dy);
        const double key = rank_key(fmaf(e1, e1, e2 * e2), __float_as_int(cd.z));
        if (key < tk[KT - 1]) topk_insert<KT>(tk, key);
      }
    }
  }

  double l1_abs = 0.0, l1_sq = 0.0;
  if (inside) {
  const int64_t pix = (int64_t)py * W + px;
  // the target of the first channel, loaded now so that it arrives during the blend
  const float *__restrict__ target = L1 ? l1.target + (int64_t)n * im.pix_off + pix : nullptr;
  float tnext = 0.f;
  if constexpr (L1) tnext = target[0];
  const int keff = min(K, cnt);
  int ts[KT];
#pragma unroll
  for (int k = 0; k < KT; ++k) ts[k] = key_valid(tk[k]) ? key_slot(tk[k]) : -1;
  float w[KT];
  int src[KT];
  float Z = 0.f, shift = 0.f;
#pragma unroll
  for (int k = 0; k < KT; ++k) {
    w[k] = 0.f;
    src[k] = 0;
    if (k < keff && ts[k] >= 0) {  // a non-finite q never enters the list
      const int slot = ts[k];
      double A, B, C, D;
      float mx, my;
      if (single) {
        A = s64[4 * slot + 0];
        B = s64[4 * slot + 1];
        C = s64[4 * slot + 2];
        D = s64[4 * slot + 3];
        mx = s_mu[slot].x;
        my = s_mu[slot].y;
        src[k] = slot;
        // keeps these LDS loads and the global loads below in their own branches (merging them
        // into loads through a pointer that is LDS or global miscompiles for gfx950)
        asm volatile("" ::: "memory");
      } else {
        const uint32_t gid = vals[start + slot];
        const double4 c = g64[gid];
        const float4 a = g32a[gid];
        A = c.x;
        B = c.y;
        C = c.z;
        D = c.w;
        mx = a.x;
        my = a.y;
        src[k] = (int)gid;
        asm volatile("" ::: "memory");
      }
      double e1, e2;
      const double q = quad_form64(fx, fy, mx, my, A, B, C, D, e1, e2);
      if (k == 0) shift = (float)q;
      w[k] = blend_weight(q, shift);
      Z += w[k];
    }
  }
  if constexpr (!P) {
  const float invZ = Z > 0.f ? 1.0f / Z : 0.0f;
  const float inv_count = L1 ? (float)(1.0 / ((double)n * (double)HW)) : 0.f;
  float gc = 0.f;
  uint32_t codes = 0;
  // finishes channel ch of the pixel: the normalized colour, and with the L1 epilogue the sign of
  // d = c_r - c_t, g . c_r and the loss sums, in channel order
  auto finish = [&](int ch, float acc, float t) {
    const float v = acc * invZ;
    image[(int64_t)ch * HW + pix] = v;
    if constexpr (L1) {
      const double d = (double)v - (double)t;
      const float g = d > 0.0 ? inv_count : (d < 0.0 ? -inv_count : 0.f);
      codes |= (d > 0.0 ? 1u : (d < 0.0 ? 3u : 0u)) << (2 * ch);
      gc = fmaf(g, v, gc);
      l1_abs += fabs(d);
      l1_sq += d * d;
    }
  };
  // channel-major: every channel sums its retained Gaussians in rank order; with the L1
  // epilogue the next channel's target is loaded one channel ahead
  float tcur = tnext;
  for (int ch = 0; ch < n; ++ch) {
    float acc = 0.f;
#pragma unroll
    for (int k = 0; k < KT; ++k) {
      if (k < keff && ts[k] >= 0) {
        const float c = single ? s_col[src[k] * ncp + ch] : params[(size_t)(5 + ch) * N + src[k]];
        acc = fmaf(w[k], c, acc);
      }
    }
    if constexpr (L1) {
      if (ch + 1 < n) tnext = target[(int64_t)(ch + 1) * HW];
    }
    finish(ch, acc, tcur);
    tcur = tnext;
  }
  if constexpr (L1) l1.rec[im.pix_off + pix] = make_float2(gc, __uint_as_float(codes));
#pragma unroll
  for (int k = 0; k < KT; ++k)
    if (k < K)
      slots[(int64_t)k * HW + pix] = (k < keff && ts[k] >= 0) ? (uint16_t)min(ts[k], 0xFFFF) : kEmptySlot;
  aux[pix] = make_float2(shift, invZ);
  } else {
  const float invZ = Z > 0.f ? 1.0f / Z : 0.0f;
  const float inv_count = L1 ? (float)(1.0 / ((double)n * (double)HW)) : 0.f;
  float gc = 0.f;
  uint32_t codes = 0;
#pragma unroll
  for (int k = 0; k < KT; ++k)
    if (k < K)
      slots[(int64_t)k * HW + pix] = (k < keff && ts[k] >= 0) ? (uint16_t)min(ts[k], 0xFFFF) : kEmptySlot;
  aux[pix] = make_float2(shift, invZ);
  // channel-major: every channel sums its retained Gaussians in rank order, then stores the
  // normalized colour; with the L1 epilogue also the sign of d = c_r - c_t, g . c_r and the loss
  // sums, in channel order, the next channel's target being loaded one channel ahead.  Entries
  // past the retained ones have weight 0 and index 0 (a valid member when cnt > 0), so they add
  // exactly 0 and the sums need no branches.  The LDS and global colour reads stay in separate
  // loops (a read through a pointer that may be either miscompiles for gfx950).
  float tcur = tnext;
  auto finish = [&](int ch, float acc) {
    if constexpr (L1) {
      if (ch + 1 < n) tnext = target[(int64_t)(ch + 1) * HW];
    }
    const float v = acc * invZ;
    image[(int64_t)ch * HW + pix] = v;
    if constexpr (L1) {
      const double d = (double)v - (double)tcur;
      const float g = d > 0.0 ? inv_count : (d < 0.0 ? -inv_count : 0.f);
      codes |= (d > 0.0 ? 1u : (d < 0.0 ? 3u : 0u)) << (2 * ch);
      gc = fmaf(g, v, gc);
      l1_abs += fabs(d);
      l1_sq += d * d;
    }
    tcur = tnext;
  };
  if (cnt == 0) {
    for (int ch = 0; ch < n; ++ch) finish(ch, 0.f);
  } else if (single) {
    for (int ch = 0; ch < n; ++ch) {
      float acc = 0.f;
#pragma unroll
      for (int k = 0; k < KT; ++k) acc = fmaf(w[k], s_col[src[k] * ncp + ch], acc);
      finish(ch, acc);
    }
  } else {
    for (int ch = 0; ch < n; ++ch) {
      float acc = 0.f;
#pragma unroll
      for (int k = 0; k < KT; ++k) acc = fmaf(w[k], params[(size_t)(5 + ch) * N + src[k]], acc);
      finish(ch, acc);
    }
  }
  if constexpr (L1) l1.rec[im.pix_off + pix] = make_float2(gc, __uint_as_float(codes));
  }
  }
  if (L1) {
    // the tile's loss sums: wave sums by shuffles, then a fixed order over the four waves
    __shared__ double s_red[2 * kWaves];
    double a = l1_abs, b = l1_sq;
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
      a += __shfl_down(a, d, 64);
      b += __shfl_down(b, d, 64);
    }
    if ((tid & 63) == 0) {
      s_red[2 * wave] = a;
      s_red[2 * wave + 1] = b;
    }
    __syncthreads();
    if (tid == 0) {
      double2 t = make_double2(0.0, 0.0);
      for (int k = 0; k < kWaves; ++k) {
        t.x += s_red[2 * k];
        t.y += s_red[2 * k + 1];
      }
      l1.part[tile] = t;
    }
  }
  __syncthreads();  // LDS is reused by the next tile
  }
}

// Per image: mean |d| and mean d^2 from the per-tile sums of its tiles (fixed order: thread t
// adds tiles t, t + 1024, ... in sequence, then a fixed tree over the threads).
constexpr int kFinalThreads = 1024;

__global__ __launch_bounds__(kFinalThreads) void l1_tiles_final_kernel(
    const double2 *__restrict__ part, Images imgs, int n, double *__restrict__ out) {
  __shared__ double sh[2 * kFinalThreads / 64];
  const ImageDesc im = imgs.at(blockIdx.x);
  const int T = im.tiles_x * im.tiles_y;
  double a = 0.0, b = 0.0;
  int t = threadIdx.x;
  for (; t + 3 * kFinalThreads < T; t += 4 * kFinalThreads) {  // four loads in flight
    double2 v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) v[u] = part[im.tile_off + t + u * kFinalThreads];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      a += v[u].x;
      b += v[u].y;
    }
  }
  for (; t < T; t += kFinalThreads) {
    const double2 v = part[im.tile_off + t];
    a += v.x;
    b += v.y;
  }
  const double2 s = block_sum2(a, b, sh, kFinalThreads / 64);
  if (threadIdx.x == 0) {
    const double inv = 1.0 / ((double)n * (double)im.H * (double)im.W);
    out[2 * blockIdx.x] = s.x * inv;
    out[2 * blockIdx.x + 1] = s.y * inv;
  }
}

template <int KT, bool L1, bool P>
hipError_t launch_fwd_t(const int2 *ranges, const uint32_t *vals, const float4 *g32a,
                        const float2 *g32b, const double4 *g64, const float *params,
                        const Dims &d, const Images &imgs, const int *tile_order, float *image,
                        uint16_t *slots, float2 *aux, const L1Out &l1, int *queue,
                        hipStream_t s) {
  const size_t lds = kFwdLdsFixed + (size_t)d.n * kFwdBatch * sizeof(float);
  const LaunchConfig cfg = launch_config();
  TileQueue q{queue, 0};
  int grid = d.T;
  if (P) {
    int per_cu = cfg.wgs_per_cu;
    if (per_cu <= 0) {
      hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
          &per_cu, (const void *)raster_fwd_kernel<KT, L1, P>, kRasterThreads, lds);
      if (e != hipSuccess) return e;
    }
    grid = persistent_grid(per_cu, d.T);
    q.persistent = 1;
    hipError_t e = launch_fill_u32(reinterpret_cast<uint32_t *>(queue), 8, 0u, s);
    if (e != hipSuccess) return e;
  }
  raster_fwd_kernel<KT, L1, P><<<grid, kRasterThreads, lds, s>>>(
      ranges, vals, g32a, g32b, g64, params, d.N, d.n, d.K, d.T, imgs, tile_order, image, slots,
      aux, l1, q, cfg.fwd_cull);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_raster_fwd(const int2 *ranges, const uint32_t *vals, const float4 *g32a,
                             const float2 *g32b, const double4 *g64, const float *params,
                             const Dims &d, const Images &imgs, const int *tile_order,
                             float *image, uint16_t *slots, float2 *aux, const float *target,
                             float2 *l1_rec, double2 *l1_part, int *queue, hipStream_t s) {
  const int kt = pick_kt(d.K);
  const L1Out l1{target, l1_rec, l1_part};
  const bool fused = target != nullptr;
  const bool pers = launch_config().persistent != 0;
#define IGS_FWD_CALL(KTV, L1V, PV)                                                             \
  return launch_fwd_t<KTV, L1V, PV>(ranges, vals, g32a, g32b, g64, params, d, imgs, tile_order, \
                                    image, slots, aux, l1, queue, s);
#define IGS_LAUNCH_FWD(KTV)                                                                    \
  if (kt == KTV) {                                                                             \
    if (fused) {                                                                               \
      if (pers) IGS_FWD_CALL(KTV, true, true)                                                  \
      IGS_FWD_CALL(KTV, true, false)                                                           \
    }                                                                                          \
    if (pers) IGS_FWD_CALL(KTV, false, true)                                                   \
    IGS_FWD_CALL(KTV, false, false)                                                            \
  }
  IGS_FOR_EACH_KT(IGS_LAUNCH_FWD)
#undef IGS_LAUNCH_FWD
#undef IGS_FWD_CALL
  return hipErrorInvalidValue;
}

hipError_t launch_l1_tiles_final(const double2 *l1_part, const Images &imgs, int n,
                                 double *loss_out, hipStream_t s) {
  l1_tiles_final_kernel<<<imgs.B, kFinalThreads, 0, s>>>(l1_part, imgs, n, loss_out);
  return hipGetLastError();
}

}  // namespace igs
