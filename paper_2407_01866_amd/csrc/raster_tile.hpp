// Per-tile phases of the rasterizers, shared by the forward (raster_fwd.hip), the adjoint
// (raster_bwd.hip) and the single-pass fitting kernel (raster_fit.hip), which runs the first two
// on one tile in one workgroup.  Everything here is inlined into its kernel.
//
//  * rank_tile: stages the tile's hit set S_j through LDS and leaves every lane with its sorted
//    top-KT (q, slot) keys (Sec. 3.2); winners: re-evaluates the retained members in double and
//    returns their blend weights (Eq. 5).
//  * adjoint_batches: given every pixel's retained slots and its row (dL/dc_r, g . c_r, weight
//    shift, 1/Z) in LDS, writes one gradient record per (tile, Gaussian) pair (Sec. 3.3).
#pragma once

#include "raster_common.hpp"

namespace igs {

// ------------------------------------------------------------------------------- forward side
//
// Candidate order and wave-level culling.  Because the keys are unique, any processing order gives
// the same lists, so each batch is visited in ascending order of a lower bound of q over the tile
// (16 coarse buckets of a counting sort).  Each wave (16 x 4 pixels) also has, per candidate, a
// lower bound of the float32 q over its own pixel rectangle, shrunk by a margin that covers float32
// evaluation error; a candidate whose bound exceeds the largest K-th key of the wave's lanes cannot
// enter any of their lists and is skipped by the whole wave, and once the bucket floor exceeds it
// the wave stops.  Winners come early in this order, so most of the tail is skipped.

// Candidates staged in LDS per batch: fb, a launch setting (default 192, which keeps the
// forward's LDS, 124 B per candidate at n = 9, small enough for six workgroups per CU).  Per
// candidate 48 B of ranking data in visiting order and 40 B of blend geometry in slot order, then
// the bucket counters, then the colour rows.
constexpr int kWaves = kRasterThreads / 64;  // each wave covers 4 rows of the tile

__host__ __device__ constexpr size_t fwd_lds_fixed(int fb) { return 88 * (size_t)fb + 2 * 16 * 4; }
__host__ __device__ constexpr size_t fwd_lds_bytes(int n, int fb) {
  return fwd_lds_fixed(fb) + (size_t)n * fb * sizeof(float);
}

// Inclusive sum over the 64 lanes of a wave by DPP: row shifts give each lane the sum of its row
// up to itself, then the last lane of each row is broadcast into the following rows.  Lanes a
// shift or a row mask leaves without a source add 0.
__device__ __forceinline__ int wave_inclusive_sum(int v) {
  v += __builtin_amdgcn_update_dpp(0, v, 0x111, 0xF, 0xF, false);  // row_shr:1
  v += __builtin_amdgcn_update_dpp(0, v, 0x112, 0xF, 0xF, false);  // row_shr:2
  v += __builtin_amdgcn_update_dpp(0, v, 0x114, 0xF, 0xF, false);  // row_shr:4
  v += __builtin_amdgcn_update_dpp(0, v, 0x118, 0xF, 0xF, false);  // row_shr:8
  v += __builtin_amdgcn_update_dpp(0, v, 0x142, 0xA, 0xF, false);  // row_bcast:15
  v += __builtin_amdgcn_update_dpp(0, v, 0x143, 0xC, 0xF, false);  // row_bcast:31
  return v;
}

// The same for a double (each step moves both words): lane 63 ends with the wave's sum, added in
// a fixed order.
template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_f64(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, ROWS, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, ROWS, 0xF, false);
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double wave_inclusive_sum_f64(double v) {
  v += dpp_f64<0x111, 0xF>(v);
  v += dpp_f64<0x112, 0xF>(v);
  v += dpp_f64<0x114, 0xF>(v);
  v += dpp_f64<0x118, 0xF>(v);
  v += dpp_f64<0x142, 0xA>(v);
  v += dpp_f64<0x143, 0xC>(v);
  return v;
}

// The forward's LDS: ranking data in visiting order (position m of the batch's candidate order),
// blend data in slot order (position j in S_j minus the batch base), bucket counters, colours.
struct FwdLds {
  float4 *pcand;  // [fb][2]: (mu_x, mu_y, A, B), (slot, C, D, bucket floor); interleaved so that
                  // one address serves both reads, the slot first so that it becomes the key's
                  // low word in place
  float *plbw;    // [kWaves][fb] bounds
  float2 *mu;     // mu_x, mu_y
  double *s64;    // [fb][4] A, B, C, D
  int *bcnt;      // [kBuckets] counters
  int *bstart;    // [kBuckets] starts
  float *col;     // [fb][n]
  int fb;         // candidates per batch
};

__device__ __forceinline__ FwdLds fwd_lds(unsigned char *smem, int fb) {
  FwdLds S;
  S.pcand = reinterpret_cast<float4 *>(smem);
  S.plbw = reinterpret_cast<float *>(smem + 32 * fb);
  S.mu = reinterpret_cast<float2 *>(smem + 48 * fb);
  S.s64 = reinterpret_cast<double *>(smem + 56 * fb);
  S.bcnt = reinterpret_cast<int *>(smem + 88 * fb);
  S.bstart = S.bcnt + kBuckets;
  S.col = reinterpret_cast<float *>(smem + fwd_lds_fixed(fb));
  S.fb = fb;
  return S;
}

// Ranks the tile's hit set S_j = vals[start, start + cnt) at the pixel centre (fx, fy) of the
// calling lane: tk receives the lane's KT smallest keys in ascending order (kKeyEmpty past the
// last member).  single (cnt <= S.fb): the blend geometry and colours of every member are
// left in LDS, in slot order, for the blend.  Every thread of the workgroup calls it.
template <int KT>
__device__ __forceinline__ void rank_tile(const FwdLds &S, int start, int cnt, bool single, int tx,
                                          int ty, float fx, float fy,
                                          const uint32_t *__restrict__ vals,
                                          const float4 *__restrict__ g32a,
                                          const float2 *__restrict__ g32b,
                                          const double4 *__restrict__ g64,
                                          const float *__restrict__ params, int N, int n, int cull,
                                          double (&tk)[KT]) {
  const int tid = threadIdx.x;
  const int ncp = n;
#pragma unroll
  for (int k = 0; k < KT; ++k) tk[k] = kKeyEmpty;

  const int wave = tid >> 6;
  if (tid < kBuckets) S.bcnt[tid] = 0;
  const int fb = S.fb;
  for (int base = 0; base < cnt; base += fb) {
    const int nb = min(fb, cnt - base);
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
        S.mu[tid] = make_float2(a.x, a.y);
        const double4 c = g64[gid];
        S.s64[4 * tid + 0] = c.x;
        S.s64[4 * tid + 1] = c.y;
        S.s64[4 * tid + 2] = c.z;
        S.s64[4 * tid + 3] = c.w;
        for (int ch = 0; ch < n; ++ch) S.col[tid * ncp + ch] = params[(size_t)(5 + ch) * N + gid];
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
      // hardware reciprocals: the 0.1% widening of kappa covers their few ulps, and an inexact
      // edge minimizer moves an edge minimum only in second order
      const float kappa =
          sqrtf(fmaxf(r1, r2) * __builtin_amdgcn_rcpf(fminf(r1, r2))) * 1.001f;
      const float i11 = __builtin_amdgcn_rcpf(p11), i22 = __builtin_amdgcn_rcpf(p22);
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
      brank = atomicAdd(&S.bcnt[bucket], 1);
    }
    __syncthreads();
    if (tid < 64) {  // bucket starts: exclusive scan of the counters (one wave)
      const int c = tid < kBuckets ? S.bcnt[tid] : 0;
      const int inc = wave_inclusive_sum(c);
      if (tid < kBuckets) S.bstart[tid] = inc - c;
    }
    __syncthreads();
    if (tid < nb) {  // scatter the ranking data into visiting order
      const int pos = (int)IGS_IDX(S.bstart[bucket] + brank, fb, kSiteStage);
      S.pcand[2 * pos] = a;
      S.pcand[2 * pos + 1] = make_float4(__int_as_float(base + tid), b.x, b.y, bucket_floor(bucket));
#pragma unroll
      for (int w = 0; w < kWaves; ++w) S.plbw[w * fb + pos] = lbw[w];
    }
    if (tid < kBuckets) S.bcnt[tid] = 0;  // ready for the next batch
    __syncthreads();
    // eight positions per step.  Every lane of a wave reads the same bound, so a skip decision is
    // uniform over the wave and a skipped candidate costs one vector compare.
    for (int m = 0; m < nb; m += 8) {
      // the largest K-th key of the wave (the lists only shrink, so a stale value is safe)
      const uint32_t th = wave_max_u32((uint32_t)__double2hiint(tk[KT - 1]));
      const float q_tau = __uint_as_float(th - kKeyBias);
      // every later candidate's bound is at least the floor of this position's bucket
      if (__int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(S.pcand[2 * m + 1].w))) >
          q_tau)
        break;
      const float4 lba = *reinterpret_cast<const float4 *>(&S.plbw[wave * fb + m]);
      const float4 lbb = *reinterpret_cast<const float4 *>(&S.plbw[wave * fb + m + 4]);
      const float lbu[8] = {lba.x, lba.y, lba.z, lba.w, lbb.x, lbb.y, lbb.z, lbb.w};
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        if (m + u >= nb) break;
        if (lbu[u] > q_tau) continue;
        const float4 g = S.pcand[2 * (m + u)];
        const float4 cd = S.pcand[2 * (m + u) + 1];
        const float dx = fx - g.x, dy = fy - g.y;
        const float e1 = fmaf(g.z, dx, g.w * dy);
        const float e2 = fmaf(cd.y, dx, cd.z * dy);
        const double key = rank_key(fmaf(e1, e1, e2 * e2), __float_as_int(cd.x));
        if (key < tk[KT - 1]) topk_insert<KT>(tk, key);
      }
    }
  }
}

// The retained members of a pixel (its first keff = min(K, |S_j|) keys), re-evaluated in double:
// ts[k] their slots (-1 when absent), src[k] where their colour is (LDS row when single, else the
// Gaussian index), w[k] their weights exp(-(q_k - shift)/2) with shift = q of the first, and Z the
// weights' sum.  No member of S_j is ever cut off (every candidate's key is finite and the
// forward skips a candidate only once the lane's list is full), so every lane's list holds
// min(|S_j|, KT) keys and the retained entries are exactly k < keff, the same for the whole
// workgroup: the loop over them is a uniform branch.
// AHEAD: in the single-batch case, issue the next winner's LDS reads before this winner's
// arithmetic (worth its ten registers in the single-pass kernel, not in the forward kernel).
template <int KT, bool AHEAD>
__device__ __forceinline__ void winners(const FwdLds &S, bool single, int start, int keff,
                                        const double (&tk)[KT], float fx, float fy,
                                        const uint32_t *__restrict__ vals,
                                        const float4 *__restrict__ g32a,
                                        const double4 *__restrict__ g64, int (&ts)[KT],
                                        float (&w)[KT], int (&src)[KT], float &Z, float &shift) {
  Z = 0.f;
  shift = 0.f;
#pragma unroll
  for (int k = 0; k < KT; ++k) {  // the slots first, so that the keys' registers are free
    ts[k] = k < keff ? key_slot(tk[k]) : -1;
    w[k] = 0.f;
    src[k] = 0;
  }
  if (single && AHEAD) {
    // one winner ahead: hoisting all of them would cost registers
    double4 cn = make_double4(0.0, 0.0, 0.0, 0.0);
    float2 mn = make_float2(0.f, 0.f);
    if (keff > 0) {
      const int sb = (int)IGS_IDX(ts[0], S.fb, kSiteSlot);
      cn = *reinterpret_cast<const double4 *>(&S.s64[4 * sb]);
      mn = S.mu[sb];
    }
#pragma unroll
    for (int k = 0; k < KT; ++k) {
      if (k < keff) {
        const double4 c = cn;
        const float2 mu = mn;
        if (k + 1 < keff) {
          const int sb = (int)IGS_IDX(ts[k + 1], S.fb, kSiteSlot);
          cn = *reinterpret_cast<const double4 *>(&S.s64[4 * sb]);
          mn = S.mu[sb];
        }
        asm volatile("" ::: "memory");
        double e1, e2;
        const double q = quad_form64(fx, fy, mu.x, mu.y, c.x, c.y, c.z, c.w, e1, e2);
        if (k == 0) shift = (float)q;
        w[k] = blend_weight(q, shift);
        Z += w[k];
        src[k] = ts[k];
      }
    }
  } else if (single) {
#pragma unroll
    for (int k = 0; k < KT; ++k) {
      if (k < keff) {
        const int slot = ts[k];
        const int sb = (int)IGS_IDX(slot, S.fb, kSiteSlot);
        const double4 c = *reinterpret_cast<const double4 *>(&S.s64[4 * sb]);
        const float2 mu = S.mu[sb];
        double e1, e2;
        const double q = quad_form64(fx, fy, mu.x, mu.y, c.x, c.y, c.z, c.w, e1, e2);
        if (k == 0) shift = (float)q;
        w[k] = blend_weight(q, shift);
        Z += w[k];
        src[k] = slot;
        // one winner's loads at a time: hoisting all of them would cost registers
        asm volatile("" ::: "memory");
      }
    }
  } else {
    // LDS and global reads stay in separate loops (a read through a pointer that may address
    // either miscompiles for gfx950)
#pragma unroll
    for (int k = 0; k < KT; ++k) {
      if (k < keff) {
        const int slot = ts[k];
        const uint32_t gid = vals[start + slot];
        const double4 c = g64[gid];
        const float4 a = g32a[gid];
        double e1, e2;
        const double q = quad_form64(fx, fy, a.x, a.y, c.x, c.y, c.z, c.w, e1, e2);
        if (k == 0) shift = (float)q;
        w[k] = blend_weight(q, shift);
        Z += w[k];
        src[k] = (int)gid;
        asm volatile("" ::: "memory");
      }
    }
  }
}

// ------------------------------------------------------------------------------- adjoint side
//
// With alpha_i = w_i / Z, c_r = sum alpha_i c_i and g = dL/dc_r at a pixel:
//   dL/dc_i += alpha_i g
//   dL/dq_i  = -1/2 alpha_i g.(c_i - c_r)
// and, with e = (A dx + B dy, C dx + D dy), q = |e|^2, the geometry enters only through five
// per-Gaussian sums  G1 = sum gq e1, G2 = sum gq e2, G11 = sum gq e1^2, G22 = sum gq e2^2,
// G12 = sum gq e1 e2  (gq = dL/dq_i at each pixel), which a per-Gaussian pass turns into the
// parameter gradients.
//
// The tile's hit set S_j is processed in batches of 256 positions: the (pixel, retained Gaussian)
// items of a batch are counting-sorted by Gaussian in LDS (item ranks come from per-wave LDS
// sub-counters and stay in registers), and each Gaussian's run is cut into chunks of at most R
// items, R chosen so that the batch has at most 256 chunks.  Lane c accumulates chunk c's 5 + n
// sums in registers and stores them to its own LDS row; lane j then adds up the rows of Gaussian
// j (in chunk order) and writes them as one record at the pair's emit index.  No atomics touch
// floating point, in LDS or in memory, so the records are reproducible bit for bit.

// Per-Gaussian item counters are split into kSub sub-counters, (wave, lane & 1): each is touched
// by one wave only, so the ranks it hands out follow the program and lane order (no dependence on
// how waves interleave) and the order of items in a run, hence every float sum, is reproducible;
// the lane split halves same-address LDS atomics.
constexpr int kSub = 8;
__device__ __forceinline__ int item_sub(int tid) { return ((tid >> 6) << 1) | (tid & 1); }

// Exclusive scan of v over the 256 threads of the block; returns the block total in *total.
__device__ __forceinline__ int block_exclusive_scan(int v, int *s_wave, int *total) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int inc = wave_inclusive_sum(v);
  if (lane == 63) s_wave[w] = inc;
  __syncthreads();
  int off = 0, tot = 0;
#pragma unroll
  for (int k = 0; k < kRasterThreads / 64; ++k) {
    const int t = s_wave[k];
    off += k < w ? t : 0;
    tot += t;
  }
  *total = tot;
  return off + inc - v;
}

// The adjoint's LDS layout (byte offsets).  The per-Gaussian counters and the placed items share
// one region, which the per-chunk sums reuse once every chunk has read its items.
struct BwdLds {
  unsigned px, part, off, cho, owner, gid, src, wave, item, total;
};

// Per-pixel row in LDS: g[0..NC), g.c_r, shift, 1/Z, padding to a multiple of 4 floats.
template <int NC>
__host__ __device__ constexpr int px_row() { return (NC + 3 + 3) & ~3; }

template <int NC, int KT>
__host__ __device__ constexpr BwdLds bwd_lds() {
  constexpr unsigned ROW = px_row<NC>();
  constexpr unsigned NACC = 5 + NC;
  constexpr unsigned cnt_bytes = 4 * (kBatch * kSub + kRasterThreads);  // + one dummy per lane
  constexpr unsigned item_bytes = 2 * kRasterThreads * KT;
  constexpr unsigned part_bytes = 4 * kRasterThreads * NACC;
  BwdLds L{};
  unsigned o = 0;
  L.px = o;
  o += 4 * kRasterThreads * ROW;
  L.part = o;
  L.item = o + cnt_bytes;
  o += part_bytes > cnt_bytes + item_bytes ? part_bytes : cnt_bytes + item_bytes;
  L.off = o;
  o += 4 * (kBatch + 4);
  L.cho = o;
  o += 4 * (kBatch + 4);
  L.owner = o;
  o += 2 * kRasterThreads;
  L.gid = o;
  o += 4 * kBatch;
  L.src = o;
  o += 4 * kBatch;
  L.wave = o;  // two scans' wave totals
  o += 32;
  L.total = (o + 15) & ~15u;
  return L;
}

// Stores the calling lane's pixel row (the first NC + 3 entries of row; the rest must be 0).
template <int NC>
__device__ __forceinline__ void store_px_row(unsigned char *smem, const float (&row)[px_row<NC>()]) {
  constexpr int ROW = px_row<NC>();
  float *s_px = reinterpret_cast<float *>(smem);
#pragma unroll
  for (int r = 0; r < ROW; r += 4)
    *reinterpret_cast<float4 *>(&s_px[threadIdx.x * ROW + r]) =
        make_float4(row[r], row[r + 1], row[r + 2], row[r + 3]);
}

// The tile's records: sl[k] are the calling lane's retained slots (-1 = none), the pixel
// rows are in LDS (store_px_row; visible after the first barrier here), S_j = vals[start,
// start + cnt) with emit indices src[start, start + cnt), and the tile's top-left pixel is
// (x0, y0).  Every thread of the workgroup calls it; LDS is free again when it returns.
template <int NC, int KT>
__device__ __forceinline__ void adjoint_batches(unsigned char *smem, int start, int cnt, int x0,
                                                int y0, const int (&sl)[KT],
                                                const uint32_t *__restrict__ vals,
                                                const uint32_t *__restrict__ src,
                                                const float4 *__restrict__ g32a,
                                                const double4 *__restrict__ g64,
                                                const float *__restrict__ params, int N, int n,
                                                float *__restrict__ part) {
  constexpr int ROW = px_row<NC>();
  constexpr int NACC = 5 + NC;
  constexpr BwdLds L = bwd_lds<NC, KT>();
  const float *s_px = reinterpret_cast<const float *>(smem + L.px);  // [256 px][ROW]
  int *s_cnt8 = reinterpret_cast<int *>(smem + L.part);            // [kBatch][kSub] + dummies
  float *s_part = reinterpret_cast<float *>(smem + L.part);        // [256 chunks][NACC]
  int *s_off = reinterpret_cast<int *>(smem + L.off);              // [kBatch + 1] run starts
  int *s_cho = reinterpret_cast<int *>(smem + L.cho);              // [kBatch + 1] chunk starts
  uint16_t *s_owner = reinterpret_cast<uint16_t *>(smem + L.owner);  // [256] chunk -> j
  uint32_t *s_gid = reinterpret_cast<uint32_t *>(smem + L.gid);    // [kBatch] j -> Gaussian
  uint32_t *s_src = reinterpret_cast<uint32_t *>(smem + L.src);    // [kBatch] j -> emit index
  int *s_wave = reinterpret_cast<int *>(smem + L.wave);
  uint16_t *s_item = reinterpret_cast<uint16_t *>(smem + L.item);  // [256 * KT] px | j << 8

  const int tid = threadIdx.x;
  const int sub = item_sub(tid);
  for (int base = 0; base < cnt; base += kBatch) {
    const int nb = min(kBatch, cnt - base);
    if (base > 0) __syncthreads();  // previous batch fully consumed
    if (tid < nb) {
      s_gid[tid] = vals[start + base + tid];
      s_src[tid] = src[start + base + tid];
    }
#pragma unroll
    for (int c = 0; c < kSub; ++c) s_cnt8[tid * kSub + c] = 0;
    __syncthreads();

    // 1a: rank of each item inside its (Gaussian, lane & 7) sub-run; items outside the batch
    // count on a private dummy counter so the atomics need no branches
    uint32_t e[KT];
#pragma unroll
    for (int k = 0; k < KT; ++k) {
      const int j = sl[k] - base;
      const bool ok = (unsigned)j < (unsigned)nb;
      const int a = ok ? j * kSub + sub : kBatch * kSub + tid;
      const int r =
          atomicAdd(&s_cnt8[IGS_IDX(a, kBatch * kSub + kRasterThreads, kSiteAdjCounter)], 1);
      e[k] = ok ? (uint32_t)(j | (r << 8)) : 0xFFFFFFFFu;
    }
    __syncthreads();

    // Gaussian tid: its run length; one packed scan gives run starts and the number of
    // Gaussians with items (a Gaussian occurs at most once per pixel, so runs are <= 256)
    int c8[kSub];
    int my_cnt = 0;
#pragma unroll
    for (int c = 0; c < kSub; ++c) {
      c8[c] = s_cnt8[tid * kSub + c];
      my_cnt += c8[c];
    }
    int packed_total;
    const int packed_off =
        block_exclusive_scan(my_cnt | ((my_cnt > 0 ? 1 : 0) << 16), s_wave, &packed_total);
    const int my_off = packed_off & 0xFFFF;
    const int total_items = packed_total & 0xFFFF;
    const int busy = packed_total >> 16;
    // chunk length R: the batch may have at most 256 chunks, sum_j ceil(cnt_j / R).  Three
    // candidates, shortest first: the ideal ceil(total / 256), an estimate that allows half a
    // partial chunk per Gaussian, and the guaranteed ceil(total / (256 - busy)), for which the
    // sum is at most total / R + busy <= 256.  One scan counts the chunks of all three (a
    // Gaussian's run is at most 256 items, so each count fits 10 bits), and the shortest that
    // fits is used.
    const int r_safe = busy < kRasterThreads
                           ? max(1, (total_items + (kRasterThreads - busy) - 1) / (kRasterThreads - busy))
                           : kRasterThreads;
    const int r_mid = min(r_safe, max(1, (2 * total_items + (2 * kRasterThreads - busy) - 1) /
                                             (2 * kRasterThreads - busy)));
    const int r_min = min(r_mid, max(1, (total_items + kRasterThreads - 1) / kRasterThreads));
    // ceil(c / R) as floor((c + R - 1/2) / R) in float with the hardware reciprocal: exact, the
    // quotient is at least 1 / (2 R) from an integer and c, R <= 256 keep its error (a few ulps
    // of a value below 512) far below that
    auto chunks_of = [&](int c, int R) {
      return (int)(((float)c + ((float)R - 0.5f)) * __builtin_amdgcn_rcpf((float)R));
    };
    const int packed_ch = chunks_of(my_cnt, r_min) | (chunks_of(my_cnt, r_mid) << 10) |
                          (chunks_of(my_cnt, r_safe) << 20);
    int packed_chunks;
    // (a second LDS slot, so the first scan's readers need no barrier before it is written)
    const int packed_cho = block_exclusive_scan(packed_ch, s_wave + 4, &packed_chunks);
    const int sel = (packed_chunks & 0x3FF) <= kRasterThreads
                        ? 0
                        : (((packed_chunks >> 10) & 0x3FF) <= kRasterThreads ? 10 : 20);
    const int R = sel == 0 ? r_min : (sel == 10 ? r_mid : r_safe);
    const int my_ch = (packed_ch >> sel) & 0x3FF;
    const int my_cho = (packed_cho >> sel) & 0x3FF;
    const int total_chunks = (packed_chunks >> sel) & 0x3FF;
    {
      int o = my_off;
#pragma unroll
      for (int c = 0; c < kSub; ++c) {
        s_cnt8[tid * kSub + c] = o;
        o += c8[c];
      }
    }
    s_off[tid] = my_off;
    s_cho[tid] = my_cho;
    for (int c = 0; c < my_ch; ++c)
      s_owner[IGS_IDX(my_cho + c, kRasterThreads, kSiteAdjChunk)] = (uint16_t)tid;
    if (tid == 0) {
      s_off[kBatch] = total_items;
      s_cho[kBatch] = total_chunks;
    }
    __syncthreads();

    // the lane's chunk: fetch its Gaussian now so the loads overlap the placement below
    const bool has = tid < total_chunks;
    const int j = has ? (int)s_owner[tid] : 0;
    const uint32_t gid = s_gid[j];
    float2 mu = make_float2(0.f, 0.f);
    double4 c64 = make_double4(0.0, 0.0, 0.0, 0.0);
    float cj[NC];
#pragma unroll
    for (int ch = 0; ch < NC; ++ch) cj[ch] = 0.f;
    if (has) {
      const float4 a = g32a[gid];
      mu = make_float2(a.x, a.y);
      c64 = g64[gid];
#pragma unroll
      for (int ch = 0; ch < NC; ++ch)
        if (ch < n) cj[ch] = params[(size_t)(5 + ch) * N + gid];
    }

    // 1b: place every item in its Gaussian's run
#pragma unroll
    for (int k = 0; k < KT; ++k) {
      if (e[k] != 0xFFFFFFFFu) {
        const int jj = e[k] & 0xFF;
        const int64_t at = IGS_IDX(s_cnt8[jj * kSub + sub] + (e[k] >> 8), kRasterThreads * KT,
                                   kSiteAdjItem);
        s_item[at] = (uint16_t)(tid | (jj << 8));
      }
    }
    __syncthreads();

    // 2: chunk tid, one Gaussian, accumulated in registers
    float G1 = 0.f, G2 = 0.f, G11 = 0.f, G22 = 0.f, G12 = 0.f;
    float gcol[NC];
#pragma unroll
    for (int ch = 0; ch < NC; ++ch) gcol[ch] = 0.f;
    if (has) {
      const int first = s_off[j] + (tid - s_cho[j]) * R;
      const int end = min(first + R, s_off[j + 1]);
      for (int it = first; it < end; ++it) {
        const int p = s_item[IGS_IDX(it, kRasterThreads * KT, kSiteAdjItem)] & 0xFF;
        float rw[ROW];
#pragma unroll
        for (int r = 0; r < ROW; r += 4) {
          const float4 v = *reinterpret_cast<const float4 *>(&s_px[p * ROW + r]);
          rw[r] = v.x;
          rw[r + 1] = v.y;
          rw[r + 2] = v.z;
          rw[r + 3] = v.w;
        }
        const float fx = (float)(x0 + (p & (kTile - 1))) + 0.5f;
        const float fy = (float)(y0 + (p >> 4)) + 0.5f;
        double d1, d2;
        const double q = quad_form64(fx, fy, mu.x, mu.y, c64.x, c64.y, c64.z, c64.w, d1, d2);
        const float alpha = blend_weight(q, rw[NC + 1]) * rw[NC + 2];
        const float e1 = (float)d1, e2 = (float)d2;
        float dot = -rw[NC];
#pragma unroll
        for (int ch = 0; ch < NC; ++ch) dot = fmaf(rw[ch], cj[ch], dot);
        const float gq = -0.5f * alpha * dot;
        const float g1 = gq * e1, g2 = gq * e2;
        G1 += g1;
        G2 += g2;
        G11 = fmaf(g1, e1, G11);
        G22 = fmaf(g2, e2, G22);
        G12 = fmaf(g1, e2, G12);
#pragma unroll
        for (int ch = 0; ch < NC; ++ch) gcol[ch] = fmaf(alpha, rw[ch], gcol[ch]);
      }
    }
    __syncthreads();  // every chunk has read its items: the sums may overwrite them
    if (has) {
      float *prow = &s_part[tid * NACC];
      prow[0] = G1;
      prow[1] = G2;
      prow[2] = G11;
      prow[3] = G22;
      prow[4] = G12;
#pragma unroll
      for (int ch = 0; ch < NC; ++ch) prow[5 + ch] = gcol[ch];
    }
    __syncthreads();

    // 3: the pair records, LP lanes per Gaussian: lane r adds up entry r of the Gaussian's chunks
    // in chunk order (zeros when no pixel of the tile retained it, and in the padding)
    {
      constexpr int NR = (NACC + 3) & ~3;
      constexpr int LP = NR <= 16 ? 16 : (NR <= 32 ? 32 : 64);
      const int stride = part_stride(n);
      const int r = tid & (LP - 1);
      if (r < stride) {
        for (int jj = tid / LP; jj < nb; jj += kRasterThreads / LP) {
          const int c1 = s_cho[jj + 1];
          const uint32_t dst = s_src[jj];
          float acc = 0.f;
          if (r < 5 + n) {
            int c = s_cho[jj];
#ifdef IGS_BOUNDS_CHECK
            if (c1 > kRasterThreads) IGS_IDX(c1, kRasterThreads + 1, kSiteAdjChunk);
#endif
            // four chunks' loads in flight, added one at a time in chunk order
            for (; c + 4 <= c1; c += 4) {
              const float v0 = s_part[c * NACC + r], v1 = s_part[(c + 1) * NACC + r];
              const float v2 = s_part[(c + 2) * NACC + r], v3 = s_part[(c + 3) * NACC + r];
              acc += v0;
              acc += v1;
              acc += v2;
              acc += v3;
            }
            for (; c < c1; ++c) acc += s_part[c * NACC + r];
          }
          part[(size_t)dst * stride + r] = acc;
        }
      }
    }
  }
  __syncthreads();  // LDS is reused by the next phase or tile
}

// Tile loss sums (sum |d|, sum d^2) over the workgroup: wave sums by DPP, then a fixed order
// over the four waves; the result is valid in thread 0.
__device__ __forceinline__ double2 tile_loss_sums(double a, double b, double *s_red) {
  a = wave_inclusive_sum_f64(a);
  b = wave_inclusive_sum_f64(b);
  const int wave = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 63) {
    s_red[2 * wave] = a;
    s_red[2 * wave + 1] = b;
  }
  __syncthreads();
  double2 t = make_double2(0.0, 0.0);
  if (threadIdx.x == 0) {
    for (int k = 0; k < kWaves; ++k) {
      t.x += s_red[2 * k];
      t.y += s_red[2 * k + 1];
    }
  }
  return t;
}

}  // namespace igs
