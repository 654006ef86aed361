// Adjoint rasterizer (Image-GS Sec. 3.3: gradients flow through the K retained Gaussians, the
// selection itself is held fixed).
//
// With alpha_i = w_i / Z, c_r = sum alpha_i c_i and g = dL/dc_r at a pixel:
//   dL/dc_i += alpha_i g
//   dL/dq_i  = -1/2 alpha_i g.(c_i - c_r)
// and, with e = (A dx + B dy, C dx + D dy), q = |e|^2, the geometry enters only through five
// per-Gaussian sums  G1 = sum gq e1, G2 = sum gq e2, G11 = sum gq e1^2, G22 = sum gq e2^2,
// G12 = sum gq e1 e2  (gq = dL/dq_i at each pixel).  A per-Gaussian pass turns them into
//   dL/dmu_x = -2 (A G1 + C G2)          dL/dmu_y = -2 (B G1 + D G2)
//   dL/dtheta = 2 (u1/u2 - u2/u1) G12    dL/ds_a = -2 u_a G_aa       (u_a = 1/s_a).
//
// One workgroup per 16 x 16 tile, one lane per pixel while reading.  The tile's hit set S_j is
// processed in batches of 256 positions: the (pixel, retained Gaussian) items of a batch are
// counting-sorted by Gaussian in LDS and split into chunks of at most R items of one Gaussian.  A
// lane loads its chunk's Gaussian once, accumulates the chunk's 5 + n sums in registers, adds
// them to the Gaussian's LDS row once (a plain store when the chunk is the Gaussian's only one),
// and each batch ends with one global atomic per (Gaussian, component) that received anything.
// The blend weights are recomputed from the saved per-pixel shift and 1/Z with the forward's
// exact double-precision expression.
#include "raster_common.hpp"

namespace igs {
namespace {

// Exclusive scan of v over the 256 threads of the block; returns the block total in *total.
__device__ __forceinline__ int block_exclusive_scan(int v, int *s_wave, int *total) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  int inc = v;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    int o = __shfl_up(inc, d, 64);
    if (lane >= d) inc += o;
  }
  if (lane == 63) s_wave[w] = inc;
  __syncthreads();
  int off = 0, tot = 0;
#pragma unroll
  for (int k = 0; k < kRasterThreads / 64; ++k) {
    const int t = s_wave[k];
    off += k < w ? t : 0;
    tot += t;
  }
  __syncthreads();
  *total = tot;
  return off + inc - v;
}

struct BwdLds {
  unsigned g, gc, aux, acc, cnt8, off, cho, owner, wave, tmp, item, total;
};

constexpr int kSub = 8;  // per-Gaussian counters are split by lane & 7 to spread LDS atomics

// LDS layout of the adjoint kernel for K retained Gaussians per pixel (byte offsets; per-pixel
// gradient rows are 16-byte aligned for float4 reads).
template <int NC>
__host__ __device__ constexpr BwdLds bwd_lds(int K) {
  constexpr unsigned NCP = (NC + 3) & ~3;
  BwdLds L{};
  unsigned o = 0;
  L.g = o;
  o += 4 * kRasterThreads * NCP;
  L.gc = o;
  o += 4 * kRasterThreads;
  L.aux = o;
  o += 8 * kRasterThreads;
  L.acc = o;
  o += 4 * kBatch * (5 + NC);
  L.cnt8 = o;
  o += 4 * kBatch * kSub;
  L.off = o;
  o += 4 * (kBatch + 4);
  L.cho = o;
  o += 4 * (kBatch + 4);
  L.owner = o;
  o += 2 * 2 * kBatch;
  L.wave = o;
  o += 16;
  L.tmp = o;
  o += 2 * kRasterThreads * (unsigned)K;
  L.item = o;
  o += 2 * kRasterThreads * (unsigned)K;
  L.total = (o + 15) & ~15u;
  return L;
}

template <int NC>
__global__ __launch_bounds__(kRasterThreads) void raster_bwd_kernel(
    const int2 *__restrict__ ranges, const uint32_t *__restrict__ vals,
    const float4 *__restrict__ g32a, const double4 *__restrict__ g64,
    const float *__restrict__ params, int N, int n, int K, int T, Images imgs,
    const int *__restrict__ tile_order, const float *__restrict__ image_all,
    const float *__restrict__ grad_image_all, const uint16_t *__restrict__ slots_all,
    const float2 *__restrict__ aux_all, float *__restrict__ gamma,
    float *__restrict__ grad_params) {
  constexpr int NCP = (NC + 3) & ~3;  // padded per-pixel gradient row
  constexpr int NACC = 5 + NC;
  extern __shared__ __align__(16) unsigned char smem[];
  const BwdLds L = bwd_lds<NC>(K);
  float *s_g = reinterpret_cast<float *>(smem + L.g);              // [256 px][NCP]
  float *s_gc = reinterpret_cast<float *>(smem + L.gc);            // [256 px] g . c_r
  float2 *s_aux = reinterpret_cast<float2 *>(smem + L.aux);        // [256 px] shift, 1/Z
  float *s_acc = reinterpret_cast<float *>(smem + L.acc);          // [kBatch][NACC]
  int *s_cnt8 = reinterpret_cast<int *>(smem + L.cnt8);            // [kBatch][kSub]
  int *s_off = reinterpret_cast<int *>(smem + L.off);              // [kBatch + 1] run starts
  int *s_cho = reinterpret_cast<int *>(smem + L.cho);              // [kBatch + 1] chunk starts
  uint16_t *s_owner = reinterpret_cast<uint16_t *>(smem + L.owner);  // [2 kBatch] chunk -> j
  int *s_wave = reinterpret_cast<int *>(smem + L.wave);            // [4]
  uint16_t *s_tmp = reinterpret_cast<uint16_t *>(smem + L.tmp);    // [256 * K] j | rank << 8
  uint16_t *s_item = reinterpret_cast<uint16_t *>(smem + L.item);  // [256 * K] px | j << 8

  const int tid = threadIdx.x;
  const int tile = __builtin_amdgcn_readfirstlane(tile_order ? tile_order[blockIdx.x]
                                                             : xcd_tile(blockIdx.x, T));
  const int2 rg = ranges[tile];
  const int start = __builtin_amdgcn_readfirstlane(rg.x);  // uniform over the workgroup
  const int cnt = __builtin_amdgcn_readfirstlane(rg.y - rg.x);
  if (cnt <= 0) return;
  const ImageDesc im = imgs.by_tile(tile);
  const int W = im.W, H = im.H;
  const int64_t HW = (int64_t)H * W;
  const float *__restrict__ image = image_all + (int64_t)n * im.pix_off;
  const float *__restrict__ grad_image = grad_image_all + (int64_t)n * im.pix_off;
  const uint16_t *__restrict__ slots = slots_all + (int64_t)K * im.pix_off;
  const float2 *__restrict__ aux = aux_all + im.pix_off;
  const int lt = tile - im.tile_off;
  const int tx = lt % im.tiles_x, ty = lt / im.tiles_x;
  const int x0 = tx * kTile, y0 = ty * kTile;
  const int px = x0 + (tid & (kTile - 1)), py = y0 + tid / kTile;
  const bool inside = px < W && py < H;
  const int64_t pix = inside ? (int64_t)py * W + px : 0;

  // per-pixel upstream gradient, g . c_r, and the forward's blend normalization
  {
    float gc = 0.f;
#pragma unroll
    for (int ch = 0; ch < NCP; ++ch) {
      float g = 0.f;
      if (ch < n && inside) {
        g = grad_image[(int64_t)ch * HW + pix];
        gc = fmaf(g, image[(int64_t)ch * HW + pix], gc);
      }
      s_g[tid * NCP + ch] = g;
    }
    s_gc[tid] = gc;
    s_aux[tid] = inside ? aux[pix] : make_float2(0.f, 0.f);
  }

  for (int base = 0; base < cnt; base += kBatch) {
    const int nb = min(kBatch, cnt - base);
    __syncthreads();  // previous batch fully consumed
#pragma unroll
    for (int c = 0; c < kSub; ++c) s_cnt8[tid * kSub + c] = 0;
#pragma unroll
    for (int r = 0; r < NACC; ++r) s_acc[tid * NACC + r] = 0.f;
    __syncthreads();

    // 1a: count the items of every Gaussian of the batch; the returned count is the item's rank
    // inside its (Gaussian, lane & 7) sub-run (at most 32 items: one per pixel of the class)
    const int sub = tid & (kSub - 1);
    if (inside)
      for (int k = 0; k < K; ++k) {
        const int j = (int)slots[(int64_t)k * HW + pix] - base;
        uint16_t e = 0xFFFF;
        if (j >= 0 && j < nb) e = (uint16_t)(j | (atomicAdd(&s_cnt8[j * kSub + sub], 1) << 8));
        s_tmp[tid * K + k] = e;
      }
    __syncthreads();
    // Gaussian tid: its run (sub-runs in lane-class order), its chunks and its sub-run starts
    int c8[kSub];
    int my_cnt = 0;
#pragma unroll
    for (int c = 0; c < kSub; ++c) {
      c8[c] = s_cnt8[tid * kSub + c];
      my_cnt += c8[c];
    }
    int total_items;
    const int my_off = block_exclusive_scan(my_cnt, s_wave, &total_items);
    // chunk length: about one chunk per lane
    const int R = max(1, (total_items + kRasterThreads - 1) / kRasterThreads + 2);
    const int my_ch = (my_cnt + R - 1) / R;
    int total_chunks;
    const int my_cho = block_exclusive_scan(my_ch, s_wave, &total_chunks);
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
    for (int c = 0; c < my_ch; ++c) s_owner[my_cho + c] = (uint16_t)tid;
    if (tid == 0) {
      s_off[kBatch] = total_items;
      s_cho[kBatch] = total_chunks;  // s_cho[j + 1] - s_cho[j] = chunks of j
    }
    __syncthreads();

    // the lane's first chunk: fetch its Gaussian now so the loads overlap the placement below
    const bool has0 = tid < total_chunks;
    const int j0 = has0 ? (int)s_owner[tid] : 0;
    const uint32_t gid0 = vals[start + base + j0];
    float4 a0 = make_float4(0.f, 0.f, 0.f, 0.f);
    double4 c640 = make_double4(0.0, 0.0, 0.0, 0.0);
    float col0[NC];
#pragma unroll
    for (int ch = 0; ch < NC; ++ch) col0[ch] = 0.f;
    if (has0) {
      a0 = g32a[gid0];
      c640 = g64[gid0];
#pragma unroll
      for (int ch = 0; ch < NC; ++ch)
        if (ch < n) col0[ch] = params[(size_t)(5 + ch) * N + gid0];
    }

    // 1b: place every item in its Gaussian's run
    if (inside)
      for (int k = 0; k < K; ++k) {
        const uint16_t e = s_tmp[tid * K + k];
        if (e != 0xFFFF) {
          const int j = e & 0xFF;
          s_item[s_cnt8[j * kSub + sub] + (e >> 8)] = (uint16_t)(tid | (j << 8));
        }
      }
    __syncthreads();

    // 2: chunks of one Gaussian each, accumulated in registers
    for (int c = tid; c < total_chunks; c += kRasterThreads) {
      const int j = c == tid ? j0 : (int)s_owner[c];
      const int first = s_off[j] + (c - s_cho[j]) * R;
      const int end = min(first + R, s_off[j + 1]);
      float4 a = a0;
      double4 c64 = c640;
      float cj[NC];
#pragma unroll
      for (int ch = 0; ch < NC; ++ch) cj[ch] = col0[ch];
      if (c != tid) {
        const uint32_t gid = vals[start + base + j];
        a = g32a[gid];
        c64 = g64[gid];
#pragma unroll
        for (int ch = 0; ch < NC; ++ch) cj[ch] = ch < n ? params[(size_t)(5 + ch) * N + gid] : 0.f;
      }
      float G1 = 0.f, G2 = 0.f, G11 = 0.f, G22 = 0.f, G12 = 0.f;
      float gcol[NC];
#pragma unroll
      for (int ch = 0; ch < NC; ++ch) gcol[ch] = 0.f;
      for (int it = first; it < end; ++it) {
        const int p = s_item[it] & 0xFF;
        const float fx = (float)(x0 + (p & (kTile - 1))) + 0.5f;
        const float fy = (float)(y0 + p / kTile) + 0.5f;
        double d1, d2;
        const double q = quad_form64(fx, fy, a.x, a.y, c64.x, c64.y, c64.z, c64.w, d1, d2);
        const float2 ax = s_aux[p];
        const float alpha = blend_weight(q, ax.x) * ax.y;
        const float e1 = (float)d1, e2 = (float)d2;
        float gv[NCP];
#pragma unroll
        for (int ch = 0; ch < NCP; ch += 4) {
          const float4 v = *reinterpret_cast<const float4 *>(&s_g[p * NCP + ch]);
          gv[ch] = v.x;
          if (ch + 1 < NCP) gv[ch + 1] = v.y;
          if (ch + 2 < NCP) gv[ch + 2] = v.z;
          if (ch + 3 < NCP) gv[ch + 3] = v.w;
        }
        float dot = -s_gc[p];
#pragma unroll
        for (int ch = 0; ch < NC; ++ch) dot = fmaf(gv[ch], cj[ch], dot);
        const float gq = -0.5f * alpha * dot;
        const float g1 = gq * e1, g2 = gq * e2;
        G1 += g1;
        G2 += g2;
        G11 = fmaf(g1, e1, G11);
        G22 = fmaf(g2, e2, G22);
        G12 = fmaf(g1, e2, G12);
#pragma unroll
        for (int ch = 0; ch < NC; ++ch) gcol[ch] = fmaf(alpha, gv[ch], gcol[ch]);
      }
      float *row = &s_acc[j * NACC];
      if (s_cho[j + 1] - s_cho[j] == 1) {  // this lane holds the Gaussian's only chunk
        row[0] = G1;
        row[1] = G2;
        row[2] = G11;
        row[3] = G22;
        row[4] = G12;
#pragma unroll
        for (int ch = 0; ch < NC; ++ch) row[5 + ch] = gcol[ch];
      } else {
        atomicAdd(&row[0], G1);
        atomicAdd(&row[1], G2);
        atomicAdd(&row[2], G11);
        atomicAdd(&row[3], G22);
        atomicAdd(&row[4], G12);
#pragma unroll
        for (int ch = 0; ch < NC; ++ch) atomicAdd(&row[5 + ch], gcol[ch]);
      }
    }
    __syncthreads();

    // 3: one global add per (Gaussian, component) of this batch
    if (tid < nb && my_cnt > 0) {
      const uint32_t gid = vals[start + base + tid];  // Gaussian tid of the batch
      const float *row = &s_acc[tid * NACC];
#pragma unroll
      for (int r = 0; r < 5; ++r) unsafeAtomicAdd(&gamma[(size_t)r * N + gid], row[r]);
#pragma unroll
      for (int ch = 0; ch < NC; ++ch)
        if (ch < n) unsafeAtomicAdd(&grad_params[(size_t)(5 + ch) * N + gid], row[5 + ch]);
    }
  }
}

__global__ __launch_bounds__(256) void grad_finalize_kernel(const float *__restrict__ params,
                                                            const float4 *__restrict__ g32a,
                                                            const float2 *__restrict__ g32b,
                                                            const float *__restrict__ gamma,
                                                            int N, float *__restrict__ grad) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const float G1 = gamma[i], G2 = gamma[(size_t)N + i], G11 = gamma[2 * (size_t)N + i];
  const float G22 = gamma[3 * (size_t)N + i], G12 = gamma[4 * (size_t)N + i];
  const float4 a = g32a[i];
  const float2 cd = g32b[i];
  const float u1 = 1.0f / params[3 * (size_t)N + i], u2 = 1.0f / params[4 * (size_t)N + i];
  grad[i] = -2.0f * (a.z * G1 + cd.x * G2);
  grad[(size_t)N + i] = -2.0f * (a.w * G1 + cd.y * G2);
  grad[2 * (size_t)N + i] = 2.0f * (u1 / u2 - u2 / u1) * G12;
  grad[3 * (size_t)N + i] = -2.0f * u1 * G11;
  grad[4 * (size_t)N + i] = -2.0f * u2 * G22;
}

template <int NC>
hipError_t launch_bwd_nc(const int2 *ranges, const uint32_t *vals, const float4 *g32a,
                         const double4 *g64, const float *params, const Dims &d,
                         const Images &imgs, const int *tile_order, const float *image,
                         const float *grad_image, const uint16_t *slots, const float2 *aux,
                         float *gamma, float *grad_params, hipStream_t s) {
  const size_t lds = bwd_lds<NC>(d.K).total;
  if (lds > 65536) {
    hipError_t e = hipFuncSetAttribute((const void *)raster_bwd_kernel<NC>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  raster_bwd_kernel<NC><<<d.T, kRasterThreads, lds, s>>>(ranges, vals, g32a, g64, params, d.N,
                                                          d.n, d.K, d.T, imgs, tile_order, image,
                                                          grad_image, slots, aux, gamma,
                                                          grad_params);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_raster_bwd(const int2 *ranges, const uint32_t *vals, const float4 *g32a,
                             const float2 *g32b, const double4 *g64, const float *params,
                             const Dims &d, const Images &imgs, const int *tile_order,
                             const float *image, const float *grad_image, const uint16_t *slots,
                             const float2 *aux, float *gamma, float *grad_params, hipStream_t s) {
  (void)g32b;
#define IGS_BWD_NC(NCV)                                                                        \
  if (d.n <= NCV)                                                                              \
    return launch_bwd_nc<NCV>(ranges, vals, g32a, g64, params, d, imgs, tile_order, image,     \
                              grad_image, slots, aux, gamma, grad_params, s);
  IGS_BWD_NC(1)
  IGS_BWD_NC(3)
  IGS_BWD_NC(4)
  IGS_BWD_NC(9)
  IGS_BWD_NC(16)
  IGS_BWD_NC(32)
#undef IGS_BWD_NC
  return hipErrorInvalidValue;
}

hipError_t launch_grad_finalize(const float *params, const float4 *g32a, const float2 *g32b,
                                const float *gamma, int N, float *grad_params, hipStream_t s) {
  if (N <= 0) return hipSuccess;
  grad_finalize_kernel<<<(N + 255) / 256, 256, 0, s>>>(params, g32a, g32b, gamma, N, grad_params);
  return hipGetLastError();
}

}  // namespace igs
