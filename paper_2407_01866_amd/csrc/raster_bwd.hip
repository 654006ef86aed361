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
// One workgroup per 16 x 16 tile.  Every per-pixel input (the KT saved slots, the upstream
// gradient, the rendered colour and the blend normalization) is loaded once, up front, with all
// loads in flight together; the pixel's row (g, g.c_r, shift, 1/Z) then lives in LDS.  The tile's
// hit set S_j is processed in batches of 256 positions: the (pixel, retained Gaussian) items of a
// batch are counting-sorted by Gaussian in LDS (item ranks come from per-wave LDS sub-counters and
// stay in registers), and each Gaussian's run is cut into chunks of at most R items,
// R chosen so that the batch has at most 256 chunks.  Lane c accumulates chunk c's 5 + n sums in
// registers and stores them to its own LDS row; lane j then adds up the rows of Gaussian j (in
// chunk order) and writes them as one record at the pair's emit index.  No atomics touch floating
// point, in LDS or in memory: a second kernel sums each Gaussian's records, which are contiguous
// in emit order (one per tile it hits, in tile order), in that fixed order, so the gradient is
// reproducible bit for bit.
// The blend weights are recomputed from the saved per-pixel shift and 1/Z with the forward's
// exact double-precision expression.
#include "raster_tile.hpp"

#include <algorithm>

namespace igs {
namespace {

// Register budget: four waves per SIMD (<= 128 VGPRs) where that fits without spilling.
__host__ __device__ constexpr int bwd_min_waves(int nc, int kt) { return nc + kt <= 25 ? 4 : 2; }

// L1 = true: the upstream gradient is the mean-absolute-error gradient recorded by the fused
// forward (per pixel: g . c_r and 2-bit sign codes, g = sign / (n H W)) instead of explicit
// gradient and colour images; image_all and grad_image_all are then unused.
template <int NC, int KT, bool L1>
__global__ __launch_bounds__(kRasterThreads)
__attribute__((amdgpu_waves_per_eu(bwd_min_waves(NC, KT)))) void raster_bwd_kernel(
    const int2 *__restrict__ ranges, const uint32_t *__restrict__ vals,
    const uint32_t *__restrict__ src, const float4 *__restrict__ g32a,
    const double4 *__restrict__ g64, const float *__restrict__ params, int N, int n, int K, int T,
    Images imgs, const int *__restrict__ tile_order, const float *__restrict__ image_all,
    const float *__restrict__ grad_image_all, const float2 *__restrict__ l1_rec,
    const uint16_t *__restrict__ slots_all, const float2 *__restrict__ aux_all,
    float *__restrict__ part, TileQueue queue) {
  constexpr int ROW = px_row<NC>();  // g[0..NC), g.c_r, shift, 1/Z, padding
  extern __shared__ __align__(16) unsigned char smem[];

  const int tid = threadIdx.x;
  int idx = 0;
  for (bool first = true; next_tile_index(queue, T, first, idx); first = false) {
  const int tile = __builtin_amdgcn_readfirstlane(tile_order ? tile_order[idx] : xcd_tile(idx, T));
  const int2 rg = ranges[tile];
  const int start = __builtin_amdgcn_readfirstlane(rg.x);  // uniform over the workgroup
  const int cnt = __builtin_amdgcn_readfirstlane(rg.y - rg.x);
  if (cnt <= 0) continue;
  const ImageDesc im = imgs.by_tile(tile);
  const int W = im.W, H = im.H;
  const int64_t HW = (int64_t)H * W;
  const int lt = tile - im.tile_off;
  const int tx = lt % im.tiles_x, ty = lt / im.tiles_x;
  const int x0 = tx * kTile, y0 = ty * kTile;
  const int px = x0 + (tid & (kTile - 1)), py = y0 + tid / kTile;
  const bool inside = px < W && py < H;
  const int64_t pix = inside ? (int64_t)py * W + px : 0;

  // every per-pixel load of the tile, issued together
  int sl[KT];
  {
    const uint16_t *__restrict__ slots = slots_all + (int64_t)K * im.pix_off + pix;
#pragma unroll
    for (int k = 0; k < KT; ++k) {
      const int v = (inside && k < K) ? (int)slots[(int64_t)k * HW] : (int)kEmptySlot;
      sl[k] = v == (int)kEmptySlot ? -1 : v;
    }
    const float2 ax = inside ? aux_all[im.pix_off + pix] : make_float2(0.f, 0.f);
    float gv[NC];
    float gc = 0.f;
    if constexpr (L1) {
      const float2 rec = inside ? l1_rec[im.pix_off + pix] : make_float2(0.f, 0.f);
      const float inv_count = (float)(1.0 / ((double)n * (double)HW));
      const uint32_t codes = __float_as_uint(rec.y);
#pragma unroll
      for (int ch = 0; ch < NC; ++ch) {
        const int sgn = (int)(codes << (30 - 2 * ch)) >> 30;  // 2-bit field, sign-extended
        gv[ch] = sgn > 0 ? inv_count : (sgn < 0 ? -inv_count : 0.f);
      }
      gc = rec.x;
    } else {
      const float *__restrict__ image = image_all + (int64_t)n * im.pix_off + pix;
      const float *__restrict__ grad_image = grad_image_all + (int64_t)n * im.pix_off + pix;
      float cv[NC];
#pragma unroll
      for (int ch = 0; ch < NC; ++ch) {
        const bool ok = ch < n && inside;
        gv[ch] = ok ? grad_image[(int64_t)ch * HW] : 0.f;
        cv[ch] = ok ? image[(int64_t)ch * HW] : 0.f;
      }
#pragma unroll
      for (int ch = 0; ch < NC; ++ch) gc = fmaf(gv[ch], cv[ch], gc);
    }
    float row[ROW];
#pragma unroll
    for (int ch = 0; ch < NC; ++ch) row[ch] = gv[ch];
    row[NC] = gc;
    row[NC + 1] = ax.x;
    row[NC + 2] = ax.y;
#pragma unroll
    for (int r = NC + 3; r < ROW; ++r) row[r] = 0.f;
    store_px_row<NC>(smem, row);
  }

  adjoint_batches<NC, KT>(smem, start, cnt, x0, y0, sl, vals, src, g32a, g64, params, N, n,
                          part);
  }
}

// Sum over the 16 lanes of a DPP row, into the row's last lane (a fixed tree: shifts by 1, 2, 4
// and 8 within the row).
__device__ __forceinline__ float row_sum16(float v) {
  v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x111, 0xF, 0xF, false));
  v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x112, 0xF, 0xF, false));
  v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x114, 0xF, 0xF, false));
  v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x118, 0xF, 0xF, false));
  return v;
}

// Per Gaussian, the sum of its pair records (contiguous in emit order, one per tile it hits, in
// tile order).  Up to kRowRecords records: one row of 16 lanes; for records of at most four
// float4 columns (n <= 11) lane l adds column l & 3 of records l >> 2, (l >> 2) + 4, ... and the
// four lanes of a column are added with a fixed tree, for wider ones lane l adds whole records
// l, l + 16, ... in that order and the row's lanes are summed with a fixed tree.  More records (a footprint of
// hundreds of tiles, which a fit can grow): the whole workgroup that holds the Gaussian's row,
// thread t adding records t, t + 256, ... in that order, then a fixed shuffle tree per wave and
// the four waves in order.  Every order depends only on the record count, so the result is
// reproducible bit for bit.  The sums become
//   dL/dmu_x = -2 (A G1 + C G2), dL/dmu_y = -2 (B G1 + D G2),
//   dL/dtheta = 2 (u1/u2 - u2/u1) G12, dL/ds_a = -2 u_a G_aa,
// and the colour sums dL/dc.  Every row of grad is written (zeros for a Gaussian that no pixel
// retained, or when the render overflowed and wrote no records).
constexpr int kReduceLanes = 16;
constexpr int kReduceThreads = 256;
constexpr int kReduceRows = kReduceThreads / kReduceLanes;  // Gaussians per workgroup
constexpr uint32_t kRowRecords = 256;

// acc += records t, t + step, t + 2 step, ... (below c), in that order.  stride4: float4s per
// record.
template <int NR>
__device__ __forceinline__ void add_records(const float4 *__restrict__ rec, int stride4,
                                            uint32_t t, uint32_t c, uint32_t step,
                                            float (&acc)[NR]) {
  for (; t < c; t += step) {
#pragma unroll
    for (int q = 0; q < NR / 4; ++q)
      if (q < stride4) {
        const float4 v = rec[(size_t)t * stride4 + q];
        acc[4 * q] += v.x;
        acc[4 * q + 1] += v.y;
        acc[4 * q + 2] += v.z;
        acc[4 * q + 3] += v.w;
      }
  }
}

// Column q (a float4) of the sum of records t, t + step, ... (below c), in that order, with four
// records' loads in flight.
__device__ __forceinline__ float4 column_sum(const float4 *__restrict__ rec, int stride4, int q,
                                             uint32_t t, uint32_t c, uint32_t step) {
  float4 a = make_float4(0.f, 0.f, 0.f, 0.f);
  for (; t + 3 * step < c; t += 4 * step) {
    float4 v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) v[u] = rec[(size_t)(t + u * step) * stride4 + q];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      a.x += v[u].x;
      a.y += v[u].y;
      a.z += v[u].z;
      a.w += v[u].w;
    }
  }
  for (; t < c; t += step) {
    const float4 v = rec[(size_t)t * stride4 + q];
    a.x += v.x;
    a.y += v.y;
    a.z += v.z;
    a.w += v.w;
  }
  return a;
}

template <int NC, int NR>
__device__ __forceinline__ void write_gradient(int i, const float (&acc)[NR],
                                               const float *__restrict__ params,
                                               const float4 *__restrict__ g32a,
                                               const float2 *__restrict__ g32b, int N, int n,
                                               float *__restrict__ grad) {
  const float G1 = acc[0], G2 = acc[1], G11 = acc[2], G22 = acc[3], G12 = acc[4];
  const float4 a = g32a[i];
  const float2 cd = g32b[i];
  const float u1 = 1.0f / params[3 * (size_t)N + i], u2 = 1.0f / params[4 * (size_t)N + i];
  grad[i] = -2.0f * (a.z * G1 + cd.x * G2);
  grad[(size_t)N + i] = -2.0f * (a.w * G1 + cd.y * G2);
  grad[2 * (size_t)N + i] = 2.0f * (u1 / u2 - u2 / u1) * G12;
  grad[3 * (size_t)N + i] = -2.0f * u1 * G11;
  grad[4 * (size_t)N + i] = -2.0f * u2 * G22;
#pragma unroll
  for (int ch = 0; ch < NC; ++ch)
    if (ch < n) grad[(size_t)(5 + ch) * N + i] = acc[5 + ch];
}

// The gradient entries that come from float4 column q of a Gaussian's record sum: column 0 holds
// (G1, G2, G11, G22), the mean and scale entries; column 1 starts with G12, the angle entry;
// entries 5 + ch are the colour sums.
template <int NC>
__device__ __forceinline__ void write_gradient_column(int i, int q, float4 a,
                                                      const float *__restrict__ params,
                                                      const float4 *__restrict__ g32a,
                                                      const float2 *__restrict__ g32b, int N,
                                                      int n, float *__restrict__ grad) {
  const float v[4] = {a.x, a.y, a.z, a.w};
  if (q == 0) {
    const float4 g = g32a[i];
    const float2 cd = g32b[i];
    const float u1 = 1.0f / params[3 * (size_t)N + i], u2 = 1.0f / params[4 * (size_t)N + i];
    grad[i] = -2.0f * (g.z * a.x + cd.x * a.y);
    grad[(size_t)N + i] = -2.0f * (g.w * a.x + cd.y * a.y);
    grad[3 * (size_t)N + i] = -2.0f * u1 * a.z;
    grad[4 * (size_t)N + i] = -2.0f * u2 * a.w;
  } else if (q == 1) {
    const float u1 = 1.0f / params[3 * (size_t)N + i], u2 = 1.0f / params[4 * (size_t)N + i];
    grad[2 * (size_t)N + i] = 2.0f * (u1 / u2 - u2 / u1) * a.x;
  }
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int ch = 4 * q + e - 5;
    if (ch >= 0 && ch < n && ch < NC) grad[(size_t)(5 + ch) * N + i] = v[e];
  }
}

template <int NC>
__global__ __launch_bounds__(kReduceThreads) void grad_reduce_kernel(
    const float *__restrict__ params, const float4 *__restrict__ g32a,
    const float2 *__restrict__ g32b, const uint32_t *__restrict__ counts,
    const int64_t *__restrict__ offsets, int64_t *__restrict__ status,
    const float *__restrict__ part, int N, int n, float *__restrict__ grad,
    const double2 *__restrict__ l1_part, Images imgs, double *__restrict__ loss_out,
    const unsigned long long *__restrict__ group_part, int groups) {
  constexpr int NR = (5 + NC + 3) & ~3;
  static_assert(kReduceThreads == 256, "sum_group_stats takes one workgroup of 256 threads");
  if (group_part && blockIdx.x == 0) sum_group_stats(group_part, groups, 0, status);
  if (l1_part && (int)blockIdx.x < imgs.B) {  // the loss of image blockIdx.x, first
    __shared__ double s_loss[2 * kLossThreads / 64];
    static_assert(kReduceThreads == kLossThreads, "one thread layout for the loss");
    tile_loss_final(l1_part, imgs.at(blockIdx.x), n, loss_out + 2 * blockIdx.x, s_loss);
  }
  if (N <= 0) return;  // (uniform) a launch for the losses alone
  __shared__ uint32_t s_big[kReduceRows];  // per row: record count if the workgroup reduces it
  __shared__ float s_wave[kReduceThreads / 64][NR];
  const int l = threadIdx.x & (kReduceLanes - 1);
  const int row = threadIdx.x / kReduceLanes;
  const int i = blockIdx.x * kReduceRows + row;
  const bool valid = i < N;
  const int ii = valid ? i : N - 1;
  const int stride4 = part_stride(n) / 4;
  const uint32_t c = (valid && status[kStatOverflow] == 0) ? counts[ii] : 0u;
  const bool big = c > kRowRecords;
  if (l == 0) s_big[row] = big ? c : 0u;
  if (!big && NR <= 16) {
    // records of at most four float4 columns (n <= 11): lane l adds column l & 3 of records
    // l >> 2, (l >> 2) + 4, ... in that order (the row reads four whole records per step), then
    // the four lanes of each column are added with a fixed tree (xor 4, then xor 8), and lane q
    // of the row writes the gradient entries of column q
    const float4 *__restrict__ rec =
        reinterpret_cast<const float4 *>(part + (size_t)offsets[ii] * (4 * stride4));
    const int q = l & 3;
    float4 a = make_float4(0.f, 0.f, 0.f, 0.f);
    if (q < stride4) {
      uint32_t t = (uint32_t)(l >> 2);
      for (; t + 12 < c; t += 16) {  // four records' loads in flight, added in record order
        float4 v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) v[u] = rec[(size_t)(t + 4 * u) * stride4 + q];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          a.x += v[u].x;
          a.y += v[u].y;
          a.z += v[u].z;
          a.w += v[u].w;
        }
      }
      // the last (at most three) records of this lane: loads issued together, added in order
      float4 v[3];
#pragma unroll
      for (int u = 0; u < 3; ++u)
        v[u] = t + 4 * u < c ? rec[(size_t)(t + 4 * u) * stride4 + q]
                             : make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
      for (int u = 0; u < 3; ++u) {
        if (t + 4 * u < c) {
          a.x += v[u].x;
          a.y += v[u].y;
          a.z += v[u].z;
          a.w += v[u].w;
        }
      }
    }
#pragma unroll
    for (int d = 4; d <= 8; d <<= 1) {
      a.x += __shfl_xor(a.x, d, 64);
      a.y += __shfl_xor(a.y, d, 64);
      a.z += __shfl_xor(a.z, d, 64);
      a.w += __shfl_xor(a.w, d, 64);
    }
    if (valid && l < 4) write_gradient_column<NC>(i, q, a, params, g32a, g32b, N, n, grad);
  } else if (!big) {
    const float4 *__restrict__ rec =
        reinterpret_cast<const float4 *>(part + (size_t)offsets[ii] * (4 * stride4));
    float acc[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) acc[r] = 0.f;
    add_records<NR>(rec, stride4, (uint32_t)l, c, kReduceLanes, acc);
#pragma unroll
    for (int r = 0; r < NR; ++r) acc[r] = row_sum16(acc[r]);
    if (valid && l == kReduceLanes - 1) write_gradient<NC>(i, acc, params, g32a, g32b, N, n, grad);
  }
  __syncthreads();
  // Gaussians with long runs: the workgroup, one float4 column at a time (a runtime loop, so the
  // path adds few registers to the kernel), wave sums in LDS, then the waves in order
  for (int r = 0; r < kReduceRows; ++r) {
    const uint32_t cb = s_big[r];
    if (cb == 0) continue;  // uniform over the workgroup
    const int ib = blockIdx.x * kReduceRows + r;
    const float4 *__restrict__ rec =
        reinterpret_cast<const float4 *>(part + (size_t)offsets[ib] * (4 * stride4));
#pragma unroll 1
    for (int q = 0; q < stride4; ++q) {
      float4 a = column_sum(rec, stride4, q, threadIdx.x, cb, kReduceThreads);
#pragma unroll
      for (int d = 32; d >= 1; d >>= 1) {
        a.x += __shfl_down(a.x, d, 64);
        a.y += __shfl_down(a.y, d, 64);
        a.z += __shfl_down(a.z, d, 64);
        a.w += __shfl_down(a.w, d, 64);
      }
      if ((threadIdx.x & 63) == 0) {
        float *wr = &s_wave[threadIdx.x >> 6][4 * q];
        wr[0] = a.x;
        wr[1] = a.y;
        wr[2] = a.z;
        wr[3] = a.w;
      }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      float tot[NR];
#pragma unroll
      for (int q = 0; q < NR; ++q) {
        tot[q] = 0.f;
        if (q < 4 * stride4) {
          tot[q] = s_wave[0][q];
          for (int w = 1; w < kReduceThreads / 64; ++w) tot[q] += s_wave[w][q];
        }
      }
      write_gradient<NC>(ib, tot, params, g32a, g32b, N, n, grad);
    }
    __syncthreads();  // s_wave is reused
  }
}

template <int NC, int KT, bool L1>
hipError_t launch_bwd_t(const int2 *ranges, const uint32_t *vals, const uint32_t *src,
                        const float4 *g32a, const double4 *g64, const float *params,
                        const Dims &d, const Images &imgs, const int *tile_order,
                        const float *image, const float *grad_image, const float2 *l1_rec,
                        const uint16_t *slots, const float2 *aux, float *part, int *queue,
                        hipStream_t s) {
  constexpr size_t lds = bwd_lds<NC, KT>().total;
  if (lds > 65536) {
    hipError_t e = hipFuncSetAttribute((const void *)raster_bwd_kernel<NC, KT, L1>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  const LaunchConfig cfg = launch_config();
  TileQueue q{queue, 0};
  int grid = d.T;
  if (cfg.persistent) {
    int per_cu = cfg.wgs_per_cu;
    if (per_cu <= 0) {
      hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
          &per_cu, (const void *)raster_bwd_kernel<NC, KT, L1>, kRasterThreads, lds);
      if (e != hipSuccess) return e;
    }
    grid = persistent_grid(per_cu, d.T);
    q.persistent = 1;
    hipError_t e = launch_fill_u32(reinterpret_cast<uint32_t *>(queue), 8, 0u, s);
    if (e != hipSuccess) return e;
  }
  raster_bwd_kernel<NC, KT, L1><<<grid, kRasterThreads, lds, s>>>(
      ranges, vals, src, g32a, g64, params, d.N, d.n, d.K, d.T, imgs, tile_order, image,
      grad_image, l1_rec, slots, aux, part, q);
  return hipGetLastError();
}

template <int NC, bool L1>
hipError_t launch_bwd_nc(const int2 *ranges, const uint32_t *vals, const uint32_t *src,
                         const float4 *g32a, const double4 *g64, const float *params,
                         const Dims &d, const Images &imgs, const int *tile_order,
                         const float *image, const float *grad_image, const float2 *l1_rec,
                         const uint16_t *slots, const float2 *aux, float *part, int *queue,
                         hipStream_t s) {
  const int kt = pick_kt(d.K);
#define IGS_BWD_KT(KTV)                                                                         \
  if (kt == KTV)                                                                                \
    return launch_bwd_t<NC, KTV, L1>(ranges, vals, src, g32a, g64, params, d, imgs, tile_order, \
                                     image, grad_image, l1_rec, slots, aux, part, queue, s);
  IGS_FOR_EACH_KT(IGS_BWD_KT)
#undef IGS_BWD_KT
  return hipErrorInvalidValue;
}

}  // namespace

hipError_t launch_raster_bwd(const int2 *ranges, const uint32_t *vals, const uint32_t *src,
                             const float4 *g32a, const double4 *g64, const float *params,
                             const Dims &d, const Images &imgs, const int *tile_order,
                             const float *image, const float *grad_image, const float2 *l1_rec,
                             const uint16_t *slots, const float2 *aux, float *part, int *queue,
                             hipStream_t s) {
  if (l1_rec != nullptr) {
#define IGS_BWD_NC(NCV)                                                                        \
  if (d.n <= NCV)                                                                              \
    return launch_bwd_nc<NCV, true>(ranges, vals, src, g32a, g64, params, d, imgs, tile_order, \
                                    image, grad_image, l1_rec, slots, aux, part, queue, s);
    IGS_BWD_NC(1)
    IGS_BWD_NC(3)
    IGS_BWD_NC(4)
    IGS_BWD_NC(9)
    IGS_BWD_NC(16)
#undef IGS_BWD_NC
    return hipErrorInvalidValue;
  }
#define IGS_BWD_NC(NCV)                                                                        \
  if (d.n <= NCV)                                                                              \
    return launch_bwd_nc<NCV, false>(ranges, vals, src, g32a, g64, params, d, imgs,            \
                                     tile_order, image, grad_image, nullptr, slots, aux, part, \
                                     queue, s);
  IGS_BWD_NC(1)
  IGS_BWD_NC(3)
  IGS_BWD_NC(4)
  IGS_BWD_NC(9)
  IGS_BWD_NC(16)
  IGS_BWD_NC(32)
#undef IGS_BWD_NC
  return hipErrorInvalidValue;
}

hipError_t launch_grad_reduce(const float *params, const float4 *g32a, const float2 *g32b,
                              const uint32_t *counts, const int64_t *offsets, int64_t *status,
                              const float *part, int N, int n, float *grad_params, hipStream_t s,
                              const double2 *l1_part, const Images *imgs, double *loss_out,
                              const uint64_t *group_part, int groups) {
  const int loss_blocks = l1_part ? imgs->B : 0;
  const int blocks = std::max((int)(((int64_t)std::max(N, 0) + kReduceRows - 1) / kReduceRows),
                              std::max(loss_blocks, group_part ? 1 : 0));
  if (blocks <= 0) return hipSuccess;
  const Images none{};
#define IGS_RED_NC(NCV)                                                                        \
  if (n <= NCV) {                                                                              \
    grad_reduce_kernel<NCV><<<blocks, kReduceThreads, 0, s>>>(                                 \
        params, g32a, g32b, counts, offsets, status, part, N, n, grad_params, l1_part,         \
        l1_part ? *imgs : none, loss_out,                                                      \
        reinterpret_cast<const unsigned long long *>(group_part), groups);                     \
    return hipGetLastError();                                                                  \
  }
  IGS_RED_NC(1)
  IGS_RED_NC(3)
  IGS_RED_NC(4)
  IGS_RED_NC(9)
  IGS_RED_NC(16)
  IGS_RED_NC(32)
#undef IGS_RED_NC
  return hipErrorInvalidValue;
}

}  // namespace igs
