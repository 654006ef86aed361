// Single-pass fitting kernel for the L1 loss (Image-GS Sec. 3.2 Eq. 5, Sec. 3.3, with the mean
// absolute error of Sec. 4.1): one workgroup per 16 x 16 tile renders the tile, compares it with
// the target and runs the adjoint of that comparison for the same tile, so that nothing per pixel
// goes through HBM: no image, retained slots, blend normalization or loss record is written or
// read back.  What leaves the workgroup is the tile's loss sums and one gradient record per
// (tile, Gaussian) pair, which the adjoint's fixed-order reduction turns into the gradient.
//
// The three phases are those of the two-pass path, in the same arithmetic:
//   1. rank_tile / winners: the lane's top-K of S_j and their double-precision blend weights;
//   2. the normalized colour per channel, d = c_r - c_t, g = sign(d) / (n H W), g . c_r and the
//      loss sums, all kept in registers; the pixel's adjoint row (g, g . c_r, shift, 1/Z) and its
//      retained slots then replace the forward's LDS;
//   3. adjoint_batches: the per-pair gradient records.
// Loss, records and hence the gradient are therefore bit for bit those of the fused forward +
// adjoint pair.  LDS is the larger of the two phases' and the register budget the adjoint's.
#include <algorithm>

#include "raster_tile.hpp"

namespace igs {
namespace {

template <int NC, int KT>
__host__ __device__ constexpr size_t fit_lds_bytes(int fb) {
  return fwd_lds_bytes(NC, fb) > bwd_lds<NC, KT>().total ? fwd_lds_bytes(NC, fb)
                                                         : (size_t)bwd_lds<NC, KT>().total;
}

// Register budget: five waves per SIMD (<= 96 VGPRs; the LDS of up to n = 9 also lets five
// workgroups share a CU) where that costs at most a few spills outside the per-candidate and
// per-item loops, else four (<= 128) or two.
__host__ __device__ constexpr int fit_min_waves(int nc, int kt) {
  return (nc <= 9 && kt <= 10) ? 5 : ((nc + kt <= 25 && !(nc >= 16 && kt >= 4)) ? 4 : 2);
}

// P: persistent scheduling, resident workgroups taking tiles from the shared queue (a
// compile-time choice so that the one-workgroup-per-tile kernel keeps the register budget of
// straight-line code).
template <int NC, int KT, bool P>
__global__ __launch_bounds__(kRasterThreads)
__attribute__((amdgpu_waves_per_eu(fit_min_waves(NC, KT)))) void raster_fit_kernel(
    const int2 *__restrict__ ranges, const uint32_t *__restrict__ vals,
    const uint32_t *__restrict__ src, const float4 *__restrict__ g32a,
    const float2 *__restrict__ g32b, const double4 *__restrict__ g64,
    const float *__restrict__ params, int N, int n, int K, int T, Images imgs,
    const int *__restrict__ tile_order, const float *__restrict__ target_all,
    double2 *__restrict__ loss_part, float *__restrict__ part, TileQueue queue, int cull,
    int fb) {
  constexpr int ROW = px_row<NC>();
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ double s_red[2 * kWaves];
  const FwdLds S = fwd_lds(smem, fb);
  const int tid = threadIdx.x;
  int idx = 0;
  if (!P) queue.persistent = 0;
  for (bool first = true; next_tile_index(queue, T, first, idx); first = false) {
  const int tile = __builtin_amdgcn_readfirstlane(tile_order ? tile_order[idx] : xcd_tile(idx, T));
  const ImageDesc im = imgs.by_tile(tile);
  const int W = im.W, H = im.H;
  const int64_t HW = (int64_t)H * W;
  const int lt = tile - im.tile_off;
  const int tx = lt % im.tiles_x, ty = lt / im.tiles_x;
  const int x0 = tx * kTile, y0 = ty * kTile;
  const int px = x0 + (tid & (kTile - 1)), py = y0 + tid / kTile;
  const bool inside = px < W && py < H;
  const float fx = (float)px + 0.5f, fy = (float)py + 0.5f;
  const int2 rg = ranges[tile];
  const int start = __builtin_amdgcn_readfirstlane(rg.x);
  const int cnt = __builtin_amdgcn_readfirstlane(rg.y - rg.x);
  const bool single = cnt <= fb;

  double tk[KT];
  rank_tile<KT>(S, start, cnt, single, tx, ty, fx, fy, vals, g32a, g32b, g64, params, N, n, cull,
                tk);

  double l1_abs = 0.0, l1_sq = 0.0;
  float row[ROW];
  int sl[KT];
#pragma unroll
  for (int r = 0; r < ROW; ++r) row[r] = 0.f;
#pragma unroll
  for (int k = 0; k < KT; ++k) sl[k] = -1;  // the slots never leave the workgroup: full width
  if (inside) {
    const int64_t pix = (int64_t)py * W + px;
    const float *__restrict__ target = target_all + (int64_t)n * im.pix_off + pix;
    float tv[NC];  // the target, loaded now so that it arrives during the blend
#pragma unroll
    for (int ch = 0; ch < NC; ++ch) tv[ch] = ch < n ? target[(int64_t)ch * HW] : 0.f;
    const int keff = min(K, cnt);
    int ts[KT], srcg[KT];
    float w[KT], Z, shift;
    winners<KT, true>(S, single, start, keff, tk, fx, fy, vals, g32a, g64, ts, w, srcg, Z,
                      shift);
    const float invZ = Z > 0.f ? 1.0f / Z : 0.0f;
    const float inv_count = (float)(1.0 / ((double)n * (double)HW));
    // channel sums in rank order; entries past the retained ones have weight 0 and index 0 (a
    // valid member when cnt > 0), so they add exactly 0.  LDS and global colour reads stay in
    // separate loops (a read through a pointer that may be either miscompiles for gfx950).
    float acc[NC];
#pragma unroll
    for (int ch = 0; ch < NC; ++ch) acc[ch] = 0.f;
    if (cnt > 0 && single) {
#pragma unroll
      for (int ch = 0; ch < NC; ++ch)
        if (ch < n) {
#pragma unroll
          for (int k = 0; k < KT; ++k) acc[ch] = fmaf(w[k], S.col[srcg[k] * n + ch], acc[ch]);
        }
    } else if (cnt > 0) {
#pragma unroll
      for (int ch = 0; ch < NC; ++ch)
        if (ch < n) {
#pragma unroll
          for (int k = 0; k < KT; ++k)
            acc[ch] = fmaf(w[k], params[(size_t)(5 + ch) * N + srcg[k]], acc[ch]);
        }
    }
    float gc = 0.f;
#pragma unroll
    for (int ch = 0; ch < NC; ++ch) {
      if (ch < n) {
        const float v = acc[ch] * invZ;
        const double d = (double)v - (double)tv[ch];
        const float g = d > 0.0 ? inv_count : (d < 0.0 ? -inv_count : 0.f);
        gc = fmaf(g, v, gc);
        l1_abs += fabs(d);
        l1_sq += d * d;
        row[ch] = g;
      }
    }
    row[NC] = gc;
    row[NC + 1] = shift;
    row[NC + 2] = invZ;
#pragma unroll
    for (int k = 0; k < KT; ++k)
      if (k < K && k < keff && ts[k] >= 0) sl[k] = ts[k];
  }
  // the tile's loss sums first, so that they hold no registers through the adjoint
  const double2 t = tile_loss_sums(l1_abs, l1_sq, s_red);
  if (tid == 0) loss_part[tile] = t;
  __syncthreads();  // the forward's LDS is dead
  store_px_row<NC>(smem, row);
  adjoint_batches<NC, KT>(smem, start, cnt, x0, y0, sl, vals, src, g32a, g64, params, N, n,
                          part);
  }
}

template <int NC, int KT, bool P>
hipError_t launch_fit_t(const int2 *ranges, const uint32_t *vals, const uint32_t *src,
                        const float4 *g32a, const float2 *g32b, const double4 *g64,
                        const float *params, const Dims &d, const Images &imgs,
                        const int *tile_order, const float *target, double2 *loss_part,
                        float *part, int *queue, hipStream_t s) {
  const LaunchConfig cfg = launch_config();
  const int fb = fwd_batch_of(cfg);
  const size_t lds = fit_lds_bytes<NC, KT>(fb);
  if (lds > 65536) {
    hipError_t e = hipFuncSetAttribute((const void *)raster_fit_kernel<NC, KT, P>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  if (d.T <= 0) return hipSuccess;
  TileQueue q{queue, 0};
  int grid = d.T;
  if (P) {
    int per_cu = cfg.wgs_per_cu;
    if (per_cu <= 0) {
      hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
          &per_cu, (const void *)raster_fit_kernel<NC, KT, P>, kRasterThreads, lds);
      if (e != hipSuccess) return e;
    }
    grid = persistent_grid(per_cu, d.T);
    q.persistent = 1;
    hipError_t e = launch_fill_u32(reinterpret_cast<uint32_t *>(queue), 8, 0u, s);
    if (e != hipSuccess) return e;
  }
  raster_fit_kernel<NC, KT, P><<<grid, kRasterThreads, lds, s>>>(
      ranges, vals, src, g32a, g32b, g64, params, d.N, d.n, d.K, d.T, imgs, tile_order, target,
      loss_part, part, q, cfg.fwd_cull, fb);
  return hipGetLastError();
}

template <int NC>
hipError_t launch_fit_nc(const int2 *ranges, const uint32_t *vals, const uint32_t *src,
                         const float4 *g32a, const float2 *g32b, const double4 *g64,
                         const float *params, const Dims &d, const Images &imgs,
                         const int *tile_order, const float *target, double2 *loss_part,
                         float *part, int *queue, hipStream_t s) {
  const LaunchConfig cfg = launch_config();
  const int kt = pick_kt(std::max(d.K, cfg.k_unroll));
  const bool pers = cfg.persistent != 0;
#define IGS_FIT_KT(KTV)                                                                         \
  if (kt == KTV) {                                                                              \
    if (pers)                                                                                   \
      return launch_fit_t<NC, KTV, true>(ranges, vals, src, g32a, g32b, g64, params, d, imgs,   \
                                         tile_order, target, loss_part, part, queue, s);        \
    return launch_fit_t<NC, KTV, false>(ranges, vals, src, g32a, g32b, g64, params, d, imgs,    \
                                        tile_order, target, loss_part, part, queue, s);         \
  }
  IGS_FOR_EACH_KT(IGS_FIT_KT)
#undef IGS_FIT_KT
  return hipErrorInvalidValue;
}

}  // namespace

hipError_t launch_raster_fit(const int2 *ranges, const uint32_t *vals, const uint32_t *src,
                             const float4 *g32a, const float2 *g32b, const double4 *g64,
                             const float *params, const Dims &d, const Images &imgs,
                             const int *tile_order, const float *target, double2 *loss_part,
                             float *part, int *queue, hipStream_t s) {
#define IGS_FIT_NC(NCV)                                                                     \
  if (d.n <= NCV)                                                                           \
    return launch_fit_nc<NCV>(ranges, vals, src, g32a, g32b, g64, params, d, imgs, tile_order, \
                              target, loss_part, part, queue, s);
  IGS_FIT_NC(1)
  IGS_FIT_NC(3)
  IGS_FIT_NC(4)
  IGS_FIT_NC(9)
  IGS_FIT_NC(16)
#undef IGS_FIT_NC
  return hipErrorInvalidValue;
}

}  // namespace igs
