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
// Candidate order and wave-level culling are described with rank_tile.
#include <algorithm>

#include "raster_tile.hpp"

namespace igs {
namespace {

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
    int cull, int fb) {
  extern __shared__ __align__(16) unsigned char smem[];
  const FwdLds S = fwd_lds(smem, fb);
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
  const bool single = cnt <= fb;  // whole S_j stays resident for the blend

  double tk[KT];
  rank_tile<KT>(S, start, cnt, single, tx, ty, fx, fy, vals, g32a, g32b, g64, params, N, n, cull,
                tk);

  double l1_abs = 0.0, l1_sq = 0.0;
  if (inside) {
  const int64_t pix = (int64_t)py * W + px;
  // the target of the first channel, loaded now so that it arrives during the blend
  const float *__restrict__ target = L1 ? l1.target + (int64_t)n * im.pix_off + pix : nullptr;
  float tnext = 0.f;
  if constexpr (L1) tnext = target[0];
  const int keff = min(K, cnt);
  int ts[KT], src[KT];
  float w[KT], Z, shift;
  winners<KT, false>(S, single, start, keff, tk, fx, fy, vals, g32a, g64, ts, w, src, Z, shift);
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
        const float c = single ? S.col[src[k] * ncp + ch] : params[(size_t)(5 + ch) * N + src[k]];
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
      for (int k = 0; k < KT; ++k) acc = fmaf(w[k], S.col[src[k] * ncp + ch], acc);
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
    __shared__ double s_red[2 * kWaves];
    const double2 t = tile_loss_sums(l1_abs, l1_sq, s_red);
    if (tid == 0) l1.part[tile] = t;
  }
  __syncthreads();  // LDS is reused by the next tile
  }
}

// Per image: mean |d| and mean d^2 from the per-tile sums of its tiles (fixed order: thread t
// adds tiles t, t + 1024, ... in sequence, then a fixed tree over the threads).
__global__ __launch_bounds__(kLossThreads) void l1_tiles_final_kernel(
    const double2 *__restrict__ part, Images imgs, int n, double *__restrict__ out) {
  __shared__ double sh[2 * kLossThreads / 64];
  tile_loss_final(part, imgs.at(blockIdx.x), n, out + 2 * blockIdx.x, sh);
}

template <int KT, bool L1, bool P>
hipError_t launch_fwd_t(const int2 *ranges, const uint32_t *vals, const float4 *g32a,
                        const float2 *g32b, const double4 *g64, const float *params,
                        const Dims &d, const Images &imgs, const int *tile_order, float *image,
                        uint16_t *slots, float2 *aux, const L1Out &l1, int *queue,
                        hipStream_t s) {
  const LaunchConfig cfg = launch_config();
  const int fb = fwd_batch_of(cfg);
  const size_t lds = fwd_lds_bytes(d.n, fb);
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
      aux, l1, q, cfg.fwd_cull, fb);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_raster_fwd(const int2 *ranges, const uint32_t *vals, const float4 *g32a,
                             const float2 *g32b, const double4 *g64, const float *params,
                             const Dims &d, const Images &imgs, const int *tile_order,
                             float *image, uint16_t *slots, float2 *aux, const float *target,
                             float2 *l1_rec, double2 *l1_part, int *queue, hipStream_t s) {
  const int kt = pick_kt(std::max(d.K, launch_config().k_unroll));
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
  l1_tiles_final_kernel<<<imgs.B, kLossThreads, 0, s>>>(l1_part, imgs, n, loss_out);
  return hipGetLastError();
}

}  // namespace igs
