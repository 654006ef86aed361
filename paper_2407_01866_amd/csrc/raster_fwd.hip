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
#include "raster_common.hpp"

namespace igs {
namespace {

constexpr uint32_t kKeyBias = 0x00800000u;
constexpr float kQMax = 1e38f;

__device__ __forceinline__ double rank_key(float q, int slot) {
  return __hiloint2double((int)(__float_as_uint(fminf(q, kQMax)) + kKeyBias), slot);
}
__device__ __forceinline__ int key_slot(double k) { return __double2loint(k); }
__device__ __forceinline__ bool key_valid(double k) {
  return (uint32_t)__double2hiint(k) < 0x7F000000u;  // not the +inf sentinel
}

// Sorted insertion of a key (ascending, unique keys): a compare-exchange down the list.
template <int KT>
__device__ __forceinline__ void topk_insert(double (&tk)[KT], double key) {
#pragma unroll
  for (int k = 0; k < KT; ++k) {
    const double hi = __builtin_fmax(key, tk[k]);
    tk[k] = __builtin_fmin(key, tk[k]);
    key = hi;
  }
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

__device__ __forceinline__ double2 block_sum2(double a, double b, double *sh) {
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
    for (int k = 0; k < kRasterThreads / 64; ++k) {
      t.x += sh[2 * k];
      t.y += sh[2 * k + 1];
    }
  return t;  // valid in thread 0
}

template <int KT, bool L1>
__global__ __launch_bounds__(kRasterThreads) void raster_fwd_kernel(
    const int2 *__restrict__ ranges, const uint32_t *__restrict__ vals,
    const float4 *__restrict__ g32a, const float2 *__restrict__ g32b,
    const double4 *__restrict__ g64, const float *__restrict__ params, int N, int n, int K, int T,
    Images imgs, const int *__restrict__ tile_order, float *__restrict__ image_all,
    uint16_t *__restrict__ slots_all, float2 *__restrict__ aux_all, L1Out l1) {
  extern __shared__ __align__(16) unsigned char smem[];
  float4 *s_geo = reinterpret_cast<float4 *>(smem);                    // mu_x, mu_y, A, B
  float2 *s_cd = reinterpret_cast<float2 *>(smem + 16 * kBatch);       // C, D
  double *s64 = reinterpret_cast<double *>(smem + 24 * kBatch);        // [kBatch][4] A,B,C,D
  float *s_col = reinterpret_cast<float *>(smem + 56 * kBatch);        // [n][kBatch]

  const int tid = threadIdx.x;
  const int tile = __builtin_amdgcn_readfirstlane(tile_order ? tile_order[blockIdx.x]
                                                             : xcd_tile(blockIdx.x, T));
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
  const bool single = cnt <= kBatch;  // whole S_j stays resident for the blend

  double tk[KT];
#pragma unroll
  for (int k = 0; k < KT; ++k) tk[k] = __longlong_as_double(0x7FF0000000000000ll);  // +inf

  for (int base = 0; base < cnt; base += kBatch) {
    const int nb = min(kBatch, cnt - base);
    __syncthreads();
    if (tid < nb) {
      const uint32_t gid = vals[start + base + tid];
      s_geo[tid] = g32a[gid];
      s_cd[tid] = g32b[gid];
      if (single) {
        const double4 c = g64[gid];
        s64[4 * tid + 0] = c.x;
        s64[4 * tid + 1] = c.y;
        s64[4 * tid + 2] = c.z;
        s64[4 * tid + 3] = c.w;
        for (int ch = 0; ch < n; ++ch) s_col[ch * kBatch + tid] = params[(size_t)(5 + ch) * N + gid];
      }
    }
    __syncthreads();
    int j = 0;
    // four candidates per step: their loads and quadratic forms overlap before the insertions
    for (; j + 4 <= nb; j += 4) {
      double key[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const float4 a = s_geo[j + u];
        const float2 b = s_cd[j + u];
        const float dx = fx - a.x, dy = fy - a.y;
        const float e1 = fmaf(a.z, dx, a.w * dy);
        const float e2 = fmaf(b.x, dx, b.y * dy);
        key[u] = rank_key(fmaf(e1, e1, e2 * e2), base + j + u);
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
        if (key[u] < tk[KT - 1]) topk_insert<KT>(tk, key[u]);
    }
    for (; j < nb; ++j) {
      const float4 a = s_geo[j];
      const float2 b = s_cd[j];
      const float dx = fx - a.x, dy = fy - a.y;
      const float e1 = fmaf(a.z, dx, a.w * dy);
      const float e2 = fmaf(b.x, dx, b.y * dy);
      const double key = rank_key(fmaf(e1, e1, e2 * e2), base + j);
      if (key < tk[KT - 1]) topk_insert<KT>(tk, key);
    }
  }

  if (!L1 && !inside) return;
  double l1_abs = 0.0, l1_sq = 0.0;
  if (inside) {
  const int64_t pix = (int64_t)py * W + px;
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
        mx = s_geo[slot].x;
        my = s_geo[slot].y;
        src[k] = slot;
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
      }
      double e1, e2;
      const double q = quad_form64(fx, fy, mx, my, A, B, C, D, e1, e2);
      if (k == 0) shift = (float)q;
      w[k] = blend_weight(q, shift);
      Z += w[k];
    }
  }
  const float invZ = Z > 0.f ? 1.0f / Z : 0.0f;
  const float *__restrict__ target = L1 ? l1.target + (int64_t)n * im.pix_off : nullptr;
  const float inv_count = L1 ? (float)(1.0 / ((double)n * (double)HW)) : 0.f;
  float gc = 0.f;
  uint32_t codes = 0;
  for (int ch = 0; ch < n; ++ch) {
    float acc = 0.f;
#pragma unroll
    for (int k = 0; k < KT; ++k) {
      if (k < keff && ts[k] >= 0) {
        const float c = single ? s_col[ch * kBatch + src[k]] : params[(size_t)(5 + ch) * N + src[k]];
        acc = fmaf(w[k], c, acc);
      }
    }
    const float v = acc * invZ;
    image[(int64_t)ch * HW + pix] = v;
    if constexpr (L1) {
      const double d = (double)v - (double)target[(int64_t)ch * HW + pix];
      const float g = d > 0.0 ? inv_count : (d < 0.0 ? -inv_count : 0.f);
      codes |= (d > 0.0 ? 1u : (d < 0.0 ? 3u : 0u)) << (2 * ch);
      gc = fmaf(g, v, gc);
      l1_abs += fabs(d);
      l1_sq += d * d;
    }
  }
  if constexpr (L1) l1.rec[im.pix_off + pix] = make_float2(gc, __uint_as_float(codes));
#pragma unroll
  for (int k = 0; k < KT; ++k)
    if (k < K)
      slots[(int64_t)k * HW + pix] = (k < keff && ts[k] >= 0) ? (uint16_t)min(ts[k], 0xFFFF) : kEmptySlot;
  aux[pix] = make_float2(shift, invZ);
  }
  if (L1) {
    __syncthreads();  // LDS staging area is reused for the reduction
    const double2 t = block_sum2(l1_abs, l1_sq, reinterpret_cast<double *>(smem));
    if (tid == 0) l1.part[tile] = t;
  }
}

// Per image: mean |d| and mean d^2 from the per-tile sums of its tiles (fixed order).
__global__ __launch_bounds__(256) void l1_tiles_final_kernel(const double2 *__restrict__ part,
                                                             Images imgs, int n,
                                                             double *__restrict__ out) {
  __shared__ double sh[8];
  const ImageDesc im = imgs.at(blockIdx.x);
  const int T = im.tiles_x * im.tiles_y;
  double a = 0.0, b = 0.0;
  for (int t = threadIdx.x; t < T; t += blockDim.x) {
    const double2 v = part[im.tile_off + t];
    a += v.x;
    b += v.y;
  }
  const double2 s = block_sum2(a, b, sh);
  if (threadIdx.x == 0) {
    const double inv = 1.0 / ((double)n * (double)im.H * (double)im.W);
    out[2 * blockIdx.x] = s.x * inv;
    out[2 * blockIdx.x + 1] = s.y * inv;
  }
}

}  // namespace

hipError_t launch_raster_fwd(const int2 *ranges, const uint32_t *vals, const float4 *g32a,
                             const float2 *g32b, const double4 *g64, const float *params,
                             const Dims &d, const Images &imgs, const int *tile_order,
                             float *image, uint16_t *slots, float2 *aux, const float *target,
                             float2 *l1_rec, double2 *l1_part, hipStream_t s) {
  const size_t lds = 56 * kBatch + (size_t)d.n * kBatch * sizeof(float);
  const int kt = pick_kt(d.K);
  const L1Out l1{target, l1_rec, l1_part};
  const bool fused = target != nullptr;
#define IGS_LAUNCH_FWD(KTV)                                                                    \
  if (kt == KTV) {                                                                             \
    if (fused)                                                                                 \
      raster_fwd_kernel<KTV, true><<<d.T, kRasterThreads, lds, s>>>(                           \
          ranges, vals, g32a, g32b, g64, params, d.N, d.n, d.K, d.T, imgs, tile_order, image,  \
          slots, aux, l1);                                                                     \
    else                                                                                       \
      raster_fwd_kernel<KTV, false><<<d.T, kRasterThreads, lds, s>>>(                          \
          ranges, vals, g32a, g32b, g64, params, d.N, d.n, d.K, d.T, imgs, tile_order, image,  \
          slots, aux, l1);                                                                     \
    return hipGetLastError();                                                                  \
  }
  IGS_FOR_EACH_KT(IGS_LAUNCH_FWD)
#undef IGS_LAUNCH_FWD
  return hipErrorInvalidValue;
}

hipError_t launch_l1_tiles_final(const double2 *l1_part, const Images &imgs, int n,
                                 double *loss_out, hipStream_t s) {
  l1_tiles_final_kernel<<<imgs.B, 256, 0, s>>>(l1_part, imgs, n, loss_out);
  return hipGetLastError();
}

}  // namespace igs
