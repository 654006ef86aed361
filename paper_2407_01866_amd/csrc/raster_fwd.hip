// Forward rasterizer (Image-GS Sec. 3.2, Eq. 5): one workgroup per 16 x 16 tile, one lane per
// pixel.  The tile's hit set S_j is staged through LDS in batches of 256 Gaussians; every lane
// ranks every member by its float32 Mahalanobis form q and keeps a register-resident sorted top-K
// of (q, slot), slot being the member's position in S_j (ties keep the earlier slot, i.e. the
// lower Gaussian index).  The K winners are then re-evaluated in double so that the normalized
// blend weights exp(-(q_i - q_min)/2) carry no float32 cancellation error.
#include "raster_common.hpp"

namespace igs {
namespace {

// Insert (q, s) into the ascending list; once a position takes the new entry every later
// position shifts down by one (the carry), so equal keys keep their arrival order.
template <int KT>
__device__ __forceinline__ void topk_insert(float (&tq)[KT], int (&ts)[KT], float q, int s) {
  bool carry = false;
#pragma unroll
  for (int k = 0; k < KT; ++k) {
    const bool take = carry || (q < tq[k]);
    const float oq = tq[k];
    const int os = ts[k];
    tq[k] = take ? q : oq;
    ts[k] = take ? s : os;
    q = take ? oq : q;
    s = take ? os : s;
    carry = take;
  }
}

template <int KT>
__global__ __launch_bounds__(kRasterThreads) void raster_fwd_kernel(
    const int2 *__restrict__ ranges, const uint32_t *__restrict__ vals,
    const float4 *__restrict__ g32a, const float2 *__restrict__ g32b,
    const double4 *__restrict__ g64, const float *__restrict__ params, int N, int n, int H,
    int W, int K, int tiles_x, int T, int64_t HW, float *__restrict__ image,
    uint16_t *__restrict__ slots, float2 *__restrict__ aux, int64_t *__restrict__ status) {
  extern __shared__ __align__(16) unsigned char smem[];
  float4 *s_geo = reinterpret_cast<float4 *>(smem);                    // mu_x, mu_y, A, B
  float2 *s_cd = reinterpret_cast<float2 *>(smem + 16 * kBatch);       // C, D
  double *s64 = reinterpret_cast<double *>(smem + 24 * kBatch);        // [kBatch][4] A,B,C,D
  float *s_col = reinterpret_cast<float *>(smem + 56 * kBatch);        // [n][kBatch]

  const int tid = threadIdx.x;
  const int tile = xcd_tile(blockIdx.x, T);
  const int tx = tile % tiles_x, ty = tile / tiles_x;
  const int px = tx * kTile + (tid & (kTile - 1)), py = ty * kTile + tid / kTile;
  const bool inside = px < W && py < H;
  const float fx = (float)px + 0.5f, fy = (float)py + 0.5f;
  const int2 rg = ranges[tile];
  const int cnt = rg.y - rg.x;
  const bool single = cnt <= kBatch;  // whole S_j stays resident for the blend

  if (tid == 0 && cnt > 0) {
    atomicMax(reinterpret_cast<unsigned long long *>(&status[kStatMaxList]),
              (unsigned long long)cnt);
    if (cnt > 0xFFFF) status[kStatSlotOverflow] = 1;
    const long long npx = (long long)(min(W - tx * kTile, kTile) * min(H - ty * kTile, kTile));
    atomicAdd(reinterpret_cast<unsigned long long *>(&status[kStatEvalsFwd]),
              (unsigned long long)(npx * cnt));
    atomicAdd(reinterpret_cast<unsigned long long *>(&status[kStatEvalsBwd]),
              (unsigned long long)(npx * min(K, cnt)));
  }

  float tq[KT];
  int ts[KT];
#pragma unroll
  for (int k = 0; k < KT; ++k) {
    tq[k] = INFINITY;
    ts[k] = -1;
  }

  for (int base = 0; base < cnt; base += kBatch) {
    const int nb = min(kBatch, cnt - base);
    __syncthreads();
    if (tid < nb) {
      const uint32_t gid = vals[rg.x + base + tid];
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
    for (int j = 0; j < nb; ++j) {
      const float4 a = s_geo[j];
      const float2 b = s_cd[j];
      const float dx = fx - a.x, dy = fy - a.y;
      const float e1 = fmaf(a.z, dx, a.w * dy);
      const float e2 = fmaf(b.x, dx, b.y * dy);
      const float q = fmaf(e1, e1, e2 * e2);
      if (q < tq[KT - 1]) topk_insert<KT>(tq, ts, q, base + j);
    }
  }

  if (!inside) return;
  const int64_t pix = (int64_t)py * W + px;
  const int keff = min(K, cnt);
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
        const uint32_t gid = vals[rg.x + slot];
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
  for (int ch = 0; ch < n; ++ch) {
    float acc = 0.f;
#pragma unroll
    for (int k = 0; k < KT; ++k) {
      if (k < keff && ts[k] >= 0) {
        const float c = single ? s_col[ch * kBatch + src[k]] : params[(size_t)(5 + ch) * N + src[k]];
        acc = fmaf(w[k], c, acc);
      }
    }
    image[(int64_t)ch * HW + pix] = acc * invZ;
  }
#pragma unroll
  for (int k = 0; k < KT; ++k)
    if (k < K)
      slots[(int64_t)k * HW + pix] = (k < keff && ts[k] >= 0) ? (uint16_t)min(ts[k], 0xFFFF) : kEmptySlot;
  aux[pix] = make_float2(shift, invZ);
}

}  // namespace

hipError_t launch_raster_fwd(const int2 *ranges, const uint32_t *vals, const float4 *g32a,
                             const float2 *g32b, const double4 *g64, const float *params,
                             const Dims &d, float *image, uint16_t *slots, float2 *aux,
                             int64_t *status, hipStream_t s) {
  const size_t lds = 56 * kBatch + (size_t)d.n * kBatch * sizeof(float);
  const int kt = pick_kt(d.K);
#define IGS_LAUNCH_FWD(KTV)                                                                    \
  if (kt == KTV) {                                                                             \
    raster_fwd_kernel<KTV><<<d.T, kRasterThreads, lds, s>>>(ranges, vals, g32a, g32b, g64,     \
                                                            params, d.N, d.n, d.H, d.W, d.K,   \
                                                            d.tiles_x, d.T, d.HW, image,       \
                                                            slots, aux, status);               \
    return hipGetLastError();                                                                  \
  }
  IGS_FOR_EACH_KT(IGS_LAUNCH_FWD)
#undef IGS_LAUNCH_FWD
  return hipErrorInvalidValue;
}

}  // namespace igs
