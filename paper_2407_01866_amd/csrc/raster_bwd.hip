// Adjoint rasterizer (Image-GS Sec. 3.3: gradients flow through the K retained Gaussians, the
// selection itself is held fixed).  One workgroup per 16 x 16 tile, one lane per pixel; the
// top-K slots saved by the forward index into the tile's hit set S_j, which is staged through LDS
// in batches of 256 together with one LDS accumulator row per gradient component.  Lanes add
// their per-(pixel, Gaussian) terms into the LDS rows; each batch then issues at most one global
// atomic per (Gaussian, component).
//
// With alpha_i = w_i / Z, c_r = sum alpha_i c_i and g = dL/dc_r at the pixel:
//   dL/dc_i += alpha_i g
//   dL/dq_i  = -1/2 alpha_i g.(c_i - c_r)
// and, with e = (A dx + B dy, C dx + D dy), q = |e|^2, the geometry enters only through the five
// per-Gaussian sums  G1 = sum gq e1, G2 = sum gq e2, G11 = sum gq e1^2, G22 = sum gq e2^2,
// G12 = sum gq e1 e2  (gq = dL/dq_i at each pixel).  A per-Gaussian pass turns them into
//   dL/dmu_x = -2 (A G1 + C G2)          dL/dmu_y = -2 (B G1 + D G2)
//   dL/dtheta = 2 (u1/u2 - u2/u1) G12    dL/ds_a = -2 u_a G_aa       (u_a = 1/s_a).
#include "raster_common.hpp"

namespace igs {
namespace {

template <int KT>
__global__ __launch_bounds__(kRasterThreads) void raster_bwd_kernel(
    const int2 *__restrict__ ranges, const uint32_t *__restrict__ vals,
    const float4 *__restrict__ g32a, const double4 *__restrict__ g64,
    const float *__restrict__ params, int N, int n, int H, int W, int K, int tiles_x, int T,
    int64_t HW, const float *__restrict__ image, const float *__restrict__ grad_image,
    const uint16_t *__restrict__ slots, const float2 *__restrict__ aux,
    float *__restrict__ gamma, float *__restrict__ grad_params) {
  extern __shared__ __align__(16) unsigned char smem[];
  float2 *s_mu = reinterpret_cast<float2 *>(smem);                        // [kBatch]
  double *s64 = reinterpret_cast<double *>(smem + 8 * kBatch);            // [kBatch][4]
  float *s_col = reinterpret_cast<float *>(smem + 40 * kBatch);           // [n][kBatch]
  float *s_g = s_col + (size_t)n * kBatch;                                // [n][256] per pixel
  float *s_acc = s_g + (size_t)n * kRasterThreads;                        // [5+n][kBatch]

  const int tid = threadIdx.x;
  const int tile = xcd_tile(blockIdx.x, T);
  const int2 rg = ranges[tile];
  const int cnt = rg.y - rg.x;
  if (cnt <= 0) return;  // uniform over the workgroup
  const int tx = tile % tiles_x, ty = tile / tiles_x;
  const int px = tx * kTile + (tid & (kTile - 1)), py = ty * kTile + tid / kTile;
  const bool inside = px < W && py < H;
  const float fx = (float)px + 0.5f, fy = (float)py + 0.5f;
  const int64_t pix = inside ? (int64_t)py * W + px : 0;

  int sl[KT];
#pragma unroll
  for (int k = 0; k < KT; ++k)
    sl[k] = (inside && k < K) ? (int)slots[(int64_t)k * HW + pix] : (int)kEmptySlot;
  const float2 ax = inside ? aux[pix] : make_float2(0.f, 0.f);
  float gc = 0.f;  // g . c_r
  for (int ch = 0; ch < n; ++ch) {
    const float g = inside ? grad_image[(int64_t)ch * HW + pix] : 0.f;
    const float c = inside ? image[(int64_t)ch * HW + pix] : 0.f;
    s_g[ch * kRasterThreads + tid] = g;
    gc = fmaf(g, c, gc);
  }

  for (int base = 0; base < cnt; base += kBatch) {
    const int nb = min(kBatch, cnt - base);
    __syncthreads();
    if (tid < nb) {
      const uint32_t gid = vals[rg.x + base + tid];
      const float4 a = g32a[gid];
      s_mu[tid] = make_float2(a.x, a.y);
      const double4 c = g64[gid];
      s64[4 * tid + 0] = c.x;
      s64[4 * tid + 1] = c.y;
      s64[4 * tid + 2] = c.z;
      s64[4 * tid + 3] = c.w;
      for (int ch = 0; ch < n; ++ch) s_col[ch * kBatch + tid] = params[(size_t)(5 + ch) * N + gid];
    }
    for (int r = 0; r < 5 + n; ++r) s_acc[r * kBatch + tid] = 0.f;
    __syncthreads();
    if (inside) {
#pragma unroll
      for (int k = 0; k < KT; ++k) {
        const int j = sl[k] - base;
        if (sl[k] != (int)kEmptySlot && j >= 0 && j < nb) {
          double e1, e2;
          const double q = quad_form64(fx, fy, s_mu[j].x, s_mu[j].y, s64[4 * j + 0],
                                       s64[4 * j + 1], s64[4 * j + 2], s64[4 * j + 3], e1, e2);
          const float alpha = blend_weight(q, ax.x) * ax.y;
          float dot = -gc;
          for (int ch = 0; ch < n; ++ch)
            dot = fmaf(s_g[ch * kRasterThreads + tid], s_col[ch * kBatch + j], dot);
          const float gq = -0.5f * alpha * dot;
          const float f1 = (float)e1, f2 = (float)e2;
          const float g1 = gq * f1, g2 = gq * f2;
          atomicAdd(&s_acc[0 * kBatch + j], g1);
          atomicAdd(&s_acc[1 * kBatch + j], g2);
          atomicAdd(&s_acc[2 * kBatch + j], g1 * f1);
          atomicAdd(&s_acc[3 * kBatch + j], g2 * f2);
          atomicAdd(&s_acc[4 * kBatch + j], g1 * f2);
          for (int ch = 0; ch < n; ++ch)
            atomicAdd(&s_acc[(5 + ch) * kBatch + j], alpha * s_g[ch * kRasterThreads + tid]);
        }
      }
    }
    __syncthreads();
    if (tid < nb) {
      const uint32_t gid = vals[rg.x + base + tid];
      for (int r = 0; r < 5; ++r) {
        const float v = s_acc[r * kBatch + tid];
        if (v != 0.f) unsafeAtomicAdd(&gamma[(size_t)r * N + gid], v);
      }
      for (int ch = 0; ch < n; ++ch) {
        const float v = s_acc[(5 + ch) * kBatch + tid];
        if (v != 0.f) unsafeAtomicAdd(&grad_params[(size_t)(5 + ch) * N + gid], v);
      }
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

}  // namespace

hipError_t launch_raster_bwd(const int2 *ranges, const uint32_t *vals, const float4 *g32a,
                             const double4 *g64, const float *params, const Dims &d,
                             const float *image, const float *grad_image, const uint16_t *slots,
                             const float2 *aux, float *gamma, float *grad_params, hipStream_t s) {
  const size_t lds = 40 * kBatch + (size_t)d.n * kBatch * 4 + (size_t)d.n * kRasterThreads * 4 +
                     (size_t)(5 + d.n) * kBatch * 4;
  const int kt = pick_kt(d.K);
#define IGS_LAUNCH_BWD(KTV)                                                                     \
  if (kt == KTV) {                                                                              \
    if (lds > 65536) {                                                                          \
      hipError_t e = hipFuncSetAttribute((const void *)raster_bwd_kernel<KTV>,                  \
                                         hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds); \
      if (e != hipSuccess) return e;                                                            \
    }                                                                                           \
    raster_bwd_kernel<KTV><<<d.T, kRasterThreads, lds, s>>>(                                    \
        ranges, vals, g32a, g64, params, d.N, d.n, d.H, d.W, d.K, d.tiles_x, d.T, d.HW, image,  \
        grad_image, slots, aux, gamma, grad_params);                                            \
    return hipGetLastError();                                                                   \
  }
  IGS_FOR_EACH_KT(IGS_LAUNCH_BWD)
#undef IGS_LAUNCH_BWD
  return hipErrorInvalidValue;
}

hipError_t launch_grad_finalize(const float *params, const float4 *g32a, const float2 *g32b,
                                const float *gamma, int N, float *grad_params, hipStream_t s) {
  if (N <= 0) return hipSuccess;
  grad_finalize_kernel<<<(N + 255) / 256, 256, 0, s>>>(params, g32a, g32b, gamma, N, grad_params);
  return hipGetLastError();
}

}  // namespace igs
