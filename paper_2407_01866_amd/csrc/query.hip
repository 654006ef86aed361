// Decoding side of the representation (Image-GS Sec. 1, Sec. 3.2, Sec. 4.1):
//
// * random access: the colour of the representation at arbitrary points of the image plane, each
//   evaluated on its own with the renderer's rule (the point's tile j, every member of S_j ranked
//   by q at the point, the top K blended by Eq. 5), using the tile lists of a binning pass.  The
//   ranking and the blend are the forward rasterizer's operations, so at a pixel centre a query
//   returns exactly the rendered pixel;
// * storage in float16 (Sec. 4.1: the trained attributes are quantized to float16): conversion
//   of the fitter's parameters (normalized mean, rotation, inverse scales, colour) to float16
//   with round-to-nearest-even, and decoding of a prefix of a stored set, its first N_prefix
//   Gaussians, into the renderer's float32 units.  Gaussians added by the error-guided schedule
//   are appended, so every prefix boundary of the schedule is a level of detail.
#include "raster_common.hpp"

#include <hip/hip_fp16.h>

#include <algorithm>

namespace igs {
namespace {

constexpr int kQueryThreads = 256;

// One thread per point.  Points outside [0, W) x [0, H) (or not finite) decode to 0.
template <int KT>
__global__ __launch_bounds__(kQueryThreads) void query_kernel(
    const float *__restrict__ params, int N, int n, int H, int W, int K, int tiles_x,
    int tiles_y, const int2 *__restrict__ ranges, const uint32_t *__restrict__ vals,
    const float4 *__restrict__ g32a, const float2 *__restrict__ g32b,
    const double4 *__restrict__ g64, const float *__restrict__ pts, int M,
    float *__restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= M) return;
  const float fx = pts[i], fy = pts[(size_t)M + i];
  const bool inside = fx >= 0.f && fx < (float)W && fy >= 0.f && fy < (float)H;
  int start = 0, cnt = 0;
  if (inside) {
    const int tx = min((int)fx / kTile, tiles_x - 1), ty = min((int)fy / kTile, tiles_y - 1);
    const int2 rg = ranges[ty * tiles_x + tx];
    start = rg.x;
    cnt = rg.y - rg.x;
  }
  double tk[KT];
#pragma unroll
  for (int k = 0; k < KT; ++k) tk[k] = kKeyEmpty;
  for (int s = 0; s < cnt; ++s) {
    const uint32_t gid = vals[start + s];
    const float4 a = g32a[gid];
    const float2 b = g32b[gid];
    const double key = rank_key(quad_q32(a.z, a.w, b.x, b.y, fx - a.x, fy - a.y), s);
    if (key < tk[KT - 1]) topk_insert<KT>(tk, key);
  }
  // blend: the winners re-evaluated in double, weights relative to the best, in rank order
  const int keff = min(K, cnt);
  float w[KT];
  uint32_t src[KT];
  float Z = 0.f, shift = 0.f;
#pragma unroll
  for (int k = 0; k < KT; ++k) {
    w[k] = 0.f;
    src[k] = 0;
    if (k < keff && key_valid(tk[k])) {
      const uint32_t gid = vals[start + key_slot(tk[k])];
      const double4 c = g64[gid];
      const float4 a = g32a[gid];
      double e1, e2;
      const double q = quad_form64(fx, fy, a.x, a.y, c.x, c.y, c.z, c.w, e1, e2);
      if (k == 0) shift = (float)q;
      w[k] = blend_weight(q, shift);
      Z += w[k];
      src[k] = gid;
    }
  }
  const float invZ = Z > 0.f ? 1.0f / Z : 0.0f;
  for (int ch = 0; ch < n; ++ch) {
    float acc = 0.f;
#pragma unroll
    for (int k = 0; k < KT; ++k)
      if (k < keff && key_valid(tk[k]))
        acc = fmaf(w[k], params[(size_t)(5 + ch) * N + src[k]], acc);
    out[(size_t)ch * M + i] = acc * invZ;
  }
}

__global__ __launch_bounds__(256) void to_fp16_kernel(const float *__restrict__ src, int64_t count,
                                                      uint16_t *__restrict__ dst) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = __half_as_ushort(__float2half_rn(src[i]));
}

// Stored float16 fitter parameters [5+n][N_src] -> float32 renderer parameters [5+n][N_prefix]
// of the first N_prefix Gaussians: mean x W and x H, rotation, scale = 1 / inverse scale, colour
// (the conversions igs_adam_step applies after each update).
__global__ __launch_bounds__(256) void decode_fp16_kernel(const uint16_t *__restrict__ src,
                                                          int N_src, int N_prefix, float W,
                                                          float H, float *__restrict__ dst) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const int r = blockIdx.y;
  if (j >= N_prefix) return;
  const float p = __half2float(__ushort_as_half(src[(size_t)r * N_src + j]));
  float v = p;
  if (r == 0) v = p * W;
  else if (r == 1) v = p * H;
  else if (r == 3 || r == 4) v = 1.0f / p;
  dst[(size_t)r * N_prefix + j] = v;
}

}  // namespace

hipError_t launch_query(const float *params, int N, int n, int H, int W, int K,
                        const int2 *ranges, const uint32_t *vals, const float4 *g32a,
                        const float2 *g32b, const double4 *g64, const float *points, int M,
                        float *out, hipStream_t s) {
  if (M <= 0) return hipSuccess;
  const int tiles_x = (W + kTile - 1) / kTile, tiles_y = (H + kTile - 1) / kTile;
  const int grid = (M + kQueryThreads - 1) / kQueryThreads;
  switch (pick_kt(K)) {
#define IGS_QUERY_CASE(KT)                                                                    \
  case KT:                                                                                    \
    query_kernel<KT><<<grid, kQueryThreads, 0, s>>>(params, N, n, H, W, K, tiles_x, tiles_y, \
                                                    ranges, vals, g32a, g32b, g64, points, M, \
                                                    out);                                     \
    break;
    IGS_FOR_EACH_KT(IGS_QUERY_CASE)
#undef IGS_QUERY_CASE
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_to_fp16(const float *src, int64_t count, uint16_t *dst, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  const int grid = (int)std::min<int64_t>((count + 255) / 256, 4096);
  to_fp16_kernel<<<grid, 256, 0, s>>>(src, count, dst);
  return hipGetLastError();
}

hipError_t launch_decode_fp16(const uint16_t *src, int N_src, int n, int N_prefix, int H, int W,
                              float *dst, hipStream_t s) {
  if (N_prefix <= 0) return hipSuccess;
  const dim3 grid((N_prefix + 255) / 256, 5 + n);
  decode_fp16_kernel<<<grid, 256, 0, s>>>(src, N_src, N_prefix, (float)W, (float)H, dst);
  return hipGetLastError();
}

}  // namespace igs
