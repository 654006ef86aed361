// Loss gradient and optimizer step around the renderer (Image-GS Sec. 3.3 and Sec. 4.1):
// the L1 term (mean absolute error, sign gradient) with a deterministic two-stage reduction, and
// Adam in the fitter's parameterization (normalized mean, inverse scales) with the chain rules
// from the renderer's units and the parameter clipping fused in.
#include "common.hpp"

namespace igs {
namespace {

constexpr int kL1Threads = 256;
constexpr int kL1MaxBlocks = 1024;

__device__ __forceinline__ double block_sum(double v, double *sh) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) v += __shfl_down(v, d, 64);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) sh[w] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0)
    for (int k = 0; k < (int)(blockDim.x >> 6); ++k) t += sh[k];
  __syncthreads();
  return t;  // valid in thread 0
}

__global__ __launch_bounds__(kL1Threads) void l1_kernel(const float *__restrict__ img,
                                                        const float *__restrict__ tgt,
                                                        int64_t count, float inv_count,
                                                        float *__restrict__ grad,
                                                        double *__restrict__ partials) {
  __shared__ double sh[kL1Threads / 64];
  double a = 0.0, q = 0.0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride) {
    const double d = (double)img[i] - (double)tgt[i];  // exact; its sign is that of a - b
    grad[i] = d > 0.0 ? inv_count : (d < 0.0 ? -inv_count : 0.f);
    a += fabs(d);
    q += d * d;
  }
  const double sa = block_sum(a, sh);
  const double sq = block_sum(q, sh);
  if (threadIdx.x == 0) {
    partials[2 * blockIdx.x] = sa;
    partials[2 * blockIdx.x + 1] = sq;
  }
}

__global__ __launch_bounds__(kL1Threads) void l1_final_kernel(const double *__restrict__ partials,
                                                              int nblocks, double inv_count,
                                                              double *__restrict__ out) {
  __shared__ double sh[kL1Threads / 64];
  double a = 0.0, q = 0.0;
  for (int b = threadIdx.x; b < nblocks; b += blockDim.x) {
    a += partials[2 * b];
    q += partials[2 * b + 1];
  }
  const double sa = block_sum(a, sh);
  const double sq = block_sum(q, sh);
  if (threadIdx.x == 0) {
    out[0] = sa * inv_count;
    out[1] = sq * inv_count;
  }
}

// Row r of the [5+n][N] arrays: 0,1 mean (fit: normalized by W, H), 2 theta, 3,4 scale (fit:
// inverse scale), 5.. colour.
__device__ __forceinline__ float to_render(int r, float p, float W, float H) {
  if (r == 0) return p * W;
  if (r == 1) return p * H;
  if (r == 3 || r == 4) return 1.0f / p;
  return p;
}

__global__ __launch_bounds__(256) void adam_kernel(
    float *__restrict__ fit, float *__restrict__ rend, const float *__restrict__ grad,
    float *__restrict__ m, float *__restrict__ v, const int32_t *__restrict__ step,
    const int64_t *__restrict__ skip, int N, int n,
    float W, float H, float lr_mu, float lr_theta, float lr_u, float lr_c, float b1, float b2,
    float eps, float u_lo, float u_hi) {
  const int64_t total = (int64_t)(5 + n) * N;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= total) return;
  if (skip != nullptr && skip[0] != 0) return;
  const int r = (int)(e / N);
  const float t = (float)(step[0] + 1);
  const float bc1 = 1.0f - powf(b1, t), bc2 = 1.0f - powf(b2, t);
  const float p = fit[e];
  float g = grad[e];
  float lr = lr_c;
  if (r == 0) {
    g *= W;
    lr = lr_mu;
  } else if (r == 1) {
    g *= H;
    lr = lr_mu;
  } else if (r == 2) {
    lr = lr_theta;
  } else if (r == 3 || r == 4) {
    g = -g / (p * p);  // dL/du = -s^2 dL/ds with u = 1/s
    lr = lr_u;
  }
  const float mm = b1 * m[e] + (1.0f - b1) * g;
  const float vv = b2 * v[e] + (1.0f - b2) * g * g;
  m[e] = mm;
  v[e] = vv;
  float np = p - lr * (mm / bc1) / (sqrtf(vv / bc2) + eps);
  if (r == 2) np = fminf(fmaxf(np, 0.0f), 3.14159265358979323846f);
  if (r == 3 || r == 4) np = fminf(fmaxf(np, u_lo), u_hi);
  fit[e] = np;
  rend[e] = to_render(r, np, W, H);
}

__global__ void step_increment_kernel(int32_t *step, const int64_t *skip) {
  if (threadIdx.x == 0 && (skip == nullptr || skip[0] == 0)) step[0] += 1;
}

__global__ __launch_bounds__(256) void fit_to_render_kernel(const float *__restrict__ fit,
                                                            float *__restrict__ rend, int N, int n,
                                                            float W, float H) {
  const int64_t total = (int64_t)(5 + n) * N;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= total) return;
  rend[e] = to_render((int)(e / N), fit[e], W, H);
}

}  // namespace

int l1_blocks(int64_t count) {
  int64_t b = (count + kL1Threads * 8 - 1) / (kL1Threads * 8);
  if (b < 1) b = 1;
  if (b > kL1MaxBlocks) b = kL1MaxBlocks;
  return (int)b;
}

hipError_t launch_l1(const float *image, const float *target, int64_t count, float *grad,
                     double *partials, double *loss_out, hipStream_t s) {
  const int nb = l1_blocks(count);
  l1_kernel<<<nb, kL1Threads, 0, s>>>(image, target, count, (float)(1.0 / (double)count), grad,
                                      partials);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  l1_final_kernel<<<1, kL1Threads, 0, s>>>(partials, nb, 1.0 / (double)count, loss_out);
  return hipGetLastError();
}

hipError_t launch_adam(float *fit, float *rend, const float *grad, float *m, float *v,
                       int32_t *step, const int64_t *skip, int N, int n, int H, int W,
                       float lr_mu, float lr_theta,
                       float lr_u, float lr_c, float b1, float b2, float eps, float u_lo,
                       float u_hi, hipStream_t s) {
  const int64_t total = (int64_t)(5 + n) * N;
  if (total > 0) {
    adam_kernel<<<(unsigned)((total + 255) / 256), 256, 0, s>>>(
        fit, rend, grad, m, v, step, skip, N, n, (float)W, (float)H, lr_mu, lr_theta, lr_u, lr_c, b1,
        b2, eps, u_lo, u_hi);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  step_increment_kernel<<<1, 64, 0, s>>>(step, skip);
  return hipGetLastError();
}

hipError_t launch_fit_to_render(const float *fit, float *rend, int N, int n, int H, int W,
                                hipStream_t s) {
  const int64_t total = (int64_t)(5 + n) * N;
  if (total <= 0) return hipSuccess;
  fit_to_render_kernel<<<(unsigned)((total + 255) / 256), 256, 0, s>>>(fit, rend, N, n, (float)W,
                                                                       (float)H);
  return hipGetLastError();
}

}  // namespace igs
