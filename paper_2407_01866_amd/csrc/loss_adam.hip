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

// Chain rule from a gradient with respect to render parameter row r to the fitter parameter p of
// that row: mu = W (mu/W) and H (mu/H), s = 1/u so dL/du = -s^2 dL/ds = -dL/ds / u^2.
__device__ __forceinline__ float grad_to_fit(int r, float g, float p, float W, float H) {
  if (r == 0) return g * W;
  if (r == 1) return g * H;
  if (r == 3 || r == 4) return -g / (p * p);
  return g;
}

// Four elements of one row per thread (Gaussians i0 + tid + 256 u of row blockIdx.y of the
// [5+n][N] arrays, so every load and store of a block is contiguous), their loads issued
// together and the bias corrections computed once.  u_lo > 0: lower clip of the inverse scales;
// u_lo <= 0: 1/max(H, W) of each Gaussian's image.
constexpr int kAdamThreads = 256;
constexpr int kAdamItems = 4;

__global__ __launch_bounds__(kAdamThreads) void adam_kernel(
    float *__restrict__ fit, float *__restrict__ rend, const float *__restrict__ grad,
    float *__restrict__ m, float *__restrict__ v, const int32_t *__restrict__ step,
    const int64_t *__restrict__ skip, int N, int n, Images imgs, float lr_mu, float lr_theta,
    float lr_u, float lr_c, float b1, float b2, float eps, float u_lo_arg, float u_hi) {
  __shared__ int s_b0;
  if (skip != nullptr && skip[0] != 0) return;  // uniform: the whole grid skips
  const int i0 = blockIdx.x * (kAdamThreads * kAdamItems);
  const int r = blockIdx.y;
  // the image of the block's first Gaussian, once per block; later ones walk forward from it
  int b = 0;
  if (imgs.arr) {
    if (threadIdx.x == 0) {
      int lo = 0, hi = imgs.B - 1;
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (imgs.arr[mid].gauss_off <= i0) lo = mid;
        else hi = mid - 1;
      }
      s_b0 = lo;
    }
    __syncthreads();
    b = s_b0;
  }
  const float t = (float)(step[0] + 1);
  const float bc1 = 1.0f - powf(b1, t), bc2 = 1.0f - powf(b2, t);
  float pv[kAdamItems], gv[kAdamItems], mv[kAdamItems], vv[kAdamItems];
#pragma unroll
  for (int u = 0; u < kAdamItems; ++u) {
    const int i = i0 + u * kAdamThreads + (int)threadIdx.x;
    const size_t e = (size_t)r * N + (i < N ? i : 0);
    pv[u] = fit[e];
    gv[u] = grad[e];
    mv[u] = m[e];
    vv[u] = v[e];
  }
#pragma unroll
  for (int u = 0; u < kAdamItems; ++u) {
    const int i = i0 + u * kAdamThreads + (int)threadIdx.x;
    if (i >= N) break;
    const size_t e = (size_t)r * N + i;
    ImageDesc im;
    if (imgs.arr) {
      while (b + 1 < imgs.B && imgs.arr[b + 1].gauss_off <= i) ++b;
      im = imgs.arr[b];
    } else {
      im = imgs.one;
    }
    const float W = (float)im.W, H = (float)im.H;
    const float u_lo = u_lo_arg > 0.f ? u_lo_arg : 1.0f / fmaxf(W, H);
    const float p = pv[u];
    const float g = grad_to_fit(r, gv[u], p, W, H);
    const float lr = r <= 1 ? lr_mu : (r == 2 ? lr_theta : (r <= 4 ? lr_u : lr_c));
    const float mm = b1 * mv[u] + (1.0f - b1) * g;
    const float vn = b2 * vv[u] + (1.0f - b2) * g * g;
    m[e] = mm;
    v[e] = vn;
    float np = p - lr * (mm / bc1) / (sqrtf(vn / bc2) + eps);
    if (r == 2) np = fminf(fmaxf(np, 0.0f), 3.14159265358979323846f);
    if (r == 3 || r == 4) np = fminf(fmaxf(np, u_lo), u_hi);
    fit[e] = np;
    rend[e] = to_render(r, np, W, H);
  }
}

__global__ void step_increment_kernel(int32_t *step, const int64_t *skip) {
  if (threadIdx.x == 0 && (skip == nullptr || skip[0] == 0)) step[0] += 1;
}

__global__ __launch_bounds__(256) void fit_to_render_kernel(const float *__restrict__ fit,
                                                            float *__restrict__ rend, int N, int n,
                                                            Images imgs) {
  const int64_t total = (int64_t)(5 + n) * N;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= total) return;
  const int r = (int)(e / N);
  const ImageDesc im = imgs.by_gauss((int)(e - (int64_t)r * N));
  rend[e] = to_render(r, fit[e], (float)im.W, (float)im.H);
}

__global__ __launch_bounds__(256) void grad_to_fit_kernel(const float *__restrict__ fit,
                                                          const float *__restrict__ grad_rend,
                                                          float *__restrict__ grad_fit, int N,
                                                          int n, Images imgs) {
  const int64_t total = (int64_t)(5 + n) * N;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= total) return;
  const int r = (int)(e / N);
  const ImageDesc im = imgs.by_gauss((int)(e - (int64_t)r * N));
  grad_fit[e] = grad_to_fit(r, grad_rend[e], fit[e], (float)im.W, (float)im.H);
}

// Batched L1: block k belongs to the image b with l1_block_off[b] <= k < l1_block_off[b+1] and
// covers kL1BatchItems consecutive values of it; each image is normalized by its own n*H*W.
constexpr int kL1BatchItems = 8192;

__device__ __forceinline__ int image_of_block(const Images &imgs, int k) {
  int lo = 0, hi = imgs.B - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (imgs.arr[mid].l1_block_off <= k) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

__global__ __launch_bounds__(kL1Threads) void l1_batched_kernel(const float *__restrict__ images,
                                                                const float *__restrict__ targets,
                                                                Images imgs, int n,
                                                                float *__restrict__ grad,
                                                                double *__restrict__ partials) {
  __shared__ double sh[kL1Threads / 64];
  const int b = image_of_block(imgs, blockIdx.x);
  const ImageDesc im = imgs.arr[b];
  const int64_t count = (int64_t)n * im.H * im.W;
  const int64_t base = (int64_t)n * im.pix_off;
  const int64_t first = (int64_t)(blockIdx.x - im.l1_block_off) * kL1BatchItems;
  const int64_t last = min(first + kL1BatchItems, count);
  const float inv_count = (float)(1.0 / (double)count);
  double a = 0.0, q = 0.0;
  for (int64_t i = first + threadIdx.x; i < last; i += kL1Threads) {
    const double d = (double)images[base + i] - (double)targets[base + i];
    grad[base + i] = d > 0.0 ? inv_count : (d < 0.0 ? -inv_count : 0.f);
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

// One block per image: its blocks' partial sums in a fixed order -> loss_out[b] = (L1, MSE).
__global__ __launch_bounds__(kL1Threads) void l1_batched_final_kernel(
    const double *__restrict__ partials, Images imgs, int n, int total_blocks,
    double *__restrict__ out) {
  __shared__ double sh[kL1Threads / 64];
  const int b = blockIdx.x;
  const ImageDesc im = imgs.arr[b];
  const int k0 = im.l1_block_off;
  const int k1 = b + 1 < imgs.B ? imgs.arr[b + 1].l1_block_off : total_blocks;
  double a = 0.0, q = 0.0;
  for (int k = k0 + threadIdx.x; k < k1; k += kL1Threads) {
    a += partials[2 * k];
    q += partials[2 * k + 1];
  }
  const double sa = block_sum(a, sh);
  const double sq = block_sum(q, sh);
  if (threadIdx.x == 0) {
    const double inv = 1.0 / ((double)n * im.H * im.W);
    out[2 * b] = sa * inv;
    out[2 * b + 1] = sq * inv;
  }
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
                       int32_t *step, const int64_t *skip, int N, int n, const Images &imgs,
                       float lr_mu, float lr_theta, float lr_u, float lr_c, float b1, float b2,
                       float eps, float u_hi, hipStream_t s) {
  return launch_adam_lo(fit, rend, grad, m, v, step, skip, N, n, imgs, lr_mu, lr_theta, lr_u,
                        lr_c, b1, b2, eps, 0.f, u_hi, s);
}

hipError_t launch_adam_lo(float *fit, float *rend, const float *grad, float *m, float *v,
                          int32_t *step, const int64_t *skip, int N, int n, const Images &imgs,
                          float lr_mu, float lr_theta, float lr_u, float lr_c, float b1, float b2,
                          float eps, float u_lo, float u_hi, hipStream_t s) {
  if (N > 0) {
    constexpr int per_block = kAdamThreads * kAdamItems;
    adam_kernel<<<dim3((unsigned)((N + per_block - 1) / per_block), (unsigned)(5 + n)),
                  kAdamThreads, 0, s>>>(
        fit, rend, grad, m, v, step, skip, N, n, imgs, lr_mu, lr_theta, lr_u, lr_c, b1, b2, eps,
        u_lo, u_hi);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  step_increment_kernel<<<1, 64, 0, s>>>(step, skip);
  return hipGetLastError();
}

hipError_t launch_fit_to_render(const float *fit, float *rend, int N, int n, const Images &imgs,
                                hipStream_t s) {
  const int64_t total = (int64_t)(5 + n) * N;
  if (total <= 0) return hipSuccess;
  fit_to_render_kernel<<<(unsigned)((total + 255) / 256), 256, 0, s>>>(fit, rend, N, n, imgs);
  return hipGetLastError();
}

hipError_t launch_grad_to_fit(const float *fit, const float *grad_rend, float *grad_fit, int N,
                              int n, const Images &imgs, hipStream_t s) {
  const int64_t total = (int64_t)(5 + n) * N;
  if (total <= 0) return hipSuccess;
  grad_to_fit_kernel<<<(unsigned)((total + 255) / 256), 256, 0, s>>>(fit, grad_rend, grad_fit, N,
                                                                      n, imgs);
  return hipGetLastError();
}

int l1_batch_block_items() { return kL1BatchItems; }

hipError_t launch_l1_batched(const float *images, const float *targets, const Images &imgs,
                             int n, int total_blocks, float *grad, double *partials,
                             double *loss_out, hipStream_t s) {
  if (total_blocks <= 0) return hipSuccess;
  l1_batched_kernel<<<total_blocks, kL1Threads, 0, s>>>(images, targets, imgs, n, grad, partials);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  l1_batched_final_kernel<<<imgs.B, kL1Threads, 0, s>>>(partials, imgs, n, total_blocks, loss_out);
  return hipGetLastError();
}

}  // namespace igs
