// The SSIM term of the fitting loss (Image-GS Sec. 3.3 and Sec. 4.1: L1 + 0.1 L_SSIM) and its
// gradient with respect to the rendered image, as two stencil kernels per call.
//
// SSIM here: local weighted means under an 11 x 11 Gaussian window (sigma 1.5, weights summing
// to 1), the image extended by zeros, C1 = 0.01^2 and C2 = 0.03^2; the map
//   S = (2 mx my + C1)(2 sxy + C2) / ((mx^2 + my^2 + C1)(sxx + syy + C2))
// with variances and covariance taken as second moments minus products of means; SSIM is the mean
// of S over every channel and pixel and L = mean|x - y| + w (1 - SSIM).
//
// Forward (ssim_fwd_kernel): per 32 x 16 output tile of one channel plane, x and y are staged in
// LDS with their 5-pixel halo, the five moments mx, my, E[x^2], E[y^2], E[xy] are blurred by a
// horizontal then a vertical 11-tap pass, in fp64 (the variances are differences of nearly equal
// moments and are compared with C2 = 9e-4, so fp32 moments would lose up to four digits), and
// each pixel writes the partial derivatives of S with respect to mx, E[x^2] and E[xy] (fp32) and
// adds S, |x - y| and (x - y)^2 to the block's sums.
// Backward (ssim_bwd_kernel): the three partial maps are blurred with the same window (the window
// is symmetric and zero outside the image, so the blur is its own adjoint) and combined,
//   dL/dx = sign(x - y)/count - (w/count)(blur(dS/dmx) + 2 x blur(dS/dE[x^2]) + y blur(dS/dE[xy])).
// Both passes are deterministic; the loss sums are reduced in a fixed order.
#include <cmath>

#include "common.hpp"

namespace igs {
namespace {

constexpr int kSsimR = 5;                      // window radius
constexpr int kSsimTW = 32;                    // output tile width
constexpr int kSsimTH = 16;                    // output tile height
constexpr int kSsimInW = kSsimTW + 2 * kSsimR;  // 42
constexpr int kSsimInH = kSsimTH + 2 * kSsimR;  // 26
constexpr int kSsimThreads = 256;
constexpr int kRunH = 4;                        // horizontal pass: outputs per thread (one row)
constexpr int kRunV = 2;                        // vertical pass: outputs per thread (one column)
constexpr int kHItems = kSsimInH * (kSsimTW / kRunH);  // 208 threads busy in the horizontal pass
static_assert(kSsimTW / kRunH * kSsimInH <= kSsimThreads, "horizontal pass: one item per thread");
static_assert(kSsimTW * (kSsimTH / kRunV) == kSsimThreads, "vertical pass: one item per thread");
constexpr double kC1 = 0.01 * 0.01;
constexpr double kC2 = 0.03 * 0.03;

__device__ __forceinline__ double wsum64(double v) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
  return v;
}

// The tile's input region (rows y0 - R .. y0 + TH + R - 1, same for columns) of one plane into
// LDS, zero outside the image.
__device__ __forceinline__ void stage_plane(const float *__restrict__ src, int H, int W, int x0,
                                            int y0, float *dst) {
  for (int i = threadIdx.x; i < kSsimInH * kSsimInW; i += kSsimThreads) {
    const int r = i / kSsimInW, c = i - r * kSsimInW;
    const int h = y0 - kSsimR + r, w = x0 - kSsimR + c;
    dst[i] = (h >= 0 && h < H && w >= 0 && w < W) ? src[(size_t)h * W + w] : 0.f;
  }
}

// Tap weight for offset k - R of the 11-tap window, k = 0..10, from the six distinct weights.
template <typename T>
__device__ __forceinline__ T tap(const T (&w)[6], int k) {
  return w[k < kSsimR ? kSsimR - k : k - kSsimR];
}

template <typename T>
struct Win {
  T w[6];  // w[j]: weight at offset +-j
};

__global__ __launch_bounds__(kSsimThreads) void ssim_fwd_kernel(
    const float *__restrict__ img, const float *__restrict__ tgt, int H, int W, int tiles_x,
    Win<double> win, float *__restrict__ d_mx, float *__restrict__ d_exx,
    float *__restrict__ d_exy, double *__restrict__ partial) {
  __shared__ float s_x[kSsimInH * kSsimInW];
  __shared__ float s_y[kSsimInH * kSsimInW];
  __shared__ double s_h[5][kSsimInH * kSsimTW];
  __shared__ double s_red[3][kSsimThreads / 64];

  const int tile = blockIdx.x;
  const int ty = tile / tiles_x, tx = tile - ty * tiles_x;
  const int x0 = tx * kSsimTW, y0 = ty * kSsimTH;
  const size_t plane = (size_t)blockIdx.y * H * W;
  const int tid = threadIdx.x;
  stage_plane(img + plane, H, W, x0, y0, s_x);
  stage_plane(tgt + plane, H, W, x0, y0, s_y);
  __syncthreads();

  // horizontal pass: row r, output columns c0 .. c0 + 3 of the tile
  if (tid < kHItems) {
    const int r = tid / (kSsimTW / kRunH), c0 = (tid - r * (kSsimTW / kRunH)) * kRunH;
    double acc[kRunH][5];
#pragma unroll
    for (int o = 0; o < kRunH; ++o)
#pragma unroll
      for (int m = 0; m < 5; ++m) acc[o][m] = 0.0;
#pragma unroll
    for (int t = 0; t < kRunH + 2 * kSsimR; ++t) {
      const double xv = (double)s_x[r * kSsimInW + c0 + t];
      const double yv = (double)s_y[r * kSsimInW + c0 + t];
      const double v[5] = {xv, yv, xv * xv, yv * yv, xv * yv};  // products exact in fp64
#pragma unroll
      for (int o = 0; o < kRunH; ++o) {
        const int k = t - o;
        if (k >= 0 && k <= 2 * kSsimR) {
          const double wk = tap(win.w, k);
#pragma unroll
          for (int m = 0; m < 5; ++m) acc[o][m] = fma(wk, v[m], acc[o][m]);
        }
      }
    }
#pragma unroll
    for (int o = 0; o < kRunH; ++o)
#pragma unroll
      for (int m = 0; m < 5; ++m) s_h[m][r * kSsimTW + c0 + o] = acc[o][m];
  }
  __syncthreads();

  // vertical pass: column c, output rows r0, r0 + 1 of the tile
  const int c = tid & (kSsimTW - 1), r0 = (tid / kSsimTW) * kRunV;
  double acc[kRunV][5];
#pragma unroll
  for (int o = 0; o < kRunV; ++o)
#pragma unroll
    for (int m = 0; m < 5; ++m) acc[o][m] = 0.0;
#pragma unroll
  for (int t = 0; t < kRunV + 2 * kSsimR; ++t) {
    double v[5];
#pragma unroll
    for (int m = 0; m < 5; ++m) v[m] = s_h[m][(r0 + t) * kSsimTW + c];
#pragma unroll
    for (int o = 0; o < kRunV; ++o) {
      const int k = t - o;
      if (k >= 0 && k <= 2 * kSsimR) {
        const double wk = tap(win.w, k);
#pragma unroll
        for (int m = 0; m < 5; ++m) acc[o][m] = fma(wk, v[m], acc[o][m]);
      }
    }
  }
  double sum_s = 0.0, sum_a = 0.0, sum_q = 0.0;
  const int w = x0 + c;
#pragma unroll
  for (int o = 0; o < kRunV; ++o) {
    const int h = y0 + r0 + o;
    if (h < H && w < W) {
      const double mx = acc[o][0], my = acc[o][1];
      const double a1 = 2.0 * mx * my + kC1;
      const double a2 = 2.0 * (acc[o][4] - mx * my) + kC2;
      const double b1 = mx * mx + my * my + kC1;
      const double b2 = (acc[o][2] - mx * mx) + (acc[o][3] - my * my) + kC2;
      const double inv = 1.0 / (b1 * b2);
      const double s = a1 * a2 * inv;
      // quotient rule on S = a1 a2 / (b1 b2): d/dmx, d/dE[x^2], d/dE[xy]
      const double gmx = (2.0 * my * (a2 - a1) - s * 2.0 * mx * (b2 - b1)) * inv;
      const double gxx = -s * b1 * inv;
      const double gxy = 2.0 * a1 * inv;
      const size_t e = plane + (size_t)h * W + w;
      d_mx[e] = (float)gmx;
      d_exx[e] = (float)gxx;
      d_exy[e] = (float)gxy;
      const int li = (r0 + o + kSsimR) * kSsimInW + c + kSsimR;
      const double d = (double)s_x[li] - (double)s_y[li];
      sum_s += s;
      sum_a += fabs(d);
      sum_q += d * d;
    }
  }
  sum_s = wsum64(sum_s);
  sum_a = wsum64(sum_a);
  sum_q = wsum64(sum_q);
  if ((tid & 63) == 0) {
    s_red[0][tid >> 6] = sum_s;
    s_red[1][tid >> 6] = sum_a;
    s_red[2][tid >> 6] = sum_q;
  }
  __syncthreads();
  if (tid < 3) {
    double t = 0.0;
#pragma unroll
    for (int k = 0; k < kSsimThreads / 64; ++k) t += s_red[tid][k];
    partial[((size_t)blockIdx.y * gridDim.x + blockIdx.x) * 3 + tid] = t;
  }
}

// One block: the blocks' sums in a fixed order; out = {L, L1, MSE, SSIM}.
__global__ __launch_bounds__(1024) void ssim_final_kernel(const double *__restrict__ partial,
                                                          int64_t nblocks, double inv_count,
                                                          double weight,
                                                          double *__restrict__ out) {
  __shared__ double s_red[3][1024 / 64];
  double t[3] = {0.0, 0.0, 0.0};
  for (int64_t b = threadIdx.x; b < nblocks; b += blockDim.x)
#pragma unroll
    for (int k = 0; k < 3; ++k) t[k] += partial[b * 3 + k];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const double v = wsum64(t[k]);
    if ((threadIdx.x & 63) == 0) s_red[k][threadIdx.x >> 6] = v;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0, a = 0.0, q = 0.0;
    for (int k = 0; k < (int)(blockDim.x >> 6); ++k) {
      s += s_red[0][k];
      a += s_red[1][k];
      q += s_red[2][k];
    }
    const double ssim = s * inv_count, l1 = a * inv_count;
    out[0] = l1 + weight * (1.0 - ssim);
    out[1] = l1;
    out[2] = q * inv_count;
    out[3] = ssim;
  }
}

__global__ __launch_bounds__(kSsimThreads) void ssim_bwd_kernel(
    const float *__restrict__ img, const float *__restrict__ tgt,
    const float *__restrict__ d_mx, const float *__restrict__ d_exx,
    const float *__restrict__ d_exy, int H, int W, int tiles_x, Win<float> win, float l1_scale,
    float ssim_scale, float *__restrict__ grad) {
  __shared__ float s_p[3][kSsimInH * kSsimInW];
  __shared__ float s_h[3][kSsimInH * kSsimTW];

  const int tile = blockIdx.x;
  const int ty = tile / tiles_x, tx = tile - ty * tiles_x;
  const int x0 = tx * kSsimTW, y0 = ty * kSsimTH;
  const size_t plane = (size_t)blockIdx.y * H * W;
  const int tid = threadIdx.x;
  stage_plane(d_mx + plane, H, W, x0, y0, s_p[0]);
  stage_plane(d_exx + plane, H, W, x0, y0, s_p[1]);
  stage_plane(d_exy + plane, H, W, x0, y0, s_p[2]);
  __syncthreads();

  if (tid < kHItems) {
    const int r = tid / (kSsimTW / kRunH), c0 = (tid - r * (kSsimTW / kRunH)) * kRunH;
    float acc[kRunH][3];
#pragma unroll
    for (int o = 0; o < kRunH; ++o)
#pragma unroll
      for (int m = 0; m < 3; ++m) acc[o][m] = 0.f;
#pragma unroll
    for (int t = 0; t < kRunH + 2 * kSsimR; ++t) {
      float v[3];
#pragma unroll
      for (int m = 0; m < 3; ++m) v[m] = s_p[m][r * kSsimInW + c0 + t];
#pragma unroll
      for (int o = 0; o < kRunH; ++o) {
        const int k = t - o;
        if (k >= 0 && k <= 2 * kSsimR) {
          const float wk = tap(win.w, k);
#pragma unroll
          for (int m = 0; m < 3; ++m) acc[o][m] = fmaf(wk, v[m], acc[o][m]);
        }
      }
    }
#pragma unroll
    for (int o = 0; o < kRunH; ++o)
#pragma unroll
      for (int m = 0; m < 3; ++m) s_h[m][r * kSsimTW + c0 + o] = acc[o][m];
  }
  __syncthreads();

  const int c = tid & (kSsimTW - 1), r0 = (tid / kSsimTW) * kRunV;
  float acc[kRunV][3];
#pragma unroll
  for (int o = 0; o < kRunV; ++o)
#pragma unroll
    for (int m = 0; m < 3; ++m) acc[o][m] = 0.f;
#pragma unroll
  for (int t = 0; t < kRunV + 2 * kSsimR; ++t) {
    float v[3];
#pragma unroll
    for (int m = 0; m < 3; ++m) v[m] = s_h[m][(r0 + t) * kSsimTW + c];
#pragma unroll
    for (int o = 0; o < kRunV; ++o) {
      const int k = t - o;
      if (k >= 0 && k <= 2 * kSsimR) {
        const float wk = tap(win.w, k);
#pragma unroll
        for (int m = 0; m < 3; ++m) acc[o][m] = fmaf(wk, v[m], acc[o][m]);
      }
    }
  }
  const int w = x0 + c;
#pragma unroll
  for (int o = 0; o < kRunV; ++o) {
    const int h = y0 + r0 + o;
    if (h < H && w < W) {
      const size_t e = plane + (size_t)h * W + w;
      const float xv = img[e], yv = tgt[e];
      const float d = xv - yv;  // exact sign; zero only when equal
      const float sg = d > 0.f ? l1_scale : (d < 0.f ? -l1_scale : 0.f);
      const float gs = acc[o][0] + 2.f * xv * acc[o][1] + yv * acc[o][2];
      grad[e] = fmaf(ssim_scale, gs, sg);
    }
  }
}

template <typename T>
Win<T> make_window() {
  // exp(-j^2 / (2 sigma^2)), sigma = 1.5, normalized over j = -5..5
  double raw[6], total = 0.0;
  for (int j = 0; j <= kSsimR; ++j) {
    raw[j] = std::exp(-(double)(j * j) / (2.0 * 1.5 * 1.5));
    total += (j == 0 ? 1.0 : 2.0) * raw[j];
  }
  Win<T> w;
  for (int j = 0; j <= kSsimR; ++j) w.w[j] = (T)(raw[j] / total);
  return w;
}

}  // namespace

int64_t ssim_blocks(int n, int H, int W) {
  const int64_t tx = (W + kSsimTW - 1) / kSsimTW, ty = (H + kSsimTH - 1) / kSsimTH;
  return tx * ty * n;
}

hipError_t launch_l1_ssim(const float *image, const float *target, int n, int H, int W,
                          double weight, float *grad, float *d_mx, float *d_exx, float *d_exy,
                          double *partial, double *loss_out, hipStream_t s) {
  const int tiles_x = (W + kSsimTW - 1) / kSsimTW, tiles_y = (H + kSsimTH - 1) / kSsimTH;
  const dim3 grid(tiles_x * tiles_y, n);
  const int64_t count = (int64_t)n * H * W;
  ssim_fwd_kernel<<<grid, kSsimThreads, 0, s>>>(image, target, H, W, tiles_x,
                                                make_window<double>(), d_mx, d_exx, d_exy,
                                                partial);
  ssim_final_kernel<<<1, 1024, 0, s>>>(partial, (int64_t)grid.x * grid.y, 1.0 / (double)count,
                                       weight, loss_out);
  ssim_bwd_kernel<<<grid, kSsimThreads, 0, s>>>(image, target, d_mx, d_exx, d_exy, H, W, tiles_x,
                                                make_window<float>(), (float)(1.0 / count),
                                                (float)(-weight / count), grad);
  return hipGetLastError();
}

}  // namespace igs
