// Placement of Gaussians around the fit (Image-GS Sec. 3.3): content-adaptive initialization
// (Eq. 6: pixels drawn with probability (1 - lambda) |grad I| / sum |grad I| + lambda / (H W)) and
// error-guided addition (Eq. 7: probability |rendered - target| / sum).  Each new Gaussian sits at
// the centre of its pixel with rotation 0, both scales `scale` pixels and the target's colour
// there (Sec. 4.1).
//
// Per call: a weight per pixel (fp64) and the blocks' sums of the weights; their total in a fixed
// order; an exclusive fp64 prefix sum of the weights; then one thread per new Gaussian inverts
// the cumulative distribution at its caller-supplied uniform by binary search and writes the
// Gaussian's parameters.  The image gradient is the per-channel central difference inside the
// image and the one-sided difference at its border (zero along an axis of length 1), its norm the
// Euclidean norm over both directions and all channels.
#include <algorithm>

#include "common.hpp"

namespace igs {
namespace {

constexpr int kPlaceThreads = 256;
constexpr int kPlaceMaxBlocks = 2048;

__device__ __forceinline__ double block_sum64(double v, double *sh) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0)
    for (int k = 0; k < kPlaceThreads / 64; ++k) t += sh[k];
  return t;  // valid in thread 0
}

// Derivative along one axis at index i of a line of length len (values a(i-1), a(i), a(i+1)).
__device__ __forceinline__ double axis_diff(int i, int len, float prev, float cur, float next) {
  if (len < 2) return 0.0;
  if (i == 0) return (double)next - (double)cur;
  if (i == len - 1) return (double)cur - (double)prev;
  return ((double)next - (double)prev) * 0.5;
}

__global__ __launch_bounds__(kPlaceThreads) void edge_weight_kernel(
    const float *__restrict__ tgt, int n, int H, int W, double *__restrict__ wgt,
    double *__restrict__ partial) {
  __shared__ double sh[kPlaceThreads / 64];
  const int64_t HW = (int64_t)H * W;
  double sum = 0.0;
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < HW;
       p += (int64_t)gridDim.x * blockDim.x) {
    const int h = (int)(p / W), w = (int)(p - (int64_t)h * W);
    double acc = 0.0;
    for (int c = 0; c < n; ++c) {
      const float *pl = tgt + (size_t)c * HW;
      const float cur = pl[p];
      const float l = w > 0 ? pl[p - 1] : cur, r = w + 1 < W ? pl[p + 1] : cur;
      const float u = h > 0 ? pl[p - W] : cur, d = h + 1 < H ? pl[p + W] : cur;
      const double gx = axis_diff(w, W, l, cur, r);
      const double gy = axis_diff(h, H, u, cur, d);
      acc += gx * gx + gy * gy;
    }
    const double g = sqrt(acc);
    wgt[p] = g;
    sum += g;
  }
  const double t = block_sum64(sum, sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = t;
}

__global__ __launch_bounds__(kPlaceThreads) void error_weight_kernel(
    const float *__restrict__ img, const float *__restrict__ tgt, int n, int64_t HW,
    double *__restrict__ wgt, double *__restrict__ partial) {
  __shared__ double sh[kPlaceThreads / 64];
  double sum = 0.0;
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < HW;
       p += (int64_t)gridDim.x * blockDim.x) {
    double e = 0.0;
    for (int c = 0; c < n; ++c) e += fabs((double)img[(size_t)c * HW + p] -
                                          (double)tgt[(size_t)c * HW + p]);
    wgt[p] = e;
    sum += e;
  }
  const double t = block_sum64(sum, sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = t;
}

__global__ __launch_bounds__(kPlaceThreads) void weight_total_kernel(
    const double *__restrict__ partial, int nblocks, double *__restrict__ total) {
  __shared__ double sh[kPlaceThreads / 64];
  double v = 0.0;
  for (int b = threadIdx.x; b < nblocks; b += blockDim.x) v += partial[b];
  const double t = block_sum64(v, sh);
  if (threadIdx.x == 0) total[0] = t;
}

// Sample i: t = u_i * G (G = sum of the weights, which is also the total of the Eq. 6 mixture
// (1 - lambda) w + lambda G / HW); the pixel is the first k whose inclusive cumulative mixture
// exceeds t.  G = 0: uniform over the pixels.
__global__ __launch_bounds__(kPlaceThreads) void sample_place_kernel(
    const double *__restrict__ excl, const double *__restrict__ wgt,
    const double *__restrict__ total, int64_t HW, double lam, const float *__restrict__ uni,
    int count, const float *__restrict__ tgt, int n, int H, int W, float scale,
    float *__restrict__ rp, float *__restrict__ fp, int N_total, int first) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const double G = total[0];
  const double u = (double)uni[i];
  int64_t k;
  if (!(G > 0.0)) {
    k = min((int64_t)(u * (double)HW), HW - 1);
  } else {
    const double t = u * G, a = 1.0 - lam, b = lam * G / (double)HW;
    int64_t lo = 0, hi = HW - 1;
    while (lo < hi) {
      const int64_t mid = (lo + hi) >> 1;
      const double incl = a * (excl[mid] + wgt[mid]) + b * (double)(mid + 1);
      if (incl > t) hi = mid;
      else lo = mid + 1;
    }
    k = lo;
  }
  const int h = (int)(k / W), w = (int)(k - (int64_t)h * W);
  const size_t j = (size_t)first + i;
  const float mx = (float)w + 0.5f, my = (float)h + 0.5f;
  rp[0 * (size_t)N_total + j] = mx;
  rp[1 * (size_t)N_total + j] = my;
  rp[2 * (size_t)N_total + j] = 0.f;
  rp[3 * (size_t)N_total + j] = scale;
  rp[4 * (size_t)N_total + j] = scale;
  for (int c = 0; c < n; ++c) rp[(size_t)(5 + c) * N_total + j] = tgt[(size_t)c * HW + k];
  if (fp) {
    fp[0 * (size_t)N_total + j] = mx / (float)W;  // the fitter's normalized mean
    fp[1 * (size_t)N_total + j] = my / (float)H;
    fp[2 * (size_t)N_total + j] = 0.f;
    fp[3 * (size_t)N_total + j] = 1.0f / scale;
    fp[4 * (size_t)N_total + j] = 1.0f / scale;
    for (int c = 0; c < n; ++c) fp[(size_t)(5 + c) * N_total + j] = tgt[(size_t)c * HW + k];
  }
}

int place_blocks(int64_t HW) {
  return (int)std::min<int64_t>((HW + kPlaceThreads - 1) / kPlaceThreads, kPlaceMaxBlocks);
}

}  // namespace

size_t place_workspace_bytes(int64_t HW) {
  return align_up((size_t)HW * sizeof(double)) * 2 +
         align_up(scan_temp_elems(HW) * sizeof(double)) +
         align_up((size_t)kPlaceMaxBlocks * sizeof(double)) + align_up(sizeof(double));
}

hipError_t launch_place(const float *image, const float *target, int n, int H, int W,
                        double lam, const float *uniforms, int count, float scale,
                        float *render_params, float *fit_params, int N_total, int first,
                        void *ws, hipStream_t s) {
  const int64_t HW = (int64_t)H * W;
  char *b = static_cast<char *>(ws);
  double *wgt = reinterpret_cast<double *>(b);
  b += align_up((size_t)HW * sizeof(double));
  double *excl = reinterpret_cast<double *>(b);
  b += align_up((size_t)HW * sizeof(double));
  double *tmp = reinterpret_cast<double *>(b);
  b += align_up(scan_temp_elems(HW) * sizeof(double));
  double *partial = reinterpret_cast<double *>(b);
  b += align_up((size_t)kPlaceMaxBlocks * sizeof(double));
  double *total = reinterpret_cast<double *>(b);
  const int nb = place_blocks(HW);
  if (image)
    error_weight_kernel<<<nb, kPlaceThreads, 0, s>>>(image, target, n, HW, wgt, partial);
  else
    edge_weight_kernel<<<nb, kPlaceThreads, 0, s>>>(target, n, H, W, wgt, partial);
  weight_total_kernel<<<1, kPlaceThreads, 0, s>>>(partial, nb, total);
  hipError_t e = scan_f64(wgt, excl, HW, tmp, s);
  if (e != hipSuccess) return e;
  if (count > 0)
    sample_place_kernel<<<(count + kPlaceThreads - 1) / kPlaceThreads, kPlaceThreads, 0, s>>>(
        excl, wgt, total, HW, image ? 0.0 : lam, uniforms, count, target, n, H, W, scale,
        render_params, fit_params, N_total, first);
  return hipGetLastError();
}

}  // namespace igs
