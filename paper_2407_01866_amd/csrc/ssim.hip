// The SSIM term of the fitting loss (Image-GS Sec. 3.3 and Sec. 4.1: L1 + 0.1 L_SSIM) and its
// gradient with respect to the rendered image, as two stencil kernels per call.
//
// SSIM here: local weighted means under an 11 x 11 Gaussian window (sigma 1.5, weights summing
// to 1), the image extended by zeros, C1 = 0.01^2 and C2 = 0.03^2; the map
//   S = (2 mx my + C1)(2 sxy + C2) / ((mx^2 + my^2 + C1)(sxx + syy + C2))
// with variances and covariance taken as second moments minus products of means; SSIM is the mean
// of S over every channel and pixel and L = mean|x - y| + w (1 - SSIM).
//
// Both kernels walk a strip of 32 output columns and up to 128 rows of one channel plane in
// chunks of 16 rows.  Each chunk stages its 16 new input rows (with the 5-column halo on either
// side) through LDS, while the next chunk's rows are already being fetched into registers; a
// horizontal 11-tap pass turns them into 16 new rows of horizontal sums, appended to the 10 rows
// kept from the previous chunk (the vertical halo is computed once per strip, not once per
// chunk), and a vertical 11-tap pass over those 26 rows gives the chunk's outputs.
//
// Forward (ssim_fwd_kernel): the five moments mx, my, E[x^2], E[y^2], E[xy] are blurred in fp64
// (the variances are differences of nearly equal moments compared with C2 = 9e-4, so fp32 moments
// would lose up to four digits); each pixel writes the partial derivatives of S with respect to
// mx, E[x^2] and E[xy] (fp32) and adds S, |x - y| and (x - y)^2 to the block's sums.
// Backward (ssim_bwd_kernel): the three partial maps are blurred with the same window (the window
// is symmetric and zero outside the image, so the blur is its own adjoint) and combined,
//   dL/dx = sign(x - y)/count - (w/count)(blur(dS/dmx) + 2 x blur(dS/dE[x^2]) + y blur(dS/dE[xy])).
// Both passes are deterministic; the loss sums are reduced in a fixed order.
#include <cmath>

#include "common.hpp"
#include "raster_common.hpp"

namespace igs {
namespace {

constexpr int kSsimR = 5;                        // window radius
constexpr int kTaps = 2 * kSsimR + 1;
constexpr int kStripW = 32;                      // output columns of a strip
constexpr int kChunkH = 16;                      // output rows per chunk
constexpr int kMaxChunks = 8;                    // chunks per strip: at most 128 rows
constexpr int kInW = kStripW + 2 * kSsimR;       // 42 staged columns
constexpr int kRing = kChunkH + 2 * kSsimR;      // 26 rows of horizontal sums
constexpr int kSsimThreads = 256;
constexpr int kRunH = 2;                         // horizontal pass: outputs per thread (one row)
constexpr int kRunsPerRow = kStripW / kRunH;     // 16
constexpr int kRunV = 2;                         // vertical pass: outputs per thread (one column)
constexpr int kStageN = kChunkH * kInW;          // 672 staged values per plane and chunk
constexpr int kStageRegs = (kStageN + kSsimThreads - 1) / kSsimThreads;  // 3
static_assert(kChunkH * kRunsPerRow == kSsimThreads, "horizontal pass: one item per thread");
static_assert(kStripW * (kChunkH / kRunV) == kSsimThreads, "vertical pass: one item per thread");
static_assert(2 * kSsimR <= kChunkH, "the carried halo rows come from the previous chunk");
constexpr double kC1 = 0.01 * 0.01;
constexpr double kC2 = 0.03 * 0.03;

template <typename T>
struct Win {
  T w[kSsimR + 1];  // w[j]: weight at offset +-j
};

// Tap weight for offset k - R of the 11-tap window, k = 0..10.
template <typename T>
__device__ __forceinline__ T tap(const Win<T> &w, int k) {
  return w.w[k < kSsimR ? kSsimR - k : k - kSsimR];
}

__device__ __forceinline__ double wsum64(double v) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
  return v;
}

// Rows row0 .. row0 + nrows - 1, columns x0 - R .. x0 + 32 + R - 1 of NP planes into registers
// (zero outside the image), then from registers into LDS.  nrows <= 16.
template <int NP>
struct Stage {
  float v[NP][kStageRegs];

  __device__ __forceinline__ void load(const float *const (&src)[NP], int H, int W, int x0,
                                       int row0, int nrows) {
#pragma unroll
    for (int k = 0; k < kStageRegs; ++k) {
      const int i = threadIdx.x + k * kSsimThreads;
      const int r = i / kInW, c = i - r * kInW;
      const int h = row0 + r, w = x0 - kSsimR + c;
      const bool in = i < nrows * kInW && h >= 0 && h < H && w >= 0 && w < W;
      const size_t e = in ? (size_t)h * W + w : 0;
#pragma unroll
      for (int p = 0; p < NP; ++p) v[p][k] = in ? src[p][e] : 0.f;
    }
  }
  __device__ __forceinline__ void store(float (*dst)[kStageN], int nrows) const {
#pragma unroll
    for (int k = 0; k < kStageRegs; ++k) {
      const int i = threadIdx.x + k * kSsimThreads;
      if (i < nrows * kInW)
#pragma unroll
        for (int p = 0; p < NP; ++p) dst[p][i] = v[p][k];
    }
  }
};

// Forward horizontal pass: staged rows 0 .. nrows - 1 of x and y (image rows row0 + r) -> rows
// ring0 + r of the five moment sums.  Every image row of the strip is staged exactly once, so the
// L1 and squared-error sums are taken here, over the staged pixels of rows [row_lo, row_hi) and
// columns < W.
__device__ __forceinline__ void fwd_horizontal(const float (*s_in)[kStageN],
                                               double (*s_h)[kRing * kStripW], int nrows,
                                               int ring0, const Win<double> &win, int row0,
                                               int row_lo, int row_hi, int x0, int W,
                                               double &sum_a, double &sum_q) {
  const int tid = threadIdx.x;
  if (tid >= nrows * kRunsPerRow) return;
  const int r = tid / kRunsPerRow, c0 = (tid - r * kRunsPerRow) * kRunH;
  const int h = row0 + r;
  if (h >= row_lo && h < row_hi) {
#pragma unroll
    for (int o = 0; o < kRunH; ++o) {
      if (x0 + c0 + o < W) {
        const int li = r * kInW + c0 + o + kSsimR;
        const double d = (double)s_in[0][li] - (double)s_in[1][li];  // exact
        sum_a += fabs(d);
        sum_q += d * d;
      }
    }
  }
  double acc[kRunH][5];
#pragma unroll
  for (int o = 0; o < kRunH; ++o)
#pragma unroll
    for (int m = 0; m < 5; ++m) acc[o][m] = 0.0;
#pragma unroll
  for (int t = 0; t < kRunH + 2 * kSsimR; ++t) {
    const double xv = (double)s_in[0][r * kInW + c0 + t];
    const double yv = (double)s_in[1][r * kInW + c0 + t];
    const double v[5] = {xv, yv, xv * xv, yv * yv, xv * yv};  // products exact in fp64
#pragma unroll
    for (int o = 0; o < kRunH; ++o) {
      const int k = t - o;
      if (k >= 0 && k < kTaps) {
        const double wk = tap(win, k);
#pragma unroll
        for (int m = 0; m < 5; ++m) acc[o][m] = fma(wk, v[m], acc[o][m]);
      }
    }
  }
#pragma unroll
  for (int o = 0; o < kRunH; ++o)
#pragma unroll
    for (int m = 0; m < 5; ++m) s_h[m][(ring0 + r) * kStripW + c0 + o] = acc[o][m];
}

// Backward horizontal pass over the three partial-derivative planes.
__device__ __forceinline__ void bwd_horizontal(const float (*s_in)[kStageN],
                                               float (*s_h)[kRing * kStripW], int nrows,
                                               int ring0, const Win<float> &win) {
  const int tid = threadIdx.x;
  if (tid >= nrows * kRunsPerRow) return;
  const int r = tid / kRunsPerRow, c0 = (tid - r * kRunsPerRow) * kRunH;
  float acc[kRunH][3];
#pragma unroll
  for (int o = 0; o < kRunH; ++o)
#pragma unroll
    for (int m = 0; m < 3; ++m) acc[o][m] = 0.f;
#pragma unroll
  for (int t = 0; t < kRunH + 2 * kSsimR; ++t) {
    float v[3];
#pragma unroll
    for (int m = 0; m < 3; ++m) v[m] = s_in[m][r * kInW + c0 + t];
#pragma unroll
    for (int o = 0; o < kRunH; ++o) {
      const int k = t - o;
      if (k >= 0 && k < kTaps) {
        const float wk = tap(win, k);
#pragma unroll
        for (int m = 0; m < 3; ++m) acc[o][m] = fmaf(wk, v[m], acc[o][m]);
      }
    }
  }
#pragma unroll
  for (int o = 0; o < kRunH; ++o)
#pragma unroll
    for (int m = 0; m < 3; ++m) s_h[m][(ring0 + r) * kStripW + c0 + o] = acc[o][m];
}

// Vertical pass for column c, chunk rows r0 .. r0 + kRunV - 1: ring rows r0 .. r0 + 2R + 1, one
// moment at a time in a loop that is not unrolled, so that only one moment's 12 loads are live
// (unrolled, the compiler issues the loads of every moment first, which exceeds the register
// budget of the fp64 forward).
template <typename T, int M>
__device__ __forceinline__ void vertical(const T (*s_h)[kRing * kStripW], int c, int r0,
                                         const Win<T> &win, T (&acc)[kRunV][M]) {
#pragma unroll 1
  for (int m = 0; m < M; ++m) {
    T v[kRunV + 2 * kSsimR];
#pragma unroll
    for (int t = 0; t < kRunV + 2 * kSsimR; ++t) v[t] = s_h[m][(r0 + t) * kStripW + c];
    T a[kRunV];
#pragma unroll
    for (int o = 0; o < kRunV; ++o) a[o] = T(0);
#pragma unroll
    for (int t = 0; t < kRunV + 2 * kSsimR; ++t)
#pragma unroll
      for (int o = 0; o < kRunV; ++o) {
        const int k = t - o;
        if (k >= 0 && k < kTaps) a[o] = fma(tap(win, k), v[t], a[o]);
      }
    // m is uniform: place the results without indexing registers dynamically
#pragma unroll
    for (int mm = 0; mm < M; ++mm)
      if (mm == m)
#pragma unroll
        for (int o = 0; o < kRunV; ++o) acc[o][mm] = a[o];
  }
}

// Ring rows 16..25 become rows 0..9 for the next chunk.
template <typename T, int M>
__device__ __forceinline__ void carry_halo(T (*s_h)[kRing * kStripW]) {
  constexpr int kCarry = 2 * kSsimR * kStripW;
  for (int i = threadIdx.x; i < M * kCarry; i += kSsimThreads) {
    const int m = i / kCarry, j = i - m * kCarry;
    s_h[m][j] = s_h[m][kChunkH * kStripW + j];
  }
}

__device__ __forceinline__ int strip_chunks(int H, int ys, int cps) {
  return min(cps, (H - ys + kChunkH - 1) / kChunkH);
}

static_assert(kStripW == 32 && kMaxChunks * kChunkH == 128, "batched strips: ssim_strips()");

// The strip a workgroup processes and its image: a single image (H, W given; strips dealt so
// that each XCD gets a contiguous run, whose 5-column halos then hit that XCD's L2), or a batch
// (the image found by its first strip, ssim_block_off; strips of up to 128 rows).  blockIdx.y is
// the channel.
struct StripSpec {
  int H, W, x0, ys, cps;
  size_t plane;   // first value of the channel plane
  int64_t count;  // n H W of the image
};

__device__ __forceinline__ StripSpec strip_of(const Images &imgs, int n, int H, int W,
                                              int strips_x, int cps) {
  StripSpec r;
  if (imgs.arr) {
    int lo = 0, hi = imgs.B - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (imgs.arr[mid].ssim_block_off <= (int64_t)blockIdx.x) lo = mid;
      else hi = mid - 1;
    }
    const ImageDesc im = imgs.arr[lo];
    const int sxn = (im.W + kStripW - 1) / kStripW;
    const int local = (int)(blockIdx.x - im.ssim_block_off);
    const int sy = local / sxn, sx = local - sy * sxn;
    r.H = im.H;
    r.W = im.W;
    r.cps = kMaxChunks;
    r.x0 = sx * kStripW;
    r.ys = sy * kMaxChunks * kChunkH;
    r.plane = (size_t)n * im.pix_off + (size_t)blockIdx.y * im.H * im.W;
  } else {
    const int strip = xcd_tile(blockIdx.x, gridDim.x);
    const int sy = strip / strips_x, sx = strip - sy * strips_x;
    r.H = H;
    r.W = W;
    r.cps = cps;
    r.x0 = sx * kStripW;
    r.ys = sy * cps * kChunkH;
    r.plane = (size_t)blockIdx.y * H * W;
  }
  r.count = (int64_t)n * r.H * r.W;
  return r;
}

// Four workgroups fit a CU's LDS; the register budget is held to match (128 VGPRs).
__global__ __launch_bounds__(kSsimThreads) __attribute__((amdgpu_waves_per_eu(4))) void
ssim_fwd_kernel(
    const float *__restrict__ img, const float *__restrict__ tgt, Images imgs, int n, int H0,
    int W0, int strips_x, int cps0, Win<double> win, float *__restrict__ d_mx,
    float *__restrict__ d_exx, float *__restrict__ d_exy, double *__restrict__ partial) {
  __shared__ float s_in[2][kStageN];
  __shared__ double s_h[5][kRing * kStripW];
  __shared__ double s_red[3][kSsimThreads / 64];

  const StripSpec sp = strip_of(imgs, n, H0, W0, strips_x, cps0);
  const int H = sp.H, W = sp.W, x0 = sp.x0, ys = sp.ys;
  const size_t plane = sp.plane;
  const float *const src[2] = {img + plane, tgt + plane};
  const int tid = threadIdx.x;
  const int nchunks = strip_chunks(H, ys, sp.cps);

  // prologue: the 10 rows above the strip's first output row
  Stage<2> st;
  st.load(src, H, W, x0, ys - kSsimR, 2 * kSsimR);
  st.store(s_in, 2 * kSsimR);
  st.load(src, H, W, x0, ys + kSsimR, kChunkH);
  __syncthreads();
  const int row_hi = min(ys + nchunks * kChunkH, H);
  double sum_s = 0.0, sum_a = 0.0, sum_q = 0.0;
  fwd_horizontal(s_in, s_h, 2 * kSsimR, 0, win, ys - kSsimR, ys, row_hi, x0, W, sum_a, sum_q);

  const int c = tid & (kStripW - 1), r0 = (tid / kStripW) * kRunV;
  const int w = x0 + c;
  for (int ch = 0; ch < nchunks; ++ch) {
    __syncthreads();  // the previous horizontal pass has read s_in, the halo carry is done
    st.store(s_in, kChunkH);
    __syncthreads();
    if (ch + 1 < nchunks) st.load(src, H, W, x0, ys + (ch + 1) * kChunkH + kSsimR, kChunkH);
    fwd_horizontal(s_in, s_h, kChunkH, 2 * kSsimR, win, ys + ch * kChunkH + kSsimR, ys, row_hi,
                   x0, W, sum_a, sum_q);
    __syncthreads();
    double acc[kRunV][5];
    vertical<double, 5>(s_h, c, r0, win, acc);
#pragma unroll
    for (int o = 0; o < kRunV; ++o) {
      const int h = ys + ch * kChunkH + r0 + o;
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
        sum_s += s;
      }
    }
    __syncthreads();
    if (ch + 1 < nchunks) carry_halo<double, 5>(s_h);
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

// One block per image of a batch: its strips' sums over every channel, in a fixed order;
// out[4 b ..] = {L, L1, MSE, SSIM} of image b.
__global__ __launch_bounds__(256) void ssim_final_batched_kernel(
    const double *__restrict__ partial, Images imgs, int n, int64_t strips_total, double weight,
    double *__restrict__ out) {
  __shared__ double s_red[3][256 / 64];
  const ImageDesc im = imgs.arr[blockIdx.x];
  const int64_t nb = (int64_t)((im.W + kStripW - 1) / kStripW) *
                     ((im.H + kMaxChunks * kChunkH - 1) / (kMaxChunks * kChunkH));
  double t[3] = {0.0, 0.0, 0.0};
  for (int c = 0; c < n; ++c)
    for (int64_t j = threadIdx.x; j < nb; j += blockDim.x) {
      const double *pr = partial + ((size_t)c * strips_total + im.ssim_block_off + j) * 3;
#pragma unroll
      for (int k = 0; k < 3; ++k) t[k] += pr[k];
    }
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const double v = wsum64(t[k]);
    if ((threadIdx.x & 63) == 0) s_red[k][threadIdx.x >> 6] = v;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double sum[3] = {0.0, 0.0, 0.0};
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w)
#pragma unroll
      for (int k = 0; k < 3; ++k) sum[k] += s_red[k][w];
    const double inv = 1.0 / ((double)n * im.H * im.W);
    const double ssim = sum[0] * inv, l1 = sum[1] * inv;
    double *o = out + 4 * (size_t)blockIdx.x;
    o[0] = l1 + weight * (1.0 - ssim);
    o[1] = l1;
    o[2] = sum[2] * inv;
    o[3] = ssim;
  }
}

// Seven waves per SIMD: the register budget (72 VGPRs) that holds the strip lookup without
// spilling; LDS would allow eight workgroups per CU.
__global__ __launch_bounds__(kSsimThreads) __attribute__((amdgpu_waves_per_eu(7))) void
ssim_bwd_kernel(
    const float *__restrict__ img, const float *__restrict__ tgt,
    const float *__restrict__ d_mx, const float *__restrict__ d_exx,
    const float *__restrict__ d_exy, Images imgs, int n, int H0, int W0, int strips_x, int cps0,
    Win<float> win, double weight, float *__restrict__ grad) {
  __shared__ float s_in[3][kStageN];
  __shared__ float s_h[3][kRing * kStripW];

  const StripSpec sp = strip_of(imgs, n, H0, W0, strips_x, cps0);
  const int H = sp.H, W = sp.W, x0 = sp.x0, ys = sp.ys;
  const size_t plane = sp.plane;
  const float l1_scale = (float)(1.0 / (double)sp.count);
  const float ssim_scale = (float)(-weight / (double)sp.count);
  const float *const src[3] = {d_mx + plane, d_exx + plane, d_exy + plane};
  const int tid = threadIdx.x;
  const int nchunks = strip_chunks(H, ys, sp.cps);

  Stage<3> st;
  st.load(src, H, W, x0, ys - kSsimR, 2 * kSsimR);
  st.store(s_in, 2 * kSsimR);
  st.load(src, H, W, x0, ys + kSsimR, kChunkH);
  __syncthreads();
  bwd_horizontal(s_in, s_h, 2 * kSsimR, 0, win);

  const int c = tid & (kStripW - 1), r0 = (tid / kStripW) * kRunV;
  const int w = x0 + c;
  for (int ch = 0; ch < nchunks; ++ch) {
    __syncthreads();
    st.store(s_in, kChunkH);
    __syncthreads();
    if (ch + 1 < nchunks) st.load(src, H, W, x0, ys + (ch + 1) * kChunkH + kSsimR, kChunkH);
    float xs[kRunV], ysv[kRunV];  // this chunk's output pixels, fetched before the passes
#pragma unroll
    for (int o = 0; o < kRunV; ++o) {
      const int h = ys + ch * kChunkH + r0 + o;
      const bool in = h < H && w < W;
      const size_t e = in ? plane + (size_t)h * W + w : 0;
      xs[o] = in ? img[e] : 0.f;
      ysv[o] = in ? tgt[e] : 0.f;
    }
    bwd_horizontal(s_in, s_h, kChunkH, 2 * kSsimR, win);
    __syncthreads();
    float acc[kRunV][3];
    vertical<float, 3>(s_h, c, r0, win, acc);
#pragma unroll
    for (int o = 0; o < kRunV; ++o) {
      const int h = ys + ch * kChunkH + r0 + o;
      if (h < H && w < W) {
        const size_t e = plane + (size_t)h * W + w;
        const float xv = xs[o], yv = ysv[o];
        const float d = xv - yv;  // exact sign; zero only when equal
        const float sg = d > 0.f ? l1_scale : (d < 0.f ? -l1_scale : 0.f);
        const float gs = acc[o][0] + 2.f * xv * acc[o][1] + yv * acc[o][2];
        grad[e] = fmaf(ssim_scale, gs, sg);
      }
    }
    __syncthreads();
    if (ch + 1 < nchunks) carry_halo<float, 3>(s_h);
  }
}

template <typename T>
Win<T> make_window() {
  // exp(-j^2 / (2 sigma^2)), sigma = 1.5, normalized over j = -5..5
  double raw[kSsimR + 1], total = 0.0;
  for (int j = 0; j <= kSsimR; ++j) {
    raw[j] = std::exp(-(double)(j * j) / (2.0 * 1.5 * 1.5));
    total += (j == 0 ? 1.0 : 2.0) * raw[j];
  }
  Win<T> w;
  for (int j = 0; j <= kSsimR; ++j) w.w[j] = (T)(raw[j] / total);
  return w;
}

}  // namespace

// Chunks per strip: the tallest strips (at most 128 rows, least halo recomputation) that still
// give at least 2048 workgroups (two rounds of four per CU), so small images fill the GPU.
static int ssim_chunks_per_strip(int n, int H, int W) {
  const int64_t sx = (W + kStripW - 1) / kStripW, rows = (H + kChunkH - 1) / kChunkH;
  int cps = kMaxChunks;
  while (cps > 1 && sx * ((rows + cps - 1) / cps) * n < 2048) --cps;
  return cps;
}

int64_t ssim_blocks(int n, int H, int W) {
  const int cps = ssim_chunks_per_strip(n, H, W);
  const int64_t sx = (W + kStripW - 1) / kStripW;
  const int64_t sy = (H + cps * kChunkH - 1) / (cps * kChunkH);
  return sx * sy * n;
}

hipError_t launch_l1_ssim(const float *image, const float *target, int n, int H, int W,
                          double weight, float *grad, float *d_mx, float *d_exx, float *d_exy,
                          double *partial, double *loss_out, hipStream_t s) {
  const int cps = ssim_chunks_per_strip(n, H, W);
  const int strips_x = (W + kStripW - 1) / kStripW;
  const int strips_y = (H + cps * kChunkH - 1) / (cps * kChunkH);
  const dim3 grid(strips_x * strips_y, n);
  const int64_t count = (int64_t)n * H * W;
  Images none{};
  none.arr = nullptr;
  none.B = 0;
  ssim_fwd_kernel<<<grid, kSsimThreads, 0, s>>>(image, target, none, n, H, W, strips_x, cps,
                                                make_window<double>(), d_mx, d_exx, d_exy,
                                                partial);
  ssim_final_kernel<<<1, 1024, 0, s>>>(partial, (int64_t)grid.x * grid.y, 1.0 / (double)count,
                                       weight, loss_out);
  ssim_bwd_kernel<<<grid, kSsimThreads, 0, s>>>(image, target, d_mx, d_exx, d_exy, none, n, H, W,
                                                strips_x, cps, make_window<float>(), weight,
                                                grad);
  return hipGetLastError();
}

hipError_t launch_l1_ssim_batched(const float *images, const float *targets, const Images &imgs,
                                  int n, int64_t strips, double weight, float *grad, float *d_mx,
                                  float *d_exx, float *d_exy, double *partial, double *loss_out,
                                  hipStream_t s) {
  if (strips <= 0) return hipSuccess;
  const dim3 grid((unsigned)strips, n);
  ssim_fwd_kernel<<<grid, kSsimThreads, 0, s>>>(images, targets, imgs, n, 0, 0, 0, kMaxChunks,
                                                make_window<double>(), d_mx, d_exx, d_exy,
                                                partial);
  ssim_final_batched_kernel<<<imgs.B, 256, 0, s>>>(partial, imgs, n, strips, weight, loss_out);
  ssim_bwd_kernel<<<grid, kSsimThreads, 0, s>>>(images, targets, d_mx, d_exx, d_exy, imgs, n, 0, 0,
                                                0, kMaxChunks, make_window<float>(), weight, grad);
  return hipGetLastError();
}

}  // namespace igs
