// Host side of the libimagegs C ABI (include/imagegs.h): argument validation, carving of the
// caller's saved-state and workspace buffers, and the launch sequence of each entry point.
// The library allocates no device memory and never synchronizes the caller's stream.
#include "../../include/imagegs.h"

#include <algorithm>

#include "common.hpp"
#include "timing.hpp"

#define IGS_API extern "C" __attribute__((visibility("default")))

namespace igs {

static int ceil_log2(int64_t x) {
  int b = 0;
  while (((int64_t)1 << b) < x) ++b;
  return b;
}

Dims make_dims(int N, int n, int H, int W, int K, int64_t cap) {
  Dims d{};
  d.N = N;
  d.n = n;
  d.H = H;
  d.W = W;
  d.K = K;
  d.cap = cap;
  d.tiles_x = (W + kTile - 1) / kTile;
  d.tiles_y = (H + kTile - 1) / kTile;
  d.T = d.tiles_x * d.tiles_y;
  d.HW = (int64_t)H * W;
  d.key_bits = std::max(1, ceil_log2(d.T));
  d.passes = (d.key_bits + 7) / 8;
  d.digit_bits = (d.key_bits + d.passes - 1) / d.passes;
  d.sort_blocks = (cap + kSortTileItems - 1) / kSortTileItems;
  return d;
}

SavedLayout saved_layout(const Dims &d) {
  SavedLayout L{};
  size_t o = 0;
  L.status = o;
  o = align_up(o + 8 * sizeof(int64_t));
  L.ranges = o;
  o = align_up(o + (size_t)d.T * sizeof(int2));
  L.vals = o;
  o = align_up(o + (size_t)d.cap * sizeof(uint32_t));
  L.g32a = o;
  o = align_up(o + (size_t)d.N * sizeof(float4));
  L.g32b = o;
  o = align_up(o + (size_t)d.N * sizeof(float2));
  L.g64 = o;
  o = align_up(o + (size_t)d.N * sizeof(double4));
  L.slots = o;
  o = align_up(o + (size_t)d.K * d.HW * sizeof(uint16_t));
  L.aux = o;
  o = align_up(o + (size_t)d.HW * sizeof(float2));
  L.total = o;
  return L;
}

WsLayout ws_layout(const Dims &d) {
  WsLayout L{};
  size_t o = 0;
  const int64_t hist_elems = ((int64_t)1 << d.digit_bits) * d.sort_blocks;
  L.counts = o;
  o = align_up(o + (size_t)d.N * sizeof(uint32_t));
  L.offsets = o;
  o = align_up(o + (size_t)d.N * sizeof(int64_t));
  L.keys = o;
  o = align_up(o + (size_t)d.cap * sizeof(uint32_t));
  L.keys_alt = o;
  o = align_up(o + (size_t)d.cap * sizeof(uint32_t));
  L.vals_alt = o;
  o = align_up(o + (size_t)d.cap * sizeof(uint32_t));
  L.hist = o;
  o = align_up(o + (size_t)hist_elems * sizeof(uint32_t));
  L.hist_off = o;
  o = align_up(o + (size_t)hist_elems * sizeof(uint32_t));
  L.scan_tmp = o;
  o = align_up(o + std::max(scan_temp_elems(d.N) * sizeof(int64_t),
                            scan_temp_elems(hist_elems) * sizeof(uint32_t)));
  L.gamma = o;
  o = align_up(o + (size_t)5 * d.N * sizeof(float));
  L.l1_tmp = o;
  L.total = o;
  return L;
}

static igs_status check_dims(int32_t N, int32_t n, int32_t H, int32_t W, int32_t K,
                             int32_t tile_h, int32_t tile_w, int64_t cap) {
  if (N < 0 || n < 1 || n > IGS_MAX_CHANNELS || K < 1 || K > IGS_MAX_K || H < 1 || W < 1 ||
      H > 65536 || W > 65536 || cap < 1 || cap > (int64_t)0x7FFFFFFF)
    return IGS_ERR_INVALID_ARG;
  if (tile_h != kTile || tile_w != kTile) return IGS_ERR_UNSUPPORTED;
  const int64_t T = (int64_t)((W + kTile - 1) / kTile) * ((H + kTile - 1) / kTile);
  if (T > ((int64_t)1 << 24)) return IGS_ERR_INVALID_ARG;
  return IGS_OK;
}

static bool aligned(const void *p) { return ((uintptr_t)p & 255u) == 0; }

template <typename T>
static T *at(void *base, size_t off) {
  return reinterpret_cast<T *>(static_cast<char *>(base) + off);
}

}  // namespace igs

using namespace igs;

#define IGS_HIP(call)                          \
  do {                                         \
    if ((call) != hipSuccess) return IGS_ERR_HIP; \
  } while (0)

IGS_API int32_t igs_abi_version(void) { return 1; }

IGS_API const char *igs_status_string(igs_status s) {
  switch (s) {
    case IGS_OK:
      return "ok";
    case IGS_ERR_INVALID_ARG:
      return "invalid argument";
    case IGS_ERR_WORKSPACE:
      return "workspace or saved buffer too small or misaligned";
    case IGS_ERR_HIP:
      return "HIP runtime or launch failure";
    case IGS_ERR_UNSUPPORTED:
      return "unsupported configuration";
    default:
      return "unknown status";
  }
}

IGS_API igs_status igs_render_buffer_sizes(int32_t N, int32_t n, int32_t H, int32_t W, int32_t K,
                                           int32_t tile_h, int32_t tile_w, int64_t pair_capacity,
                                           size_t *ws_bytes, size_t *saved_bytes) {
  if (!ws_bytes || !saved_bytes) return IGS_ERR_INVALID_ARG;
  igs_status st = check_dims(N, n, H, W, K, tile_h, tile_w, pair_capacity);
  if (st != IGS_OK) return st;
  const Dims d = make_dims(N, n, H, W, K, pair_capacity);
  *ws_bytes = ws_layout(d).total;
  *saved_bytes = saved_layout(d).total;
  return IGS_OK;
}

IGS_API igs_status igs_saved_offsets(int32_t N, int32_t n, int32_t H, int32_t W, int32_t K,
                                     int32_t tile_h, int32_t tile_w, int64_t pair_capacity,
                                     int64_t out[6]) {
  if (!out) return IGS_ERR_INVALID_ARG;
  igs_status st = check_dims(N, n, H, W, K, tile_h, tile_w, pair_capacity);
  if (st != IGS_OK) return st;
  const SavedLayout L = saved_layout(make_dims(N, n, H, W, K, pair_capacity));
  out[0] = (int64_t)L.status;
  out[1] = (int64_t)L.ranges;
  out[2] = (int64_t)L.vals;
  out[3] = (int64_t)L.slots;
  out[4] = (int64_t)L.aux;
  out[5] = (int64_t)L.total;
  return IGS_OK;
}

IGS_API igs_status igs_render(const float *params, int32_t N, int32_t n, int32_t H, int32_t W,
                              int32_t K, int32_t tile_h, int32_t tile_w, int64_t pair_capacity,
                              float *image, void *saved, size_t saved_bytes, void *workspace,
                              size_t ws_bytes, void *stream) {
  igs_status st = check_dims(N, n, H, W, K, tile_h, tile_w, pair_capacity);
  if (st != IGS_OK) return st;
  if ((N > 0 && !params) || !image || !workspace) return IGS_ERR_INVALID_ARG;
  const Dims d = make_dims(N, n, H, W, K, pair_capacity);
  const SavedLayout SL = saved_layout(d);
  const WsLayout WL = ws_layout(d);
  void *sv = saved;
  if (!sv) {
    if (ws_bytes < WL.total + SL.total) return IGS_ERR_WORKSPACE;
    sv = static_cast<char *>(workspace) + WL.total;
  } else if (saved_bytes < SL.total || ws_bytes < WL.total) {
    return IGS_ERR_WORKSPACE;
  }
  if (!aligned(sv) || !aligned(workspace)) return IGS_ERR_WORKSPACE;
  hipStream_t s = static_cast<hipStream_t>(stream);

  int64_t *status = at<int64_t>(sv, SL.status);
  int2 *ranges = at<int2>(sv, SL.ranges);
  uint32_t *vals = at<uint32_t>(sv, SL.vals);
  float4 *g32a = at<float4>(sv, SL.g32a);
  float2 *g32b = at<float2>(sv, SL.g32b);
  double4 *g64 = at<double4>(sv, SL.g64);
  uint16_t *slots = at<uint16_t>(sv, SL.slots);
  float2 *aux = at<float2>(sv, SL.aux);
  uint32_t *counts = at<uint32_t>(workspace, WL.counts);
  int64_t *offsets = at<int64_t>(workspace, WL.offsets);
  uint32_t *keys = at<uint32_t>(workspace, WL.keys);
  uint32_t *keys_alt = at<uint32_t>(workspace, WL.keys_alt);
  uint32_t *vals_alt = at<uint32_t>(workspace, WL.vals_alt);
  uint32_t *hist = at<uint32_t>(workspace, WL.hist);
  uint32_t *hist_off = at<uint32_t>(workspace, WL.hist_off);
  void *scan_tmp = at<void>(workspace, WL.scan_tmp);

  {
    PhaseTimer timer(kPhaseBinning, s);
    IGS_HIP(launch_status_reset(status, s));
    IGS_HIP(launch_fill_u32(reinterpret_cast<uint32_t *>(ranges), 2 * (int64_t)d.T, 0u, s));
  IGS_HIP(launch_preprocess(params, N, H, W, d.tiles_x, d.tiles_y, g32a, g32b, g64, counts, s));
  IGS_HIP(scan_u32_to_i64(counts, offsets, N, static_cast<int64_t *>(scan_tmp), s));
  IGS_HIP(launch_pair_total(counts, offsets, N, pair_capacity, status, s));
  const bool alt = sort_starts_in_alt(d.passes);
  IGS_HIP(launch_emit(params, N, H, W, d.tiles_x, d.tiles_y, counts, offsets, pair_capacity,
                      alt ? keys_alt : keys, alt ? vals_alt : vals, s));
  IGS_HIP(radix_sort_pairs(keys, vals, keys_alt, vals_alt, status, pair_capacity, d.key_bits,
                           d.passes, d.digit_bits, hist, hist_off,
                           static_cast<uint32_t *>(scan_tmp), s));
    IGS_HIP(launch_tile_ranges(keys, status, pair_capacity, ranges, s));
    IGS_HIP(launch_tile_stats(ranges, d.T, d.tiles_x, H, W, K, status, s));
  }
  PhaseTimer timer(kPhaseRasterFwd, s);
  IGS_HIP(launch_raster_fwd(ranges, vals, g32a, g32b, g64, params, d, image, slots, aux, status,
                            s));
  return IGS_OK;
}

IGS_API igs_status igs_render_backward(const float *params, int32_t N, int32_t n, int32_t H,
                                       int32_t W, int32_t K, int32_t tile_h, int32_t tile_w,
                                       int64_t pair_capacity, const float *image,
                                       const float *grad_image, const void *saved,
                                       size_t saved_bytes, float *grad_params, void *workspace,
                                       size_t ws_bytes, void *stream) {
  igs_status st = check_dims(N, n, H, W, K, tile_h, tile_w, pair_capacity);
  if (st != IGS_OK) return st;
  if ((N > 0 && (!params || !grad_params)) || !image || !grad_image || !saved || !workspace)
    return IGS_ERR_INVALID_ARG;
  const Dims d = make_dims(N, n, H, W, K, pair_capacity);
  const SavedLayout SL = saved_layout(d);
  const WsLayout WL = ws_layout(d);
  if (saved_bytes < SL.total || ws_bytes < WL.total) return IGS_ERR_WORKSPACE;
  if (!aligned(saved) || !aligned(workspace)) return IGS_ERR_WORKSPACE;
  if (N == 0) return IGS_OK;
  hipStream_t s = static_cast<hipStream_t>(stream);
  void *sv = const_cast<void *>(saved);
  const int2 *ranges = at<int2>(sv, SL.ranges);
  const uint32_t *vals = at<uint32_t>(sv, SL.vals);
  const float4 *g32a = at<float4>(sv, SL.g32a);
  const float2 *g32b = at<float2>(sv, SL.g32b);
  const double4 *g64 = at<double4>(sv, SL.g64);
  const uint16_t *slots = at<uint16_t>(sv, SL.slots);
  const float2 *aux = at<float2>(sv, SL.aux);
  float *gamma = at<float>(workspace, WL.gamma);

  PhaseTimer timer(kPhaseRasterBwd, s);
  IGS_HIP(launch_fill_f32(gamma, 5 * (int64_t)N, 0.f, s));
  IGS_HIP(launch_fill_f32(grad_params + 5 * (size_t)N, (int64_t)n * N, 0.f, s));
  IGS_HIP(launch_raster_bwd(ranges, vals, g32a, g32b, g64, params, d, image, grad_image, slots,
                            aux, gamma, grad_params, s));
  IGS_HIP(launch_grad_finalize(params, g32a, g32b, gamma, N, grad_params, s));
  return IGS_OK;
}

IGS_API igs_status igs_l1_workspace_size(int64_t count, size_t *ws_bytes) {
  if (count < 1 || !ws_bytes) return IGS_ERR_INVALID_ARG;
  *ws_bytes = align_up((size_t)l1_blocks(count) * 2 * sizeof(double));
  return IGS_OK;
}

IGS_API igs_status igs_l1_loss_grad(const float *image, const float *target, int32_t n, int32_t H,
                                    int32_t W, float *grad_image, double *loss_out,
                                    void *workspace, size_t ws_bytes, void *stream) {
  if (n < 1 || H < 1 || W < 1 || !image || !target || !grad_image || !loss_out || !workspace)
    return IGS_ERR_INVALID_ARG;
  const int64_t count = (int64_t)n * H * W;
  if (ws_bytes < (size_t)l1_blocks(count) * 2 * sizeof(double)) return IGS_ERR_WORKSPACE;
  PhaseTimer timer(kPhaseLoss, static_cast<hipStream_t>(stream));
  IGS_HIP(launch_l1(image, target, count, grad_image, static_cast<double *>(workspace), loss_out,
                    static_cast<hipStream_t>(stream)));
  return IGS_OK;
}

IGS_API igs_status igs_adam_step(float *fit_params, float *render_params, const float *grad_render,
                                 float *m, float *v, int32_t *step, const int64_t *skip_flag,
                                 int32_t N, int32_t n,
                                 int32_t H, int32_t W, float lr_mu, float lr_theta,
                                 float lr_inv_scale, float lr_color, float beta1, float beta2,
                                 float eps, float inv_scale_lo, float inv_scale_hi, void *stream) {
  if (N < 0 || n < 1 || n > IGS_MAX_CHANNELS || H < 1 || W < 1 || !step) return IGS_ERR_INVALID_ARG;
  if (N > 0 && (!fit_params || !render_params || !grad_render || !m || !v)) return IGS_ERR_INVALID_ARG;
  if (!(beta1 >= 0.f && beta1 < 1.f && beta2 >= 0.f && beta2 < 1.f && eps >= 0.f &&
        inv_scale_lo > 0.f && inv_scale_hi >= inv_scale_lo))
    return IGS_ERR_INVALID_ARG;
  PhaseTimer timer(kPhaseAdam, static_cast<hipStream_t>(stream));
  IGS_HIP(launch_adam(fit_params, render_params, grad_render, m, v, step, skip_flag, N, n, H, W, lr_mu,
                      lr_theta, lr_inv_scale, lr_color, beta1, beta2, eps, inv_scale_lo,
                      inv_scale_hi, static_cast<hipStream_t>(stream)));
  return IGS_OK;
}

IGS_API igs_status igs_fit_to_render(const float *fit_params, float *render_params, int32_t N,
                                     int32_t n, int32_t H, int32_t W, void *stream) {
  if (N < 0 || n < 1 || n > IGS_MAX_CHANNELS || H < 1 || W < 1) return IGS_ERR_INVALID_ARG;
  if (N > 0 && (!fit_params || !render_params)) return IGS_ERR_INVALID_ARG;
  IGS_HIP(launch_fit_to_render(fit_params, render_params, N, n, H, W,
                               static_cast<hipStream_t>(stream)));
  return IGS_OK;
}

IGS_API igs_status igs_timing_enable(int32_t on) {
  timing_enable(on != 0);
  return IGS_OK;
}

IGS_API igs_status igs_timing_read(double ms_out[IGS_NUM_PHASES], int64_t calls_out[IGS_NUM_PHASES],
                                   int32_t reset) {
  if (!ms_out || !calls_out) return IGS_ERR_INVALID_ARG;
  IGS_HIP(timing_read(ms_out, calls_out, reset != 0));
  return IGS_OK;
}
