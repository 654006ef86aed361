// Host side of the libimagegs C ABI (include/imagegs.h): argument validation, carving of the
// caller's saved-state and workspace buffers, and the launch sequence of each entry point.
// The library allocates no device memory and never synchronizes the caller's stream.
#include "../../include/imagegs.h"

#include <algorithm>
#include <mutex>
#include <vector>

#include "common.hpp"
#include "timing.hpp"

#define IGS_API extern "C" __attribute__((visibility("default")))

namespace igs {

static int ceil_log2(int64_t x) {
  int b = 0;
  while (((int64_t)1 << b) < x) ++b;
  return b;
}

// Pair sort plan: up to 16 key bits, a partition by the top min(8, key_bits) bits and one
// workgroup per group for the rest (at most 8 bits); the Gaussian index rides in the key when
// tile and Gaussian bits fit 32 bits together.
static void set_group_sort(Dims &d) {
  d.group_sort = d.key_bits <= 16;
  d.hb = std::min(8, d.key_bits);
  d.lb = d.key_bits - d.hb;
  d.gid_shift =
      d.group_sort && ceil_log2(std::max(d.N, 1)) + d.key_bits <= 32 ? d.key_bits : 0;
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
  set_group_sort(d);
  return d;
}

Dims make_batch_dims(const ImageDesc *descs, int B, int n, int K, int64_t cap) {
  Dims d{};
  int64_t N = 0, T = 0, HW = 0;
  for (int b = 0; b < B; ++b) {
    N += descs[b].N;
    T += (int64_t)descs[b].tiles_x * descs[b].tiles_y;
    HW += (int64_t)descs[b].H * descs[b].W;
  }
  d.N = (int)N;
  d.n = n;
  d.K = K;
  d.cap = cap;
  d.T = (int)T;
  d.HW = HW;
  d.H = d.W = d.tiles_x = d.tiles_y = 0;
  d.key_bits = std::max(1, ceil_log2(d.T));
  d.passes = (d.key_bits + 7) / 8;
  d.digit_bits = (d.key_bits + d.passes - 1) / d.passes;
  d.sort_blocks = (std::max<int64_t>(cap, d.T) + kSortTileItems - 1) / kSortTileItems;
  set_group_sort(d);
  return d;
}

SavedLayout saved_layout(const Dims &d) {
  SavedLayout L{};
  size_t o = 0;
  L.status = o;
  o = align_up(o + 8 * sizeof(int64_t));
  L.ranges = o;
  o = align_up(o + (size_t)d.T * sizeof(int2));
  L.order = o;
  o = align_up(o + (size_t)d.T * sizeof(int32_t));
  L.vals = o;
  o = align_up(o + (size_t)d.cap * sizeof(uint32_t));
  L.src = o;
  o = align_up(o + (size_t)d.cap * sizeof(uint32_t));
  L.counts = o;
  o = align_up(o + (size_t)d.N * sizeof(uint32_t));
  L.offsets = o;
  o = align_up(o + (size_t)d.N * sizeof(int64_t));
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
  L.l1_rec = o;
  o = align_up(o + (size_t)d.HW * sizeof(float2));
  L.total = o;
  return L;
}

WsLayout ws_layout(const Dims &d) {
  WsLayout L{};
  size_t o = 0;
  // 256 digits: the widest pass of either sort (pairs, or the batch's 16-bit tile queue keys)
  const int64_t hist_elems = (int64_t)256 * d.sort_blocks;
  L.keys = o;
  o = align_up(o + (size_t)d.cap * sizeof(uint32_t));
  L.keys_alt = o;
  o = align_up(o + (size_t)d.cap * sizeof(uint32_t));
  L.vals_alt = o;
  o = align_up(o + (size_t)d.cap * sizeof(uint32_t));
  L.pair_gid = o;
  o = align_up(o + (size_t)d.cap * sizeof(uint32_t));
  L.hist = o;
  o = align_up(o + (size_t)hist_elems * sizeof(uint32_t));
  L.hist_off = o;
  o = align_up(o + (size_t)hist_elems * sizeof(uint32_t));
  L.scan_tmp = o;
  o = align_up(o + scan_temp_elems(hist_elems) * sizeof(uint32_t));
  L.part = o;
  o = align_up(o + (size_t)d.cap * part_stride(d.n) * sizeof(float));
  L.order_keys = o;  // largest-first tile queue of a batch: sort scratch
  o = align_up(o + (size_t)d.T * sizeof(uint32_t));
  L.order_keys_alt = o;
  o = align_up(o + (size_t)d.T * sizeof(uint32_t));
  L.order_vals_alt = o;
  o = align_up(o + (size_t)d.T * sizeof(uint32_t));
  L.order_count = o;
  o = align_up(o + sizeof(int64_t));
  L.l1_part = o;
  o = align_up(o + (size_t)d.T * sizeof(double2));
  L.queue_fwd = o;
  o = align_up(o + 8 * sizeof(int));
  L.queue_bwd = o;
  o = align_up(o + 8 * sizeof(int));
  L.group_part = o;
  o = align_up(o + 3 * kMaxGroups * sizeof(uint64_t));
  L.block_tot = o;
  o = align_up(o + (size_t)std::max(gauss_blocks(d.N), 1) * sizeof(uint32_t));
  L.hit_mask = o;
  o = align_up(o + (size_t)d.N * sizeof(uint64_t));
  L.hit_box = o;
  o = align_up(o + (size_t)d.N * sizeof(uint32_t));
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

namespace igs {

// per host thread: each thread starts from the defaults, and a fitter applies its own settings
// on the thread that enqueues its work
static thread_local LaunchConfig g_launch_config{0, 0, 1, 0, 0};

LaunchConfig launch_config() { return g_launch_config; }
void set_launch_config(const LaunchConfig &c) { g_launch_config = c; }

int persistent_grid(int per_cu, int T) {
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      cus <= 0)
    cus = 256;
  int64_t g = (int64_t)cus * std::max(per_cu, 1);
  const int64_t need = ((int64_t)T + 7) / 8 * 8;
  g = std::min(g, std::max<int64_t>(need, 8));
  g = std::max<int64_t>(g / 8 * 8, 8);
  return (int)g;
}

}  // namespace igs

using namespace igs;

#define IGS_HIP(call)                          \
  do {                                         \
    if ((call) != hipSuccess) return IGS_ERR_HIP; \
  } while (0)

IGS_API int32_t igs_abi_version(void) { return 3; }

#ifdef IGS_BOUNDS_CHECK
namespace igs {
static std::vector<BoundsReader> &bounds_readers() {
  static std::vector<BoundsReader> r;
  return r;
}
void register_bounds_reader(BoundsReader r) { bounds_readers().push_back(r); }
}  // namespace igs
#endif

IGS_API igs_status igs_bounds_violations(uint32_t *out) {
  if (!out) return IGS_ERR_INVALID_ARG;
  *out = 0;
#ifdef IGS_BOUNDS_CHECK
  if (hipDeviceSynchronize() != hipSuccess) return IGS_ERR_HIP;
  for (BoundsReader r : bounds_readers()) *out |= r();
  return IGS_OK;
#else
  return IGS_ERR_UNSUPPORTED;
#endif
}

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

namespace {

// Forward of one call (single image or batch); saved may be NULL (inference).  target != NULL
// selects the fused mean-absolute-error epilogue (loss_out: double[B][2]).
igs_status render_impl(const float *params, const Dims &d, const Images &imgs, bool batched,
                       float *image, void *saved, size_t saved_bytes, void *workspace,
                       size_t ws_bytes, hipStream_t s, const float *target = nullptr,
                       double *loss_out = nullptr, bool raster = true,
                       bool defer_stats = false) {
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

  int64_t *status = at<int64_t>(sv, SL.status);
  int2 *ranges = at<int2>(sv, SL.ranges);
  int *order = at<int>(sv, SL.order);
  uint32_t *vals = at<uint32_t>(sv, SL.vals);
  uint32_t *src = at<uint32_t>(sv, SL.src);
  float4 *g32a = at<float4>(sv, SL.g32a);
  float2 *g32b = at<float2>(sv, SL.g32b);
  double4 *g64 = at<double4>(sv, SL.g64);
  uint16_t *slots = at<uint16_t>(sv, SL.slots);
  float2 *aux = at<float2>(sv, SL.aux);
  uint32_t *counts = at<uint32_t>(sv, SL.counts);
  int64_t *offsets = at<int64_t>(sv, SL.offsets);
  uint32_t *pair_gid = at<uint32_t>(workspace, WL.pair_gid);
  uint32_t *keys = at<uint32_t>(workspace, WL.keys);
  uint32_t *keys_alt = at<uint32_t>(workspace, WL.keys_alt);
  uint32_t *vals_alt = at<uint32_t>(workspace, WL.vals_alt);
  uint32_t *hist = at<uint32_t>(workspace, WL.hist);
  uint32_t *hist_off = at<uint32_t>(workspace, WL.hist_off);
  void *scan_tmp = at<void>(workspace, WL.scan_tmp);

  {
    PhaseTimer timer(kPhaseBinning, s);
    // the group sort writes every tile's range itself; the LSD path needs them zeroed
    uint32_t *block_tot = at<uint32_t>(workspace, WL.block_tot);
    uint64_t *hit_mask = at<uint64_t>(workspace, WL.hit_mask);
    uint32_t *hit_box = at<uint32_t>(workspace, WL.hit_box);
    IGS_HIP(launch_preprocess(params, d.N, imgs, g32a, g32b, g64, counts, offsets, block_tot,
                              hit_mask, hit_box, status, ranges, d.group_sort ? 0 : d.T, s));
    if (d.group_sort) {
      IGS_HIP(launch_offsets_emit(params, d.N, imgs, counts, offsets, d.cap, status, keys,
                                  pair_gid, d.gid_shift, block_tot, hit_mask, hit_box, s));
      PartitionOffsets po;
      IGS_HIP(radix_partition_pairs(keys, keys_alt, vals_alt, status, d.cap, d.lb, d.hb, hist,
                                    hist_off, static_cast<uint32_t *>(scan_tmp), s, &po));
      IGS_HIP(launch_group_sort(keys_alt, vals_alt, po, d.cap, d.hb, d.lb, d.gid_shift, pair_gid,
                                imgs, d.T, d.K, raster, status,
                                at<uint64_t>(workspace, WL.group_part), src, vals, ranges,
                                !defer_stats, s));
    } else {
      const bool alt = sort_starts_in_alt(d.passes);
      IGS_HIP(launch_offsets_emit(params, d.N, imgs, counts, offsets, d.cap, status,
                                  alt ? keys_alt : keys, pair_gid, 0, block_tot, hit_mask,
                                  hit_box, s));
      IGS_HIP(radix_sort_pairs(keys, src, keys_alt, vals_alt, status, d.cap, d.key_bits,
                               d.passes, d.digit_bits, hist, hist_off,
                               static_cast<uint32_t *>(scan_tmp), s, true, true));
      IGS_HIP(launch_resolve_ranges(src, pair_gid, keys, status, d.cap, vals, ranges, s));
      IGS_HIP(launch_tile_stats(ranges, d.T, imgs, d.K, raster, status, s));
    }
    if (batched) {
      // largest-first queue: tiles by descending |S_j| (16-bit keys, stable, so ties keep the
      // tile order)
      uint32_t *ok = at<uint32_t>(workspace, WL.order_keys);
      uint32_t *oka = at<uint32_t>(workspace, WL.order_keys_alt);
      uint32_t *ova = at<uint32_t>(workspace, WL.order_vals_alt);
      int64_t *ocount = at<int64_t>(workspace, WL.order_count);
      IGS_HIP(launch_tile_order_keys(ranges, d.T, ok, reinterpret_cast<uint32_t *>(order), ocount,
                                     s));
      IGS_HIP(radix_sort_pairs(ok, reinterpret_cast<uint32_t *>(order), oka, ova, ocount, d.T, 16,
                               2, 8, hist, hist_off, static_cast<uint32_t *>(scan_tmp), s,
                               false));
    }
  }
  if (!raster) return IGS_OK;
  float2 *l1_rec = target ? at<float2>(sv, SL.l1_rec) : nullptr;
  double2 *l1_part = target ? at<double2>(workspace, WL.l1_part) : nullptr;
  {
    PhaseTimer timer(kPhaseRasterFwd, s);
    IGS_HIP(launch_raster_fwd(ranges, vals, g32a, g32b, g64, params, d, imgs,
                              batched ? order : nullptr, image, slots, aux, target, l1_rec,
                              l1_part, at<int>(workspace, WL.queue_fwd), s));
  }
  if (target) {
    PhaseTimer timer(kPhaseLoss, s);
    IGS_HIP(launch_l1_tiles_final(l1_part, imgs, d.n, loss_out, s));
  }
  return IGS_OK;
}

// fused = true: the upstream gradient is the L1 record of a fused forward (image and
// grad_image unused).
igs_status backward_impl(const float *params, const Dims &d, const Images &imgs, bool batched,
                         const float *image, const float *grad_image, const void *saved,
                         size_t saved_bytes, float *grad_params, void *workspace, size_t ws_bytes,
                         hipStream_t s, bool fused = false) {
  const SavedLayout SL = saved_layout(d);
  const WsLayout WL = ws_layout(d);
  if (saved_bytes < SL.total || ws_bytes < WL.total) return IGS_ERR_WORKSPACE;
  if (!aligned(saved) || !aligned(workspace)) return IGS_ERR_WORKSPACE;
  if (d.N == 0) return IGS_OK;
  void *sv = const_cast<void *>(saved);
  const int2 *ranges = at<int2>(sv, SL.ranges);
  const int *order = at<int>(sv, SL.order);
  const uint32_t *vals = at<uint32_t>(sv, SL.vals);
  const uint32_t *src = at<uint32_t>(sv, SL.src);
  const uint32_t *counts = at<uint32_t>(sv, SL.counts);
  const int64_t *offsets = at<int64_t>(sv, SL.offsets);
  const float4 *g32a = at<float4>(sv, SL.g32a);
  const float2 *g32b = at<float2>(sv, SL.g32b);
  const double4 *g64 = at<double4>(sv, SL.g64);
  const uint16_t *slots = at<uint16_t>(sv, SL.slots);
  const float2 *aux = at<float2>(sv, SL.aux);
  float *part = at<float>(workspace, WL.part);

  const float2 *l1_rec = fused ? at<float2>(sv, SL.l1_rec) : nullptr;
  {
    PhaseTimer timer(kPhaseRasterBwd, s);
    IGS_HIP(launch_raster_bwd(ranges, vals, src, g32a, g64, params, d, imgs,
                              batched ? order : nullptr, image, grad_image, l1_rec, slots, aux,
                              part, at<int>(workspace, WL.queue_bwd), s));
  }
  PhaseTimer timer(kPhaseGradReduce, s);
  IGS_HIP(launch_grad_reduce(params, g32a, g32b, counts, offsets, at<int64_t>(sv, SL.status),
                             part, d.N, d.n, grad_params, s));
  return IGS_OK;
}

// Single-pass L1 evaluation: binning as render_impl, then the fitting kernel (loss sums and
// per-pair records), the loss reduction and the adjoint's per-Gaussian reduction, which also
// sums the binning's per-group statistics (one launch less).
igs_status fit_l1_impl(const float *params, const Dims &d, const Images &imgs, bool batched,
                       const float *target, double *loss_out, float *grad_params, void *saved,
                       size_t saved_bytes, void *workspace, size_t ws_bytes, hipStream_t s) {
  igs_status st = render_impl(params, d, imgs, batched, nullptr, saved, saved_bytes, workspace,
                              ws_bytes, s, nullptr, nullptr, false, d.group_sort);
  if (st != IGS_OK) return st;
  const SavedLayout SL = saved_layout(d);
  const WsLayout WL = ws_layout(d);
  const int2 *ranges = at<int2>(saved, SL.ranges);
  const int *order = at<int>(saved, SL.order);
  const uint32_t *vals = at<uint32_t>(saved, SL.vals);
  const uint32_t *src = at<uint32_t>(saved, SL.src);
  const float4 *g32a = at<float4>(saved, SL.g32a);
  const float2 *g32b = at<float2>(saved, SL.g32b);
  const double4 *g64 = at<double4>(saved, SL.g64);
  double2 *l1_part = at<double2>(workspace, WL.l1_part);
  float *part = at<float>(workspace, WL.part);
  {
    PhaseTimer timer(kPhaseRasterFit, s);
    IGS_HIP(launch_raster_fit(ranges, vals, src, g32a, g32b, g64, params, d, imgs,
                              batched ? order : nullptr, target, l1_part, part,
                              at<int>(workspace, WL.queue_fwd), s));
  }
  // the gradient reduction also finishes the loss and the binning's statistics (two launches less)
  PhaseTimer timer(kPhaseGradReduce, s);
  IGS_HIP(launch_grad_reduce(params, g32a, g32b, at<uint32_t>(saved, SL.counts),
                             at<int64_t>(saved, SL.offsets), at<int64_t>(saved, SL.status), part,
                             d.N, d.n, grad_params, s, l1_part, &imgs, loss_out,
                             d.group_sort ? at<uint64_t>(workspace, WL.group_part) : nullptr,
                             1 << d.hb));
  return IGS_OK;
}

Images single_view(int H, int W, int N) {
  Images v{};
  v.one = single_image(H, W, N);
  v.arr = nullptr;
  v.B = 1;
  return v;
}

// Checks a host descriptor array as written by igs_batch_describe for n channels; *blocks_out
// receives the number of loss blocks.
igs_status check_descs(const igs_image_desc *descs, int32_t B, int32_t n, int64_t *blocks_out) {
  if (!descs || B < 1 || n < 1 || n > IGS_MAX_CHANNELS) return IGS_ERR_INVALID_ARG;
  const int64_t items = l1_batch_block_items();
  int64_t g = 0, t = 0, p = 0, blk = 0, sblk = 0;
  for (int b = 0; b < B; ++b) {
    const igs_image_desc &d = descs[b];
    if (d.H < 1 || d.W < 1 || d.H > 65536 || d.W > 65536 || d.N < 0) return IGS_ERR_INVALID_ARG;
    if (d.tiles_x != (d.W + kTile - 1) / kTile || d.tiles_y != (d.H + kTile - 1) / kTile ||
        d.gauss_off != g || d.tile_off != t || d.pix_off != p || d.l1_block_off != blk ||
        d.ssim_block_off != sblk)
      return IGS_ERR_INVALID_ARG;
    sblk += ssim_strips(d.H, d.W);
    g += d.N;
    t += (int64_t)d.tiles_x * d.tiles_y;
    p += (int64_t)d.H * d.W;
    blk += ((int64_t)n * d.H * d.W + items - 1) / items;
  }
  if (g > 0x7FFFFFFF || t > ((int64_t)1 << 24) || blk > 0x7FFFFFFF) return IGS_ERR_INVALID_ARG;
  if (blocks_out) *blocks_out = blk;
  return IGS_OK;
}

igs_status check_batch(const igs_image_desc *descs, int32_t B, int32_t n, int32_t K, int64_t cap) {
  if (K < 1 || K > IGS_MAX_K || cap < 1 || cap > (int64_t)0x7FFFFFFF) return IGS_ERR_INVALID_ARG;
  return check_descs(descs, B, n, nullptr);
}

Images batch_view(const igs_image_desc *descs_dev, int32_t B) {
  Images v{};
  v.arr = reinterpret_cast<const ImageDesc *>(descs_dev);
  v.B = B;
  return v;
}

}  // namespace

IGS_API igs_status igs_render(const float *params, int32_t N, int32_t n, int32_t H, int32_t W,
                              int32_t K, int32_t tile_h, int32_t tile_w, int64_t pair_capacity,
                              float *image, void *saved, size_t saved_bytes, void *workspace,
                              size_t ws_bytes, void *stream) {
  igs_status st = check_dims(N, n, H, W, K, tile_h, tile_w, pair_capacity);
  if (st != IGS_OK) return st;
  if ((N > 0 && !params) || !image || !workspace) return IGS_ERR_INVALID_ARG;
  return render_impl(params, make_dims(N, n, H, W, K, pair_capacity), single_view(H, W, N), false,
                     image, saved, saved_bytes, workspace, ws_bytes,
                     static_cast<hipStream_t>(stream));
}

IGS_API igs_status igs_bin(const float *params, int32_t N, int32_t n, int32_t H, int32_t W,
                           int32_t K, int32_t tile_h, int32_t tile_w, int64_t pair_capacity,
                           void *saved, size_t saved_bytes, void *workspace, size_t ws_bytes,
                           void *stream) {
  igs_status st = check_dims(N, n, H, W, K, tile_h, tile_w, pair_capacity);
  if (st != IGS_OK) return st;
  if ((N > 0 && !params) || !saved || !workspace) return IGS_ERR_INVALID_ARG;
  return render_impl(params, make_dims(N, n, H, W, K, pair_capacity), single_view(H, W, N), false,
                     nullptr, saved, saved_bytes, workspace, ws_bytes,
                     static_cast<hipStream_t>(stream), nullptr, nullptr, false);
}

IGS_API igs_status igs_query_workspace_size(int32_t M, int32_t N, int32_t n, int32_t H,
                                            int32_t W, size_t *ws_bytes) {
  if (M < 0 || N < 0 || n < 1 || n > IGS_MAX_CHANNELS || H < 1 || W < 1 || !ws_bytes)
    return IGS_ERR_INVALID_ARG;
  *ws_bytes = query_workspace_bytes(M, N, n, H, W);
  return IGS_OK;
}

IGS_API igs_status igs_query(const float *params, int32_t N, int32_t n, int32_t H, int32_t W,
                             int32_t K, int32_t tile_h, int32_t tile_w, int64_t pair_capacity,
                             const void *saved, size_t saved_bytes, const float *points,
                             int32_t M, float *out, void *workspace, size_t ws_bytes,
                             void *stream) {
  igs_status st = check_dims(N, n, H, W, K, tile_h, tile_w, pair_capacity);
  if (st != IGS_OK) return st;
  if ((N > 0 && !params) || !saved || M < 0 || (M > 0 && (!points || !out)))
    return IGS_ERR_INVALID_ARG;
  const Dims d = make_dims(N, n, H, W, K, pair_capacity);
  const SavedLayout SL = saved_layout(d);
  if (saved_bytes < SL.total) return IGS_ERR_WORKSPACE;
  if (!aligned(saved)) return IGS_ERR_WORKSPACE;
  if (workspace && (ws_bytes < query_workspace_bytes(M, N, n, H, W) || !aligned(workspace)))
    return IGS_ERR_WORKSPACE;
  void *sv = const_cast<void *>(saved);
  IGS_HIP(launch_query(params, N, n, H, W, K, at<int2>(sv, SL.ranges), at<uint32_t>(sv, SL.vals),
                       at<float4>(sv, SL.g32a), at<float2>(sv, SL.g32b), at<double4>(sv, SL.g64),
                       points, M, out, workspace, static_cast<hipStream_t>(stream)));
  return IGS_OK;
}

IGS_API igs_status igs_params_to_fp16(const float *params, int32_t N, int32_t n, uint16_t *out,
                                      void *stream) {
  if (N < 0 || n < 1 || n > IGS_MAX_CHANNELS || (N > 0 && (!params || !out)))
    return IGS_ERR_INVALID_ARG;
  IGS_HIP(launch_to_fp16(params, (int64_t)(5 + n) * N, out, static_cast<hipStream_t>(stream)));
  return IGS_OK;
}

IGS_API igs_status igs_decode_fp16(const uint16_t *stored, int32_t N_stored, int32_t n,
                                   int32_t N_prefix, int32_t H, int32_t W, float *render_params,
                                   void *stream) {
  if (N_stored < 0 || n < 1 || n > IGS_MAX_CHANNELS || N_prefix < 0 || N_prefix > N_stored ||
      H < 1 || W < 1 || (N_prefix > 0 && (!stored || !render_params)))
    return IGS_ERR_INVALID_ARG;
  IGS_HIP(launch_decode_fp16(stored, N_stored, n, N_prefix, H, W, render_params,
                             static_cast<hipStream_t>(stream)));
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
  return backward_impl(params, make_dims(N, n, H, W, K, pair_capacity), single_view(H, W, N),
                       false, image, grad_image, saved, saved_bytes, grad_params, workspace,
                       ws_bytes, static_cast<hipStream_t>(stream));
}

IGS_API igs_status igs_render_l1(const float *params, int32_t N, int32_t n, int32_t H, int32_t W,
                                 int32_t K, int32_t tile_h, int32_t tile_w, int64_t pair_capacity,
                                 const float *target, float *image, double *loss_out, void *saved,
                                 size_t saved_bytes, void *workspace, size_t ws_bytes,
                                 void *stream) {
  igs_status st = check_dims(N, n, H, W, K, tile_h, tile_w, pair_capacity);
  if (st != IGS_OK) return st;
  if (n > kMaxFusedChannels) return IGS_ERR_UNSUPPORTED;
  if ((N > 0 && !params) || !target || !image || !loss_out || !saved || !workspace)
    return IGS_ERR_INVALID_ARG;
  return render_impl(params, make_dims(N, n, H, W, K, pair_capacity), single_view(H, W, N), false,
                     image, saved, saved_bytes, workspace, ws_bytes,
                     static_cast<hipStream_t>(stream), target, loss_out);
}

IGS_API igs_status igs_render_backward_l1(const float *params, int32_t N, int32_t n, int32_t H,
                                          int32_t W, int32_t K, int32_t tile_h, int32_t tile_w,
                                          int64_t pair_capacity, const void *saved,
                                          size_t saved_bytes, float *grad_params, void *workspace,
                                          size_t ws_bytes, void *stream) {
  igs_status st = check_dims(N, n, H, W, K, tile_h, tile_w, pair_capacity);
  if (st != IGS_OK) return st;
  if (n > kMaxFusedChannels) return IGS_ERR_UNSUPPORTED;
  if ((N > 0 && (!params || !grad_params)) || !saved || !workspace) return IGS_ERR_INVALID_ARG;
  return backward_impl(params, make_dims(N, n, H, W, K, pair_capacity), single_view(H, W, N),
                       false, nullptr, nullptr, saved, saved_bytes, grad_params, workspace,
                       ws_bytes, static_cast<hipStream_t>(stream), true);
}

IGS_API igs_status igs_render_l1_grad(const float *params, int32_t N, int32_t n, int32_t H,
                                      int32_t W, int32_t K, int32_t tile_h, int32_t tile_w,
                                      int64_t pair_capacity, const float *target,
                                      double *loss_out, float *grad_params, void *saved,
                                      size_t saved_bytes, void *workspace, size_t ws_bytes,
                                      void *stream) {
  igs_status st = check_dims(N, n, H, W, K, tile_h, tile_w, pair_capacity);
  if (st != IGS_OK) return st;
  if (n > kMaxFusedChannels) return IGS_ERR_UNSUPPORTED;
  if ((N > 0 && (!params || !grad_params)) || !target || !loss_out || !saved || !workspace)
    return IGS_ERR_INVALID_ARG;
  return fit_l1_impl(params, make_dims(N, n, H, W, K, pair_capacity), single_view(H, W, N), false,
                     target, loss_out, grad_params, saved, saved_bytes, workspace, ws_bytes,
                     static_cast<hipStream_t>(stream));
}

// --------------------------------------------------------------- no-allocation variant

namespace {

// Workspace of igs_render_l1_grad_noalloc.  Every device the library runs on holds its own copy
// until the process ends; host code only ever uses its per-device address (scratch_address),
// never this name.
static __device__ __align__(256) unsigned char scratch[IGS_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxScratchDevices = 256;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxScratchDevices] = {};

// The address of the current device's copy of `scratch`, looked up once per device.
igs_status scratch_address(void **out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return IGS_ERR_HIP;
  if (dev < 0 || dev >= kMaxScratchDevices) return IGS_ERR_UNSUPPORTED;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return IGS_ERR_HIP;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return IGS_OK;
}

}  // namespace

IGS_API igs_status igs_render_l1_grad_noalloc(const float *params, int32_t N, int32_t n,
                                              int32_t H, int32_t W, int32_t K, int32_t tile_h,
                                              int32_t tile_w, int64_t pair_capacity,
                                              const float *target, double *loss_out,
                                              float *grad_params, void *saved, size_t saved_bytes,
                                              void *stream) {
  igs_status st = check_dims(N, n, H, W, K, tile_h, tile_w, pair_capacity);
  if (st != IGS_OK) return st;
  if (n > kMaxFusedChannels) return IGS_ERR_UNSUPPORTED;
  if ((N > 0 && (!params || !grad_params)) || !target || !loss_out || !saved)
    return IGS_ERR_INVALID_ARG;
  const Dims d = make_dims(N, n, H, W, K, pair_capacity);
  if (ws_layout(d).total > (size_t)IGS_NOALLOC_SCRATCH_BYTES) return IGS_ERR_WORKSPACE;
  void *ws = nullptr;
  st = scratch_address(&ws);
  if (st != IGS_OK) return st;
  return fit_l1_impl(params, d, single_view(H, W, N), false, target, loss_out, grad_params, saved,
                     saved_bytes, ws, (size_t)IGS_NOALLOC_SCRATCH_BYTES,
                     static_cast<hipStream_t>(stream));
}

// ------------------------------------------------------------------------------ batches

IGS_API igs_status igs_batch_describe(int32_t B, int32_t n, const int32_t *H, const int32_t *W,
                                      const int32_t *N, igs_image_desc *descs_out,
                                      int64_t totals_out[4]) {
  if (B < 1 || n < 1 || n > IGS_MAX_CHANNELS || !H || !W || !N || !descs_out || !totals_out)
    return IGS_ERR_INVALID_ARG;
  int64_t g = 0, t = 0, p = 0, blk = 0, sblk = 0;
  const int64_t items = l1_batch_block_items();
  for (int b = 0; b < B; ++b) {
    if (H[b] < 1 || W[b] < 1 || H[b] > 65536 || W[b] > 65536 || N[b] < 0) return IGS_ERR_INVALID_ARG;
    igs_image_desc &d = descs_out[b];
    d.H = H[b];
    d.W = W[b];
    d.N = N[b];
    d.tiles_x = (W[b] + kTile - 1) / kTile;
    d.tiles_y = (H[b] + kTile - 1) / kTile;
    d.tile_off = (int32_t)t;
    d.gauss_off = (int32_t)g;
    d.l1_block_off = (int32_t)blk;
    d.pix_off = p;
    d.ssim_block_off = sblk;
    sblk += ssim_strips(H[b], W[b]);
    g += N[b];
    t += (int64_t)d.tiles_x * d.tiles_y;
    p += (int64_t)H[b] * W[b];
    blk += ((int64_t)n * H[b] * W[b] + items - 1) / items;
    if (g > 0x7FFFFFFF || t > ((int64_t)1 << 24) || blk > 0x7FFFFFFF) return IGS_ERR_INVALID_ARG;
  }
  totals_out[0] = g;
  totals_out[1] = t;
  totals_out[2] = p;
  totals_out[3] = blk;
  return IGS_OK;
}

IGS_API igs_status igs_batch_buffer_sizes(const igs_image_desc *descs, int32_t B, int32_t n,
                                          int32_t K, int64_t pair_capacity, size_t *ws_bytes,
                                          size_t *saved_bytes) {
  if (!ws_bytes || !saved_bytes) return IGS_ERR_INVALID_ARG;
  igs_status st = check_batch(descs, B, n, K, pair_capacity);
  if (st != IGS_OK) return st;
  const Dims d = make_batch_dims(reinterpret_cast<const ImageDesc *>(descs), B, n, K, pair_capacity);
  *ws_bytes = ws_layout(d).total;
  *saved_bytes = saved_layout(d).total;
  return IGS_OK;
}

IGS_API igs_status igs_batch_saved_offsets(const igs_image_desc *descs, int32_t B, int32_t n,
                                           int32_t K, int64_t pair_capacity, int64_t out[7]) {
  if (!out) return IGS_ERR_INVALID_ARG;
  igs_status st = check_batch(descs, B, n, K, pair_capacity);
  if (st != IGS_OK) return st;
  const SavedLayout L = saved_layout(
      make_batch_dims(reinterpret_cast<const ImageDesc *>(descs), B, n, K, pair_capacity));
  out[0] = (int64_t)L.status;
  out[1] = (int64_t)L.ranges;
  out[2] = (int64_t)L.vals;
  out[3] = (int64_t)L.slots;
  out[4] = (int64_t)L.aux;
  out[5] = (int64_t)L.total;
  out[6] = (int64_t)L.order;
  return IGS_OK;
}

IGS_API igs_status igs_render_batched(const float *params, const igs_image_desc *descs_host,
                                      const igs_image_desc *descs_dev, int32_t B, int32_t n,
                                      int32_t K, int64_t pair_capacity, float *images, void *saved,
                                      size_t saved_bytes, void *workspace, size_t ws_bytes,
                                      void *stream) {
  igs_status st = check_batch(descs_host, B, n, K, pair_capacity);
  if (st != IGS_OK) return st;
  const Dims d =
      make_batch_dims(reinterpret_cast<const ImageDesc *>(descs_host), B, n, K, pair_capacity);
  if ((d.N > 0 && !params) || !descs_dev || !images || !workspace) return IGS_ERR_INVALID_ARG;
  return render_impl(params, d, batch_view(descs_dev, B), true, images, saved, saved_bytes,
                     workspace, ws_bytes, static_cast<hipStream_t>(stream));
}

IGS_API igs_status igs_render_backward_batched(const float *params, const igs_image_desc *descs_host,
                                               const igs_image_desc *descs_dev, int32_t B,
                                               int32_t n, int32_t K, int64_t pair_capacity,
                                               const float *images, const float *grad_images,
                                               const void *saved, size_t saved_bytes,
                                               float *grad_params, void *workspace,
                                               size_t ws_bytes, void *stream) {
  igs_status st = check_batch(descs_host, B, n, K, pair_capacity);
  if (st != IGS_OK) return st;
  const Dims d =
      make_batch_dims(reinterpret_cast<const ImageDesc *>(descs_host), B, n, K, pair_capacity);
  if ((d.N > 0 && (!params || !grad_params)) || !descs_dev || !images || !grad_images || !saved ||
      !workspace)
    return IGS_ERR_INVALID_ARG;
  return backward_impl(params, d, batch_view(descs_dev, B), true, images, grad_images, saved,
                       saved_bytes, grad_params, workspace, ws_bytes,
                       static_cast<hipStream_t>(stream));
}

IGS_API igs_status igs_render_l1_batched(const float *params, const igs_image_desc *descs_host,
                                         const igs_image_desc *descs_dev, int32_t B, int32_t n,
                                         int32_t K, int64_t pair_capacity, const float *targets,
                                         float *images, double *loss_out, void *saved,
                                         size_t saved_bytes, void *workspace, size_t ws_bytes,
                                         void *stream) {
  igs_status st = check_batch(descs_host, B, n, K, pair_capacity);
  if (st != IGS_OK) return st;
  if (n > kMaxFusedChannels) return IGS_ERR_UNSUPPORTED;
  const Dims d =
      make_batch_dims(reinterpret_cast<const ImageDesc *>(descs_host), B, n, K, pair_capacity);
  if ((d.N > 0 && !params) || !descs_dev || !targets || !images || !loss_out || !saved ||
      !workspace)
    return IGS_ERR_INVALID_ARG;
  return render_impl(params, d, batch_view(descs_dev, B), true, images, saved, saved_bytes,
                     workspace, ws_bytes, static_cast<hipStream_t>(stream), targets, loss_out);
}

IGS_API igs_status igs_render_backward_l1_batched(const float *params,
                                                  const igs_image_desc *descs_host,
                                                  const igs_image_desc *descs_dev, int32_t B,
                                                  int32_t n, int32_t K, int64_t pair_capacity,
                                                  const void *saved, size_t saved_bytes,
                                                  float *grad_params, void *workspace,
                                                  size_t ws_bytes, void *stream) {
  igs_status st = check_batch(descs_host, B, n, K, pair_capacity);
  if (st != IGS_OK) return st;
  if (n > kMaxFusedChannels) return IGS_ERR_UNSUPPORTED;
  const Dims d =
      make_batch_dims(reinterpret_cast<const ImageDesc *>(descs_host), B, n, K, pair_capacity);
  if ((d.N > 0 && (!params || !grad_params)) || !descs_dev || !saved || !workspace)
    return IGS_ERR_INVALID_ARG;
  return backward_impl(params, d, batch_view(descs_dev, B), true, nullptr, nullptr, saved,
                       saved_bytes, grad_params, workspace, ws_bytes,
                       static_cast<hipStream_t>(stream), true);
}

IGS_API igs_status igs_render_l1_grad_batched(const float *params,
                                              const igs_image_desc *descs_host,
                                              const igs_image_desc *descs_dev, int32_t B,
                                              int32_t n, int32_t K, int64_t pair_capacity,
                                              const float *targets, double *loss_out,
                                              float *grad_params, void *saved, size_t saved_bytes,
                                              void *workspace, size_t ws_bytes, void *stream) {
  igs_status st = check_batch(descs_host, B, n, K, pair_capacity);
  if (st != IGS_OK) return st;
  if (n > kMaxFusedChannels) return IGS_ERR_UNSUPPORTED;
  const Dims d =
      make_batch_dims(reinterpret_cast<const ImageDesc *>(descs_host), B, n, K, pair_capacity);
  if ((d.N > 0 && (!params || !grad_params)) || !descs_dev || !targets || !loss_out || !saved ||
      !workspace)
    return IGS_ERR_INVALID_ARG;
  return fit_l1_impl(params, d, batch_view(descs_dev, B), true, targets, loss_out, grad_params,
                     saved, saved_bytes, workspace, ws_bytes, static_cast<hipStream_t>(stream));
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

namespace {
struct SsimWs {
  size_t d_mx, d_exx, d_exy, partial, total;
};
SsimWs ssim_ws(int n, int H, int W) {
  const size_t plane = align_up((size_t)n * H * W * sizeof(float));
  SsimWs L{};
  L.d_mx = 0;
  L.d_exx = plane;
  L.d_exy = 2 * plane;
  L.partial = 3 * plane;
  L.total = L.partial + align_up((size_t)ssim_blocks(n, H, W) * 3 * sizeof(double));
  return L;
}
}  // namespace

IGS_API igs_status igs_l1_ssim_workspace_size(int32_t n, int32_t H, int32_t W, size_t *ws_bytes) {
  if (n < 1 || H < 1 || W < 1 || !ws_bytes) return IGS_ERR_INVALID_ARG;
  *ws_bytes = ssim_ws(n, H, W).total;
  return IGS_OK;
}

IGS_API igs_status igs_l1_ssim_loss_grad(const float *image, const float *target, int32_t n,
                                         int32_t H, int32_t W, double ssim_weight,
                                         float *grad_image, double *loss_out, void *workspace,
                                         size_t ws_bytes, void *stream) {
  if (n < 1 || H < 1 || W < 1 || !image || !target || !grad_image || !loss_out || !workspace ||
      !(ssim_weight >= 0.0 && ssim_weight <= 1.0e30))
    return IGS_ERR_INVALID_ARG;
  const SsimWs L = ssim_ws(n, H, W);
  if (ws_bytes < L.total) return IGS_ERR_WORKSPACE;
  PhaseTimer timer(kPhaseLoss, static_cast<hipStream_t>(stream));
  IGS_HIP(launch_l1_ssim(image, target, n, H, W, ssim_weight, grad_image,
                         at<float>(workspace, L.d_mx), at<float>(workspace, L.d_exx),
                         at<float>(workspace, L.d_exy), at<double>(workspace, L.partial),
                         loss_out, static_cast<hipStream_t>(stream)));
  return IGS_OK;
}

IGS_API igs_status igs_place_workspace_size(int32_t H, int32_t W, size_t *ws_bytes) {
  if (H < 1 || W < 1 || !ws_bytes) return IGS_ERR_INVALID_ARG;
  *ws_bytes = place_workspace_bytes((int64_t)H * W);
  return IGS_OK;
}

static igs_status place_impl(const float *image, const float *target, int32_t n, int32_t H,
                             int32_t W, double lam, const float *uniforms, int32_t count,
                             float scale, float *render_params, float *fit_params,
                             int32_t N_total, int32_t first, void *workspace, size_t ws_bytes,
                             void *stream) {
  if (n < 1 || n > IGS_MAX_CHANNELS || H < 1 || W < 1 || !target || count < 0 || first < 0 ||
      N_total < 0 || (int64_t)first + count > N_total || !(scale > 0.f && scale < 1e30f) ||
      !(lam >= 0.0 && lam <= 1.0) || !workspace)
    return IGS_ERR_INVALID_ARG;
  if (count > 0 && (!uniforms || !render_params)) return IGS_ERR_INVALID_ARG;
  if (ws_bytes < place_workspace_bytes((int64_t)H * W)) return IGS_ERR_WORKSPACE;
  IGS_HIP(launch_place(image, target, n, H, W, lam, uniforms, count, scale, render_params,
                       fit_params, N_total, first, workspace, static_cast<hipStream_t>(stream)));
  return IGS_OK;
}

IGS_API igs_status igs_init_gaussians(const float *target, int32_t n, int32_t H, int32_t W,
                                      double lambda_init, const float *uniforms, int32_t count,
                                      float scale, float *render_params, float *fit_params,
                                      int32_t N_total, int32_t first, void *workspace,
                                      size_t ws_bytes, void *stream) {
  return place_impl(nullptr, target, n, H, W, lambda_init, uniforms, count, scale, render_params,
                    fit_params, N_total, first, workspace, ws_bytes, stream);
}

IGS_API igs_status igs_add_gaussians(const float *image, const float *target, int32_t n,
                                     int32_t H, int32_t W, const float *uniforms, int32_t count,
                                     float scale, float *render_params, float *fit_params,
                                     int32_t N_total, int32_t first, void *workspace,
                                     size_t ws_bytes, void *stream) {
  if (!image) return IGS_ERR_INVALID_ARG;
  return place_impl(image, target, n, H, W, 0.0, uniforms, count, scale, render_params,
                    fit_params, N_total, first, workspace, ws_bytes, stream);
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
  IGS_HIP(launch_adam_lo(fit_params, render_params, grad_render, m, v, step, skip_flag, N, n,
                         single_view(H, W, N), lr_mu, lr_theta, lr_inv_scale, lr_color, beta1,
                         beta2, eps, inv_scale_lo, inv_scale_hi, static_cast<hipStream_t>(stream)));
  return IGS_OK;
}

IGS_API igs_status igs_fit_to_render(const float *fit_params, float *render_params, int32_t N,
                                     int32_t n, int32_t H, int32_t W, void *stream) {
  if (N < 0 || n < 1 || n > IGS_MAX_CHANNELS || H < 1 || W < 1) return IGS_ERR_INVALID_ARG;
  if (N > 0 && (!fit_params || !render_params)) return IGS_ERR_INVALID_ARG;
  IGS_HIP(launch_fit_to_render(fit_params, render_params, N, n, single_view(H, W, N),
                               static_cast<hipStream_t>(stream)));
  return IGS_OK;
}

IGS_API igs_status igs_grad_to_fit(const float *fit_params, const float *grad_render,
                                   float *grad_fit, int32_t N, int32_t n, int32_t H, int32_t W,
                                   void *stream) {
  if (N < 0 || n < 1 || n > IGS_MAX_CHANNELS || H < 1 || W < 1) return IGS_ERR_INVALID_ARG;
  if (N > 0 && (!fit_params || !grad_render || !grad_fit)) return IGS_ERR_INVALID_ARG;
  IGS_HIP(launch_grad_to_fit(fit_params, grad_render, grad_fit, N, n, single_view(H, W, N),
                             static_cast<hipStream_t>(stream)));
  return IGS_OK;
}

IGS_API igs_status igs_l1_batched_workspace_size(const igs_image_desc *descs, int32_t B, int32_t n,
                                                 size_t *ws_bytes) {
  int64_t blocks = 0;
  if (!ws_bytes) return IGS_ERR_INVALID_ARG;
  igs_status st = check_descs(descs, B, n, &blocks);
  if (st != IGS_OK) return st;
  *ws_bytes = align_up((size_t)std::max<int64_t>(blocks, 1) * 2 * sizeof(double));
  return IGS_OK;
}

IGS_API igs_status igs_l1_loss_grad_batched(const float *images, const float *targets,
                                            const igs_image_desc *descs_host,
                                            const igs_image_desc *descs_dev, int32_t B, int32_t n,
                                            float *grad_images, double *loss_out,
                                            void *workspace, size_t ws_bytes, void *stream) {
  int64_t blocks = 0;
  igs_status st = check_descs(descs_host, B, n, &blocks);
  if (st != IGS_OK) return st;
  if (!images || !targets || !descs_dev || !grad_images || !loss_out || !workspace)
    return IGS_ERR_INVALID_ARG;
  if (ws_bytes < (size_t)blocks * 2 * sizeof(double)) return IGS_ERR_WORKSPACE;
  PhaseTimer timer(kPhaseLoss, static_cast<hipStream_t>(stream));
  IGS_HIP(launch_l1_batched(images, targets, batch_view(descs_dev, B), n, (int)blocks, grad_images,
                            static_cast<double *>(workspace), loss_out,
                            static_cast<hipStream_t>(stream)));
  return IGS_OK;
}

static int64_t ssim_total_strips(const igs_image_desc *descs, int32_t B) {
  int64_t t = 0;
  for (int b = 0; b < B; ++b) t += ssim_strips(descs[b].H, descs[b].W);
  return t;
}

static size_t ssim_batched_bytes(const igs_image_desc *descs, int32_t B, int32_t n,
                                 size_t *maps_plane) {
  int64_t P = 0;
  for (int b = 0; b < B; ++b) P += (int64_t)descs[b].H * descs[b].W;
  const size_t plane = align_up((size_t)n * P * sizeof(float));
  if (maps_plane) *maps_plane = plane;
  return 3 * plane + align_up((size_t)n * ssim_total_strips(descs, B) * 3 * sizeof(double));
}

IGS_API igs_status igs_l1_ssim_batched_workspace_size(const igs_image_desc *descs, int32_t B,
                                                      int32_t n, size_t *ws_bytes) {
  if (!ws_bytes) return IGS_ERR_INVALID_ARG;
  igs_status st = check_descs(descs, B, n, nullptr);
  if (st != IGS_OK) return st;
  *ws_bytes = ssim_batched_bytes(descs, B, n, nullptr);
  return IGS_OK;
}

IGS_API igs_status igs_l1_ssim_loss_grad_batched(const float *images, const float *targets,
                                                 const igs_image_desc *descs_host,
                                                 const igs_image_desc *descs_dev, int32_t B,
                                                 int32_t n, double ssim_weight, float *grad_images,
                                                 double *loss_out, void *workspace,
                                                 size_t ws_bytes, void *stream) {
  igs_status st = check_descs(descs_host, B, n, nullptr);
  if (st != IGS_OK) return st;
  if (!images || !targets || !descs_dev || !grad_images || !loss_out || !workspace ||
      !(ssim_weight >= 0.0 && ssim_weight <= 1.0e30))
    return IGS_ERR_INVALID_ARG;
  size_t plane = 0;
  if (ws_bytes < ssim_batched_bytes(descs_host, B, n, &plane)) return IGS_ERR_WORKSPACE;
  char *w = static_cast<char *>(workspace);
  PhaseTimer timer(kPhaseLoss, static_cast<hipStream_t>(stream));
  IGS_HIP(launch_l1_ssim_batched(images, targets, batch_view(descs_dev, B), n,
                                 ssim_total_strips(descs_host, B), ssim_weight, grad_images,
                                 reinterpret_cast<float *>(w), reinterpret_cast<float *>(w + plane),
                                 reinterpret_cast<float *>(w + 2 * plane),
                                 reinterpret_cast<double *>(w + 3 * plane), loss_out,
                                 static_cast<hipStream_t>(stream)));
  return IGS_OK;
}

IGS_API igs_status igs_adam_step_batched(float *fit_params, float *render_params,
                                         const float *grad_render, float *m, float *v,
                                         int32_t *step, const int64_t *skip_flag,
                                         const igs_image_desc *descs_host,
                                         const igs_image_desc *descs_dev, int32_t B, int32_t n,
                                         float lr_mu, float lr_theta, float lr_inv_scale,
                                         float lr_color, float beta1, float beta2, float eps,
                                         float inv_scale_hi, void *stream) {
  igs_status st = check_descs(descs_host, B, n, nullptr);
  if (st != IGS_OK) return st;
  int64_t N = 0;
  for (int b = 0; b < B; ++b) N += descs_host[b].N;
  if (!step || !descs_dev || (N > 0 && (!fit_params || !render_params || !grad_render || !m || !v)))
    return IGS_ERR_INVALID_ARG;
  if (!(beta1 >= 0.f && beta1 < 1.f && beta2 >= 0.f && beta2 < 1.f && eps >= 0.f &&
        inv_scale_hi > 0.f))
    return IGS_ERR_INVALID_ARG;
  PhaseTimer timer(kPhaseAdam, static_cast<hipStream_t>(stream));
  IGS_HIP(launch_adam_lo(fit_params, render_params, grad_render, m, v, step, skip_flag, (int)N, n,
                         batch_view(descs_dev, B), lr_mu, lr_theta, lr_inv_scale, lr_color, beta1,
                         beta2, eps, 0.f, inv_scale_hi, static_cast<hipStream_t>(stream)));
  return IGS_OK;
}

IGS_API igs_status igs_fit_to_render_batched(const float *fit_params, float *render_params,
                                             const igs_image_desc *descs_host,
                                             const igs_image_desc *descs_dev, int32_t B,
                                             int32_t n, void *stream) {
  igs_status st = check_descs(descs_host, B, n, nullptr);
  if (st != IGS_OK) return st;
  int64_t N = 0;
  for (int b = 0; b < B; ++b) N += descs_host[b].N;
  if (!descs_dev || (N > 0 && (!fit_params || !render_params))) return IGS_ERR_INVALID_ARG;
  IGS_HIP(launch_fit_to_render(fit_params, render_params, (int)N, n, batch_view(descs_dev, B),
                               static_cast<hipStream_t>(stream)));
  return IGS_OK;
}

IGS_API igs_status igs_set_launch_config(const igs_launch_config *cfg) {
  if (!cfg || (cfg->persistent != 0 && cfg->persistent != 1) || cfg->wgs_per_cu < 0 ||
      cfg->wgs_per_cu > 64 || (cfg->fwd_cull != 0 && cfg->fwd_cull != 1) ||
      (cfg->fwd_batch != 0 && (cfg->fwd_batch < 64 || cfg->fwd_batch > kFwdBatchMax ||
                               cfg->fwd_batch % 32 != 0)) ||
      cfg->k_unroll < 0 || cfg->k_unroll > IGS_MAX_K)
    return IGS_ERR_INVALID_ARG;
  set_launch_config(LaunchConfig{cfg->persistent, cfg->wgs_per_cu, cfg->fwd_cull, cfg->fwd_batch,
                                 cfg->k_unroll});
  return IGS_OK;
}
IGS_API igs_status igs_get_launch_config(igs_launch_config *cfg) {
  if (!cfg) return IGS_ERR_INVALID_ARG;
  const LaunchConfig c = launch_config();
  cfg->persistent = c.persistent;
  cfg->wgs_per_cu = c.wgs_per_cu;
  cfg->fwd_cull = c.fwd_cull;
  cfg->fwd_batch = c.fwd_batch;
  cfg->k_unroll = c.k_unroll;
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
