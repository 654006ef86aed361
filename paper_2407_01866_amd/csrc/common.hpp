// Internal declarations shared by the HIP kernels and the C-ABI host code of libimagegs.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace igs {

constexpr int kTile = 16;             // tile side (pixels)
constexpr int kTilePixels = kTile * kTile;
constexpr int kRasterThreads = 256;   // one thread per pixel of a 16 x 16 tile
constexpr int kBatch = 256;           // Gaussians staged in LDS per batch (one per thread)
constexpr int kMaxK = 32;
constexpr int kMaxChannels = 32;
constexpr uint16_t kEmptySlot = 0xFFFF;

// Bounds-checked build (compiled with IGS_BOUNDS_CHECK, libimagegs_debug.so): an index checked
// with IGS_IDX that falls outside its buffer sets the bit of its site in this translation unit's
// violation word and is replaced by 0, so the access stays inside the buffer;
// igs_bounds_violations collects and clears the words.  In the normal build IGS_IDX is the index
// itself and nothing is compiled.
enum BoundsSite : unsigned {
  kSiteEmit = 0,         // pair emission: emit index < pair capacity
  kSiteSortScatter = 1,  // radix scatter: destination < pair capacity
  kSiteResolve = 2,      // sorted emit index < pair capacity
  kSiteStage = 3,        // forward LDS batch: visiting position < batch size
  kSiteSlot = 4,         // a retained slot of a single-batch tile < batch size
  kSiteAdjCounter = 5,   // adjoint LDS: per-Gaussian sub-counters
  kSiteAdjItem = 6,      // adjoint LDS: placed items
  kSiteAdjChunk = 7,     // adjoint LDS: chunk owners and chunk rows
};
#ifdef IGS_BOUNDS_CHECK
namespace {
__device__ unsigned int g_bounds_word;
}
__device__ __forceinline__ int64_t check_index(int64_t i, int64_t n, unsigned site) {
  if (i < 0 || i >= n) {
    atomicOr(&g_bounds_word, 1u << site);
    return 0;
  }
  return i;
}
#define IGS_IDX(i, n, site) ::igs::check_index((int64_t)(i), (int64_t)(n), (site))
using BoundsReader = unsigned (*)();
void register_bounds_reader(BoundsReader r);  // api.cpp
namespace {
// reads and clears this translation unit's word (synchronous)
inline unsigned take_bounds_word() {
  unsigned v = 0, z = 0;
  if (hipMemcpyFromSymbol(&v, HIP_SYMBOL(g_bounds_word), sizeof(v)) != hipSuccess) return ~0u;
  if (hipMemcpyToSymbol(HIP_SYMBOL(g_bounds_word), &z, sizeof(z)) != hipSuccess) return ~0u;
  return v;
}
struct BoundsRegistrar {
  BoundsRegistrar() { register_bounds_reader(&take_bounds_word); }
};
const BoundsRegistrar g_bounds_registrar;
}  // namespace
#else
#define IGS_IDX(i, n, site) (i)
#endif

// Device status block (int64 words), see include/imagegs.h.
enum StatusWord {
  kStatPairs = 0,
  kStatOverflow = 1,
  kStatMaxList = 2,
  kStatSlotOverflow = 3,
  kStatEvalsFwd = 4,
  kStatEvalsBwd = 5,
  kStatSkip = 6  // the render's gradient must not be applied (pair overflow, or 16-bit slots
                 // that cannot address a hit set)
};

// The tile statistics of the status block from per-group shares (part[3 g + 0..2] = largest
// |S_j|, E_fwd and E_bwd of group g < G; integers, exact in any order), by one workgroup of 256
// threads: a plain store per word, so no atomics contend for the block's one cache line.  The
// preprocess kernel zeroed the words and the emit kernel set the skip word on a pair overflow,
// which this only ever raises (slots16: a hit set beyond 16-bit slots also sets it).
__device__ inline void sum_group_stats(const unsigned long long *__restrict__ part, int G,
                                       int slots16, int64_t *__restrict__ status) {
  __shared__ unsigned long long s_st[4][3];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  unsigned long long mx = 0, ef = 0, eb = 0;
  for (int g = tid; g < G; g += 256) {
    const unsigned long long m = part[3 * g];
    mx = m > mx ? m : mx;
    ef += part[3 * g + 1];
    eb += part[3 * g + 2];
  }
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) {
    const unsigned long long omx = __shfl_down(mx, d, 64);
    mx = omx > mx ? omx : mx;
    ef += __shfl_down(ef, d, 64);
    eb += __shfl_down(eb, d, 64);
  }
  if (lane == 0) {
    s_st[w][0] = mx;
    s_st[w][1] = ef;
    s_st[w][2] = eb;
  }
  __syncthreads();
  if (tid == 0) {
    for (int k = 1; k < 4; ++k) {
      mx = s_st[k][0] > mx ? s_st[k][0] : mx;
      ef += s_st[k][1];
      eb += s_st[k][2];
    }
    status[kStatMaxList] = (int64_t)mx;
    status[kStatSlotOverflow] = mx > 0xFFFF ? 1 : 0;
    if (slots16 && mx > 0xFFFF) status[kStatSkip] = 1;
    status[kStatEvalsFwd] = (int64_t)ef;
    status[kStatEvalsBwd] = (int64_t)eb;
  }
}

// Radix sort geometry.
constexpr int kSortThreads = 256;
constexpr int kSortItems = 8;
constexpr int kSortTileItems = kSortThreads * kSortItems;  // keys per sort block

// Scan geometry.
constexpr int kScanThreads = 256;
constexpr int kScanItems = 8;
constexpr int kScanBlockItems = kScanThreads * kScanItems;

inline size_t align_up(size_t x, size_t a = 256) { return (x + a - 1) / a * a; }

// Launch settings of the raster kernels, per host thread (igs_set_launch_config).  None of them
// changes a result bit: they choose how tiles are scheduled, whether the forward may skip
// candidates that provably cannot enter a list, how many candidates the forward stages in LDS at
// a time and how long its register-resident list is (its first K entries are the top-K whatever
// its length, because keys are unique).
struct LaunchConfig {
  int persistent;  // 0: one workgroup per tile; 1: resident workgroups pulling tiles
  int wgs_per_cu;  // persistent grid size per CU; <= 0: as many as fit
  int fwd_cull;    // forward candidate ordering and wave-level culling
  int fwd_batch;   // candidates per forward LDS batch, a multiple of 32 in [64, 256]; 0: 192
  int k_unroll;    // list length: the smallest compiled one >= max(K, k_unroll); 0: >= K
};
LaunchConfig launch_config();
void set_launch_config(const LaunchConfig &c);
constexpr int kFwdBatchDefault = 192;
constexpr int kFwdBatchMax = 256;
inline int fwd_batch_of(const LaunchConfig &c) { return c.fwd_batch > 0 ? c.fwd_batch : kFwdBatchDefault; }
// Persistent grid: per_cu workgroups on every CU of the current device, a multiple of 8 (one
// share per XCD), at least 8, and no more than needed for T tiles (rounded up to 8).
int persistent_grid(int per_cu, int T);

// One image of a render call.  A batch concatenates its images: the Gaussians of image b are the
// global indices [gauss_off, gauss_off + N) (parameter row stride = total N of the batch), its
// tiles [tile_off, tile_off + tiles_x * tiles_y) of the global tile numbering, and its pixels
// [pix_off, pix_off + H * W): its image and image gradient start at float n * pix_off, its top-K
// slots at K * pix_off, its per-pixel blend normalization at pix_off.  l1_block_off numbers the
// loss kernel's blocks (image b owns blocks [l1_block_off[b], l1_block_off[b + 1])), and
// ssim_block_off the SSIM stencils' strips (ssim_strips(H, W) per image and channel).
// Layout identical to igs_image_desc in include/imagegs.h.
struct ImageDesc {
  int32_t H, W, N, tiles_x;
  int32_t tiles_y, tile_off, gauss_off, l1_block_off;
  int64_t pix_off, ssim_block_off;
};
static_assert(sizeof(ImageDesc) == 48, "ImageDesc layout");

// The images of a call, passed by value: a single image inline, or a device array.
struct Images {
  ImageDesc one;
  const ImageDesc *arr;  // nullptr: the single image `one`
  int B;

  __device__ __forceinline__ ImageDesc at(int b) const { return arr ? arr[b] : one; }
  // the image owning global Gaussian gi (the last image whose first Gaussian is <= gi)
  __device__ __forceinline__ ImageDesc by_gauss(int gi) const {
    if (!arr) return one;
    int lo = 0, hi = B - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (arr[mid].gauss_off <= gi) lo = mid;
      else hi = mid - 1;
    }
    return arr[lo];
  }
  // the image owning global tile gt
  __device__ __forceinline__ ImageDesc by_tile(int gt) const {
    if (!arr) return one;
    int lo = 0, hi = B - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (arr[mid].tile_off <= gt) lo = mid;
      else hi = mid - 1;
    }
    return arr[lo];
  }
};

inline ImageDesc single_image(int H, int W, int N) {
  ImageDesc d{};
  d.H = H;
  d.W = W;
  d.N = N;
  d.tiles_x = (W + kTile - 1) / kTile;
  d.tiles_y = (H + kTile - 1) / kTile;
  return d;
}

// Sizes of a call.  For a batch N, T and HW are totals over its images (H, W, tiles_x, tiles_y
// then describe no single image and are unused by the kernels).
struct Dims {
  int N, n, H, W, K;
  int64_t cap;
  int tiles_x, tiles_y, T;
  int64_t HW;
  int key_bits, passes, digit_bits;
  int64_t sort_blocks;
  // Pair sort by tile.  group_sort (key_bits <= 16): a stable partition by the key's top hb bits,
  // then one workgroup per group sorting by the low lb bits (launch_group_sort); otherwise LSD
  // passes of digit_bits.  gid_shift > 0: the emitted keys carry the Gaussian index above the
  // tile bits (key = tile | gid << gid_shift), so the sorted keys give it without a lookup.
  bool group_sort;
  int hb, lb, gid_shift;
};

Dims make_dims(int N, int n, int H, int W, int K, int64_t cap);
Dims make_batch_dims(const ImageDesc *descs, int B, int n, int K, int64_t cap);

// Byte offsets inside the caller's `saved` buffer.
struct SavedLayout {
  size_t status, ranges, order, vals, src, counts, offsets, g32a, g32b, g64, slots, aux, l1_rec,
      total;
};
// Byte offsets inside the caller's workspace.
struct WsLayout {
  size_t keys, keys_alt, vals_alt, pair_gid, hist, hist_off, scan_tmp, part, order_keys,
      order_keys_alt, order_vals_alt, order_count, l1_part, queue_fwd, queue_bwd, group_part,
      block_tot, hit_mask, hit_box, l1_tmp, total;
};
// Floats per (tile, Gaussian) partial-gradient record of the adjoint: 5 geometry sums and n
// colour sums, padded to a multiple of four (16-byte aligned records).
__host__ __device__ inline int part_stride(int n) { return (5 + n + 3) & ~3; }

SavedLayout saved_layout(const Dims &d);
WsLayout ws_layout(const Dims &d);
size_t scan_temp_elems(int64_t n);

// ------------------------------------------------------------------ launchers (return hipError_t)

// binning.hip
hipError_t launch_fill_u32(uint32_t *p, int64_t count, uint32_t value, hipStream_t s);
hipError_t launch_fill_f32(float *p, int64_t count, float value, hipStream_t s);
// Workgroups of the preprocess and emit kernels for N Gaussians (one block_tot word each).
int gauss_blocks(int N);
// Per-Gaussian geometry and tile-hit counts, with their exclusive prefix inside each workgroup
// (offsets) and each workgroup's total (block_tot), and for the emit kernel each Gaussian's
// candidate box and hit pattern (hit_box, hit_mask; N each).  Also zeroes the status block and
// the T tile ranges (launched even for N = 0).
hipError_t launch_preprocess(const float *params, int N, const Images &imgs, float4 *g32a,
                             float2 *g32b, double4 *g64, uint32_t *counts, int64_t *offsets,
                             uint32_t *block_tot, uint64_t *hit_mask, uint32_t *hit_box,
                             int64_t *status, int2 *ranges, int T, hipStream_t s);
// Pair offsets and emission: offsets = exclusive scan of counts (finished inside the emit kernel
// from the preprocess kernel's per-workgroup prefixes and totals; it also writes the pair total
// and overflow flag into the status block); then every Gaussian's tile keys at their emit
// indices and pair_gid[u], the Gaussian of emit index u.  The sort carries the emit indices as
// values (generated by its first pass); the Gaussian of a sorted pair then comes from its key
// (gid_shift > 0: keys carry the Gaussian above the tile bits and pair_gid is not written) or
// from pair_gid.
hipError_t launch_offsets_emit(const float *params, int N, const Images &imgs,
                               const uint32_t *counts, int64_t *offsets, int64_t cap,
                               int64_t *status, uint32_t *keys, uint32_t *pair_gid, int gid_shift,
                               const uint32_t *block_tot, const uint64_t *hit_mask,
                               const uint32_t *hit_box, hipStream_t s);
hipError_t launch_resolve_ranges(const uint32_t *src, const uint32_t *pair_gid,
                                const uint32_t *keys, const int64_t *status, int64_t cap,
                                uint32_t *vals, int2 *ranges, hipStream_t s);
// slots16: the render saves 16-bit top-K slots for a separate adjoint, so a hit set longer than
// 65535 also sets the status block's skip word.
hipError_t launch_tile_stats(const int2 *ranges, int T, const Images &imgs, int K, bool slots16,
                             int64_t *status, hipStream_t s);
// Where the segments of a stable partition's digits start (radix_partition_pairs): digit g's
// first pair is hist_off[g * nblocks] plus, when run_sums is set, the sum of run_sums over the
// runs before run (g * nblocks) / kScanBlockItems.
struct PartitionOffsets {
  const uint32_t *hist_off;
  const uint32_t *run_sums;  // nullptr: hist_off holds full prefixes
  int nruns;
  int64_t nblocks;
};
// Second stage of the pair sort: one workgroup per group g < 2^hb of the partitioned pairs
// (keys, emit indices) sorts its segment stably by the low lb key bits and writes the sorted emit
// indices (src), the Gaussian of each sorted pair (vals: the key's bits from gid_shift on, or
// pair_gid[emit index] when gid_shift is 0), every tile's range (empty tiles [0, 0)) and the
// tile statistics of the status block (largest |S_j|, slot overflow, E_fwd, E_bwd; slots16 as
// in launch_tile_stats), summed from per-group shares in group_part (kMaxGroups x 3 words) by a
// one-workgroup kernel, or, with stats_kernel false, by a later kernel of the caller's
// (launch_grad_reduce's group_part).
constexpr int kMaxGroups = 256;
hipError_t launch_group_sort(const uint32_t *keys, const uint32_t *emit_idx,
                             const PartitionOffsets &po, int64_t cap, int hb, int lb,
                             int gid_shift, const uint32_t *pair_gid, const Images &imgs, int T,
                             int K, bool slots16, int64_t *status, uint64_t *group_part,
                             uint32_t *src, uint32_t *vals, int2 *ranges, bool stats_kernel,
                             hipStream_t s);
// Sort keys for the largest-first tile queue: key = 0xFFFF - min(|S_j|, 0xFFFF), value = tile;
// also writes T to *count.
hipError_t launch_tile_order_keys(const int2 *ranges, int T, uint32_t *keys, uint32_t *vals,
                                  int64_t *count, hipStream_t s);

// scan.hip: exclusive scans; temp must hold scan_temp_elems(n) elements of the output type.
hipError_t scan_u32_to_u32(const uint32_t *in, uint32_t *out, int64_t n, uint32_t *temp,
                           hipStream_t s);
// Level one of scan_u32_to_u32 alone: exclusive prefixes within each run of kScanBlockItems
// inputs, and each run's total in block_sums[ceil(n / kScanBlockItems)]; the full prefix of
// input i is out[i] plus the exclusive prefix of block_sums at i / kScanBlockItems.
hipError_t scan_u32_blocks(const uint32_t *in, uint32_t *out, int64_t n, uint32_t *block_sums,
                           hipStream_t s);

// radix_sort.hip: stable LSD sort of (key, val) by the low key_bits bits; the count is read
// from status on the device.  Result lands in (keys, vals); (keys_alt, vals_alt) are scratch.
// count_word: the device word holding the number of pairs (a render's status block, whose
// overflow flag then also empties the sort), or a plain count when status_semantics is false.
// identity_vals: the input value of key i is i (the first pass generates it; vals is not read).
hipError_t radix_sort_pairs(uint32_t *keys, uint32_t *vals, uint32_t *keys_alt,
                            uint32_t *vals_alt, const int64_t *status, int64_t cap, int key_bits,
                            int passes, int digit_bits, uint32_t *hist, uint32_t *hist_off,
                            uint32_t *scan_tmp, hipStream_t s, bool status_semantics = true,
                            bool identity_vals = false);
// One stable pass of the pair sort by bits [shift, shift + bits) of keys, from emit order (the
// values are the emit indices); the pair count comes from the render status block.  Result in
// (keys_out, emit_out); po receives where each digit's segment starts.
hipError_t radix_partition_pairs(const uint32_t *keys, uint32_t *keys_out, uint32_t *emit_out,
                                 const int64_t *status, int64_t cap, int shift, int bits,
                                 uint32_t *hist, uint32_t *hist_off, uint32_t *scan_tmp,
                                 hipStream_t s, PartitionOffsets *po);
// Which buffer emit must write into so the sort's final pass ends in (keys, vals).
inline bool sort_starts_in_alt(int passes) { return (passes & 1) != 0; }

// raster_fwd.hip
// tile_order: optional device array of the T global tile ids in the order workgroups take them
// (a largest-first queue for batches); nullptr = XCD-aware order of a single image's tiles.
// target != nullptr: fused mean-absolute-error epilogue (n <= kMaxFusedChannels) writing the
// per-pixel adjoint record l1_rec [pixels] and the per-tile sums l1_part [T].
constexpr int kMaxFusedChannels = 16;
hipError_t launch_raster_fwd(const int2 *ranges, const uint32_t *vals, const float4 *g32a,
                             const float2 *g32b, const double4 *g64, const float *params,
                             const Dims &d, const Images &imgs, const int *tile_order,
                             float *image, uint16_t *slots, float2 *aux, const float *target,
                             float2 *l1_rec, double2 *l1_part, int *queue, hipStream_t s);
// Per image b: loss_out[2b] = mean |d|, loss_out[2b+1] = mean d^2 from the per-tile sums.
hipError_t launch_l1_tiles_final(const double2 *l1_part, const Images &imgs, int n,
                                 double *loss_out, hipStream_t s);

// raster_bwd.hip: the adjoint writes one partial record (part_stride(n) floats) per pair at its
// emit index src[pos]; launch_grad_reduce sums each Gaussian's records in emit order.
hipError_t launch_raster_bwd(const int2 *ranges, const uint32_t *vals, const uint32_t *src,
                             const float4 *g32a, const double4 *g64, const float *params,
                             const Dims &d, const Images &imgs, const int *tile_order,
                             const float *image, const float *grad_image, const float2 *l1_rec,
                             const uint16_t *slots, const float2 *aux, float *part, int *queue,
                             hipStream_t s);
// With l1_part, its first workgroups also finish the tile loss sums of the images into
// loss_out (as launch_l1_tiles_final, bit for bit), saving that launch.  With group_part, its
// first workgroup also sums the binning's per-group statistics into the status block (a binning
// launched with stats_kernel false; 16-bit slots are not involved).
hipError_t launch_grad_reduce(const float *params, const float4 *g32a, const float2 *g32b,
                              const uint32_t *counts, const int64_t *offsets, int64_t *status,
                              const float *part, int N, int n, float *grad_params, hipStream_t s,
                              const double2 *l1_part = nullptr, const Images *imgs = nullptr,
                              double *loss_out = nullptr, const uint64_t *group_part = nullptr,
                              int groups = 0);

// raster_fit.hip: render, L1 comparison and adjoint of every tile in one pass; writes the tile loss
// sums (as the fused forward) and the adjoint's per-pair records (as launch_raster_bwd), nothing
// per pixel.
hipError_t launch_raster_fit(const int2 *ranges, const uint32_t *vals, const uint32_t *src,
                             const float4 *g32a, const float2 *g32b, const double4 *g64,
                             const float *params, const Dims &d, const Images &imgs,
                             const int *tile_order, const float *target, double2 *loss_part,
                             float *part, int *queue, hipStream_t s);

// loss_adam.hip
// SSIM strips of one channel plane of an H x W image in the batched stencils (32 x 128 each).
inline int64_t ssim_strips(int H, int W) { return (int64_t)((W + 31) / 32) * ((H + 127) / 128); }
hipError_t launch_l1_ssim_batched(const float *images, const float *targets, const Images &imgs,
                                  int n, int64_t strips, double weight, float *grad, float *d_mx,
                                  float *d_exx, float *d_exy, double *partial, double *loss_out,
                                  hipStream_t s);

// Decoding (query.hip): colours at arbitrary points from a binning pass's tile lists; float16
// storage of the fitter's parameters and decoding of a prefix into renderer units.
size_t query_workspace_bytes(int64_t M, int N, int n, int H, int W);
// ws == nullptr: points processed in input order; else they are first sorted by tile.
hipError_t launch_query(const float *params, int N, int n, int H, int W, int K,
                        const int2 *ranges, const uint32_t *vals, const float4 *g32a,
                        const float2 *g32b, const double4 *g64, const float *points, int M,
                        float *out, void *ws, hipStream_t s);
hipError_t launch_to_fp16(const float *src, int64_t count, uint16_t *dst, hipStream_t s);
hipError_t launch_decode_fp16(const uint16_t *src, int N_src, int n, int N_prefix, int H, int W,
                              float *dst, hipStream_t s);

// Placement of new Gaussians (place.hip): workspace bytes for an H x W image; image == nullptr
// samples Eq. 6 from the target's gradient, otherwise Eq. 7 from |image - target|.
size_t place_workspace_bytes(int64_t HW);
hipError_t launch_place(const float *image, const float *target, int n, int H, int W,
                        double lam, const float *uniforms, int count, float scale,
                        float *render_params, float *fit_params, int N_total, int first,
                        void *ws, hipStream_t s);
hipError_t scan_f64(const double *in, double *out, int64_t n, double *temp, hipStream_t s);

// SSIM term of the loss (ssim.hip): blocks of the stencil kernels for an [n][H][W] image, and
// the forward, final reduction and backward kernels of one call.
int64_t ssim_blocks(int n, int H, int W);
hipError_t launch_l1_ssim(const float *image, const float *target, int n, int H, int W,
                          double weight, float *grad, float *d_mx, float *d_exx, float *d_exy,
                          double *partial, double *loss_out, hipStream_t s);
int l1_blocks(int64_t count);
hipError_t launch_l1(const float *image, const float *target, int64_t count, float *grad,
                     double *partials, double *loss_out, hipStream_t s);
hipError_t launch_adam(float *fit, float *rend, const float *grad, float *m, float *v,
                       int32_t *step, const int64_t *skip, int N, int n, const Images &imgs,
                       float lr_mu, float lr_theta, float lr_u, float lr_c, float b1, float b2,
                       float eps, float u_hi, hipStream_t s);
hipError_t launch_adam_lo(float *fit, float *rend, const float *grad, float *m, float *v,
                          int32_t *step, const int64_t *skip, int N, int n, const Images &imgs,
                          float lr_mu, float lr_theta, float lr_u, float lr_c, float b1, float b2,
                          float eps, float u_lo, float u_hi, hipStream_t s);
hipError_t launch_fit_to_render(const float *fit, float *rend, int N, int n, const Images &imgs,
                                hipStream_t s);
// Gradient with respect to render parameters -> gradient with respect to fitter parameters.
hipError_t launch_grad_to_fit(const float *fit, const float *grad_rend, float *grad_fit, int N,
                              int n, const Images &imgs, hipStream_t s);
// Batched L1: per-image mean normalization; loss_out is double[B][2].
int l1_batch_block_items();
hipError_t launch_l1_batched(const float *images, const float *targets, const Images &imgs,
                             int n, int total_blocks, float *grad, double *partials,
                             double *loss_out, hipStream_t s);

}  // namespace igs
