// Stable LSD radix sort of (tile key, Gaussian index) pairs.  Stability keeps each tile's hit set
// S_j in ascending Gaussian index after the sort, which makes S_j canonical (Sec. 3.2 defines
// the set; the order fixes how equal values are ranked).  The pair count is read on the device
// so the host never waits for it.
#include "common.hpp"

namespace igs {
namespace {

// Number of pairs to sort: a render status block (pairs, overflow flag) or a plain count.
__device__ __forceinline__ int64_t live_pairs(const int64_t *status, int64_t cap, bool st) {
  int64_t P = st ? (status[kStatOverflow] ? 0 : status[kStatPairs]) : status[0];
  return P > cap ? 0 : P;
}

// Per-block digit histogram, stored digit-major: hist[d * nblocks + b].
__global__ __launch_bounds__(kSortThreads) void radix_upsweep_kernel(
    const uint32_t *__restrict__ keys, const int64_t *__restrict__ status, int64_t cap, int shift,
    int digit_bits, uint32_t *__restrict__ hist, int64_t nblocks, bool st) {
  __shared__ uint32_t lh[256];
  const int tid = threadIdx.x;
  const int R = 1 << digit_bits;
  const uint32_t mask = (uint32_t)R - 1;
  const int64_t P = live_pairs(status, cap, st);
  const int64_t base = (int64_t)blockIdx.x * kSortTileItems;
  if (tid < R) lh[tid] = 0;
  __syncthreads();
  if (base < P) {
#pragma unroll
    for (int r = 0; r < kSortItems; ++r) {
      int64_t i = base + (int64_t)r * kSortThreads + tid;
      if (i < P) atomicAdd(&lh[(keys[i] >> shift) & mask], 1u);
    }
  }
  __syncthreads();
  if (tid < R) hist[(int64_t)tid * nblocks + blockIdx.x] = lh[tid];
}

// Stable scatter: block b places its keys, round by round and lane by lane, at
// hist_off[d * nblocks + b] + (earlier rounds) + (earlier waves of this round) + (earlier lanes
// of this wave with the same digit).  Lanes with equal digits are found with one ballot per bit.
// Every thread loads its keys and values of all rounds first, so the loads are in flight together
// instead of one round trip per round.  identity: the value of key i is i itself (vals_in unread).
// With block_sums, hist_off holds the digit-offset scan's
// per-run prefixes only (scan_u32_blocks, at most kSortThreads runs), and the block adds the
// exclusive prefix of the run totals itself, scanned in LDS.
__global__ __launch_bounds__(kSortThreads) void radix_downsweep_kernel(
    const uint32_t *__restrict__ keys_in, const uint32_t *__restrict__ vals_in,
    uint32_t *__restrict__ keys_out, uint32_t *__restrict__ vals_out,
    const int64_t *__restrict__ status, int64_t cap, int shift, int digit_bits,
    const uint32_t *__restrict__ hist_off, const uint32_t *__restrict__ block_sums, int nsums,
    int64_t nblocks, bool st, bool identity) {
  constexpr int kWaves = kSortThreads / 64;
  __shared__ uint32_t digit_run[256];
  __shared__ uint32_t wave_cnt[2][kWaves][256];
  __shared__ uint32_t run_off[kSortThreads];
  __shared__ uint32_t wave_sum[kWaves];
  const int tid = threadIdx.x;
  const int lane = tid & 63, w = tid >> 6;
  const int R = 1 << digit_bits;
  const uint32_t mask = (uint32_t)R - 1;
  const int64_t P = live_pairs(status, cap, st);
  const int64_t base = (int64_t)blockIdx.x * kSortTileItems;
  if (base >= P) return;  // uniform over the block
  if (block_sums) {  // exclusive scan of the run totals
    const uint32_t v = tid < nsums ? block_sums[tid] : 0u;
    uint32_t inc = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const uint32_t o = __shfl_up(inc, d, 64);
      if (lane >= d) inc += o;
    }
    if (lane == 63) wave_sum[w] = inc;
    __syncthreads();
    uint32_t off = 0;
    for (int k = 0; k < w; ++k) off += wave_sum[k];
    run_off[tid] = off + inc - v;
    __syncthreads();
  }
  if (tid < R) {
    const int64_t h = (int64_t)tid * nblocks + blockIdx.x;
    digit_run[tid] = hist_off[h] + (block_sums ? run_off[h / kScanBlockItems] : 0u);
    for (int k = 0; k < kWaves; ++k) wave_cnt[0][k][tid] = wave_cnt[1][k][tid] = 0;
  }
  __syncthreads();
  const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  uint32_t kk[kSortItems], vv[kSortItems];
#pragma unroll
  for (int r = 0; r < kSortItems; ++r) {
    const int64_t i = base + (int64_t)r * kSortThreads + tid;
    kk[r] = i < P ? keys_in[i] : 0u;
    vv[r] = identity ? (uint32_t)i : (i < P ? vals_in[i] : 0u);
  }
#pragma unroll
  for (int r = 0; r < kSortItems; ++r) {
    const int buf = r & 1;
    const int64_t i = base + (int64_t)r * kSortThreads + tid;
    const bool valid = i < P;
    const uint32_t key = kk[r];
    const uint32_t val = vv[r];
    uint32_t d = (key >> shift) & mask;
    uint64_t peers = __ballot(valid);
    for (int b = 0; b < digit_bits; ++b) {
      bool bit = (d >> b) & 1u;
      uint64_t m = __ballot(bit);
      peers &= bit ? m : ~m;
    }
    const int rank = __popcll(peers & lt_mask);
    if (valid && rank == 0) wave_cnt[buf][w][d] = (uint32_t)__popcll(peers);
    __syncthreads();
    if (tid < R) {
      uint32_t run = digit_run[tid];
#pragma unroll
      for (int k = 0; k < kWaves; ++k) {
        uint32_t c = wave_cnt[buf][k][tid];
        wave_cnt[buf][k][tid] = run;
        run += c;
        wave_cnt[buf ^ 1][k][tid] = 0;  // last read in the previous round, next written after
                                        // this round's second barrier
      }
      digit_run[tid] = run;
    }
    __syncthreads();
    if (valid) {
      const int64_t pos = IGS_IDX(wave_cnt[buf][w][d] + (uint32_t)rank, cap, kSiteSortScatter);
      keys_out[pos] = key;
      vals_out[pos] = val;
    }
  }
}

}  // namespace

// One stable scatter pass by the digit at bits [shift, shift + bits): per-block histograms, the
// digit-offset scan and the scatter from (src_k, src_v) into (dst_k, dst_v).  The scan leaves
// per-run prefixes in hist_off and the run totals in scan_tmp (*run_sums = scan_tmp, *nruns runs)
// when there are at most kSortThreads runs, else the full prefixes (*run_sums = nullptr).
static hipError_t sort_pass(const uint32_t *src_k, const uint32_t *src_v, uint32_t *dst_k,
                            uint32_t *dst_v, const int64_t *status, int64_t cap, int shift,
                            int bits, uint32_t *hist, uint32_t *hist_off, uint32_t *scan_tmp,
                            int64_t nblocks, hipStream_t s, bool st, bool identity,
                            const uint32_t **run_sums, int *nruns) {
  radix_upsweep_kernel<<<(unsigned)nblocks, kSortThreads, 0, s>>>(src_k, status, cap, shift, bits,
                                                                   hist, nblocks, st);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int64_t hn = (int64_t)(1 << bits) * nblocks;
  const int64_t runs = (hn + kScanBlockItems - 1) / kScanBlockItems;
  *run_sums = nullptr;
  *nruns = (int)runs;
  if (runs <= kSortThreads) {
    e = scan_u32_blocks(hist, hist_off, hn, scan_tmp, s);
    *run_sums = scan_tmp;
  } else {
    e = scan_u32_to_u32(hist, hist_off, hn, scan_tmp, s);
  }
  if (e != hipSuccess) return e;
  radix_downsweep_kernel<<<(unsigned)nblocks, kSortThreads, 0, s>>>(
      src_k, src_v, dst_k, dst_v, status, cap, shift, bits, hist_off, *run_sums, (int)runs,
      nblocks, st, identity);
  return hipGetLastError();
}

hipError_t radix_sort_pairs(uint32_t *keys, uint32_t *vals, uint32_t *keys_alt,
                            uint32_t *vals_alt, const int64_t *status, int64_t cap, int key_bits,
                            int passes, int digit_bits, uint32_t *hist, uint32_t *hist_off,
                            uint32_t *scan_tmp, hipStream_t s, bool status_semantics,
                            bool identity_vals) {
  const int64_t nblocks = (cap + kSortTileItems - 1) / kSortTileItems;
  // pass p reads from src and writes to dst; with an odd pass count the data starts in alt
  uint32_t *src_k = sort_starts_in_alt(passes) ? keys_alt : keys;
  uint32_t *src_v = sort_starts_in_alt(passes) ? vals_alt : vals;
  uint32_t *dst_k = sort_starts_in_alt(passes) ? keys : keys_alt;
  uint32_t *dst_v = sort_starts_in_alt(passes) ? vals : vals_alt;
  for (int p = 0; p < passes; ++p) {
    int shift = p * digit_bits;
    int bits = digit_bits;
    if (shift + bits > key_bits) bits = key_bits - shift;
    if (bits < 1) bits = 1;
    const uint32_t *run_sums;
    int nruns;
    hipError_t e = sort_pass(src_k, src_v, dst_k, dst_v, status, cap, shift, bits, hist, hist_off,
                             scan_tmp, nblocks, s, status_semantics, identity_vals && p == 0,
                             &run_sums, &nruns);
    if (e != hipSuccess) return e;
    uint32_t *tk = src_k, *tv = src_v;
    src_k = dst_k;
    src_v = dst_v;
    dst_k = tk;
    dst_v = tv;
  }
  return hipSuccess;
}

hipError_t radix_partition_pairs(const uint32_t *keys, uint32_t *keys_out, uint32_t *emit_out,
                                 const int64_t *status, int64_t cap, int shift, int bits,
                                 uint32_t *hist, uint32_t *hist_off, uint32_t *scan_tmp,
                                 hipStream_t s, PartitionOffsets *po) {
  po->nblocks = (cap + kSortTileItems - 1) / kSortTileItems;
  po->hist_off = hist_off;
  return sort_pass(keys, nullptr, keys_out, emit_out, status, cap, shift, bits, hist, hist_off,
                   scan_tmp, po->nblocks, s, true, true, &po->run_sums, &po->nruns);
}

}  // namespace igs
