// Exclusive prefix sums (reduce-then-scan, recursive over block totals), used for the per-Gaussian
// pair offsets, the radix-sort digit offsets and the sampling distributions of the placement
// kernels (fp64, in a fixed order).  The pair offsets and the digit offsets use level one only;
// the kernel that consumes them adds the prefix of the run totals itself.
#include "common.hpp"

namespace igs {
namespace {

template <typename T>
__device__ __forceinline__ T wave_inclusive_scan(T v) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    T o = __shfl_up(v, d, 64);
    if (lane >= d) v += o;
  }
  return v;
}

// Each block scans kScanBlockItems consecutive inputs; writes exclusive local prefixes and the
// block total.
template <typename Tin, typename Tout>
__global__ __launch_bounds__(kScanThreads) void scan_block_kernel(const Tin *__restrict__ in,
                                                                   Tout *__restrict__ out,
                                                                   int64_t n,
                                                                   Tout *__restrict__ block_sums) {
  __shared__ Tout wave_tot[kScanThreads / 64];
  const int tid = threadIdx.x;
  const int64_t base = (int64_t)blockIdx.x * kScanBlockItems + (int64_t)tid * kScanItems;
  Tout v[kScanItems];
  Tout sum = 0;
#pragma unroll
  for (int j = 0; j < kScanItems; ++j) {
    int64_t i = base + j;
    v[j] = i < n ? (Tout)in[i] : (Tout)0;
    sum += v[j];
  }
  Tout inc = wave_inclusive_scan(sum);
  const int w = tid >> 6;
  if ((tid & 63) == 63) wave_tot[w] = inc;
  __syncthreads();
  Tout wave_off = 0;
  for (int k = 0; k < w; ++k) wave_off += wave_tot[k];
  Tout run = wave_off + inc - sum;
#pragma unroll
  for (int j = 0; j < kScanItems; ++j) {
    int64_t i = base + j;
    if (i < n) out[i] = run;
    run += v[j];
  }
  if (tid == kScanThreads - 1) {
    Tout tot = 0;
    for (int k = 0; k < kScanThreads / 64; ++k) tot += wave_tot[k];
    block_sums[blockIdx.x] = tot;
  }
}

template <typename T>
__global__ __launch_bounds__(kScanThreads) void scan_add_kernel(T *__restrict__ out, int64_t n,
                                                                const T *__restrict__ offs) {
  const int64_t base = (int64_t)blockIdx.x * kScanBlockItems;
  const T o = offs[blockIdx.x];
  for (int j = threadIdx.x; j < kScanBlockItems; j += kScanThreads) {
    int64_t i = base + j;
    if (i < n) out[i] += o;
  }
}

int64_t blocks_for(int64_t n) { return (n + kScanBlockItems - 1) / kScanBlockItems; }

// temp layout per level: [block sums][scanned block sums], then the next level.
template <typename Tin, typename Tout>
hipError_t scan_rec(const Tin *in, Tout *out, int64_t n, Tout *temp, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  int64_t nb = blocks_for(n);
  Tout *sums = temp;
  Tout *sums_scanned = temp + nb;
  scan_block_kernel<Tin, Tout><<<(unsigned)nb, kScanThreads, 0, s>>>(in, out, n, sums);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || nb == 1) return e;
  e = scan_rec<Tout, Tout>(sums, sums_scanned, nb, temp + 2 * nb, s);
  if (e != hipSuccess) return e;
  scan_add_kernel<Tout><<<(unsigned)nb, kScanThreads, 0, s>>>(out, n, sums_scanned);
  return hipGetLastError();
}

}  // namespace

size_t scan_temp_elems(int64_t n) {
  size_t total = 0;
  while (n > 1) {
    int64_t nb = blocks_for(n);
    total += 2 * (size_t)nb;
    if (nb == 1) break;
    n = nb;
  }
  return total + 2;
}

hipError_t scan_u32_to_u32(const uint32_t *in, uint32_t *out, int64_t n, uint32_t *temp,
                           hipStream_t s) {
  return scan_rec<uint32_t, uint32_t>(in, out, n, temp, s);
}

hipError_t scan_u32_blocks(const uint32_t *in, uint32_t *out, int64_t n, uint32_t *block_sums,
                           hipStream_t s) {
  if (n <= 0) return hipSuccess;
  scan_block_kernel<uint32_t, uint32_t>
      <<<(unsigned)blocks_for(n), kScanThreads, 0, s>>>(in, out, n, block_sums);
  return hipGetLastError();
}

hipError_t scan_f64(const double *in, double *out, int64_t n, double *temp, hipStream_t s) {
  return scan_rec<double, double>(in, out, n, temp, s);
}

}  // namespace igs
