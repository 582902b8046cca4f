// Stable LSD radix sort of the (tile, depth) keys with their pair values, and
// per-tile ranges of the sorted list ("ascending order of original depth",
// Sec. 3.3.1; ties keep the emission order, i.e. surfel id).
//
// Each pass: per-block digit histograms (LDS atomics) -> one exclusive scan
// over the digit-major histogram table -> stable scatter.  In the scatter a
// block owns kSortTile consecutive keys; each of its four waves ranks a
// contiguous quarter, 64 keys at a time, finding lanes with equal digits by
// eight ballots (one per digit bit), so the rank inside the block follows the
// input order exactly.
#include "rogs_internal.h"

namespace rogs {

namespace {

__device__ __forceinline__ uint32_t count_n(const uint32_t* n_dev, int64_t n_host, int64_t cap) {
  if (!n_dev) return (uint32_t)n_host;
  int64_t n = (int64_t)(*n_dev);
  return (uint32_t)(n < cap ? n : cap);
}

__global__ __launch_bounds__(kSortBlock) void k_hist(const unsigned long long* __restrict__ keys,
                                                     const uint32_t* __restrict__ n_dev,
                                                     int64_t n_host, int64_t cap, int shift,
                                                     uint32_t mask, uint32_t* __restrict__ hist,
                                                     int64_t nblk) {
  __shared__ uint32_t h[kRadix];
  h[threadIdx.x] = 0;
  __syncthreads();
  const uint32_t n = count_n(n_dev, n_host, cap);
  const int64_t base = (int64_t)blockIdx.x * kSortTile;
  for (int it = 0; it < kSortIPT; ++it) {
    int64_t idx = base + it * kSortBlock + threadIdx.x;
    if (idx < (int64_t)n) {
      uint32_t d = (uint32_t)(keys[idx] >> shift) & mask;
      atomicAdd(&h[d], 1u);
    }
  }
  __syncthreads();
  hist[(int64_t)threadIdx.x * nblk + blockIdx.x] = h[threadIdx.x];
}

__global__ __launch_bounds__(kSortBlock) void k_scatter(
    const unsigned long long* __restrict__ kin, const uint32_t* __restrict__ vin,
    unsigned long long* __restrict__ kout, uint32_t* __restrict__ vout,
    const uint32_t* __restrict__ n_dev, int64_t n_host, int64_t cap, int shift, uint32_t mask,
    int nbits, const uint32_t* __restrict__ hist_scan, int64_t nblk) {
  constexpr int kWaves = kSortBlock / 64;
  constexpr int kPerWave = kSortTile / kWaves;
  constexpr int kIters = kPerWave / 64;
  __shared__ uint32_t wcnt[kWaves][kRadix];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const uint32_t n = count_n(n_dev, n_host, cap);
  const int64_t base = (int64_t)blockIdx.x * kSortTile;
  if (base >= (int64_t)n) return;
  for (int k = threadIdx.x; k < kWaves * kRadix; k += kSortBlock) (&wcnt[0][0])[k] = 0;
  __syncthreads();
  const unsigned long long lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  uint32_t rank[kIters];
  uint32_t dig[kIters];
  for (int it = 0; it < kIters; ++it) {
    const int64_t idx = base + (int64_t)wv * kPerWave + it * 64 + lane;
    const bool valid = idx < (int64_t)n;
    uint32_t d = valid ? ((uint32_t)(kin[idx] >> shift) & mask) : 0u;
    unsigned long long m = __ballot(valid);
    for (int b = 0; b < nbits; ++b) {
      const bool bit = (d >> b) & 1u;
      unsigned long long bb = __ballot(valid && bit);
      m &= bit ? bb : ~bb;
    }
    uint32_t before = __popcll(m & lt_mask);
    uint32_t pre = 0;
    if (valid) pre = wcnt[wv][d];
    __builtin_amdgcn_wave_barrier();
    if (valid && before == 0) wcnt[wv][d] = pre + (uint32_t)__popcll(m);
    __builtin_amdgcn_wave_barrier();
    rank[it] = pre + before;
    dig[it] = d;
  }
  __syncthreads();
  // per digit: global start of this block, then the waves one after another
  {
    const int d = threadIdx.x;   // kSortBlock == kRadix
    uint32_t run = hist_scan[(int64_t)d * nblk + blockIdx.x];
    for (int w = 0; w < kWaves; ++w) {
      uint32_t c = wcnt[w][d];
      wcnt[w][d] = run;
      run += c;
    }
  }
  __syncthreads();
  for (int it = 0; it < kIters; ++it) {
    const int64_t idx = base + (int64_t)wv * kPerWave + it * 64 + lane;
    if (idx < (int64_t)n) {
      uint32_t dst = wcnt[wv][dig[it]] + rank[it];
      kout[dst] = kin[idx];
      vout[dst] = vin[idx];
    }
  }
}

__global__ void k_ranges(const unsigned long long* __restrict__ keys,
                         const uint32_t* __restrict__ n_dev, int64_t n_host, int64_t cap,
                         uint2* __restrict__ ranges) {
  const uint32_t n = count_n(n_dev, n_host, cap);
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)n) return;
  const uint32_t t = (uint32_t)(keys[i] >> 32);
  if (i == 0 || (uint32_t)(keys[i - 1] >> 32) != t) ranges[t].x = (uint32_t)i;
  if (i == (int64_t)n - 1 || (uint32_t)(keys[i + 1] >> 32) != t) ranges[t].y = (uint32_t)(i + 1);
}

}  // namespace

// Sort the batch's keys/vals.  n_host >= 0: the pair count is known on the
// host; < 0: it is read on the device.  Returns 1 when the sorted result is in
// the alternate buffers (o_keys2 / o_vals2), 0 when it is in o_keys / o_vals.
int launch_sort(const Layout& L, void* ws, int64_t n_host, hipStream_t st) {
  const uint32_t* n_dev = n_host < 0 ? at<uint32_t>(ws, L.o_misc) + kMiscPairs : nullptr;
  const int64_t n_grid = n_host < 0 ? L.cap : n_host;
  const int key_bits = 32 + L.tile_bits;
  const int passes = (key_bits + kRadixBits - 1) / kRadixBits;
  if (n_grid <= 0) return passes & 1;
  const int64_t nblk = (n_grid + kSortTile - 1) / kSortTile;
  unsigned long long* k0 = at<unsigned long long>(ws, L.o_keys);
  unsigned long long* k1 = at<unsigned long long>(ws, L.o_keys2);
  uint32_t* v0 = at<uint32_t>(ws, L.o_vals);
  uint32_t* v1 = at<uint32_t>(ws, L.o_vals2);
  uint32_t* hist = at<uint32_t>(ws, L.o_hist);
  for (int shift = 0; shift < key_bits; shift += kRadixBits) {
    const int nbits = (key_bits - shift) < kRadixBits ? (key_bits - shift) : kRadixBits;
    const uint32_t mask = (1u << nbits) - 1u;
    hipLaunchKernelGGL(k_hist, dim3((unsigned)nblk), dim3(kSortBlock), 0, st, k0, n_dev,
                       n_grid, L.cap, shift, mask, hist, nblk);
    scan_u32(hist, hist, (int64_t)kRadix * nblk, nullptr, at<uint32_t>(ws, L.o_histtmp), st);
    hipLaunchKernelGGL(k_scatter, dim3((unsigned)nblk), dim3(kSortBlock), 0, st, k0, v0, k1, v1,
                       n_dev, n_grid, L.cap, shift, mask, nbits, hist, nblk);
    unsigned long long* tk = k0; k0 = k1; k1 = tk;
    uint32_t* tv = v0; v0 = v1; v1 = tv;
  }
  return passes & 1;
}

void launch_ranges(const Layout& L, void* ws, int64_t n_host, hipStream_t st) {
  uint2* ranges = at<uint2>(ws, L.o_ranges);
  fill_u32(reinterpret_cast<uint32_t*>(ranges), 0u, 2 * L.total_tiles, st);
  const uint32_t* n_dev = n_host < 0 ? at<uint32_t>(ws, L.o_misc) + kMiscPairs : nullptr;
  const int64_t n_grid = n_host < 0 ? L.cap : n_host;
  if (n_grid <= 0) return;
  hipLaunchKernelGGL(k_ranges, dim3((unsigned)((n_grid + 255) / 256)), dim3(256), 0, st,
                     at<const unsigned long long>(ws, L.o_keys), n_dev, n_grid, L.cap, ranges);
}

}  // namespace rogs
