// Per-(view, surfel) culling and EWA projection (Eq. 5, supp. Sec. 2.1), tile
// counts and visible counts per block, their scans, and the generic scan.
//
// One block per (range of 256 surfels, view): a thread projects one surfel
// into one view (the other views' blocks of a surfel range find its
// parameters in the cache); per-view results land in "slot" arrays indexed
// v * N + i.
#include "rogs_internal.h"

namespace rogs {

namespace {

__device__ __forceinline__ uint32_t nonzero_bytes4(uint32_t x) {
  return ((x & 0xffu) != 0u) + ((x & 0xff00u) != 0u) + ((x & 0xff0000u) != 0u) +
         ((x & 0xff000000u) != 0u);
}

// Extra blocks of the fused step's projection launch, block (nb + c, v):
// the nonzero bytes of chunk c (kMaskChunk bytes) of view v's loss mask into
// mpart[v * nmb + c] (summed per view by the count-table scan), and a share
// of clearing the n_zero per-tile pair counters.  Work the step needs
// anyway, done here instead of in two launches of its own.
__device__ void project_side_block(const ViewDev* __restrict__ views, int V, int nb,
                                   const uint8_t* __restrict__ mask, int nmb,
                                   uint32_t* __restrict__ mpart, uint32_t* __restrict__ zero_words,
                                   int64_t n_zero, uint32_t* s_w) {
  const int c = blockIdx.x - nb, v = blockIdx.y;
  const ViewDev& vw = views[v];
  const int64_t npix = (int64_t)vw.w * vw.h;
  const uint8_t* m = mask + vw.pix_off;
  uint32_t cnt = 0;
#pragma unroll
  for (int it = 0; it < kMaskChunk / (16 * kProjBlock); ++it) {
    const int64_t p = (int64_t)c * kMaskChunk + 16 * ((int64_t)it * kProjBlock + threadIdx.x);
    if (p >= npix) continue;
    const uint8_t* g = m + p;
    if (p + 16 <= npix && (reinterpret_cast<uintptr_t>(g) & 15u) == 0) {
      const uint4 x = *reinterpret_cast<const uint4*>(g);
      cnt += nonzero_bytes4(x.x) + nonzero_bytes4(x.y) + nonzero_bytes4(x.z) + nonzero_bytes4(x.w);
    } else {
      const int n = (int)min<int64_t>(16, npix - p);
      for (int k = 0; k < n; ++k) cnt += g[k] ? 1u : 0u;
    }
  }
  cnt = wave_sum_u32(cnt);
  if ((threadIdx.x & 63) == 0) s_w[threadIdx.x >> 6] = cnt;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t t = 0;
    for (int w = 0; w < kProjBlock / 64; ++w) t += s_w[w];
    mpart[(size_t)v * nmb + c] = t;
  }
  const int64_t nside = (int64_t)V * nmb;
  for (int64_t k = ((int64_t)v * nmb + c) * kProjBlock + threadIdx.x; k < n_zero;
       k += nside * kProjBlock)
    zero_words[k] = 0u;
}

// Feature records feat[N][FS] (rgb, sem[C], alpha, zero padding) from the
// surfel SoA: one thread per float4 of the output, so the stores are
// contiguous; the four values of a float4 are read from four rows.
__global__ __launch_bounds__(256) void k_pack_feat(int N, int C, int FS,
                                                   const float* __restrict__ pa,
                                                   const float* __restrict__ prgb,
                                                   const float* __restrict__ psem,
                                                   float4* __restrict__ feat) {
  const int Q = FS / 4;
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= (int64_t)N * Q) return;
  const int64_t i = t / Q;
  const int q = (int)(t - i * Q);
  float v[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int r = 4 * q + k;      // record column: rgb 0-2, sem 3..3+C-1, alpha 3+C
    v[k] = r < 3 ? prgb[(size_t)r * N + i]
                 : r < 3 + C ? psem[(size_t)(r - 3) * N + i] : r == 3 + C ? pa[i] : 0.0f;
  }
  feat[t] = make_float4(v[0], v[1], v[2], v[3]);
}

__global__ __launch_bounds__(kProjBlock) void k_project(
    const ViewDev* __restrict__ views, int V, int N, int nb, float eps, float qcut,
    const float* __restrict__ px, const float* __restrict__ py, const float* __restrict__ pz,
    const float* __restrict__ pq, const float* __restrict__ ps,
    uint32_t* __restrict__ cnt, float4* __restrict__ rec, uint2* __restrict__ rect,
    uint16_t* __restrict__ rspan, uint32_t* __restrict__ part, uint32_t* __restrict__ partv,
    const uint8_t* __restrict__ mask, int nmb,
    uint32_t* __restrict__ mpart, uint32_t* __restrict__ zero_words, int64_t n_zero) {
  __shared__ uint32_t s_w[kProjBlock / 64];
  if (blockIdx.x >= (unsigned)nb) {
    project_side_block(views, V, nb, mask, nmb, mpart, zero_words, n_zero, s_w);
    return;
  }
  __shared__ uint32_t s_v[kProjBlock / 64];
  __shared__ Span s_sp[kProjBlock];           // per-record span set-up
  __shared__ uint32_t s_roff[kProjBlock];     // first row item of each lane in its wave
  __shared__ uint32_t s_y0[kProjBlock];
  __shared__ uint32_t s_y1[kProjBlock];
  __shared__ uint32_t s_cnt[kProjBlock];
  const int i = blockIdx.x * kProjBlock + threadIdx.x;
  const int v = blockIdx.y;
  const int lane = threadIdx.x & 63, wbase = threadIdx.x & ~63;
  const bool valid = i < N;
  (void)V;
  const ViewDev& vw = views[v];
  const size_t slot = (size_t)v * N + i;
  // a block none of whose surfels lies in the view's ground rectangle (most
  // blocks of a long road) is culled whole: the same test the contract takes
  // first, without the projection, scans and barriers of the full path.  Its
  // slots' counts are not written: every reader of per-slot arrays tests the
  // block's visible count (partv) first.
  if (!__syncthreads_or(valid && ground_inside(vw, px[i], py[i]))) {
    if (threadIdx.x == 0) {
      part[(size_t)v * nb + blockIdx.x] = 0u;
      partv[(size_t)v * nb + blockIdx.x] = 0u;
    }
    return;
  }
  uint32_t nt = 0, rows = 0;
  Proj p;
  p.vis = false;
  p.y0 = 0;
  if (valid) {
    p = project_contract(vw, eps, qcut, px[i], py[i], pz[i], pq[i], pq[N + i],
                         pq[2 * (size_t)N + i], pq[3 * (size_t)N + i], ps[i], ps[N + i]);
    if (p.vis) {
      const Span sp = span_setup(p.uh, p.vh, p.ul, p.vl, p.A, p.B, p.C, qcut, p.x0, p.x1);
      if (sp.full) {
        nt = (uint32_t)((p.x1 - p.x0) * (p.y1 - p.y0));
        if (span_desc_ok(p.x0, p.x1, p.y0, p.y1))
          for (int r = 0; r < p.y1 - p.y0; ++r)
            rspan[slot * kSpanRows + r] = (uint16_t)((p.x1 - p.x0) << 8);
      } else {
        rows = (uint32_t)(p.y1 - p.y0);
      }
      s_sp[threadIdx.x] = sp;
      rec[2 * slot] = make_float4(p.uh, p.vh, p.ul, p.vl);
      rec[2 * slot + 1] = make_float4(p.A, p.B, p.C, p.tz);
      rect[slot] = make_uint2((uint32_t)p.x0 | ((uint32_t)p.x1 << 16),
                              (uint32_t)p.y0 | ((uint32_t)p.y1 << 16));
    }
  }
  // the wave's rectangle rows, spread evenly over its lanes: the row spans
  // of one record are summed into its lane's counter (integer adds)
  const uint32_t incl = wave_incl_scan(rows, lane);
  const uint32_t R = __shfl(incl, 63, 64);
  s_roff[threadIdx.x] = incl - rows;
  s_y0[threadIdx.x] = (uint32_t)p.y0;
  s_y1[threadIdx.x] = (uint32_t)p.y1;
  s_cnt[threadIdx.x] = 0;
  __syncthreads();
  for (uint32_t k = (uint32_t)lane; k < R; k += 64) {
    const int j = wbase + last_le(s_roff + wbase, 64, k);
    const int r = (int)(k - s_roff[j]);
    const Span& sj = s_sp[j];
    int lo, hi;
    span_row(sj, vw.tw, vw.th, vw.w, vw.h, (int)s_y0[j] + r, lo, hi);
    if (hi > lo) atomicAdd(&s_cnt[j], (uint32_t)(hi - lo));
    if (span_desc_ok(sj.x0, sj.x1, (int)s_y0[j], (int)s_y1[j]))
      rspan[((size_t)v * N + blockIdx.x * kProjBlock + (j & (kProjBlock - 1))) * kSpanRows + r] =
          (uint16_t)((lo - sj.x0) | ((hi - sj.x0) << 8));
  }
  __syncthreads();
  nt += s_cnt[threadIdx.x];
  if (valid) cnt[slot] = nt;
  uint32_t ws = wave_sum_u32(nt);
  const uint32_t wvis = (uint32_t)__popcll(__ballot(nt != 0));
  if (lane == 0) {
    s_w[threadIdx.x >> 6] = ws;
    s_v[threadIdx.x >> 6] = wvis;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t t = 0, tv = 0;
    for (int w = 0; w < kProjBlock / 64; ++w) {
      t += s_w[w];
      tv += s_v[w];
    }
    part[(size_t)v * nb + blockIdx.x] = t;
    partv[(size_t)v * nb + blockIdx.x] = tv;
  }
}

// Per-view mask counts from the projection's side blocks (exact integer
// sums): per view, the block's threads stride over the chunks, then a wave
// sum and the waves' totals.  blockDim.x is a multiple of 64, at most 1024.
// One block for all views (small batches, inside k_scan_part) ...
__device__ __forceinline__ void sum_mask_parts_all(const uint32_t* __restrict__ mpart, int nmb,
                                                   int V, uint32_t* __restrict__ mcount) {
  __shared__ uint32_t s_t[16];
  for (int v = 0; v < V; ++v) {
    uint32_t t = 0;
    for (int c = threadIdx.x; c < nmb; c += blockDim.x) t += mpart[(size_t)v * nmb + c];
    t = wave_sum_u32(t);
    if ((threadIdx.x & 63) == 0) s_t[threadIdx.x >> 6] = t;
    __syncthreads();
    if (threadIdx.x == 0) {
      uint32_t a = 0;
      for (int w = 0; w < (int)(blockDim.x >> 6); ++w) a += s_t[w];
      mcount[v] = a;
    }
    __syncthreads();
  }
}

// ... or one 64-lane block per view (view v's count).
__device__ __forceinline__ void sum_mask_parts(const uint32_t* __restrict__ mpart, int nmb, int v,
                                               uint32_t* __restrict__ mcount) {
  uint32_t t = 0;
  for (int c = threadIdx.x; c < nmb; c += 64) t += mpart[(size_t)v * nmb + c];
  t = wave_sum_u32(t);
  if (threadIdx.x == 0) mcount[v] = t;
}

// ------------------------------------------------------------ generic scan

__device__ __forceinline__ int64_t scan_count(const uint32_t* n_dev, int64_t n) {
  if (!n_dev) return n;
  const int64_t d = (int64_t)(*n_dev);
  return d < n ? d : n;
}

// The three passes of the multi-block scan as block bodies: the single-table
// kernels below and the paired ones (both projection count tables in one set
// of launches) share them.
__device__ __forceinline__ void scan_reduce_block(const uint32_t* __restrict__ in, int64_t n,
                                                  uint32_t* __restrict__ sums) {
  __shared__ uint32_t s_w[4];
  const int64_t base = (int64_t)blockIdx.x * kScanChunk;
  uint32_t acc = 0;
  for (int k = threadIdx.x; k < kScanChunk; k += 256) {
    int64_t j = base + k;
    if (j < n) acc += in[j];
  }
  acc = wave_sum_u32(acc);
  if ((threadIdx.x & 63) == 0) s_w[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) sums[blockIdx.x] = s_w[0] + s_w[1] + s_w[2] + s_w[3];
}

__global__ __launch_bounds__(256) void k_scan_reduce(const uint32_t* __restrict__ in, int64_t n_cap,
                                                     const uint32_t* __restrict__ n_dev,
                                                     uint32_t* __restrict__ sums) {
  scan_reduce_block(in, scan_count(n_dev, n_cap), sums);
}

// Exclusive scan in place of m values with one block of 1024 threads.
__device__ __forceinline__ void scan_top_block(uint32_t* __restrict__ sums, int64_t m,
                                               uint32_t* __restrict__ total) {
  __shared__ uint32_t s_w[16];
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  const int64_t per = (m + 1023) / 1024;
  const int64_t b = t * per, e = (b + per < m) ? b + per : m;
  uint32_t loc = 0;
  for (int64_t j = b; j < e; ++j) loc += sums[j];
  uint32_t inc = wave_incl_scan(loc, lane);
  if (lane == 63) s_w[wv] = inc;
  __syncthreads();
  uint32_t pre = 0, tot = 0;
  for (int w = 0; w < 16; ++w) {
    pre += (w < wv) ? s_w[w] : 0u;
    tot += s_w[w];
  }
  uint32_t run = pre + inc - loc;
  for (int64_t j = b; j < e; ++j) {
    uint32_t x = sums[j];
    sums[j] = run;
    run += x;
  }
  if (t == 0 && total) *total = tot;
}

__global__ __launch_bounds__(1024) void k_scan_top(uint32_t* __restrict__ sums, int64_t m,
                                                   uint32_t* __restrict__ total) {
  scan_top_block(sums, m, total);
}

// in and out may be the same array (each block reads its chunk before writing it).
__device__ __forceinline__ void scan_down_block(const uint32_t* in, uint32_t* out, int64_t n,
                                                const uint32_t* __restrict__ sums) {
  __shared__ uint32_t s_v[kScanChunk];
  __shared__ uint32_t s_w[4];
  const int64_t base = (int64_t)blockIdx.x * kScanChunk;
  if (base >= n) return;
  for (int k = threadIdx.x; k < kScanChunk; k += 256) {
    int64_t j = base + k;
    s_v[k] = (j < n) ? in[j] : 0u;
  }
  __syncthreads();
  constexpr int per = kScanChunk / 256;
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  uint32_t loc = 0;
  for (int k = 0; k < per; ++k) loc += s_v[t * per + k];
  uint32_t inc = wave_incl_scan(loc, lane);
  if (lane == 63) s_w[wv] = inc;
  __syncthreads();
  uint32_t pre = sums[blockIdx.x];
  for (int w = 0; w < 4; ++w) pre += (w < wv) ? s_w[w] : 0u;
  uint32_t run = pre + inc - loc;
  for (int k = 0; k < per; ++k) {
    uint32_t x = s_v[t * per + k];
    s_v[t * per + k] = run;
    run += x;
  }
  __syncthreads();
  for (int k = threadIdx.x; k < kScanChunk; k += 256) {
    int64_t j = base + k;
    if (j < n) out[j] = s_v[k];
  }
}

__global__ __launch_bounds__(256) void k_scan_down(const uint32_t* in, uint32_t* out, int64_t n_cap,
                                                   const uint32_t* __restrict__ n_dev,
                                                   const uint32_t* __restrict__ sums) {
  scan_down_block(in, out, scan_count(n_dev, n_cap), sums);
}

// Both projection count tables (pairs, visible slots; n values each, scanned
// in place): table blockIdx.y of the reduce and down passes, block b of the
// top pass; the sums of table a at sums + a * ms.
__global__ __launch_bounds__(256) void k_scan2_reduce(uint32_t* t0, uint32_t* t1, int64_t n,
                                                      uint32_t* __restrict__ sums, int64_t ms) {
  scan_reduce_block(blockIdx.y ? t1 : t0, n, sums + blockIdx.y * ms);
}

__global__ __launch_bounds__(1024) void k_scan2_top(uint32_t* __restrict__ sums, int64_t ms,
                                                    int64_t m, uint32_t* __restrict__ total0,
                                                    uint32_t* __restrict__ total1) {
  scan_top_block(sums + blockIdx.x * ms, m, blockIdx.x ? total1 : total0);
}

// A third row of blocks (blockIdx.y == 2) runs once the totals are known:
// block 0 sets the overflow flag, and with mpart block x sums view x's mask
// count.
__global__ __launch_bounds__(256) void k_scan2_down(uint32_t* t0, uint32_t* t1, int64_t n,
                                                    const uint32_t* __restrict__ sums,
                                                    int64_t ms, uint32_t* misc, int64_t cap,
                                                    int64_t scap,
                                                    const uint32_t* __restrict__ mpart, int nmb,
                                                    int V, uint32_t* __restrict__ mcount) {
  if (blockIdx.y == 2) {
    if (threadIdx.x == 0 && blockIdx.x == 0)
      misc[kMiscOverflow] =
          ((int64_t)misc[kMiscPairs] > cap || (int64_t)misc[kMiscVisible] > scap) ? 1u : 0u;
    // one wave per view
    if (mpart && (int)blockIdx.x < V && threadIdx.x < 64)
      sum_mask_parts(mpart, nmb, (int)blockIdx.x, mcount);
    return;
  }
  uint32_t* t = blockIdx.y ? t1 : t0;
  scan_down_block(t, t, n, sums + blockIdx.y * ms);
}

// Exclusive scan of at most kSmallScan values in one block of 1024 threads
// (one launch instead of three for the small tables).  Rounds of kSmallChunk
// values: a coalesced load into LDS (padded by one word per 32 against bank
// conflicts), 8 consecutive values per thread, a block scan of the thread
// sums, the results back through LDS and a coalesced store; a carry links
// the rounds.  Every round reads its values before it writes them, so
// in == out is allowed.
constexpr int kSmallScan = 1024 * 32;
constexpr int kSmallChunk = 1024 * 8;

__device__ __forceinline__ int pad32(int i) { return i + (i >> 5); }

__device__ __forceinline__ void block_scan_small(const uint32_t* in, uint32_t* out, int64_t n,
                                                 uint32_t* __restrict__ total) {
  __shared__ uint32_t s[kSmallChunk + kSmallChunk / 32];
  __shared__ uint32_t s_w[16];
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  uint32_t carry = 0;
  for (int64_t c0 = 0; c0 < n; c0 += kSmallChunk) {
    const int m = (int)((n - c0) < kSmallChunk ? (n - c0) : kSmallChunk);
    for (int i = t; i < kSmallChunk; i += 1024) s[pad32(i)] = (i < m) ? in[c0 + i] : 0u;
    __syncthreads();
    uint32_t v[8];
    uint32_t loc = 0;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      v[j] = s[pad32(8 * t + j)];
      loc += v[j];
    }
    const uint32_t inc = wave_incl_scan(loc, lane);
    if (lane == 63) s_w[wv] = inc;
    __syncthreads();
    uint32_t pre = 0, tot = 0;
    for (int w = 0; w < 16; ++w) {
      pre += (w < wv) ? s_w[w] : 0u;
      tot += s_w[w];
    }
    uint32_t run = carry + pre + inc - loc;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      s[pad32(8 * t + j)] = run;
      run += v[j];
    }
    __syncthreads();
    for (int i = t; i < m; i += 1024) out[c0 + i] = s[pad32(i)];
    carry += tot;
    __syncthreads();
  }
  if (t == 0 && total) *total = carry;
}

__global__ __launch_bounds__(1024) void k_scan_small(const uint32_t* in, uint32_t* out,
                                                     int64_t n_cap,
                                                     const uint32_t* __restrict__ n_dev,
                                                     uint32_t* __restrict__ total) {
  block_scan_small(in, out, scan_count(n_dev, n_cap), total);
}

// Both per-block count tables of the projection (pairs, visible slots) in one
// launch, one block each, and with mpart a third block for the per-view mask
// counts; the last block sets the overflow flag.
__global__ __launch_bounds__(1024) void k_scan_part(uint32_t* part, uint32_t* partv, int64_t n,
                                                    uint32_t* __restrict__ misc, int64_t cap,
                                                    int64_t scap,
                                                    const uint32_t* __restrict__ mpart, int nmb,
                                                    int V, uint32_t* __restrict__ mcount,
                                                    int check) {
  if (blockIdx.x == 2) {
    sum_mask_parts_all(mpart, nmb, V, mcount);
  } else {
    uint32_t* a = blockIdx.x == 0 ? part : partv;
    block_scan_small(a, a, n, misc + (blockIdx.x == 0 ? kMiscPairs : kMiscVisible));
  }
  if (check && last_block(misc + kMiscTicketScan) && threadIdx.x == 0) {
    const uint32_t pairs = __atomic_load_n(misc + kMiscPairs, __ATOMIC_RELAXED);
    const uint32_t vis = __atomic_load_n(misc + kMiscVisible, __ATOMIC_RELAXED);
    misc[kMiscOverflow] = ((int64_t)pairs > cap || (int64_t)vis > scap) ? 1u : 0u;
  }
}

__global__ void k_fill_u32(uint32_t* __restrict__ p, uint32_t value, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) p[i] = value;
}

}  // namespace

size_t scan_tmp_words(int64_t n) { return (size_t)((n + kScanChunk - 1) / kScanChunk) + 1; }

void scan_u32(const uint32_t* in, uint32_t* out, int64_t n, uint32_t* total, uint32_t* tmp,
              hipStream_t st) {
  if (n <= 0) return;
  if (n <= kSmallScan) {
    hipLaunchKernelGGL(k_scan_small, dim3(1), dim3(1024), 0, st, in, out, n,
                       (const uint32_t*)nullptr, total);
    return;
  }
  int64_t m = (n + kScanChunk - 1) / kScanChunk;
  hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)m), dim3(256), 0, st, in, n,
                     (const uint32_t*)nullptr, tmp);
  hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(1024), 0, st, tmp, m, total);
  hipLaunchKernelGGL(k_scan_down, dim3((unsigned)m), dim3(256), 0, st, in, out, n,
                     (const uint32_t*)nullptr, tmp);
}

void fill_u32(uint32_t* p, uint32_t value, int64_t n, hipStream_t st) {
  if (n <= 0) return;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)blocks), dim3(256), 0, st, p, value, n);
}

void launch_project(const Layout& L, void* ws, const rogs_surfels* s, bool pack_feat,
                    hipStream_t st, const uint8_t* mask) {
  fill_u32(at<uint32_t>(ws, L.o_misc), 0u, kMiscCount, st);
  if (pack_feat) {
    const int64_t n4 = (int64_t)L.N * (L.FS / 4);
    hipLaunchKernelGGL(k_pack_feat, dim3((unsigned)((n4 + 255) / 256)), dim3(256), 0, st, L.N,
                       L.C, L.FS, s->alpha, s->rgb, s->sem, at<float4>(ws, L.o_feat));
  }
  const int nmb = mask ? mask_chunks(L) : 0;
  hipLaunchKernelGGL(k_project, dim3(L.nb + nmb, L.V), dim3(kProjBlock), 0, st,
                     at<const ViewDev>(ws, L.o_views), L.V, L.N, L.nb, L.eps2d, L.q_cut, s->x, s->y, s->z,
                     s->q, s->s, at<uint32_t>(ws, L.o_cnt),
                     at<float4>(ws, L.o_rec), at<uint2>(ws, L.o_rect),
                     at<uint16_t>(ws, L.o_rspan), at<uint32_t>(ws, L.o_part),
                     at<uint32_t>(ws, L.o_partv), mask, nmb,
                     mask ? at<uint32_t>(ws, L.o_mpart) : nullptr,
                     mask ? at<uint32_t>(ws, L.o_tcnt) : nullptr,
                     mask ? L.total_tiles : (int64_t)0);
}

void launch_scan_part(const Layout& L, void* ws, hipStream_t st, bool mask_parts) {
  uint32_t* misc = at<uint32_t>(ws, L.o_misc);
  const uint32_t* mpart = mask_parts ? at<const uint32_t>(ws, L.o_mpart) : nullptr;
  const int nmb = mask_parts ? mask_chunks(L) : 0;
  uint32_t* mcount = at<uint32_t>(ws, L.o_mcount);
  if ((int64_t)L.V * L.nb <= kSmallScan) {
    hipLaunchKernelGGL(k_scan_part, dim3(mask_parts ? 3 : 2), dim3(1024), 0, st,
                       at<uint32_t>(ws, L.o_part), at<uint32_t>(ws, L.o_partv),
                       (int64_t)L.V * L.nb, misc, L.cap, L.scap, mpart, nmb, L.V, mcount,
                       mask_parts ? 0 : 1);   // the fused step's compaction sets the flag
    return;
  }
  // both tables at once: three launches instead of six
  const int64_t n = (int64_t)L.V * L.nb;
  const int64_t m = (n + kScanChunk - 1) / kScanChunk;
  const int64_t ms = (int64_t)scan_tmp_words(n);   // sums of one table
  uint32_t* sums = at<uint32_t>(ws, L.o_parttmp);
  uint32_t* part = at<uint32_t>(ws, L.o_part);
  uint32_t* partv = at<uint32_t>(ws, L.o_partv);
  hipLaunchKernelGGL(k_scan2_reduce, dim3((unsigned)m, 2), dim3(256), 0, st, part, partv, n, sums,
                     ms);
  hipLaunchKernelGGL(k_scan2_top, dim3(2), dim3(1024), 0, st, sums, ms, m, misc + kMiscPairs,
                     misc + kMiscVisible);
  const int64_t gx = std::max<int64_t>(m, mpart ? L.V : 1);   // the scan's blocks, the views
  hipLaunchKernelGGL(k_scan2_down, dim3((unsigned)gx, 3), dim3(256), 0, st, part, partv, n, sums,
                     ms, misc, L.cap, L.scap, mpart, nmb, L.V, mcount);
}

}  // namespace rogs
