// Binning: the visible (view, surfel) slots in (view, surfel id) order,
// emission of one (tile) pair per covered tile in that order with a rank in
// its tile's counter, the tiles' list starts, ranges and compositing launch
// order from the counters, the pairs placed into their tiles' lists, then
// each tile's list ordered by depth inside the tile.  The result is every
// tile's list in ascending order of original depth with ties by surfel id
// (Sec. 3.3.1), the order a stable sort by (tile, depth) gives.
#include "rogs_internal.h"

namespace rogs {

namespace {

__device__ __forceinline__ uint32_t count_n(const uint32_t* n_dev, int64_t n_host, int64_t cap) {
  if (!n_dev) return (uint32_t)n_host;
  int64_t n = (int64_t)(*n_dev);
  return (uint32_t)(n < cap ? n : cap);
}

constexpr int kEmitThreads = 256;
constexpr int kEmitRows = 1024;
constexpr int kEmitWin = 2 * kEmitRows;   // tiles of a block's count window

// Visible slots in (view, surfel) order: each slot's position in that order
// (from the per-block visible counts, scanned), its emission count and first
// pair (from the per-block pair counts, scanned, plus the block's exclusive
// scan of the counts), and the first slot of every emission block of
// kEmitPairs pairs (each block start lies in exactly one slot; only the nblk
// launched blocks).  Block 0 also sets the overflow flag from the totals of
// the count scans (the fused step's scan launch leaves it to this one).
__global__ __launch_bounds__(kProjBlock) void k_compact(int V, int N, int nb,
                                                        const uint32_t* __restrict__ cnt,
                                                        const uint32_t* __restrict__ part,
                                                        const uint32_t* __restrict__ partv,
                                                        int64_t scap,
                                                        uint32_t* __restrict__ sval,
                                                        uint32_t* __restrict__ scnt,
                                                        uint32_t* __restrict__ soff,
                                                        uint32_t* __restrict__ spos,
                                                        uint32_t* __restrict__ bstart,
                                                        uint32_t nblk, uint32_t* __restrict__ misc,
                                                        int64_t cap) {
  __shared__ uint32_t s_w[kProjBlock / 64];
  __shared__ uint32_t s_p[kProjBlock / 64];
  if (blockIdx.x == 0 && threadIdx.x == 0)
    misc[kMiscOverflow] =
        ((int64_t)misc[kMiscPairs] > cap || (int64_t)misc[kMiscVisible] > scap) ? 1u : 0u;
  const int i = blockIdx.x * kProjBlock + threadIdx.x;
  const bool valid = i < N;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const unsigned long long lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  const size_t nparts = (size_t)V * nb;
  for (int v = 0; v < V; ++v) {
    const size_t slot = (size_t)v * N + i;
    // the scanned visible counts give this block's count in view v: none
    // visible (a block the view's ground rectangle misses) needs no scan, and
    // its slots get no position (the projection adjoint makes the same test)
    const size_t pb = (size_t)v * nb + blockIdx.x;
    const uint32_t vnext = pb + 1 < nparts ? partv[pb + 1] : misc[kMiscVisible];
    if (vnext == partv[pb]) continue;
    const uint32_t c = valid ? cnt[slot] : 0u;
    const bool vis = c != 0;
    const unsigned long long b = __ballot(vis);
    const uint32_t inc = wave_incl_scan(c, lane);
    if (lane == 0) s_w[wv] = (uint32_t)__popcll(b);
    if (lane == 63) s_p[wv] = inc;
    __syncthreads();
    uint32_t pre = partv[(size_t)v * nb + blockIdx.x];
    uint32_t off = part[(size_t)v * nb + blockIdx.x] + inc - c;
    for (int w = 0; w < wv; ++w) {
      pre += s_w[w];
      off += s_p[w];
    }
    __syncthreads();
    // every slot's position in a block with visible slots, 0xffffffff for a
    // culled one or one beyond the slot capacity
    uint32_t sp = 0xffffffffu;
    if (vis) {
      const uint32_t pos = pre + (uint32_t)__popcll(b & lt_mask);
      if ((int64_t)pos < scap) {
        sval[pos] = (uint32_t)slot;
        scnt[pos] = c;
        soff[pos] = off;
        sp = pos;
        if (nblk) {
          const uint32_t b0 = (off + (uint32_t)kEmitPairs - 1u) / (uint32_t)kEmitPairs;
          const uint32_t b1 = min((off + c - 1u) / (uint32_t)kEmitPairs, nblk - 1u);
          for (uint32_t bb = b0; bb <= b1; ++bb) bstart[bb] = pos;
        }
      }
    }
    if (valid) spos[slot] = sp;
  }
}

// Ranks of pairs among the pairs of their tiles, from the tiles' counters,
// for kR rounds of one wave at once: in each round the lanes that hold the
// same tile form one group whose lowest lane adds the group's size, and each
// lane's rank is the count before that add plus its place among the group's
// lanes.  The adds of all rounds are issued before the first result is used,
// so the wave waits for one atomic round trip, not kR.  Per tile the ranks
// are a permutation of 0 ... count - 1 whose order depends on timing; the
// depth sort inside each tile (key t_z bits, then emission index) removes it.
// Every lane of the wave calls this together (act = holds a pair).
template <int kR>
__device__ __forceinline__ void tile_ranks(uint32_t* __restrict__ tcnt, const uint32_t (&t)[kR],
                                           const bool (&act)[kR], uint32_t (&rank)[kR]) {
  const uint32_t lane = threadIdx.x & 63u;
  const unsigned long long lt = (1ull << lane) - 1ull;
  uint32_t lead[kR], base[kR];
#pragma unroll
  for (int r = 0; r < kR; ++r) {
    unsigned long long todo = __ballot(act[r]);
    uint32_t size = 0u;
    lead[r] = 0u;
    rank[r] = 0u;
    while (todo) {
      const int l = __ffsll((unsigned long long)todo) - 1;
      const uint32_t tl = (uint32_t)__builtin_amdgcn_readlane((int)t[r], l);
      const bool mine = act[r] && t[r] == tl;
      const unsigned long long grp = __ballot(mine);
      if (mine) {
        lead[r] = (uint32_t)l;
        rank[r] = (uint32_t)__popcll(grp & lt);
        size = (uint32_t)__popcll(grp);
      }
      todo &= ~grp;
    }
    base[r] = 0u;
    if (act[r] && lane == lead[r]) base[r] = atomicAdd(&tcnt[t[r]], size);
  }
#pragma unroll
  for (int r = 0; r < kR; ++r) rank[r] += (uint32_t)__shfl((int)base[r], (int)lead[r], 64);
}

// Emission in (view, surfel id) slot order, balanced by pairs: block b writes the
// pairs e in [b * kEmitPairs, (b + 1) * kEmitPairs).  Its first slot comes from
// the compaction (bstart); the following slots that start before the block's end (each
// visible slot has at least one pair, so the offsets are strictly increasing
// and the range holds at most kEmitPairs slots) are staged in LDS.  The rectangle rows of the staged slots
// become row items: each gets its tile span (the same row spans that gave the
// counts: from the projection's row-span descriptor, or recomputed where the
// slot has more rows or a wider rectangle than a descriptor holds), an
// exclusive scan turns the span lengths into pair offsets, and each pair
// finds its row by binary search.  A block whose slots hold more
// than kEmitRows rows walks each pair's rows instead.  Per pair e: keys[e] =
// global tile, rank[e] = its rank in that tile's counter tcnt, pslot[e] =
// slot, pdep[e] = the slot's t_z bits.  The number of pairs written (the pair
// count, clipped to the capacity and to the pairs of the slots within the
// slot capacity) goes to *n_emit.

__device__ __forceinline__ Span emit_span(const float4* __restrict__ rec, uint32_t slot, float qcut,
                                          int x0, int x1) {
  const float4 r0 = rec[2 * (size_t)slot], r1 = rec[2 * (size_t)slot + 1];
  return span_setup(r0.x, r0.y, r0.z, r0.w, r1.x, r1.y, r1.z, qcut, x0, x1);
}

// In-place exclusive scan of n <= kEmitRows values in LDS; returns the total.
__device__ uint32_t emit_scan(uint32_t* a, int n, uint32_t* s_w) {
  constexpr int kPer = kEmitRows / kEmitThreads;
  const int b = threadIdx.x * kPer;
  uint32_t v[kPer], sum = 0;
#pragma unroll
  for (int k = 0; k < kPer; ++k) {
    v[k] = (b + k < n) ? a[b + k] : 0u;
    sum += v[k];
  }
  uint32_t total;
  uint32_t pre = block_excl_scan(sum, s_w, &total);
#pragma unroll
  for (int k = 0; k < kPer; ++k) {
    if (b + k < n) a[b + k] = pre;
    pre += v[k];
  }
  __syncthreads();
  return total;
}

__global__ __launch_bounds__(kEmitThreads) void k_emit(
    const ViewDev* __restrict__ views, int N, const uint32_t* __restrict__ p_dev, int64_t p_host,
    const uint32_t* __restrict__ s_dev, int64_t s_host, int64_t scap, int64_t cap,
    const uint32_t* __restrict__ sval, const uint32_t* __restrict__ soff,
    const uint32_t* __restrict__ scnt, const uint2* __restrict__ rect,
    const uint16_t* __restrict__ rspan, const float4* __restrict__ rec, float qcut,
    const uint32_t* __restrict__ bstart, uint32_t* __restrict__ keys,
    uint32_t* __restrict__ rank, uint32_t* __restrict__ pslot, uint32_t* __restrict__ pdep,
    uint32_t* __restrict__ tcnt, uint32_t* __restrict__ n_emit) {
  static_assert(kEmitThreads == kProjBlock, "block scan width");
  __shared__ uint32_t s_off[kEmitPairs + 1];
  __shared__ uint32_t s_slot[kEmitPairs];
  __shared__ uint32_t s_dep[kEmitPairs];        // t_z bits of each staged slot
  __shared__ uint32_t s_roff[kEmitPairs + 1];   // first row item of each slot
  // row items while the tiles are found, then the block's tile-count window
  __shared__ uint32_t s_rows[2 * kEmitRows];
  uint32_t* s_rx = s_rows;                      // row span length, then its first pair
  uint32_t* s_rinfo = s_rows + kEmitRows;       // span start tile | tile row << 16
  __shared__ uint16_t s_rslot[kEmitRows];
  __shared__ uint32_t s_w[kEmitThreads / 64];
  __shared__ uint32_t s_mm[8 * (kEmitThreads / 64)];
  const uint32_t S = count_n(s_dev, s_host, scap);
  const uint32_t P = count_n(p_dev, p_host, cap);
  const uint32_t pend = S ? soff[S - 1] + scnt[S - 1] : 0u;
  const uint32_t E = min(P, pend);
  if (n_emit && blockIdx.x == 0 && threadIdx.x == 0) *n_emit = E;
  const uint32_t e0 = blockIdx.x * (uint32_t)kEmitPairs;
  if (e0 >= E) return;
  const uint32_t e1 = min(E, e0 + (uint32_t)kEmitPairs);
  // the block's slots are ka (holding e0) and the following ones that start
  // before e1: at most kEmitPairs, since every listed slot has a pair
  const uint32_t ka = bstart[blockIdx.x];
  const uint32_t avail = min(S - ka, (uint32_t)kEmitPairs);
  constexpr int kPer = kEmitPairs / kEmitThreads;
  uint32_t nrow[kPer], rsum = 0, mine = 0;
#pragma unroll
  for (int k = 0; k < kPer; ++k) {
    const int t = threadIdx.x * kPer + k;
    nrow[k] = 0;
    if ((uint32_t)t < avail) {
      const uint32_t o = soff[ka + t];
      if (o < e1) {
        const uint32_t slot = sval[ka + t];
        s_off[t] = o;
        s_slot[t] = slot;
        s_dep[t] = __float_as_uint(rec[2 * (size_t)slot + 1].w);
        const uint2 r = rect[slot];
        nrow[k] = (r.y >> 16) - (r.y & 0xffff);
        mine += 1;
      }
    }
    rsum += nrow[k];
  }
  // the staged slots are a prefix of the candidates; their count is ns
  uint32_t ns_u;
  (void)block_excl_scan(mine, s_w, &ns_u);
  const int ns = (int)ns_u;
  uint32_t R;
  uint32_t pre = block_excl_scan(rsum, s_w, &R);
#pragma unroll
  for (int k = 0; k < kPer; ++k) {
    const int t = threadIdx.x * kPer + k;
    if (t < ns) s_roff[t] = pre;
    pre += nrow[k];
  }
  __syncthreads();
  uint32_t tile[kPer], vq[kPer], txq[kPer], tyq[kPer];   // global tile; view, column, row
  bool act[kPer];
  if (R <= (uint32_t)kEmitRows) {
    // row items: span of each rectangle row of the staged slots
    for (int k = threadIdx.x; k < (int)R; k += kEmitThreads) {
      const int j = last_le(s_roff, ns, (uint32_t)k);
      const uint32_t slot = s_slot[j];
      const uint2 r = rect[slot];
      const int x0 = r.x & 0xffff, x1 = r.x >> 16, y0 = r.y & 0xffff, y1 = r.y >> 16;
      const int row = k - (int)s_roff[j];
      const int ty = y0 + row;
      int lo, hi;
      if (span_desc_ok(x0, x1, y0, y1)) {
        const uint32_t d = rspan[(size_t)slot * kSpanRows + row];
        lo = x0 + (int)(d & 0xffu);
        hi = x0 + (int)(d >> 8);
      } else {
        const ViewDev& vw = views[slot / (uint32_t)N];
        span_row(emit_span(rec, slot, qcut, x0, x1), vw.tw, vw.th, vw.w, vw.h, ty, lo, hi);
      }
      s_rx[k] = (uint32_t)(hi - lo);
      s_rinfo[k] = (uint32_t)lo | ((uint32_t)ty << 16);
      s_rslot[k] = (uint16_t)j;
    }
    __syncthreads();
    emit_scan(s_rx, (int)R, s_w);                 // pair offsets from the first slot's first pair
    // pair e0 + threadIdx.x + r * kEmitThreads in round r
#pragma unroll
    for (int r = 0; r < kPer; ++r) {
      const uint32_t e = e0 + threadIdx.x + (uint32_t)(r * kEmitThreads);
      act[r] = e < e1;
      tile[r] = vq[r] = txq[r] = tyq[r] = 0u;
      if (act[r]) {
        const uint32_t t = e - s_off[0];
        const int rr = last_le(s_rx, (int)R, t);
        const uint32_t info = s_rinfo[rr];
        const uint32_t js = s_rslot[rr];
        const uint32_t slot = s_slot[js];
        const int tx = (int)(info & 0xffff) + (int)(t - s_rx[rr]);
        const int ty = (int)(info >> 16);
        const ViewDev& vw = views[slot / (uint32_t)N];
        tile[r] = (uint32_t)vw.tile_off + (uint32_t)(ty * vw.tiles_x + tx);
        vq[r] = slot / (uint32_t)N;
        txq[r] = (uint32_t)tx;
        tyq[r] = (uint32_t)ty;
        keys[e] = tile[r];
        pslot[e] = slot;
        pdep[e] = s_dep[js];
      }
    }
  } else {
#pragma unroll
  for (int q = 0; q < kPer; ++q) {
    const uint32_t e = e0 + threadIdx.x + (uint32_t)(q * kEmitThreads);
    act[q] = e < e1;
    tile[q] = vq[q] = txq[q] = tyq[q] = 0u;
    if (act[q]) {
      const int j = last_le(s_off, ns, e);
      const uint32_t slot = s_slot[j];
      const uint2 r = rect[slot];
      const int x0 = r.x & 0xffff, x1 = r.x >> 16, y0 = r.y & 0xffff, y1 = r.y >> 16;
      const ViewDev& vw = views[slot / (uint32_t)N];
      const bool desc = span_desc_ok(x0, x1, y0, y1);
      const Span sp = desc ? Span{} : emit_span(rec, slot, qcut, x0, x1);
      // walk the rectangle's rows to the one holding the kk-th reached tile
      int kk = (int)(e - s_off[j]);
      int ty = y0, tx = x0;
      for (; ty < y1; ++ty) {
        int a, b;
        if (desc) {
          const uint32_t d = rspan[(size_t)slot * kSpanRows + (ty - y0)];
          a = x0 + (int)(d & 0xffu);
          b = x0 + (int)(d >> 8);
        } else {
          span_row(sp, vw.tw, vw.th, vw.w, vw.h, ty, a, b);
        }
        if (kk < b - a) {
          tx = a + kk;
          break;
        }
        kk -= b - a;
      }
      if (ty >= y1) ty = y1 - 1;   // unreachable: the counts come from the same spans
      tile[q] = (uint32_t)vw.tile_off + (uint32_t)(ty * vw.tiles_x + tx);
      vq[q] = slot / (uint32_t)N;
      txq[q] = (uint32_t)tx;
      tyq[q] = (uint32_t)ty;
      keys[e] = tile[q];
      pslot[e] = slot;
      pdep[e] = s_dep[j];
    }
  }
  }
  // ranks: the block's extent in tile index, view, column and row (maxima
  // kept as complements so that every reduction is a minimum)
  constexpr int kX = 8;
  uint32_t m[kX];
#pragma unroll
  for (int k = 0; k < kX; ++k) m[k] = 0xffffffffu;
#pragma unroll
  for (int q = 0; q < kPer; ++q)
    if (act[q]) {
      const uint32_t x[4] = {tile[q], vq[q], txq[q], tyq[q]};
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        m[2 * k] = min(m[2 * k], x[k]);
        m[2 * k + 1] = min(m[2 * k + 1], ~x[k]);
      }
    }
#pragma unroll
  for (uint32_t d = 1; d < 64u; d <<= 1)
#pragma unroll
    for (int k = 0; k < kX; ++k) m[k] = min(m[k], lane_xor(m[k], d));
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  constexpr int kWaves = kEmitThreads / 64;
  if (lane < kX) {
    uint32_t mine = m[0];
#pragma unroll
    for (int k = 1; k < kX; ++k) mine = (lane == k) ? m[k] : mine;
    s_mm[lane * kWaves + wv] = mine;
  }
  __syncthreads();                      // the row items are no longer read
#pragma unroll
  for (int k = 0; k < kX; ++k) {
    m[k] = s_mm[k * kWaves];
#pragma unroll
    for (int w = 1; w < kWaves; ++w) m[k] = min(m[k], s_mm[k * kWaves + w]);
  }
  const uint32_t lo = m[0], hi = ~m[1];
  const uint32_t v0 = m[2], v1 = ~m[3], x0 = m[4], x1 = ~m[5], y0 = m[6], y1 = ~m[7];
  // window layout: a single-view block whose rows x (columns rounded up to a
  // power of two) fit counts by (row, column); otherwise by tile index when
  // the index span fits
  int lwx = 0;
  while (lwx < 31 && (1u << lwx) < x1 - x0 + 1u) ++lwx;
  const bool win2d = v0 == v1 && (uint64_t)(y1 - y0 + 1u) << lwx <= (uint64_t)kEmitWin;
  const bool win1d = hi - lo < (uint32_t)kEmitWin;
  uint32_t toff = 0u, tcols = 0u;
  if (win2d) {
    toff = (uint32_t)views[v0].tile_off;
    tcols = (uint32_t)views[v0].tiles_x;
  }
  auto widx = [&](int q) -> uint32_t {
    return win2d ? ((tyq[q] - y0) << lwx) + (txq[q] - x0) : tile[q] - lo;
  };
  auto wtile = [&](uint32_t w) -> uint32_t {
    return win2d ? toff + (y0 + (w >> lwx)) * tcols + x0 + (w & ((1u << lwx) - 1u)) : lo + w;
  };
  uint32_t rk[kPer];
  if (win2d || win1d) {
    // one global add per distinct tile of the block: local ranks from LDS
    // counters over the window, then each nonzero window count takes its
    // tile's global base
    constexpr int kWinPer = kEmitWin / kEmitThreads;
    uint32_t* s_win = s_rows;
#pragma unroll
    for (int k = 0; k < kWinPer; ++k) s_win[threadIdx.x + k * kEmitThreads] = 0u;
    __syncthreads();
#pragma unroll
    for (int q = 0; q < kPer; ++q) rk[q] = act[q] ? atomicAdd(&s_win[widx(q)], 1u) : 0u;
    __syncthreads();
    uint32_t c[kWinPer];
#pragma unroll
    for (int k = 0; k < kWinPer; ++k) {
      const uint32_t w = threadIdx.x + (uint32_t)(k * kEmitThreads);
      c[k] = s_win[w];
      if (c[k]) c[k] = atomicAdd(&tcnt[wtile(w)], c[k]);
    }
#pragma unroll
    for (int k = 0; k < kWinPer; ++k) s_win[threadIdx.x + k * kEmitThreads] = c[k];
    __syncthreads();
#pragma unroll
    for (int q = 0; q < kPer; ++q)
      if (act[q]) rk[q] += s_win[widx(q)];
  } else {
    tile_ranks<kPer>(tcnt, tile, act, rk);
  }
#pragma unroll
  for (int q = 0; q < kPer; ++q)
    if (act[q]) rank[e0 + threadIdx.x + (uint32_t)(q * kEmitThreads)] = rk[q];
}

// Pairs grouped by tile: pair e goes to the first list position of its tile
// plus its rank (n = the emitted pairs).
__global__ __launch_bounds__(256) void k_place(const uint32_t* __restrict__ keys,
                                               const uint32_t* __restrict__ rank,
                                               const uint32_t* __restrict__ tstart,
                                               const uint32_t* __restrict__ n_dev, int64_t n_host,
                                               int64_t cap, uint32_t* __restrict__ vals) {
  const uint32_t n = count_n(n_dev, n_host, cap);
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= (int64_t)n) return;
  vals[tstart[keys[e]] + rank[e]] = (uint32_t)e;
}

// Compositing work item of each launch position b: (tile, list begin, list
// end, view | the tile's row in its view << kViewBits) of the tile order[b],
// so a compositing wave starts from one load and needs no division.
// Depth order inside each tile.  A tile's list holds its pairs in the order
// the counters ranked them; these kernels order it by (t_z bits, emission
// index e), which is the binary32 depth with ties by surfel id (emission runs
// in (view, surfel id) order and a tile belongs to one view), and write each
// sorted pair's slot.  t_z > 0 for a visible slot, so its bits order like its
// value; padding takes (0xffffffff, 0xffffffff) and sorts last.
__device__ __forceinline__ bool key_less(uint32_t ka, uint32_t ia, uint32_t kb, uint32_t ib) {
  return ka < kb || (ka == kb && ia < ib);
}

// One wave's bitonic network over 64 R elements held R per lane (element
// r * 64 + lane in register r): distances of 64 and more compare registers of
// the same lane, shorter ones exchange across lanes.
template <int R>
__device__ __forceinline__ void wave_sort_regs(uint32_t (&key)[R], uint32_t (&e)[R], int lane) {
  constexpr uint32_t P = 64u * R;
#pragma unroll
  for (uint32_t k = 2; k <= P; k <<= 1) {
#pragma unroll
    for (uint32_t j = k >> 1; j > 0; j >>= 1) {
      if (j >= 64u) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const int pr = r ^ (int)(j >> 6);
          if (r < pr) {
            const uint32_t i = (uint32_t)r * 64u + (uint32_t)lane;
            const bool up = (i & k) == 0u;
            if (up == key_less(key[pr], e[pr], key[r], e[r])) {
              const uint32_t tk = key[r], te = e[r];
              key[r] = key[pr];
              e[r] = e[pr];
              key[pr] = tk;
              e[pr] = te;
            }
          }
        }
      } else {
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const uint32_t ok = lane_xor(key[r], j);
          const uint32_t oe = lane_xor(e[r], j);
          const uint32_t i = (uint32_t)r * 64u + (uint32_t)lane;
          const bool keep_min = (((uint32_t)lane & j) == 0u) == ((i & k) == 0u);
          if (keep_min == key_less(ok, oe, key[r], e[r])) {
            key[r] = ok;
            e[r] = oe;
          }
        }
      }
    }
  }
}

// One list of 64 R / 2 to 64 R entries on one wave: loaded R per lane,
// sorted in registers, written back with each pair's slot.
template <int R>
__device__ __forceinline__ void wave_sort_list(uint32_t beg, uint32_t len,
                                               uint32_t* __restrict__ vals,
                                               const uint32_t* __restrict__ pslot,
                                               const uint32_t* __restrict__ pdep,
                                               uint32_t* __restrict__ spair, int lane) {
  uint32_t key[R], e[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const uint32_t i = (uint32_t)r * 64u + (uint32_t)lane;
    e[r] = key[r] = 0xffffffffu;
    if (i < len) e[r] = vals[beg + i];
  }
#pragma unroll
  for (int r = 0; r < R; ++r)
    if ((uint32_t)r * 64u + (uint32_t)lane < len) key[r] = pdep[e[r]];
  wave_sort_regs<R>(key, e, lane);
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const uint32_t i = (uint32_t)r * 64u + (uint32_t)lane;
    if (i < len) {
      vals[beg + i] = e[r];
      spair[beg + i] = pslot[e[r]];
    }
  }
}

// Lists of 1 to 511 entries.  The launch order groups the tiles by the bit
// length bl of their list length.  For bl <= 6 a wave takes 64 / 2^bl
// consecutive tiles of one group, each on a segment of 2^bl lanes, and sorts
// every segment with one bitonic network over (key, e) (the e of a tile are
// distinct, so the order is strict); for bl = 7, 8, 9 (64 to 511 entries) a
// wave takes one tile and holds 2, 4 or 8 entries per lane (wave_sort_list).
// Work items (waves) of a group: ceil(tiles / tiles per wave); the blocks
// stride over all groups' items, longest lists first.  Lists of 512 or more
// entries are left to k_tile_sort_long.
constexpr uint32_t kWaveSortMax = 511;

__global__ __launch_bounds__(64) void k_tile_sort_short(const uint4* __restrict__ tinfo,
                                                        const uint32_t* __restrict__ bucket_tot,
                                                        uint32_t* __restrict__ vals,
                                                        const uint32_t* __restrict__ pslot,
                                                        const uint32_t* __restrict__ pdep,
                                                        uint32_t* __restrict__ spair) {
  // launch-order buckets: key 15 - bl, so bucket d holds bit length 15 - d
  __shared__ uint32_t s_start[16], s_cnt[16], s_items[16];
  const int lane = threadIdx.x;
  if (lane < 16) s_cnt[lane] = bucket_tot[lane];
  __syncthreads();
  if (lane == 0) {
    uint32_t st = 0;
    for (int d = 0; d < 16; ++d) {
      const int bl = 15 - d;
      s_start[d] = st;
      st += s_cnt[d];
      s_items[d] = 0u;
      if (bl >= 1 && bl <= 9) {
        const uint32_t per = bl >= 6 ? 1u : 64u >> bl;         // tiles per wave
        s_items[d] = (s_cnt[d] + per - 1u) / per;
      }
    }
  }
  __syncthreads();
  uint32_t total = 0;
  for (int d = 0; d < 16; ++d) total += s_items[d];
  for (uint32_t w = blockIdx.x; w < total; w += gridDim.x) {
    int d = 0;
    uint32_t wi = w;
    while (wi >= s_items[d]) { wi -= s_items[d]; ++d; }
    const int bl = 15 - d;
    if (bl >= 7) {
      const uint4 ti = tinfo[s_start[d] + wi];
      const uint32_t beg = ti.y, len = ti.z - ti.y;
      if (bl == 7) wave_sort_list<2>(beg, len, vals, pslot, pdep, spair, lane);
      else if (bl == 8) wave_sort_list<4>(beg, len, vals, pslot, pdep, spair, lane);
      else wave_sort_list<8>(beg, len, vals, pslot, pdep, spair, lane);
      continue;
    }
    const int S = 1 << bl;                                     // segment lanes
    const uint32_t per = 64u / (uint32_t)S;
    const uint32_t pos = s_start[d] + wi * per + (uint32_t)(lane / S);
    const uint32_t seg_lane = (uint32_t)(lane & (S - 1));
    uint32_t beg = 0u, len = 0u;
    if (pos < s_start[d] + s_cnt[d]) {
      const uint4 ti = tinfo[pos];
      beg = ti.y;
      len = ti.z - ti.y;
    }
    uint32_t e = 0xffffffffu, key = 0xffffffffu;
    if (seg_lane < len) {
      e = vals[beg + seg_lane];
      key = pdep[e];
    }
    for (int k = 2; k <= S; k <<= 1) {
      for (int j = k >> 1; j > 0; j >>= 1) {
        // partner lane ^ j (inside the wave: j < 64), one address for both
        const int src = (lane ^ j) << 2;
        const uint32_t ok = (uint32_t)__builtin_amdgcn_ds_bpermute(src, (int)key);
        const uint32_t oe = (uint32_t)__builtin_amdgcn_ds_bpermute(src, (int)e);
        const bool keep_min = ((lane & j) == 0) == ((seg_lane & (uint32_t)k) == 0u);
        const bool other_less = key_less(ok, oe, key, e);
        if (keep_min == other_less) {
          key = ok;
          e = oe;
        }
      }
    }
    if (seg_lane < len) {
      vals[beg + seg_lane] = e;
      spair[beg + seg_lane] = pslot[e];
    }
  }
}

// Lists of more than kWaveSortMax entries, taken in launch order (longest
// first, so a block stops at the first shorter list): up to kLongSort
// entries in an LDS bitonic network; longer lists by ranking every entry
// against all others through the free sort buffers (quadratic, for rare
// extreme lists).
constexpr int kLongSort = 4096;
constexpr int kLongBlocks = 4096;
constexpr int kShortBlocks = 16384;

__global__ __launch_bounds__(256) void k_tile_sort_long(const uint4* __restrict__ tinfo, int64_t T,
                                                        uint32_t* __restrict__ vals,
                                                        const uint32_t* __restrict__ pslot,
                                                        const uint32_t* __restrict__ pdep,
                                                        uint32_t* __restrict__ spair,
                                                        uint32_t* __restrict__ tmpk,
                                                        uint32_t* __restrict__ tmpv) {
  __shared__ uint32_t s_k[kLongSort];
  __shared__ uint32_t s_i[kLongSort];   // e of each entry
  const int tid = threadIdx.x;
  for (int64_t b = blockIdx.x; b < T; b += gridDim.x) {
    const uint4 ti = tinfo[b];
    const uint32_t beg = ti.y, len = ti.z - ti.y;
    if (len <= kWaveSortMax) break;
    if (len <= (uint32_t)kLongSort) {
      uint32_t P = 128u;
      while (P < len) P <<= 1;
      for (uint32_t i = tid; i < P; i += 256u) {
        uint32_t key = 0xffffffffu, e = 0xffffffffu;
        if (i < len) {
          e = vals[beg + i];
          key = pdep[e];
        }
        s_k[i] = key;
        s_i[i] = e;
      }
      __syncthreads();
      // distances below 64 stay inside a wave's 64-element chunk: those steps
      // run on registers with cross-lane exchanges, the longer ones on LDS
      const int lane = tid & 63, wave = tid >> 6;
      auto chunk_steps = [&](uint32_t kfrom, uint32_t kto) {   // stages kfrom ... kto
        for (uint32_t c = (uint32_t)wave; c < (P >> 6); c += 4u) {
          const uint32_t gi = (c << 6) | (uint32_t)lane;
          uint32_t key = s_k[gi], idx = s_i[gi];
          for (uint32_t kk = kfrom; kk <= kto; kk <<= 1) {
            for (uint32_t j = min(kk >> 1, 32u); j > 0u; j >>= 1) {
              const uint32_t ok = (uint32_t)__shfl_xor((int)key, (int)j, 64);
              const uint32_t oi = (uint32_t)__shfl_xor((int)idx, (int)j, 64);
              const bool keep_min = (((uint32_t)lane & j) == 0u) == ((gi & kk) == 0u);
              if (keep_min == key_less(ok, oi, key, idx)) {
                key = ok;
                idx = oi;
              }
            }
          }
          s_k[gi] = key;
          s_i[gi] = idx;
        }
        __syncthreads();
      };
      chunk_steps(2u, 64u);
      for (uint32_t k = 128u; k <= P; k <<= 1) {
        for (uint32_t j = k >> 1; j >= 64u; j >>= 1) {
          for (uint32_t t = tid; t < (P >> 1); t += 256u) {
            const uint32_t i = ((t & ~(j - 1u)) << 1) | (t & (j - 1u));   // lower element
            const uint32_t p = i | j;
            const uint32_t ka = s_k[i], ia = s_i[i], kb = s_k[p], ib = s_i[p];
            const bool up = (i & k) == 0u;
            if (up == key_less(kb, ib, ka, ia)) {
              s_k[i] = kb; s_i[i] = ib;
              s_k[p] = ka; s_i[p] = ia;
            }
          }
          __syncthreads();
        }
        chunk_steps(k, k);
      }
      for (uint32_t rk = tid; rk < len; rk += 256u) {
        const uint32_t e = s_i[rk];
        vals[beg + rk] = e;
        spair[beg + rk] = pslot[e];
      }
      __syncthreads();
    } else {
      for (uint32_t i = tid; i < len; i += 256u) {
        tmpk[beg + i] = pdep[vals[beg + i]];
      }
      __syncthreads();
      for (uint32_t i = tid; i < len; i += 256u) {
        const uint32_t ki = tmpk[beg + i], ei = vals[beg + i];
        uint32_t rank = 0u;
        for (uint32_t j = 0; j < len; ++j)
          rank += key_less(tmpk[beg + j], vals[beg + j], ki, ei) ? 1u : 0u;
        tmpv[beg + rank] = ei;
      }
      __syncthreads();
      for (uint32_t rk = tid; rk < len; rk += 256u) {
        const uint32_t e = tmpv[beg + rk];
        vals[beg + rk] = e;
        spair[beg + rk] = pslot[e];
      }
      __syncthreads();
    }
  }
}

// Tile layout: list start and range of every tile, and the compositing launch
// order with a work item per launch position.  The launch order takes the
// longest lists first: bucket d = 15 - (bit length of the list length,
// capped at 15) ascending, tile index order inside a bucket (a tile's results
// do not depend on when it runs; the order keeps the few very long far-field
// lists from starting last and setting the kernel's end).  Inside each bucket
// the launch positions are permuted in blocks of 64 (an 8 x 8 transpose), so
// that runs of 8 consecutive tiles of the order (one tile row, mostly the
// same surfels) take launch positions 8 apart: the workgroups of one launch
// go to the 8 XCDs in turn, so such a run is composited by one XCD and its
// surfels' records stay in that XCD's L2.  Three launches: per block of
// kTileBlk tiles the pair count and the bucket sizes (k_tile_part), their
// exclusive scans down the blocks and the totals (k_tile_top), then the
// placement (k_tile_layout).

__device__ __forceinline__ uint32_t tile_bucket(uint32_t len) {
  const int bl = len ? 32 - __clz((int)len) : 0;
  return 15u - (uint32_t)min(bl, 15);
}

__global__ __launch_bounds__(256) void k_tile_part(const uint32_t* __restrict__ tcnt, int64_t T,
                                                   uint32_t* __restrict__ tpart) {
  __shared__ uint32_t s_h[16];
  __shared__ uint32_t s_w[4];
  if (threadIdx.x < 16) s_h[threadIdx.x] = 0u;
  __syncthreads();
  uint32_t sum = 0u;
#pragma unroll
  for (int r = 0; r < kTileBlk / 256; ++r) {
    const int64_t i = (int64_t)blockIdx.x * kTileBlk + r * 256 + threadIdx.x;
    if (i < T) {
      const uint32_t c = tcnt[i];
      sum += c;
      atomicAdd(&s_h[tile_bucket(c)], 1u);
    }
  }
  uint32_t total;
  (void)block_excl_scan(sum, s_w, &total);
  uint32_t* row = tpart + (size_t)blockIdx.x * kTPart;
  if (threadIdx.x == 0) row[0] = total;
  if (threadIdx.x < 16) row[1 + threadIdx.x] = s_h[threadIdx.x];
}

// One wave per column j of the nblk x kTPart table: its exclusive scan down
// the blocks, in place, and its total; the bucket sizes also go to
// bucket_tot for the depth sorts.
__global__ __launch_bounds__(64) void k_tile_top(uint32_t* __restrict__ tpart, int64_t nblk,
                                                 uint32_t* __restrict__ tot,
                                                 uint32_t* __restrict__ bucket_tot) {
  const int j = blockIdx.x, lane = threadIdx.x;
  uint32_t carry = 0u;
  for (int64_t r0 = 0; r0 < nblk; r0 += 64) {
    const int64_t r = r0 + lane;
    const uint32_t v = r < nblk ? tpart[r * kTPart + j] : 0u;
    const uint32_t inc = wave_incl_scan(v, lane);
    if (r < nblk) tpart[r * kTPart + j] = carry + inc - v;
    carry += (uint32_t)__shfl((int)inc, 63, 64);
  }
  if (lane == 0) {
    tot[j] = carry;
    if (j > 0) bucket_tot[j - 1] = carry;
  }
}

__global__ __launch_bounds__(256) void k_tile_layout(const uint32_t* __restrict__ tcnt, int64_t T,
                                                     const uint32_t* __restrict__ tpart,
                                                     const uint32_t* __restrict__ tot,
                                                     const ViewDev* __restrict__ views, int V,
                                                     uint32_t* __restrict__ tstart,
                                                     uint2* __restrict__ ranges,
                                                     uint4* __restrict__ tinfo) {
  __shared__ uint32_t s_bst[16], s_bsz[16], s_run[16];
  __shared__ uint32_t s_wc[4][16];
  __shared__ uint32_t s_ws[4];
  __shared__ uint32_t s_prun;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const unsigned long long lt = (1ull << lane) - 1ull;
  const uint32_t* row = tpart + (size_t)blockIdx.x * kTPart;
  if (threadIdx.x < 16) {
    const int d = threadIdx.x;
    uint32_t st = 0u;
    for (int k = 0; k < d; ++k) st += tot[1 + k];
    s_bst[d] = st;
    s_bsz[d] = tot[1 + d];
    s_run[d] = row[1 + d];                 // this block's first rank in bucket d
  }
  if (threadIdx.x == 0) s_prun = row[0];
  if (threadIdx.x < 64) (&s_wc[0][0])[threadIdx.x] = 0u;
  __syncthreads();
  for (int r = 0; r < kTileBlk / 256; ++r) {
    const int64_t i = (int64_t)blockIdx.x * kTileBlk + r * 256 + threadIdx.x;
    const bool valid = i < T;
    const uint32_t c = valid ? tcnt[i] : 0u;
    const uint32_t d = tile_bucket(c);
    const uint32_t inc = wave_incl_scan(c, lane);
    // lanes of the wave in the same bucket
    unsigned long long m = __ballot(valid);
#pragma unroll
    for (int bit = 0; bit < 4; ++bit) {
      const bool on = (d >> bit) & 1u;
      const unsigned long long bb = __ballot(valid && on);
      m &= on ? bb : ~bb;
    }
    const uint32_t below = (uint32_t)__popcll(m & lt);
    if (valid && below == 0u) s_wc[wv][d] = (uint32_t)__popcll(m);
    if (lane == 63) s_ws[wv] = inc;
    __syncthreads();
    if (valid) {
      uint32_t pst = s_prun + inc - c, rk = s_run[d] + below;
      for (int w = 0; w < wv; ++w) {
        pst += s_ws[w];
        rk += s_wc[w][d];
      }
      tstart[i] = pst;
      ranges[i] = c ? make_uint2(pst, pst + c) : make_uint2(0u, 0u);
      // launch position: the 8 x 8 transpose inside full blocks of 64
      uint32_t q = rk;
      if (q < (s_bsz[d] & ~63u)) q = (q & ~63u) + 8u * (q & 7u) + ((q >> 3) & 7u);
      int lo = 0, hi = V - 1;
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (views[mid].tile_off <= (int32_t)i) lo = mid; else hi = mid - 1;
      }
      // the view and the tile's row in it (images are at most 16384 rows)
      const uint32_t row_in_view = (uint32_t)(((int32_t)i - views[lo].tile_off) / views[lo].tiles_x);
      const uint32_t vr = (uint32_t)lo | (row_in_view << kViewBits);
      tinfo[s_bst[d] + q] = c ? make_uint4((uint32_t)i, pst, pst + c, vr)
                              : make_uint4((uint32_t)i, 0u, 0u, vr);
    }
    __syncthreads();
    if (threadIdx.x < 16) {
      uint32_t add = 0u;
      for (int w = 0; w < 4; ++w) add += s_wc[w][threadIdx.x];
      s_run[threadIdx.x] += add;
    }
    if (threadIdx.x == 0) s_prun += s_ws[0] + s_ws[1] + s_ws[2] + s_ws[3];
    __syncthreads();
    if (threadIdx.x < 64) (&s_wc[0][0])[threadIdx.x] = 0u;
    __syncthreads();
  }
}

}  // namespace

// Binning of the current batch.  n_pairs / n_vis >= 0: counts known on the
// host (exact grids); < 0: read on the device (grids sized by the capacity).
void launch_binning(const Layout& L, void* ws, int64_t n_pairs, int64_t n_vis, hipStream_t st,
                    bool counts_cleared) {
  uint32_t* misc = at<uint32_t>(ws, L.o_misc);
  const uint32_t* p_dev = n_pairs < 0 ? misc + kMiscPairs : nullptr;
  const uint32_t* s_dev = n_vis < 0 ? misc + kMiscVisible : nullptr;
  const int64_t s_grid = n_vis < 0 ? L.scap : n_vis;
  const int64_t p_grid = n_pairs < 0 ? L.cap : n_pairs;
  const int64_t T = L.total_tiles;
  uint32_t* tcnt = at<uint32_t>(ws, L.o_tcnt);
  uint32_t* tstart = at<uint32_t>(ws, L.o_tstart);
  if (!counts_cleared) fill_u32(tcnt, 0u, T, st);
  // 1. visible slots in (view, surfel id) order, with their emission counts
  uint32_t* sv = at<uint32_t>(ws, L.o_sval);
  uint32_t* scnt = at<uint32_t>(ws, L.o_scnt);
  uint32_t* soff = at<uint32_t>(ws, L.o_soff);
  //    and first pairs, and the first slot of every emission block
  const uint32_t nblk_emit = (uint32_t)((p_grid + kEmitPairs - 1) / kEmitPairs);
  hipLaunchKernelGGL(k_compact, dim3(L.nb), dim3(kProjBlock), 0, st, L.V, L.N, L.nb,
                     at<const uint32_t>(ws, L.o_cnt), at<const uint32_t>(ws, L.o_part),
                     at<const uint32_t>(ws, L.o_partv), L.scap, sv, scnt, soff,
                     at<uint32_t>(ws, L.o_pos), at<uint32_t>(ws, L.o_bstart), nblk_emit, misc,
                     L.cap);
  uint32_t* n_emit = p_dev ? misc + kMiscEmit : nullptr;
  // 2. one (tile, rank) per covered tile, counted per tile
  uint32_t* keys = at<uint32_t>(ws, L.o_keys);
  uint32_t* rank = at<uint32_t>(ws, L.o_vals2);
  if (p_grid > 0) {
    if (s_grid > 0) {
      const uint32_t nblk = nblk_emit;
      hipLaunchKernelGGL(k_emit, dim3(nblk), dim3(kEmitThreads), 0, st,
                         at<const ViewDev>(ws, L.o_views), L.N, p_dev, p_grid, s_dev, s_grid,
                         L.scap, L.cap, sv, soff, scnt, at<const uint2>(ws, L.o_rect),
                         at<const uint16_t>(ws, L.o_rspan), at<const float4>(ws, L.o_rec),
                         L.q_cut, at<const uint32_t>(ws, L.o_bstart), keys, rank,
                         at<uint32_t>(ws, L.o_pslot), at<uint32_t>(ws, L.o_pdep), tcnt, n_emit);
    } else if (n_emit) {
      fill_u32(n_emit, 0u, 1, st);
    }
  }
  // 3. first list position and range of every tile and the compositing
  //    launch order, then the pairs grouped by tile (launch_ranges orders
  //    each tile's list by depth)
  const int64_t nbt = (T + kTileBlk - 1) / kTileBlk;
  uint32_t* tpart = at<uint32_t>(ws, L.o_tscan);
  uint32_t* ttot = tpart + nbt * kTPart;
  hipLaunchKernelGGL(k_tile_part, dim3((unsigned)nbt), dim3(256), 0, st, tcnt, T, tpart);
  hipLaunchKernelGGL(k_tile_top, dim3(kTPart), dim3(64), 0, st, tpart, nbt, ttot,
                     at<uint32_t>(ws, L.o_histtmp));
  hipLaunchKernelGGL(k_tile_layout, dim3((unsigned)nbt), dim3(256), 0, st, tcnt, T, tpart, ttot,
                     at<const ViewDev>(ws, L.o_views), L.V, tstart, at<uint2>(ws, L.o_ranges),
                     at<uint4>(ws, L.o_tinfo));
  if (p_grid > 0 && s_grid > 0)
    hipLaunchKernelGGL(k_place, dim3((unsigned)((p_grid + 255) / 256)), dim3(256), 0, st, keys,
                       rank, tstart, n_emit, p_grid, L.cap, at<uint32_t>(ws, L.o_vals));
}

hipError_t launch_ranges(const Layout& L, void* ws, hipStream_t st, hipStream_t side,
                         hipEvent_t fork, hipEvent_t join) {
  // each tile's list by depth, and the slot of every sorted pair; the two
  // kernels touch disjoint tiles
  const int64_t T = L.total_tiles;
  hipStream_t lst = st;
  if (side) {
    hipError_t e = hipEventRecord(fork, st);
    if (e == hipSuccess) e = hipStreamWaitEvent(side, fork, 0);
    if (e != hipSuccess) return e;
    lst = side;
  }
  hipLaunchKernelGGL(k_tile_sort_long, dim3((unsigned)std::min<int64_t>(T, kLongBlocks)), dim3(256),
                     0, lst, at<const uint4>(ws, L.o_tinfo), T, at<uint32_t>(ws, L.o_vals),
                     at<const uint32_t>(ws, L.o_pslot), at<const uint32_t>(ws, L.o_pdep),
                     at<uint32_t>(ws, L.o_spair), at<uint32_t>(ws, L.o_keys2),
                     at<uint32_t>(ws, L.o_vals2));
  if (side) {
    hipError_t e = hipEventRecord(join, side);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_tile_sort_short, dim3((unsigned)std::min<int64_t>(T, kShortBlocks)),
                     dim3(64), 0, st, at<const uint4>(ws, L.o_tinfo),
                     at<const uint32_t>(ws, L.o_histtmp), at<uint32_t>(ws, L.o_vals),
                     at<const uint32_t>(ws, L.o_pslot), at<const uint32_t>(ws, L.o_pdep),
                     at<uint32_t>(ws, L.o_spair));
  return side ? hipStreamWaitEvent(st, join, 0) : hipSuccess;
}

}  // namespace rogs
