// Tile render mask and per-tile depth order (Supp. "Local Optimization Kernel", item 1).
//
// Pipeline for V views of n Gaussians (entry e = v*n + i):
//   1. mask    : tiles covered by the rectangles of the changed Gaussians (LDS bitmap per
//                block, OR-ed into the global bitmap), or all tiles in full mode; then
//                its index: the sorted list of set tiles (the tiles to render) and a
//                corner table of prefix counts that gives the set tiles of any
//                rectangle in O(1);
//   2. count   : pairs each entry emits = masked tiles of its rectangle;
//   3. compact : entries with at least one pair, keyed by their float32 depth bits;
//   4. sort    : stable LSD radix sort of those keys (equal depths keep entry order);
//   5. emit    : in depth order, each entry writes (global tile, entry) for its masked
//                tiles at its prefix-sum offset;
//   6. sort    : stable LSD radix sort of the pairs by global tile only — the depth
//                order within a tile comes from step 4, so only ceil(log2(V*T)) key bits
//                are sorted instead of tile + 32 depth bits;
//   7. ranges  : [start, end) of each tile's run.
// Masked slabs whose per-chunk tile counts fit a budget replace 5-7 by a counting
// placement (see "5-7 by counting"): per chunk of 64 entries and per tile, which of
// the chunk's entries cover the tile; the counts' prefix over the chunks gives every
// pair its position in tile order directly.
// Every kernel reads its element count from device memory, so nothing is read back.
//
// Depth-sliced lists: steps 5-7 first run for the nearest slab of the depth order
// only; after the forward pass has rendered it, steps 5-6 run again for the remaining
// entries, emitting only into the tiles that still have compositing pixels (the
// "alive" tiles, indexed like the mask), and the forward continues those tiles, each
// finding its run of the second slab by a search over the sorted tiles (step 7).
#include <algorithm>

#include "internal.hpp"

namespace clsp {
namespace {

constexpr int NT = 256;                     // threads per block
constexpr int RS_ITEMS = 4;                 // keys per thread per chunk
constexpr int RS_CHUNK = NT * RS_ITEMS;     // 1024 keys staged in LDS per chunk
constexpr int RS_WAVE_SPAN = 64 * RS_ITEMS; // consecutive keys one wave ranks per chunk
constexpr int MAX_SORT_BLOCKS = 2048;
constexpr int RS_RAW_BLOCKS = 64;  // sorts of at most this many blocks skip the digit-scan launch
constexpr int SCAN_ITEMS = 8;
constexpr int SCAN_CHUNK = NT * SCAN_ITEMS;
constexpr int MAX_SCAN_BLOCKS = 1024;

// Counter slots (see clsp_bins).
constexpr int C_PAIRS = 0, C_OVERFLOW = 1, C_TILES = 2, C_WRITTEN = 3, C_ENTRIES = 4, C_STICKY = 5, C_SLAB1 = 6,
              C_PAIRS1 = 7, C_ALIVE = 8;
// scratch counter slots used while a slab is listed
constexpr int C_SLAB_LO = 9, C_SLAB_N = 10, C_SLAB_PAIRS = 11, C_SLAB_BASE = 12;
// scratch counter slots of lists built from a stored depth order of the unchanged rows
constexpr int C_FSPLIT = 13, C_NACT = 14;

__device__ __forceinline__ uint32_t lane_id() { return threadIdx.x & 63u; }

__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t x) {
  const uint32_t lane = lane_id();
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t y = __shfl_up(x, o, 64);
    if (lane >= (uint32_t)o) x += y;
  }
  return x;
}

// Exclusive scan across a 256-thread block; s4 is 4 words of LDS.
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t x, uint32_t* s4, uint32_t& total) {
  const uint32_t inc = wave_incl_scan(x);
  const int w = threadIdx.x >> 6;
  if (lane_id() == 63) s4[w] = inc;
  __syncthreads();
  uint32_t off = 0;
  for (int k = 0; k < w; ++k) off += s4[k];
  total = s4[0] + s4[1] + s4[2] + s4[3];
  __syncthreads();
  return off + inc - x;
}

__device__ __forceinline__ uint32_t load_count(const uint32_t* p, uint32_t fallback) { return p ? *p : fallback; }

// Contiguous element span of block b out of G for n elements (multiples of `quant`).
__device__ __forceinline__ void block_span(uint32_t n, int G, int b, uint32_t quant, uint32_t& beg, uint32_t& end) {
  uint64_t per = ((uint64_t)n + G - 1) / G;
  per = (per + quant - 1) / quant * quant;
  uint64_t bg = (uint64_t)b * per;
  if (bg > n) bg = n;
  uint64_t en = bg + per;
  if (en > n) en = n;
  beg = (uint32_t)bg;
  end = (uint32_t)en;
}

// Sum of a[lo, hi) across the block (every thread calls it; s4 is 4 words of LDS).
__device__ __forceinline__ uint32_t block_sum_range(const uint32_t* __restrict__ a, uint32_t lo, uint32_t hi,
                                                    uint32_t* s4) {
  uint32_t x = 0;
  for (uint32_t i = lo + threadIdx.x; i < hi; i += NT) x += a[i];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
  if ((threadIdx.x & 63u) == 0) s4[threadIdx.x >> 6] = x;
  __syncthreads();
  x = s4[0] + s4[1] + s4[2] + s4[3];
  __syncthreads();
  return x;
}

// ------------------------------------------------------------------ fills
// Zero up to CLEAR_SEGS buffers in one launch.
constexpr int CLEAR_SEGS = 6;
struct ClearList {
  uint32_t* p[CLEAR_SEGS];
  int64_t n[CLEAR_SEGS];
  int k;
};

__global__ void clear_kernel(ClearList c) {
  for (int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x;; i += (int64_t)gridDim.x * NT) {
    int64_t j = i;
    int s = 0;
    while (s < c.k && j >= c.n[s]) j -= c.n[s++];
    if (s == c.k) return;
    c.p[s][j] = 0u;
  }
}

__global__ void fill_u32_kernel(uint32_t* p, uint32_t value, int64_t count) {
  for (int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x; i < count; i += (int64_t)gridDim.x * NT) p[i] = value;
}

// Full mode: every valid tile bit of every view.
__global__ void mask_all_kernel(uint32_t* mask, int views, int T, int wpv) {
  const int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x;
  if (i >= (int64_t)views * wpv) return;
  const int w = (int)(i % wpv);
  const int lo = w * 32;
  uint32_t bits = 0;
  if (lo + 32 <= T) bits = 0xffffffffu;
  else if (lo < T) bits = (1u << (T - lo)) - 1u;
  mask[i] = bits;
}

// ------------------------------------------------------------------ 1. render mask
__global__ void __launch_bounds__(NT) mask_kernel(const uint2* __restrict__ rect, const uint32_t* __restrict__ flags,
                                                  int64_t n, int64_t a0, int64_t a1, int TX, int wpv,
                                                  uint32_t* __restrict__ mask) {
  extern __shared__ uint32_t smask[];
  const int v = blockIdx.y;
  for (int w = threadIdx.x; w < wpv; w += NT) smask[w] = 0;
  __syncthreads();
  const int64_t i = a0 + (int64_t)blockIdx.x * NT + threadIdx.x;
  if (i < a1) {
    const int64_t e = (int64_t)v * n + i;
    if (flags[e] & CLSP_FLAG_VISIBLE) {
      const uint2 r = rect[e];
      const uint32_t x0 = r.x & 0xffffu, x1 = r.x >> 16, y0 = r.y & 0xffffu, y1 = r.y >> 16;
      for (uint32_t ty = y0; ty < y1; ++ty)
        for (uint32_t tx = x0; tx < x1; ++tx) {
          const uint32_t t = ty * TX + tx;
          atomicOr(&smask[t >> 5], 1u << (t & 31));
        }
    }
  }
  __syncthreads();
  for (int w = threadIdx.x; w < wpv; w += NT)
    if (smask[w]) atomicOr(&mask[(int64_t)v * wpv + w], smask[w]);
}

// Number of set bits of `m` in [lo, hi).
__device__ __forceinline__ uint32_t count_bits(const uint32_t* m, uint32_t lo, uint32_t hi) {
  uint32_t c = 0;
  while (lo < hi) {
    const uint32_t w = lo >> 5, b = lo & 31;
    const uint32_t take = min(32u - b, hi - lo);
    const uint32_t sel = (take == 32 ? 0xffffffffu : ((1u << take) - 1u)) << b;
    c += __popc(m[w] & sel);
    lo += take;
  }
  return c;
}

// Corner table of a tile bitmap (built by mask_index_kernel): for view v, row ty in
// [0, TY] and column x in [0, TX], tab[(v*(TY+1) + ty)*(TX+1) + x] = set tiles in rows
// < ty and columns < x.  The set tiles of a rectangle, and the rank of a tile among
// the view's set tiles in row-major order, follow from four and three entries.
__device__ __forceinline__ uint32_t tab_rect(const uint32_t* tab, uint32_t vrow, uint32_t TXp, uint32_t x0, uint32_t x1,
                                             uint32_t ya, uint32_t yb) {
  const uint32_t* a = tab + (size_t)(vrow + ya) * TXp;
  const uint32_t* b = tab + (size_t)(vrow + yb) * TXp;
  return (b[x1] - b[x0]) - (a[x1] - a[x0]);
}

// Set tiles of the view before (ty, x), row-major (TX = TXp - 1).
__device__ __forceinline__ uint32_t tab_rank(const uint32_t* tab, uint32_t vrow, uint32_t TXp, uint32_t ty, uint32_t x) {
  const uint32_t* a = tab + (size_t)(vrow + ty) * TXp;
  return a[TXp - 1] + (a[TXp + x] - a[x]);
}

// ------------------------------------------------------------------ 2. counts
// Pairs of each entry: the rectangle's area, or its set tiles in the mask (corner table).
// Block b takes the span block_span(E, G, b, NT) of entries e = v*n + i, and also
// writes how many of them have pairs to blk[b]: the first step of the compaction's
// exclusive scan (scan_compact_kernel uses the same spans).  Rows i >= row_lim count
// no pairs (row_lim = n: every row).
__global__ void __launch_bounds__(NT) count_kernel(const uint2* __restrict__ rect, const uint32_t* __restrict__ flags,
                                                   const uint32_t* __restrict__ tab, uint32_t n, uint32_t E, int G,
                                                   int TX, int TY, int use_mask, uint32_t row_lim,
                                                   uint32_t* __restrict__ cnt, uint32_t* __restrict__ blk) {
  __shared__ uint32_t s4[4];
  uint32_t beg, end;
  block_span(E, G, blockIdx.x, NT, beg, end);
  uint32_t has = 0;
  constexpr int U = 4;  // entries per thread per round, their loads issued together
  const uint32_t TXp = (uint32_t)TX + 1, TYp = (uint32_t)TY + 1;
  for (uint32_t e0 = beg + threadIdx.x; e0 < end; e0 += U * NT) {
    uint32_t fl[U];
    uint2 r[U];
#pragma unroll
    for (int k = 0; k < U; ++k) {
      const uint32_t e = e0 + k * NT;
      fl[k] = e < end ? flags[e] : 0u;
      r[k] = e < end ? rect[e] : make_uint2(0u, 0u);
    }
#pragma unroll
    for (int k = 0; k < U; ++k) {
      const uint32_t e = e0 + k * NT;
      // a rectangle within the tile grid (preprocess writes no other), or none
      const uint32_t x0 = min(r[k].x & 0xffffu, (uint32_t)TX), x1 = min(r[k].x >> 16, (uint32_t)TX);
      const uint32_t y0 = min(r[k].y & 0xffffu, (uint32_t)TY), y1 = min(r[k].y >> 16, (uint32_t)TY);
      bool ok = (fl[k] & CLSP_FLAG_VISIBLE) && x1 > x0 && y1 > y0;
      if (row_lim < n) ok = ok && e % n < row_lim;
      uint32_t c = 0;
      if (!use_mask) {
        c = (x1 - x0) * (y1 - y0);
      } else {
        const uint32_t v = e < end ? e / n : 0u;
        c = tab_rect(tab, v * TYp, TXp, ok ? x0 : 0u, ok ? x1 : 0u, ok ? y0 : 0u, ok ? y1 : 0u);
      }
      c = ok ? c : 0u;
      if (e < end) cnt[e] = c;
      has += c != 0u ? 1u : 0u;
    }
  }
  uint32_t tot;
  block_excl_scan(has, s4, tot);
  if (threadIdx.x == 0) blk[blockIdx.x] = tot;
}

// Capacity check after a slab's pair count: P = first-slab pairs + this slab's pairs.
__device__ void capacity_check(uint32_t* counters, uint64_t capacity, int which) {
  const uint32_t sp = counters[C_SLAB_PAIRS];
  const uint32_t p = (which == 1 ? 0u : counters[C_PAIRS1]) + sp;
  if (which == 1) counters[C_PAIRS1] = sp;
  const bool over = (uint64_t)p > capacity || counters[C_OVERFLOW];
  counters[C_PAIRS] = p;
  counters[C_OVERFLOW] = over ? 1u : 0u;
  counters[C_WRITTEN] = over ? 0u : p;
  if (over) {
    counters[C_STICKY] = 1u;
    if (which == 1) counters[C_TILES] = 0u;  // no tile is rendered
    counters[C_SLAB_PAIRS] = 0u;  // nothing is emitted or sorted
    counters[C_SLAB_N] = 0u;
  }
}

// The rest of the exclusive scan over the entries' has-pairs flags (pair count > 0), as
// a compaction: entry e with a pair goes to position p (its exclusive prefix) as
// (depth key, e).  Block b's base is the sum of the count pass's block sums blk[0, b);
// block 0 writes the total (the entries with pairs) to *total_out.
__global__ void __launch_bounds__(NT) scan_compact_kernel(const uint32_t* __restrict__ cnt, uint32_t n,
                                                          const uint32_t* __restrict__ blk, int G,
                                                          const float* __restrict__ depth, uint32_t* __restrict__ keys,
                                                          uint32_t* __restrict__ vals, uint32_t* __restrict__ total_out) {
  __shared__ uint32_t s4[4];
  if (blockIdx.x == 0) {
    const uint32_t all = block_sum_range(blk, 0, (uint32_t)G, s4);
    if (threadIdx.x == 0) *total_out = all;
  }
  uint32_t beg, end;
  block_span(n, G, blockIdx.x, NT, beg, end);
  uint32_t base = block_sum_range(blk, 0, blockIdx.x, s4);
  for (uint32_t c = beg; c < end; c += SCAN_CHUNK) {
    uint32_t v[SCAN_ITEMS], dk[SCAN_ITEMS];
    uint32_t sum = 0;
    const uint32_t t0 = c + threadIdx.x * SCAN_ITEMS;
#pragma unroll
    for (int k = 0; k < SCAN_ITEMS; ++k) {
      const bool in = t0 + k < end;
      v[k] = (in && cnt[t0 + k] != 0u) ? 1u : 0u;
      dk[k] = in ? __float_as_uint(depth[t0 + k]) : 0u;  // depth > 0.2: the bit pattern orders like the value
      sum += v[k];
    }
    uint32_t tot;
    uint32_t off = base + block_excl_scan(sum, s4, tot);
#pragma unroll
    for (int k = 0; k < SCAN_ITEMS; ++k) {
      if (v[k]) {
        keys[off] = dk[k];
        vals[off] = t0 + k;
      }
      off += v[k];
    }
    base += tot;
  }
}

// ------------------------------------------------------------------ 2-3 from a stored order
// The unchanged rows [0, a0) of local optimisation keep their projection, so their
// entries' depth order can be built once and reused (Supp. "Local Optimization Kernel",
// item 1 reuses the projection for the per-tile depth ordering).  The stored order is
// one buffer of 32-bit words: a header of ORD_HDR words ([0]: the number of entries
// nF), then for cap = views * a0 slots the entry indices (ascending (depth key, entry)
// order), their depth keys and their rectangles (uint2, 8-byte aligned).  It holds the
// entries of the unchanged rows that are visible with a nonempty rectangle, the ones
// that can have pairs under any mask.
constexpr uint32_t ORD_HDR = 64;
__host__ __device__ inline uint64_t ord_rect_word(uint64_t cap) { return (ORD_HDR + 2 * cap + 1) & ~1ull; }

// Stored order of the build: its nF sorted entries and their rectangles.
__global__ void __launch_bounds__(NT) order_store_kernel(const uint32_t* __restrict__ keys,
                                                         const uint32_t* __restrict__ vals,
                                                         const uint2* __restrict__ rect, uint32_t cap,
                                                         uint32_t* __restrict__ ord) {
  const uint32_t nF = min(ord[0], cap);
  uint2* rects = reinterpret_cast<uint2*>(ord + ord_rect_word(cap));
  for (uint32_t p = blockIdx.x * NT + threadIdx.x; p < nF; p += gridDim.x * NT) {
    const uint32_t e = vals[p];
    ord[ORD_HDR + p] = e;
    ord[ORD_HDR + cap + p] = keys[p];
    rects[p] = rect[e];
  }
}

// Count pass over positions p in [0, cap + views * (n - a0)): position p < cap is slot p
// of the stored order (no pairs when p >= nF), the others are the changed entries
// v*n + i, i in [a0, n), view-major.  cnt[p] = masked tiles of the rectangle; blk[b] /
// blkF[b] = positions of block b with pairs, all / those of the stored order (the
// compaction then knows where the stored entries end).
__global__ void __launch_bounds__(NT) count_frozen_kernel(const uint32_t* __restrict__ ord, uint32_t cap,
                                                          const uint2* __restrict__ rect,
                                                          const uint32_t* __restrict__ flags,
                                                          const uint32_t* __restrict__ tab, uint32_t n, uint32_t a0,
                                                          uint32_t NP, int G, int TX, int TY,
                                                          uint32_t* __restrict__ cnt, uint32_t* __restrict__ blk,
                                                          uint32_t* __restrict__ blkF) {
  __shared__ uint32_t s4[4];
  const uint32_t nF = min(ord[0], cap);
  const uint32_t* fvals = ord + ORD_HDR;
  const uint2* frect = reinterpret_cast<const uint2*>(ord + ord_rect_word(cap));
  const uint32_t na = n - a0;
  uint32_t beg, end;
  block_span(NP, G, blockIdx.x, NT, beg, end);
  uint32_t hasF = 0, hasA = 0;
  constexpr int U = 4;
  const uint32_t TXp = (uint32_t)TX + 1, TYp = (uint32_t)TY + 1;
  for (uint32_t p0 = beg + threadIdx.x; p0 < end; p0 += U * NT) {
    uint32_t fl[U], e[U];
    uint2 r[U];
#pragma unroll
    for (int k = 0; k < U; ++k) {
      const uint32_t p = p0 + k * NT;
      fl[k] = 0u;
      e[k] = 0u;
      r[k] = make_uint2(0u, 0u);
      if (p < end) {
        if (p < cap) {
          if (p < nF) {
            e[k] = fvals[p];
            r[k] = frect[p];
            fl[k] = e[k] < NP ? CLSP_FLAG_VISIBLE : 0u;  // (an order built for these sizes holds no other)
            e[k] = e[k] < NP ? e[k] : 0u;
          }
        } else {
          const uint32_t q = p - cap;
          e[k] = (q / na) * n + a0 + q % na;
          r[k] = rect[e[k]];
          fl[k] = flags[e[k]];
        }
      }
    }
#pragma unroll
    for (int k = 0; k < U; ++k) {
      const uint32_t p = p0 + k * NT;
      const uint32_t x0 = min(r[k].x & 0xffffu, (uint32_t)TX), x1 = min(r[k].x >> 16, (uint32_t)TX);
      const uint32_t y0 = min(r[k].y & 0xffffu, (uint32_t)TY), y1 = min(r[k].y >> 16, (uint32_t)TY);
      const bool ok = (fl[k] & CLSP_FLAG_VISIBLE) && x1 > x0 && y1 > y0;
      const uint32_t v = e[k] / n;
      uint32_t c = tab_rect(tab, v * TYp, TXp, ok ? x0 : 0u, ok ? x1 : 0u, ok ? y0 : 0u, ok ? y1 : 0u);
      c = ok ? c : 0u;
      if (p < end) cnt[p] = c;
      if (p < cap) hasF += c != 0u ? 1u : 0u;
      else hasA += c != 0u ? 1u : 0u;
    }
  }
  uint32_t totF, totA;
  block_excl_scan(hasF, s4, totF);
  block_excl_scan(hasA, s4, totA);
  if (threadIdx.x == 0) {
    blk[blockIdx.x] = totF + totA;
    blkF[blockIdx.x] = totF;
  }
}

// Compaction of the positions with pairs, in position order, as (depth key, entry): the
// stored order's entries first (already in depth order), then the changed ones (entry
// order).  Block 0 writes the total (counters[C_ENTRIES]), the stored entries among
// them (counters[C_FSPLIT]) and the changed ones (counters[C_NACT]).
__global__ void __launch_bounds__(NT) scan_compact_frozen_kernel(const uint32_t* __restrict__ cnt, uint32_t NP,
                                                                 const uint32_t* __restrict__ blk,
                                                                 const uint32_t* __restrict__ blkF, int G,
                                                                 const uint32_t* __restrict__ ord, uint32_t cap,
                                                                 const float* __restrict__ depth, uint32_t n,
                                                                 uint32_t a0, uint32_t* __restrict__ keys,
                                                                 uint32_t* __restrict__ vals,
                                                                 uint32_t* __restrict__ counters) {
  __shared__ uint32_t s4[4];
  if (blockIdx.x == 0) {
    const uint32_t all = block_sum_range(blk, 0, (uint32_t)G, s4);
    const uint32_t fr = block_sum_range(blkF, 0, (uint32_t)G, s4);
    if (threadIdx.x == 0) {
      counters[C_ENTRIES] = all;
      counters[C_FSPLIT] = fr;
      counters[C_NACT] = all - fr;
    }
  }
  const uint32_t na = n - a0;
  uint32_t beg, end;
  block_span(NP, G, blockIdx.x, NT, beg, end);
  uint32_t base = block_sum_range(blk, 0, blockIdx.x, s4);
  for (uint32_t c = beg; c < end; c += SCAN_CHUNK) {
    uint32_t v[SCAN_ITEMS];
    uint32_t sum = 0;
    const uint32_t t0 = c + threadIdx.x * SCAN_ITEMS;
#pragma unroll
    for (int k = 0; k < SCAN_ITEMS; ++k) {
      v[k] = (t0 + k < end && cnt[t0 + k] != 0u) ? 1u : 0u;
      sum += v[k];
    }
    uint32_t tot;
    uint32_t off = base + block_excl_scan(sum, s4, tot);
#pragma unroll
    for (int k = 0; k < SCAN_ITEMS; ++k) {
      if (v[k]) {
        const uint32_t p = t0 + k;
        uint32_t e, key;
        if (p < cap) {
          e = ord[ORD_HDR + p];
          key = ord[ORD_HDR + cap + p];
        } else {
          const uint32_t q = p - cap;
          e = (q / na) * n + a0 + q % na;
          key = __float_as_uint(depth[e]);
        }
        keys[off] = key;
        vals[off] = e;
      }
      off += v[k];
    }
    base += tot;
  }
}

// (key, entry) order; entries are distinct, so it is a strict total order.
__device__ __forceinline__ bool key_entry_less(uint32_t ka, uint32_t ea, uint32_t kb, uint32_t eb) {
  return ka < kb || (ka == kb && ea < eb);
}

// Merge of the two sorted runs A = [0, s) (stored entries) and B = [s, M) (changed
// entries, sorted) of (keys, vals), s = counters[C_FSPLIT], M = counters[C_ENTRIES], into
// out[0, M) (entries only).  Each thread writes MG_ITEMS consecutive outputs from output
// position d: the number i of A entries among the first d outputs is the first mid
// with A[mid] not before B[d - 1 - mid] (a binary search on the merge path), then it
// merges sequentially.
constexpr int MG_ITEMS = 8;
__global__ void __launch_bounds__(NT) merge_runs_kernel(const uint32_t* __restrict__ keys,
                                                        const uint32_t* __restrict__ vals,
                                                        const uint32_t* __restrict__ counters,
                                                        uint32_t* __restrict__ out) {
  const uint32_t M = counters[C_ENTRIES], na = min(counters[C_FSPLIT], M), nb = M - na;
  const uint32_t *ka = keys, *va = vals, *kb = keys + na, *vb = vals + na;
  for (uint64_t d0 = ((uint64_t)blockIdx.x * NT + threadIdx.x) * MG_ITEMS; d0 < M;
       d0 += (uint64_t)gridDim.x * NT * MG_ITEMS) {
    const uint32_t d = (uint32_t)d0;
    uint32_t lo = d > nb ? d - nb : 0u, hi = min(d, na);
    while (lo < hi) {
      const uint32_t mid = (lo + hi) >> 1, j = d - 1u - mid;
      if (key_entry_less(ka[mid], va[mid], kb[j], vb[j])) lo = mid + 1u; else hi = mid;
    }
    uint32_t i = lo, j = d - lo;
    const uint32_t end = min(d + (uint32_t)MG_ITEMS, M);
    for (uint32_t o = d; o < end; ++o) {
      const bool take_a = i < na && (j >= nb || key_entry_less(ka[i], va[i], kb[j], vb[j]));
      out[o] = take_a ? va[i++] : vb[j++];
    }
  }
}

// ------------------------------------------------------------------ 3. compaction
// ------------------------------------------------------------------ radix sort
// All sort kernels work on keys[off + e], e < n, with n and off read from device memory.
__device__ __forceinline__ uint32_t load_off(const uint32_t* p) { return p ? *p : 0u; }

// Blocks that hold keys: one chunk each up to G (the grid), more per block beyond.
__device__ __forceinline__ int rs_blocks(uint32_t n, int G) {
  const uint32_t c = (n + RS_CHUNK - 1) / RS_CHUNK;
  return (int)min((uint32_t)G, max(c, 1u));
}

// Digit histogram of each block's span: hist[d * Ge + b], Ge = rs_blocks(n, G).
__global__ void __launch_bounds__(NT) rs_upsweep_kernel(const uint32_t* __restrict__ keys, const uint32_t* n_ptr,
                                                        const uint32_t* off_ptr, int shift, int bits,
                                                        uint32_t* __restrict__ hist, int G, int raw) {
  __shared__ uint32_t h[4][256];
  const uint32_t n = *n_ptr;
  const int Ge = rs_blocks(n, G);
  if ((int)blockIdx.x >= Ge) return;
  keys += load_off(off_ptr);
  const int radix = 1 << bits;
  const uint32_t msk = (uint32_t)radix - 1u;
  uint32_t beg, end;
  block_span(n, Ge, blockIdx.x, RS_CHUNK, beg, end);
  const int w = threadIdx.x >> 6;
  // the first keys are in flight while the histograms are cleared
  uint32_t e0 = beg + threadIdx.x;
  uint32_t k[RS_ITEMS];
#pragma unroll
  for (int u = 0; u < RS_ITEMS; ++u) k[u] = e0 + u * NT < end ? keys[e0 + u * NT] : 0u;
  for (int d = threadIdx.x; d < 4 * 256; d += NT) (&h[0][0])[d] = 0;
  __syncthreads();
  while (e0 < end) {
#pragma unroll
    for (int u = 0; u < RS_ITEMS; ++u)
      if (e0 + u * NT < end) atomicAdd(&h[w][(k[u] >> shift) & msk], 1u);
    e0 += RS_ITEMS * NT;
#pragma unroll
    for (int u = 0; u < RS_ITEMS; ++u) k[u] = e0 + u * NT < end ? keys[e0 + u * NT] : 0u;
  }
  __syncthreads();
  // digit-major for the scan kernel; block-major (raw) for a downsweep that reads every
  // block's counts itself
  for (int d = threadIdx.x; d < radix; d += NT)
    hist[raw ? (int64_t)blockIdx.x * radix + d : (int64_t)d * Ge + blockIdx.x] = h[0][d] + h[1][d] + h[2][d] + h[3][d];
}

// Block d: exclusive scan over blocks of digit d's counts; digit total -> tot[d].
__global__ void __launch_bounds__(NT) rs_scan_kernel(uint32_t* __restrict__ hist, const uint32_t* n_ptr, int G,
                                                     uint32_t* __restrict__ tot) {
  __shared__ uint32_t s4[4];
  constexpr int PER = MAX_SORT_BLOCKS / NT;
  G = rs_blocks(*n_ptr, G);
  uint32_t* row = hist + (int64_t)blockIdx.x * G;
  uint32_t v[PER];
  uint32_t sum = 0;
  for (int k = 0; k < PER; ++k) {
    const int idx = threadIdx.x * PER + k;
    v[k] = idx < G ? row[idx] : 0u;
    sum += v[k];
  }
  uint32_t total;
  uint32_t off = block_excl_scan(sum, s4, total);
  for (int k = 0; k < PER; ++k) {
    const int idx = threadIdx.x * PER + k;
    if (idx < G) row[idx] = off;
    off += v[k];
  }
  if (threadIdx.x == 0) tot[blockIdx.x] = total;
}

// Stable scatter of each block's span.  Each wave ranks RS_WAVE_SPAN consecutive keys with
// ballot-based digit matching; the block then stages the chunk in LDS ordered by digit
// and writes every digit's run contiguously.
template <bool RAW>
__global__ void __launch_bounds__(NT) rs_downsweep_kernel(const uint32_t* __restrict__ kin,
                                                          const uint32_t* __restrict__ vin,
                                                          uint32_t* __restrict__ kout, uint32_t* __restrict__ vout,
                                                          const uint32_t* n_ptr, const uint32_t* off_ptr, int shift,
                                                          int bits, const uint32_t* __restrict__ hist,
                                                          const uint32_t* __restrict__ tot, int G) {
  __shared__ uint32_t s_key[RS_CHUNK];
  __shared__ uint32_t s_val[RS_CHUNK];
  __shared__ uint32_t s_wcnt[4][256];
  __shared__ uint32_t s_base[256];
  __shared__ uint32_t s_choff[256];
  __shared__ uint32_t s_tot[256];
  __shared__ uint32_t s4[4];

  const uint32_t n = *n_ptr;
  const uint32_t off = load_off(off_ptr);
  kin += off;
  vin += off;
  kout += off;
  vout += off;
  G = rs_blocks(n, G);
  if ((int)blockIdx.x >= G) return;
  uint32_t beg, end;
  block_span(n, G, blockIdx.x, RS_CHUNK, beg, end);
  if (beg >= end) return;
  const int radix = 1 << bits;
  const uint32_t msk = (uint32_t)radix - 1u;
  const int tid = threadIdx.x, w = tid >> 6;
  const uint32_t lane = lane_id();
  const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));


  for (uint32_t c = beg; c < end; c += RS_CHUNK) {
    const uint32_t clen = min((uint32_t)RS_CHUNK, end - c);
    // the chunk's keys and values: all loads in flight while the counts are cleared
    uint32_t key[RS_ITEMS], val[RS_ITEMS], rnk[RS_ITEMS];
    const uint32_t wbase = c + w * RS_WAVE_SPAN;
#pragma unroll
    for (int it = 0; it < RS_ITEMS; ++it) {
      const uint32_t e = wbase + it * 64 + lane;
      key[it] = e < end ? kin[e] : 0u;
      val[it] = e < end ? vin[e] : 0u;
    }
    if (c == beg) {
      // the global base of each digit for this block, while the first loads are in flight:
      // from the digit totals and the scanned block counts, or (raw: a sort of at most
      // RS_RAW_BLOCKS blocks, no scan launch) from the upsweep's counts of every block
      uint32_t t = 0, before = 0;
      if (tid < radix) {
        if (RAW) {
          // (block-major counts: coalesced, all in flight together)
          uint32_t x[RS_RAW_BLOCKS];
#pragma unroll
          for (int b = 0; b < RS_RAW_BLOCKS; ++b) x[b] = b < G ? hist[(int64_t)b * radix + tid] : 0u;
#pragma unroll
          for (int b = 0; b < RS_RAW_BLOCKS; ++b) {
            t += x[b];
            before += b < (int)blockIdx.x ? x[b] : 0u;
          }
        } else {
          t = tot[tid];
          before = hist[(int64_t)tid * G + blockIdx.x];
        }
      }
      uint32_t all;
      const uint32_t ex = block_excl_scan(t, s4, all);
      if (tid < radix) s_base[tid] = ex + before;
    }
    for (int d = tid; d < 4 * 256; d += NT) (&s_wcnt[0][0])[d] = 0;
    __syncthreads();
#pragma unroll
    for (int it = 0; it < RS_ITEMS; ++it) {
      const uint32_t e = wbase + it * 64 + lane;
      const bool valid = e < end;
      const uint32_t d = (key[it] >> shift) & msk;
      uint64_t peers = __ballot(valid);
#pragma unroll
      for (int b = 0; b < 8; ++b) {
        if (b >= bits) break;
        const uint64_t bal = __ballot((d >> b) & 1u);
        peers &= ((d >> b) & 1u) ? bal : ~bal;
      }
      const uint32_t base = valid ? s_wcnt[w][d] : 0u;
      rnk[it] = base + (uint32_t)__popcll(peers & lt_mask);
      // the highest lane of each digit group advances the wave's running count
      if (valid && (peers >> lane) == 1ull) s_wcnt[w][d] = base + (uint32_t)__popcll(peers);
    }
    __syncthreads();
    // per digit: offsets of the four waves and the chunk total
    {
      uint32_t t = 0;
      if (tid < radix) {
        const uint32_t c0 = s_wcnt[0][tid], c1 = s_wcnt[1][tid], c2 = s_wcnt[2][tid], c3 = s_wcnt[3][tid];
        s_wcnt[0][tid] = 0;
        s_wcnt[1][tid] = c0;
        s_wcnt[2][tid] = c0 + c1;
        s_wcnt[3][tid] = c0 + c1 + c2;
        t = c0 + c1 + c2 + c3;
        s_tot[tid] = t;
      }
      uint32_t all;
      const uint32_t ex = block_excl_scan(t, s4, all);
      if (tid < radix) s_choff[tid] = ex;
    }
    __syncthreads();
#pragma unroll
    for (int it = 0; it < RS_ITEMS; ++it) {
      const uint32_t e = wbase + it * 64 + lane;
      if (e < end) {
        const uint32_t d = (key[it] >> shift) & msk;
        const uint32_t p = s_choff[d] + s_wcnt[w][d] + rnk[it];
        s_key[p] = key[it];
        s_val[p] = val[it];
      }
    }
    __syncthreads();
    for (uint32_t p = tid; p < clen; p += NT) {
      const uint32_t k = s_key[p];
      const uint32_t d = (k >> shift) & msk;
      const uint32_t o = s_base[d] + (p - s_choff[d]);
      kout[o] = k;
      vout[o] = s_val[p];
    }
    __syncthreads();
    if (tid < radix) s_base[tid] += s_tot[tid];
    __syncthreads();
  }
}

// ------------------------------------------------------------------ slabs of the depth order
// Slab `which` (1: [0, S1), 2: [S1, M)) of the depth order: its first sorted entry lo,
// entry count m and first pair position base.  The first slab is the nearest
// max(M/16, 16384) entries (all of them for complete lists); the second is listed only
// if some tile is still alive.  The kernel that computes it first (gather_counts or
// recount) also stores it in the counters for the kernels after it.
__device__ __forceinline__ void slab_params(uint32_t* counters, int which, int sliced, uint32_t& lo, uint32_t& m) {
  const uint32_t M = counters[C_ENTRIES];
  const uint32_t s1 = which == 1 ? (sliced ? min(M, max(M >> 4, 16384u)) : M) : counters[C_SLAB1];
  lo = which == 1 ? 0u : s1;
  m = which == 1 ? s1 : (counters[C_ALIVE] ? M - s1 : 0u);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    if (which == 1) counters[C_SLAB1] = s1;
    counters[C_SLAB_LO] = lo;
    counters[C_SLAB_N] = m;
    counters[C_SLAB_BASE] = which == 1 ? 0u : counters[C_PAIRS1];
  }
}

// Sum of x over groups of `group` consecutive threads (64 or NT), valid in every thread
// of the group; every thread of the block calls it.
__device__ __forceinline__ uint32_t group_sum(uint32_t x, int group, uint32_t* s4) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
  if (group == 64) return x;
  if (lane_id() == 0) s4[threadIdx.x >> 6] = x;
  __syncthreads();
  x = s4[0] + s4[1] + s4[2] + s4[3];
  __syncthreads();
  return x;
}

// The slab's entries are taken in chunks of `epb` (the emission's entries per block):
// chunk q = slab entries [q*epb, (q+1)*epb), its pair count -> blk[q], from which the
// emission takes each chunk's pair offset and the slab's pair count.
// Pairs each slab entry emits: its count from the count pass (first slab) ...
// Both also copy the slab entries' rectangles into depth order (rsort) for the emission.
__global__ void __launch_bounds__(NT) gather_counts_kernel(const uint32_t* __restrict__ order,
                                                           const uint32_t* __restrict__ cnt,
                                                           const uint2* __restrict__ rect, uint32_t* counters,
                                                           int sliced, int epb, uint32_t* __restrict__ out,
                                                           uint2* __restrict__ rsort, uint32_t* __restrict__ blk) {
  __shared__ uint32_t s4[4];
  uint32_t lo, m;
  slab_params(counters, 1, sliced, lo, m);
  const uint32_t nq = (m + epb - 1) / epb, per_iter = NT / epb;
  const uint32_t g = threadIdx.x / epb, t = threadIdx.x % epb;
  for (uint32_t q0 = blockIdx.x * per_iter; q0 < nq; q0 += gridDim.x * per_iter) {
    const uint32_t q = q0 + g, j = q * epb + t;
    uint32_t c = 0;
    if (q < nq && j < m) {
      const uint32_t e = order[lo + j];
      c = cnt[e];
      out[j] = c;
      rsort[j] = rect[e];
    }
    c = group_sum(c, epb, s4);
    if (t == 0 && q < nq) blk[q] = c;
  }
}

// ... or recounted from the rectangle against the corner table `tab` (second slab: the
// tiles still alive; first slab of lists built from a stored depth order of the
// unchanged entries, whose count pass ran in another order).
__global__ void __launch_bounds__(NT) recount_kernel(const uint32_t* __restrict__ order, const uint2* __restrict__ rect,
                                                     const uint32_t* __restrict__ tab, uint32_t* counters, uint32_t n,
                                                     int TX, int TY, int which, int sliced, int epb,
                                                     uint32_t* __restrict__ out, uint2* __restrict__ rsort,
                                                     uint32_t* __restrict__ blk) {
  __shared__ uint32_t s4[4];
  uint32_t lo, m;
  slab_params(counters, which, sliced, lo, m);
  const uint32_t nq = (m + epb - 1) / epb, per_iter = NT / epb;
  const uint32_t g = threadIdx.x / epb, t = threadIdx.x % epb;
  for (uint32_t q0 = blockIdx.x * per_iter; q0 < nq; q0 += gridDim.x * per_iter) {
    const uint32_t q = q0 + g, j = q * epb + t;
    uint32_t c = 0;
    if (q < nq && j < m) {
      const uint32_t e = order[lo + j];
      const uint2 r = rect[e];
      rsort[j] = r;
      const uint32_t x0 = r.x & 0xffffu, x1 = r.x >> 16, y0 = r.y & 0xffffu, y1 = r.y >> 16;
      c = tab_rect(tab, (e / n) * (uint32_t)(TY + 1), (uint32_t)(TX + 1), x0, x1, y0, y1);
      out[j] = c;
    }
    c = group_sum(c, epb, s4);
    if (t == 0 && q < nq) blk[q] = c;
  }
}

// ------------------------------------------------------------------ 5. emission
// Words (corner table + tile list) up to which the masked emission stages both in LDS
// (with the static arrays, within 64 KB).
constexpr int EMIT_TAB_WORDS = 10240;
// Pairs one thread emits per round: a contiguous run, so the owner search and the
// row search are paid once per run.
constexpr int EMIT_RUN = 8;
constexpr int EMIT_ROUND = NT * EMIT_RUN;
// Entries per block: the first slab holds the nearest (largest) footprints, so its
// entries are spread over more blocks.
constexpr int EMIT_EPB_NEAR = 64;
constexpr int EMIT_EPB = NT;

// LDS slot of run position p (runs padded to EMIT_RUN + 1 words against bank conflicts).
__device__ __forceinline__ uint32_t run_slot(uint32_t p) { return (p / EMIT_RUN) * (EMIT_RUN + 1) + p % EMIT_RUN; }

// Emission of one slab: entry j of the slab (in depth order) writes (global tile,
// entry) for its counts[j] tiles from position offs[j] on, offs being the exclusive
// prefix sum of the counts: a chunk's offset is the sum of the earlier chunks' counts
// qsum[], an entry's the chunk's plus a block scan of the chunk's counts.  The sum of
// all of qsum is the slab's pair count; block 0 stores it and runs the capacity check,
// and no block writes a pair of a slab that does not fit.  Without MASKED every
// tile of the rectangle is a pair (row-major); with MASKED only the tiles set in the
// mask: those of row ty are the run [rank(ty, x0), rank(ty, x1)) of the mask's sorted
// tile list `list`, ranks taken from the corner table `tab` plus the view's first list
// position `vfirst[v]`.  A block takes `epb` consecutive entries; its threads take
// contiguous runs of EMIT_RUN positions of the block's pair range, find the run's
// owner entry (the last one whose offset is <= the position: an entry without pairs
// shares its offset with the next one) and the pair's row (binary search over the
// rectangle's rows on the table's prefix counts), and step through the row's tiles,
// searching the row again whenever a row or an entry is exhausted.  Runs are staged in
// LDS and written out with coalesced stores.
// LDS_TAB: the corner table and the first V*T words of the list are copied into
// dynamic LDS.
template <bool MASKED, bool LDS_TAB>
__global__ void __launch_bounds__(NT) emit_kernel(const uint32_t* __restrict__ order, const uint32_t* __restrict__ counts,
                                                  const uint32_t* __restrict__ qsum, const uint2* __restrict__ rsort,
                                                  const uint32_t* __restrict__ tab,
                                                  const uint32_t* __restrict__ vfirst, const uint32_t* __restrict__ list,
                                                  uint32_t* __restrict__ counters, int64_t n, int TX, int TY,
                                                  int views, int epb, int which, uint64_t capacity,
                                                  uint32_t* __restrict__ pk, uint32_t* __restrict__ pv) {
  extern __shared__ uint32_t s_tab[];  // LDS_TAB: the corner table, then the tile list
  __shared__ uint32_t s_off[NT + 1];
  __shared__ uint32_t s_e[NT];
  __shared__ uint2 s_r[NT];
  __shared__ uint32_t s_vb[NT];  // MASKED: first table row of the view; else first global tile
  __shared__ uint32_t s_vf[NT];  // MASKED: the view's first list position
  __shared__ uint32_t s_k[NT * (EMIT_RUN + 1)];
  __shared__ uint32_t s_v[NT * (EMIT_RUN + 1)];
  __shared__ uint32_t s4[4];
  __shared__ uint32_t s_c[3];
  // Block 0 writes counters below (the capacity check) that other blocks read here, so
  // each block reads them once, in one thread: whichever values it sees, an overflowing
  // slab writes no pair and the others see their own values.
  if (threadIdx.x == 0) {
    s_c[0] = counters[C_OVERFLOW];  // set when the first slab overflowed
    s_c[1] = counters[C_SLAB_N];
    s_c[2] = which == 1 ? 0u : counters[C_PAIRS1];
  }
  __syncthreads();
  if (s_c[0]) return;
  const uint32_t m = s_c[1];
  // the slab's pair count from the chunk sums; block 0 records it and runs the capacity
  // check, and every block leaves on overflow before writing anything
  const uint32_t nq = (m + epb - 1) / epb;
  const uint32_t slab_pairs = block_sum_range(qsum, 0, nq, s4);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    counters[C_SLAB_PAIRS] = slab_pairs;
    capacity_check(counters, capacity, which);
  }
  if ((uint64_t)s_c[2] + slab_pairs > capacity) return;
  if ((uint64_t)blockIdx.x * epb >= m) return;
  const uint32_t TXp = (uint32_t)TX + 1, TYp = (uint32_t)TY + 1;
  const uint32_t tab_words = (uint32_t)views * TYp * TXp;
  if (MASKED && LDS_TAB) {
    // the table and the list's valid part (the rendered tiles; the second slab's list
    // of alive tiles is shorter still); eight loads in flight per thread
    const uint32_t words = tab_words + min((uint32_t)views * (uint32_t)(TX * TY), counters[C_TILES]);
    for (uint32_t w0 = threadIdx.x; w0 < words; w0 += 8 * NT) {
      uint32_t t[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const uint32_t w = w0 + u * NT;
        t[u] = w < tab_words ? tab[w] : (w < words ? list[w - tab_words] : 0u);
      }
#pragma unroll
      for (int u = 0; u < 8; ++u)
        if (w0 + u * NT < words) s_tab[w0 + u * NT] = t[u];
    }
  }
  const uint32_t* tb = LDS_TAB ? s_tab : tab;
  const uint32_t* tl = LDS_TAB ? s_tab + tab_words : list;
  order += counters[C_SLAB_LO];
  const uint32_t pbase = counters[C_SLAB_BASE];
  pk += pbase;
  pv += pbase;
  // tiles of row ty of the current rectangle: global tiles a + [0, c) (full) or list
  // entries a + [0, c) (masked)
  auto row_span = [&](uint32_t vb, uint32_t vf, uint32_t ty, uint32_t x0, uint32_t x1, uint32_t& a, uint32_t& c) {
    if (MASKED) {
      a = vf + tab_rank(tb, vb, TXp, ty, x0);
      c = vf + tab_rank(tb, vb, TXp, ty, x1) - a;
    } else {
      a = vb + ty * TX + x0;
      c = x1 - x0;
    }
  };
  uint32_t qdone = 0, qb = 0;  // qb: pairs of the chunks [0, qdone)
  for (uint32_t j0 = blockIdx.x * epb; j0 < m; j0 += gridDim.x * epb) {
    const uint32_t cnt = min((uint32_t)epb, m - j0);
    __syncthreads();
    // the entries' pair offsets: the chunk's offset (the sum of the earlier chunks'
    // counts) plus an exclusive scan of its own counts
    qb += block_sum_range(qsum, qdone, j0 / epb, s4);
    qdone = j0 / epb;
    const uint32_t ce = threadIdx.x < cnt ? counts[j0 + threadIdx.x] : 0u;
    uint32_t ctot;
    const uint32_t ex = block_excl_scan(ce, s4, ctot);
    if (threadIdx.x < cnt) {
      const uint32_t e = order[j0 + threadIdx.x];
      const uint32_t v = (uint32_t)(e / n);
      s_off[threadIdx.x] = qb + ex;
      s_e[threadIdx.x] = e;
      s_r[threadIdx.x] = rsort[j0 + threadIdx.x];
      s_vb[threadIdx.x] = MASKED ? v * TYp : v * (uint32_t)(TX * TY);
      s_vf[threadIdx.x] = MASKED ? vfirst[v] : 0u;
    }
    if (threadIdx.x == 0) s_off[cnt] = qb + ctot;
    __syncthreads();
    const uint32_t base = s_off[0], end = s_off[cnt];
    for (uint32_t rb = base; rb < end; rb += EMIT_ROUND) {
      const uint32_t q0 = rb + threadIdx.x * EMIT_RUN;
      const uint32_t q1 = min(q0 + EMIT_RUN, end);
      if (q0 < q1) {
        uint32_t lo = 0, hi = cnt;
        while (hi - lo > 1) {
          const uint32_t mid = (lo + hi) >> 1;
          if (s_off[mid] <= q0) lo = mid; else hi = mid;
        }
        // state of the current pair: entry lo, its rectangle, the pair's index re among
        // the entry's pairs, its row ty, the row's tiles a + [0, c) and the index r in it
        uint32_t x0 = 0, x1 = 0, y0 = 0, y1 = 0, vb = 0, vf = 0, e = 0, ne = 0;
        uint32_t re = q0 - s_off[lo], ty = 0, a = 0, c = 0, r = 0;
        auto load_entry = [&]() {
          const uint2 rc = s_r[lo];
          x0 = rc.x & 0xffffu;
          x1 = rc.x >> 16;
          y0 = rc.y & 0xffffu;
          y1 = rc.y >> 16;
          vb = s_vb[lo];
          vf = s_vf[lo];
          e = s_e[lo];
          ne = s_off[lo + 1] - s_off[lo];
        };
        // the row holding pair re of the entry
        auto locate = [&]() {
          if (MASKED) {
            // largest row t in [y0, y1) with (set tiles of rows [y0, t)) <= re
            uint32_t ylo = y0, yhi = y1;
            while (yhi - ylo > 1) {
              const uint32_t mid = (ylo + yhi) >> 1;
              if (tab_rect(tb, vb, TXp, x0, x1, y0, mid) <= re) ylo = mid; else yhi = mid;
            }
            ty = ylo;
            r = re - tab_rect(tb, vb, TXp, x0, x1, y0, ty);
          } else {
            const uint32_t w = x1 - x0;
            ty = y0 + re / w;
            r = re % w;
          }
          row_span(vb, vf, ty, x0, x1, a, c);
        };
        load_entry();
        locate();
        for (uint32_t q = q0; q < q1; ++q) {
          const uint32_t slot = run_slot(q - rb);
          s_k[slot] = MASKED ? tl[a + r] : a + r;
          s_v[slot] = e;
          ++re;
          if (++r < c || q + 1 == q1) continue;
          if (re == ne) {
            // the entry is done: the owner of position q + 1 (entries without pairs
            // share their offset with it)
            ++lo;
            while (lo + 1 < cnt && s_off[lo + 1] <= q + 1) ++lo;
            if (lo >= cnt) break;  // cannot happen with consistent counts
            load_entry();
            re = 0;
          }
          locate();
        }
      }
      __syncthreads();
      const uint32_t len = min((uint32_t)EMIT_ROUND, end - rb);
      for (uint32_t p = threadIdx.x; p < len; p += NT) {
        const uint32_t slot = run_slot(p);
        pk[rb + p] = s_k[slot];
        pv[rb + p] = s_v[slot];
      }
      __syncthreads();
    }
  }
}

// ------------------------------------------------------------------ 5-7 by counting
// Counting placement of a masked slab's pairs, when its count matrix fits (see
// list_slab): the pairs are written straight into tile order, with no tile sort and no
// range scan.  The slab's entries are taken in chunks of CM_EPB (depth order).  A tile's
// "slot" is its position in the slab's tile list (the rank of the tile among the view's
// set tiles, from the corner table).  For a chunk, each slot's mask has bit j set when
// the chunk's entry j covers the slot, so the chunk's entries of a tile, in depth
// order, are the mask's set bits in order.
//   count : row q of the count matrix, cm[q * S + s] = popcount(mask of slot s, chunk q)
//   scan  : each column's exclusive prefix over the chunks, and its total (the tile's
//           pair count)
//   emit  : the tiles' first positions (an exclusive scan of the totals), then pair k of
//           slot s in chunk q goes to first(s) + cm[q][s] + k, its entry the mask's k-th
//           set bit; block 0 also writes the tiles' ranges and runs the capacity check.
constexpr int CM_EPB = 64;                     // one bit per entry of a chunk
constexpr int64_t CM_MAX_WORDS = 64ll << 20;   // count matrix budget (256 MB)
constexpr int CM_MAX_SLOTS = 3840;             // the emission keeps 16 B per slot in LDS
// With at most CM_SMALL_SLOTS slots (and a corner table of at most CM_TAB_WORDS) the
// kernels also keep the corner table, and the emission the chunk's count-matrix row,
// in LDS.
constexpr int CM_SMALL_SLOTS = 1024;
constexpr int CM_TAB_WORDS = 8192;
constexpr int64_t CM_MASK_WORDS = 8ll << 20;  // kept tile masks (64-bit words): 64 MB
constexpr int CM_PAIR_ROUND = 2048;  // a chunk's pairs placed at once by the small-layout emission (16-bit words in LDS)
__host__ __device__ inline size_t cm_count_lds(int64_t gt, int64_t tab_words) {
  const size_t big = (size_t)gt * 8, small = (size_t)CM_SMALL_SLOTS * 8 + (size_t)tab_words * 4;
  return tab_words <= CM_TAB_WORDS && small > big ? small : big;
}
__host__ __device__ inline size_t cm_emit_lds(int64_t gt, int64_t tab_words) {
  const size_t big = (size_t)gt * 16 + 4, small = (size_t)CM_SMALL_SLOTS * 24 + 4 + (size_t)tab_words * 4;
  return tab_words <= CM_TAB_WORDS && small > big ? small : big;
}

// Slots [a, a + c) of row ty of the rectangle [x0, x1): list positions of the row's set
// tiles (vb: the view's first table row; vf: the view's first list position).
__device__ __forceinline__ void cm_row_slots(const uint32_t* tb, uint32_t vb, uint32_t vf, uint32_t TXp, uint32_t ty,
                                             uint32_t x0, uint32_t x1, uint32_t& a, uint32_t& c) {
  a = vf + tab_rank(tb, vb, TXp, ty, x0);
  c = vf + tab_rank(tb, vb, TXp, ty, x1) - a;
}

// Sets bit t of the mask of every slot entry t (t < cnt) of the chunk covers: the block's
// threads take (entry, row) pairs, four rows of an entry at a time.
__device__ __forceinline__ void cm_build_masks(unsigned long long* s_mask, const uint2* s_r, const uint32_t* s_vb,
                                               const uint32_t* s_vf, uint32_t cnt, const uint32_t* tb, uint32_t TXp) {
  const uint32_t t = threadIdx.x % CM_EPB, g = threadIdx.x / CM_EPB;
  if (t >= cnt) return;
  const uint2 r = s_r[t];
  const uint32_t x0 = r.x & 0xffffu, x1 = r.x >> 16, y0 = r.y & 0xffffu, y1 = r.y >> 16;
  for (uint32_t ty = y0 + g; ty < y1; ty += NT / CM_EPB) {
    uint32_t a, c;
    cm_row_slots(tb, s_vb[t], s_vf[t], TXp, ty, x0, x1, a, c);
    for (uint32_t i = 0; i < c; ++i) atomicOr(&s_mask[a + i], 1ull << t);
  }
}

// The chunk's entries: index, rectangle and view bases (s_e, s_r, s_vb, s_vf).
__device__ __forceinline__ void cm_load_chunk(const uint32_t* __restrict__ order, const uint2* __restrict__ rect,
                                              const uint32_t* __restrict__ vfirst, uint32_t j0, uint32_t cnt,
                                              uint32_t n, uint32_t TYp, uint32_t* s_e, uint2* s_r, uint32_t* s_vb,
                                              uint32_t* s_vf) {
  if (threadIdx.x < cnt) {
    const uint32_t e = order[j0 + threadIdx.x];
    const uint32_t v = e / n;
    const uint2 r = rect[e];
    s_e[threadIdx.x] = e;
    s_r[threadIdx.x] = r;
    s_vb[threadIdx.x] = v * TYp;
    s_vf[threadIdx.x] = vfirst[v];
  }
}

// (Copies the corner table into LDS.)
__device__ __forceinline__ void cm_stage_table(uint32_t* s_tab, const uint32_t* __restrict__ tab, uint32_t words) {
  for (uint32_t w0 = threadIdx.x; w0 < words; w0 += 4 * NT) {
    uint32_t t[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) t[u] = w0 + u * NT < words ? tab[w0 + u * NT] : 0u;
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (w0 + u * NT < words) s_tab[w0 + u * NT] = t[u];
  }
}

template <bool STAGED>
__device__ __forceinline__ void cm_count_chunks(unsigned long long* s_mask, const uint32_t* tb,
                                                const uint32_t* __restrict__ order, const uint2* __restrict__ rect,
                                                const uint32_t* __restrict__ vfirst, uint32_t m, uint32_t S,
                                                uint32_t n, uint32_t TXp, uint32_t TYp, uint32_t* s_e, uint2* s_r,
                                                uint32_t* s_vb, uint32_t* s_vf, uint32_t* __restrict__ cm,
                                                unsigned long long* __restrict__ cmask) {
  const uint32_t nq = (m + CM_EPB - 1) / CM_EPB;
  for (uint32_t q = blockIdx.x; q < nq; q += gridDim.x) {
    const uint32_t j0 = q * CM_EPB, cnt = min((uint32_t)CM_EPB, m - j0);
    __syncthreads();
    for (uint32_t s = threadIdx.x; s < S; s += NT) s_mask[s] = 0ull;
    cm_load_chunk(order, rect, vfirst, j0, cnt, n, TYp, s_e, s_r, s_vb, s_vf);
    __syncthreads();
    cm_build_masks(s_mask, s_r, s_vb, s_vf, cnt, tb, TXp);
    __syncthreads();
    for (uint32_t s = threadIdx.x; s < S; s += NT) {
      const unsigned long long msk = s_mask[s];
      cm[(size_t)q * S + s] = (uint32_t)__popcll(msk);
      if (cmask) cmask[(size_t)q * S + s] = msk;
    }
  }
}

__global__ void __launch_bounds__(NT) cm_count_kernel(const uint32_t* __restrict__ order,
                                                      const uint2* __restrict__ rect,
                                                      const uint32_t* __restrict__ tab,
                                                      const uint32_t* __restrict__ vfirst, uint32_t* counters,
                                                      int which, int sliced, uint32_t n, int TX, int TY,
                                                      uint32_t tab_words, uint32_t* __restrict__ cm,
                                                      unsigned long long* __restrict__ cmask, uint64_t cmask_words) {
  extern __shared__ unsigned long long s_mask[];  // [S], then (small) the corner table
  __shared__ uint32_t s_e[CM_EPB], s_vb[CM_EPB], s_vf[CM_EPB];
  __shared__ uint2 s_r[CM_EPB];
  uint32_t lo, m;
  slab_params(counters, which, sliced, lo, m);
  const uint32_t S = counters[which == 1 ? C_TILES : C_ALIVE];
  if ((uint64_t)((m + CM_EPB - 1) / CM_EPB) * S > cmask_words) cmask = nullptr;
  const uint32_t TXp = (uint32_t)TX + 1, TYp = (uint32_t)TY + 1;
  order += lo;
  if (m == 0) return;
  if (S <= CM_SMALL_SLOTS && tab_words <= CM_TAB_WORDS) {
    uint32_t* s_tab = reinterpret_cast<uint32_t*>(s_mask + CM_SMALL_SLOTS);
    cm_stage_table(s_tab, tab, tab_words);
    cm_count_chunks<true>(s_mask, s_tab, order, rect, vfirst, m, S, n, TXp, TYp, s_e, s_r, s_vb, s_vf, cm, cmask);
  } else {
    cm_count_chunks<false>(s_mask, tab, order, rect, vfirst, m, S, n, TXp, TYp, s_e, s_r, s_vb, s_vf, cm, cmask);
  }
}

// Column scan of the count matrix (nq rows of S): each column's exclusive prefix over the
// rows in place, and its total -> tot[s].  A block takes CS_COLS columns and splits the
// rows into CS_SEGS contiguous segments, one thread per (segment, column) with the
// columns fastest (coalesced row pieces): each thread sums its segment, the segment
// sums are scanned per column in LDS (one wave pair per column), and each thread
// rewrites its segment from its base.
constexpr int CS_COLS = 8, CS_SEGS = 128, CS_NT = CS_COLS * CS_SEGS, CS_BATCH = 8;
__global__ void __launch_bounds__(CS_NT) cm_scan_kernel(uint32_t* __restrict__ cm, const uint32_t* counters,
                                                        int which, uint32_t* __restrict__ tot) {
  __shared__ uint32_t s_seg[CS_SEGS][CS_COLS];
  __shared__ uint32_t s_wave[CS_NT / 64];
  const uint32_t m = counters[C_SLAB_N], S = counters[which == 1 ? C_TILES : C_ALIVE];
  if (blockIdx.x * CS_COLS >= S) return;
  const uint32_t nq = (m + CM_EPB - 1) / CM_EPB;
  const uint32_t c = threadIdx.x % CS_COLS, seg = threadIdx.x / CS_COLS;
  const uint32_t col = blockIdx.x * CS_COLS + c;
  const bool ok = col < S;
  const uint32_t per = (nq + CS_SEGS - 1) / CS_SEGS;
  const uint32_t r0 = min(seg * per, nq), r1 = min(r0 + per, nq);
  uint32_t sum = 0;
  for (uint32_t r = r0; r < r1; r += CS_BATCH) {
    uint32_t x[CS_BATCH];
#pragma unroll
    for (int u = 0; u < CS_BATCH; ++u) x[u] = (ok && r + u < r1) ? cm[(size_t)(r + u) * S + col] : 0u;
#pragma unroll
    for (int u = 0; u < CS_BATCH; ++u) sum += x[u];
  }
  s_seg[seg][c] = sum;
  __syncthreads();
  {
    // column-major pass: thread t scans segment t % CS_SEGS of column t / CS_SEGS
    const uint32_t cc = threadIdx.x / CS_SEGS, sg = threadIdx.x % CS_SEGS;
    const uint32_t v = s_seg[sg][cc];
    const uint32_t inc = wave_incl_scan(v);
    const uint32_t w = threadIdx.x >> 6;
    if (lane_id() == 63) s_wave[w] = inc;
    __syncthreads();
    // the waves before this one within the column (CS_SEGS / 64 waves per column)
    uint32_t carry = 0;
    for (uint32_t k = cc * (CS_SEGS / 64); k < w; ++k) carry += s_wave[k];
    s_seg[sg][cc] = carry + inc - v;  // exclusive base of the segment
    if (sg == CS_SEGS - 1 && blockIdx.x * CS_COLS + cc < S) tot[blockIdx.x * CS_COLS + cc] = carry + inc;
  }
  __syncthreads();
  if (!ok) return;
  uint32_t run = s_seg[seg][c];
  for (uint32_t r = r0; r < r1; r += CS_BATCH) {
    uint32_t x[CS_BATCH];
#pragma unroll
    for (int u = 0; u < CS_BATCH; ++u) x[u] = r + u < r1 ? cm[(size_t)(r + u) * S + col] : 0u;
#pragma unroll
    for (int u = 0; u < CS_BATCH; ++u)
      if (r + u < r1) {
        cm[(size_t)(r + u) * S + col] = run;
        run += x[u];
      }
  }
}

// The k-th (0-based) set bit of m (m has more than k set bits).
__device__ __forceinline__ uint32_t kth_set_bit(unsigned long long m, uint32_t k) {
  uint32_t pos = 0;
#pragma unroll
  for (int w = 32; w > 0; w >>= 1) {
    const uint32_t c = (uint32_t)__popcll(m & ((1ull << w) - 1ull));
    if (k >= c) {
      k -= c;
      m >>= w;
      pos += (uint32_t)w;
    }
  }
  return pos;
}

// Emission by counting.  Dynamic LDS: the slots' masks (8 B each), the slots' first
// positions (4 B) and the chunk's exclusive pair scan (4 B, S + 1 words); with the
// small layout (S <= CM_SMALL_SLOTS, arrays of CM_SMALL_SLOTS) also the chunk's
// count-matrix row, the slots' tiles and the corner table.
template <bool SMALL>
__device__ __forceinline__ void cm_emit_chunks(unsigned long long* s_mask, uint32_t* s_first, uint32_t* s_scan,
                                               uint32_t* s_row, const uint32_t* s_list, const uint32_t* tb,
                                               const uint32_t* __restrict__ order, const uint2* __restrict__ rect,
                                               const uint32_t* __restrict__ vfirst, const uint32_t* __restrict__ list,
                                               const uint32_t* __restrict__ cm, uint32_t m, uint32_t S, uint32_t n,
                                               uint32_t TXp, uint32_t TYp, uint32_t* s_e, uint2* s_r,
                                               uint32_t* s_vb, uint32_t* s_vf, uint32_t* s4, uint16_t* s_pair,
                                               uint32_t* __restrict__ pk, uint32_t* __restrict__ pv,
                                               const unsigned long long* __restrict__ cmask) {
  const uint32_t nq = (m + CM_EPB - 1) / CM_EPB;
  for (uint32_t q = blockIdx.x; q < nq; q += gridDim.x) {
    const uint32_t j0 = q * CM_EPB, cnt = min((uint32_t)CM_EPB, m - j0);
    const uint32_t* row = cm + (size_t)q * S;
    __syncthreads();
    // the chunk's tile masks: kept by the count pass, or built again from the rectangles
    for (uint32_t s = threadIdx.x; s < S; s += NT) {
      s_mask[s] = cmask ? cmask[(size_t)q * S + s] : 0ull;
      if (SMALL) s_row[s] = row[s];
    }
    if (cmask) {
      if (threadIdx.x < cnt) s_e[threadIdx.x] = order[j0 + threadIdx.x];
      __syncthreads();
    } else {
      cm_load_chunk(order, rect, vfirst, j0, cnt, n, TYp, s_e, s_r, s_vb, s_vf);
      __syncthreads();
      cm_build_masks(s_mask, s_r, s_vb, s_vf, cnt, tb, TXp);
      __syncthreads();
    }
    // the chunk's pairs per slot, scanned: pair i of the chunk belongs to the slot s with
    // s_scan[s] <= i < s_scan[s + 1]
    uint32_t chunk_pairs;
    {
      const uint32_t per = (S + NT - 1) / NT, s0 = min(threadIdx.x * per, S), s1 = min(s0 + per, S);
      uint32_t sum = 0;
      for (uint32_t s = s0; s < s1; ++s) sum += (uint32_t)__popcll(s_mask[s]);
      uint32_t run = block_excl_scan(sum, s4, chunk_pairs);
      for (uint32_t s = s0; s < s1; ++s) {
        s_scan[s] = run;
        run += (uint32_t)__popcll(s_mask[s]);
      }
      if (threadIdx.x == 0) s_scan[S] = chunk_pairs;
    }
    if (SMALL) {
      // pair i of the chunk, in rounds of CM_PAIR_ROUND: first each slot's thread writes
      // (slot, entry) of the slot's pairs in the round (its mask's set bits in order)
      // into s_pair, then every thread stores pairs i, i + NT, ... (consecutive pairs
      // of a slot go to consecutive positions)
      for (uint32_t r0 = 0; r0 < chunk_pairs; r0 += CM_PAIR_ROUND) {
        const uint32_t r1 = min(chunk_pairs, r0 + (uint32_t)CM_PAIR_ROUND);
        __syncthreads();
        for (uint32_t s = threadIdx.x; s < S; s += NT) {
          const uint32_t i0 = max(s_scan[s], r0), i1 = min(s_scan[s + 1], r1);
          if (i0 >= i1) continue;
          unsigned long long msk = s_mask[s];
          // drop the slot's pairs before the round
          const uint32_t skip = i0 - s_scan[s];
          if (skip) msk &= ~0ull << kth_set_bit(msk, skip);
          for (uint32_t i = i0; i < i1; ++i) {
            const uint32_t j = (uint32_t)__ffsll(msk) - 1u;
            msk &= msk - 1ull;
            s_pair[i - r0] = (uint16_t)((s << 6) | j);
          }
        }
        __syncthreads();
        for (uint32_t i = r0 + threadIdx.x; i < r1; i += NT) {
          const uint32_t wd = s_pair[i - r0], s = wd >> 6, j = wd & 63u;
          const uint32_t pos = s_first[s] + s_row[s] + (i - s_scan[s]);
          pk[pos] = s_list[s];
          pv[pos] = s_e[j];
        }
      }
    } else {
      __syncthreads();
      for (uint32_t i = threadIdx.x; i < chunk_pairs; i += NT) {
        uint32_t lo = 0, hi = S;  // the last slot with s_scan[s] <= i
        while (hi - lo > 1) {
          const uint32_t mid = (lo + hi) >> 1;
          if (s_scan[mid] <= i) lo = mid; else hi = mid;
        }
        const uint32_t s = lo, k = i - s_scan[s];
        const uint32_t j = kth_set_bit(s_mask[s], k);
        const uint32_t pos = s_first[s] + row[s] + k;
        pk[pos] = list[s];
        pv[pos] = s_e[j];
      }
    }
  }
}

__global__ void __launch_bounds__(NT) cm_emit_kernel(const uint32_t* __restrict__ order,
                                                     const uint2* __restrict__ rect,
                                                     const uint32_t* __restrict__ tab,
                                                     const uint32_t* __restrict__ vfirst,
                                                     const uint32_t* __restrict__ list,
                                                     const uint32_t* __restrict__ cm, const uint32_t* __restrict__ tot,
                                                     uint32_t* __restrict__ counters, int which, uint32_t n, int TX,
                                                     int TY, uint32_t tab_words, uint64_t capacity,
                                                     uint32_t* __restrict__ pk, uint32_t* __restrict__ pv,
                                                     uint2* __restrict__ ranges,
                                                     const unsigned long long* __restrict__ cmask,
                                                     uint64_t cmask_words) {
  extern __shared__ unsigned long long s_mask[];
  __shared__ uint32_t s_e[CM_EPB], s_vb[CM_EPB], s_vf[CM_EPB];
  __shared__ uint2 s_r[CM_EPB];
  __shared__ uint32_t s4[4];
  __shared__ uint32_t s_c[4];
  __shared__ uint16_t s_pair[CM_PAIR_ROUND];
  if (threadIdx.x == 0) {
    s_c[0] = counters[C_OVERFLOW];  // set when the first slab overflowed
    s_c[1] = counters[C_SLAB_N];
    s_c[2] = which == 1 ? 0u : counters[C_PAIRS1];
    s_c[3] = counters[which == 1 ? C_TILES : C_ALIVE];
  }
  __syncthreads();
  if (s_c[0]) return;
  const uint32_t m = s_c[1], S = s_c[3];
  // (the count pass kept the masks under the same condition)
  if ((uint64_t)((m + CM_EPB - 1) / CM_EPB) * S > cmask_words) cmask = nullptr;
  const bool small = S <= CM_SMALL_SLOTS && tab_words <= CM_TAB_WORDS;
  const uint32_t SA = small ? (uint32_t)CM_SMALL_SLOTS : S;       // array length of the layout
  uint32_t* s_first = reinterpret_cast<uint32_t*>(s_mask + SA);  // first position of the slot's run
  uint32_t* s_scan = s_first + SA;                               // [S + 1]
  uint32_t* s_row = s_scan + SA + 1;                             // small: the chunk's count-matrix row
  uint32_t* s_list = s_row + SA;                                 // small: the slots' tiles
  uint32_t* s_tab = s_list + SA;                                 // small: the corner table
  const uint32_t base = s_c[2];
  // the tiles' first positions: an exclusive scan of the column totals (runs of
  // consecutive slots per thread), after the pairs of earlier slabs
  uint32_t slab_pairs;
  {
    const uint32_t per = (S + NT - 1) / NT, s0 = min(threadIdx.x * per, S), s1 = min(s0 + per, S);
    uint32_t sum = 0;
    for (uint32_t s = s0; s < s1; ++s) sum += tot[s];
    uint32_t run = block_excl_scan(sum, s4, slab_pairs);
    for (uint32_t s = s0; s < s1; ++s) {
      s_first[s] = base + run;
      run += tot[s];
    }
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    counters[C_SLAB_PAIRS] = slab_pairs;
    capacity_check(counters, capacity, which);
  }
  if ((uint64_t)base + slab_pairs > capacity) return;
  __syncthreads();
  if (blockIdx.x == 0 && which == 1) {
    for (uint32_t s = threadIdx.x; s < S; s += NT) {
      const uint32_t c = tot[s];
      if (c) ranges[list[s]] = make_uint2(s_first[s], s_first[s] + c);
    }
  }
  const uint32_t TXp = (uint32_t)TX + 1, TYp = (uint32_t)TY + 1;
  order += counters[C_SLAB_LO];
  if ((uint64_t)blockIdx.x * CM_EPB >= m) return;
  if (small) {
    if (!cmask) cm_stage_table(s_tab, tab, tab_words);
    for (uint32_t s2 = threadIdx.x; s2 < S; s2 += NT) s_list[s2] = list[s2];
    cm_emit_chunks<true>(s_mask, s_first, s_scan, s_row, s_list, s_tab, order, rect, vfirst, list, cm, m, S, n, TXp,
                         TYp, s_e, s_r, s_vb, s_vf, s4, s_pair, pk, pv, cmask);
  } else {
    cm_emit_chunks<false>(s_mask, s_first, s_scan, s_row, nullptr, tab, order, rect, vfirst, list, cm, m, S, n, TXp,
                          TYp, s_e, s_r, s_vb, s_vf, s4, s_pair, pk, pv, cmask);
  }
}

// ------------------------------------------------------------------ 7. ranges, tile list
// [start, end) of each tile's run among the slab's sorted pairs (absolute positions).
__global__ void __launch_bounds__(NT) ranges_kernel(const uint32_t* __restrict__ keys,
                                                    const uint32_t* __restrict__ counters, uint2* __restrict__ ranges) {
  const uint32_t P = counters[C_SLAB_PAIRS], base = counters[C_SLAB_BASE];
  for (uint32_t p = blockIdx.x * NT + threadIdx.x; p < P; p += gridDim.x * NT) {
    const uint32_t q = base + p;
    const uint32_t k = keys[q];
    if (p == 0 || keys[q - 1] != k) ranges[k].x = q;
    if (p + 1 == P || keys[q + 1] != k) ranges[k].y = q + 1;
  }
}

// Index of a tile bitmap (V views of TX x TY tiles, wpv words per view): `list` = the
// set tiles as global indices v*T + t in ascending order, vfirst[v] = the list
// position of view v's first set tile, and the corner table `tab` (see tab_rect).
// One block of MI_NT threads walks the words in chunks with a running carry (wpre[w]
// = set bits in words [0, w) is kept as scratch), then builds the table column by
// column; the total goes to *count_out when given.
constexpr int MI_NT = 1024;
constexpr int MI_ITEMS = 4;
constexpr int MI_TAB_WORDS = 12288;  // corner tables up to 48 KB are built in LDS
constexpr int MI_MASK_WORDS = 2048;  // masks up to 8 KB are kept in LDS

__global__ void __launch_bounds__(MI_NT) mask_index_kernel(const uint32_t* __restrict__ mask, int views, int wpv,
                                                           int TX, int TY, uint32_t* __restrict__ wpre,
                                                           uint32_t* __restrict__ list, uint32_t* __restrict__ vfirst,
                                                           uint32_t* __restrict__ tab, uint32_t* __restrict__ count_out,
                                                           int lds_tab, const uint32_t* __restrict__ skip_if_zero) {
  extern __shared__ uint32_t s_tab[];  // lds_tab: the corner table under construction
  // an index nobody will read (no tile is alive: the second slab is empty)
  if (skip_if_zero && *skip_if_zero == 0u) return;
  const int T = TX * TY;
  __shared__ uint32_t s_w[MI_NT / 64];
  __shared__ uint32_t s_carry;
  __shared__ uint32_t s_words[MI_MASK_WORDS];  // the mask, when it fits, for the corner table
  const uint32_t nw = (uint32_t)views * (uint32_t)wpv;
  const bool lds_mask = nw <= MI_MASK_WORDS;
  if (threadIdx.x == 0) s_carry = 0;
  __syncthreads();
  for (uint32_t base = 0; base < nw; base += MI_NT * MI_ITEMS) {
    uint32_t wd[MI_ITEMS];
    uint32_t sum = 0;
#pragma unroll
    for (int k = 0; k < MI_ITEMS; ++k) {
      const uint32_t idx = base + threadIdx.x * MI_ITEMS + k;
      wd[k] = idx < nw ? mask[idx] : 0u;
      sum += __popc(wd[k]);
    }
    const uint32_t inc = wave_incl_scan(sum);
    const int wave = threadIdx.x >> 6;
    if (lane_id() == 63) s_w[wave] = inc;
    __syncthreads();
    uint32_t off = 0, total = 0;
    for (int k = 0; k < MI_NT / 64; ++k) {
      if (k < wave) off += s_w[k];
      total += s_w[k];
    }
    uint32_t run = s_carry + off + inc - sum;
#pragma unroll
    for (int k = 0; k < MI_ITEMS; ++k) {
      const uint32_t idx = base + threadIdx.x * MI_ITEMS + k;
      if (idx < nw) {
        if (lds_mask) s_words[idx] = wd[k];
        wpre[idx] = run;
        if (idx % (uint32_t)wpv == 0u) vfirst[idx / (uint32_t)wpv] = run;  // a view's first word
        const uint32_t v = idx / (uint32_t)wpv, t0 = (idx % (uint32_t)wpv) * 32u;
        for (uint32_t bits = wd[k]; bits; bits &= bits - 1u) list[run++] = v * (uint32_t)T + t0 + (__ffs(bits) - 1u);
      }
    }
    __syncthreads();
    if (threadIdx.x == 0) s_carry += total;
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    wpre[nw] = s_carry;
    if (count_out) *count_out = s_carry;
  }
  __syncthreads();
  // corner table, built in LDS when it fits (lds_tab): each row's prefix counts summed
  // down each column
  const uint32_t TXp = (uint32_t)TX + 1, TYp = (uint32_t)TY + 1;
  const uint32_t words = (uint32_t)views * TYp * TXp;
  uint32_t* tb = lds_tab ? s_tab : tab;
  const uint32_t* mk = lds_mask ? s_words : mask;
  if (TYp <= 64) {
    // one wave per column x, a lane per table row: each lane counts the set bits of its
    // row left of x, and a wave scan sums them down the column
    const uint32_t lane = lane_id();
    for (uint32_t i = threadIdx.x >> 6; i < (uint32_t)views * TXp; i += MI_NT / 64) {
      const uint32_t v = i / TXp, x = i % TXp;
      const uint32_t c = lane >= 1 && lane < TYp ? count_bits(mk + (size_t)v * wpv, (lane - 1) * TX, (lane - 1) * TX + x)
                                                 : 0u;
      const uint32_t inc = wave_incl_scan(c);
      if (lane < TYp) tb[((size_t)v * TYp + lane) * TXp + x] = inc;
    }
  } else {
    for (uint32_t i = threadIdx.x; i < words; i += MI_NT) {
      const uint32_t x = i % TXp, row = i / TXp, v = row / TYp, ty = row % TYp;
      tb[i] = ty == 0 ? 0u : count_bits(mk + (size_t)v * wpv, (ty - 1) * TX, (ty - 1) * TX + x);
    }
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < (uint32_t)views * TXp; i += MI_NT) {
      uint32_t* col = tb + (size_t)(i / TXp) * TYp * TXp + i % TXp;
      uint32_t acc = 0;
      for (uint32_t ty = 1; ty < TYp; ++ty) {
        acc += col[(size_t)ty * TXp];
        col[(size_t)ty * TXp] = acc;
      }
    }
  }
  if (lds_tab) {
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < words; i += MI_NT) tab[i] = s_tab[i];
  }
}

// ------------------------------------------------------------------ host helpers
size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

int sort_blocks(int64_t nmax) {
  int64_t g = (nmax + RS_CHUNK - 1) / RS_CHUNK;
  if (g < 1) g = 1;
  if (g > MAX_SORT_BLOCKS) g = MAX_SORT_BLOCKS;
  return (int)g;
}

// Blocks of the count pass and of the compaction (spans of whole NT groups).
int count_blocks(int64_t nmax) {
  int64_t g = (nmax + NT - 1) / NT;
  if (g < 1) g = 1;
  if (g > MAX_SCAN_BLOCKS) g = MAX_SCAN_BLOCKS;
  return (int)g;
}

int grid_for(int64_t count, int cap = 8192) {
  int64_t g = (count + NT - 1) / NT;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (int)g;
}

// Stable LSD radix sort of (keys, vals)[off + e], e < n, on bits [0, total_bits); n and
// off read from device memory.  Passes alternate between (k0, v0) and (k1, v1); returns
// 0 when the result is in (k0, v0).
int radix_sort(uint32_t* k0, uint32_t* v0, uint32_t* k1, uint32_t* v1, const uint32_t* n_ptr, const uint32_t* off_ptr,
               int64_t nmax, int total_bits, uint32_t* hist, uint32_t* tot, hipStream_t s) {
  if (total_bits <= 0) return 0;
  const int passes = (total_bits + 7) / 8;
  const int per = (total_bits + passes - 1) / passes;
  const int G = sort_blocks(nmax);
  int shift = 0, cur = 0;
  for (int p = 0; p < passes; ++p) {
    const int bits = min(per, total_bits - shift);
    uint32_t* ki = cur ? k1 : k0;
    uint32_t* vi = cur ? v1 : v0;
    uint32_t* ko = cur ? k0 : k1;
    uint32_t* vo = cur ? v0 : v1;
    // few blocks: the downsweep sums the block counts itself (one launch fewer per pass)
    const int raw = G <= RS_RAW_BLOCKS ? 1 : 0;
    hipLaunchKernelGGL(rs_upsweep_kernel, dim3(G), dim3(NT), 0, s, ki, n_ptr, off_ptr, shift, bits, hist, G, raw);
    if (!raw) hipLaunchKernelGGL(rs_scan_kernel, dim3(1 << bits), dim3(NT), 0, s, hist, n_ptr, G, tot);
    if (raw)
      hipLaunchKernelGGL(rs_downsweep_kernel<true>, dim3(G), dim3(NT), 0, s, ki, vi, ko, vo, n_ptr, off_ptr, shift, bits,
                         hist, tot, G);
    else
      hipLaunchKernelGGL(rs_downsweep_kernel<false>, dim3(G), dim3(NT), 0, s, ki, vi, ko, vo, n_ptr, off_ptr, shift, bits,
                         hist, tot, G);
    shift += bits;
    cur ^= 1;
  }
  return cur;
}

int passes_for(int bits) { return bits <= 0 ? 0 : (bits + 7) / 8; }

struct WsPtrs {
  uint32_t *cnt, *tmp, *keyA, *valA, *keyB, *valB, *blk, *hist, *dtot, *pairK, *pairV, *wpre, *tlist, *vfirst, *tab;
  uint32_t *cm, *ctot;
  unsigned long long* cmask;
  uint2* rsort;
};

WsPtrs carve(const BinPlan& p, char* ws) {
  WsPtrs w;
  w.cnt = reinterpret_cast<uint32_t*>(ws + p.off_cnt);
  w.tmp = reinterpret_cast<uint32_t*>(ws + p.off_flag);
  w.keyA = reinterpret_cast<uint32_t*>(ws + p.off_keyA);
  w.valA = reinterpret_cast<uint32_t*>(ws + p.off_valA);
  w.keyB = reinterpret_cast<uint32_t*>(ws + p.off_keyB);
  w.valB = reinterpret_cast<uint32_t*>(ws + p.off_valB);
  w.blk = reinterpret_cast<uint32_t*>(ws + p.off_scanBlk);
  w.hist = reinterpret_cast<uint32_t*>(ws + p.off_hist);
  w.dtot = reinterpret_cast<uint32_t*>(ws + p.off_digit);
  w.pairK = reinterpret_cast<uint32_t*>(ws + p.off_pairK);
  w.pairV = reinterpret_cast<uint32_t*>(ws + p.off_pairV);
  w.wpre = reinterpret_cast<uint32_t*>(ws + p.off_tflag);
  w.tlist = w.wpre + ((int64_t)p.views * p.T + 1);
  w.vfirst = reinterpret_cast<uint32_t*>(ws + p.off_vfirst);
  w.tab = reinterpret_cast<uint32_t*>(ws + p.off_tab);
  w.rsort = reinterpret_cast<uint2*>(ws + p.off_rsort);
  w.cm = p.cm_words > 0 ? reinterpret_cast<uint32_t*>(ws + p.off_cm) : nullptr;
  w.ctot = w.cm ? w.cm + p.cm_words : nullptr;
  w.cmask = p.cmask_words > 0 ? reinterpret_cast<unsigned long long*>(ws + p.off_cmask) : nullptr;
  return w;
}

// Index of `mask`: sorted tile list into `list`, view first positions and corner table
// into w.vfirst and w.tab.
void index_mask(const BinPlan& p, const uint32_t* mask, const WsPtrs& w, uint32_t* list, uint32_t* count_out,
                hipStream_t s, const uint32_t* skip_if_zero = nullptr) {
  const int wpv = (p.T + 31) / 32;
  const int64_t words = (int64_t)p.views * (p.TY + 1) * (p.TX + 1);
  const int lds = words <= MI_TAB_WORDS;
  hipLaunchKernelGGL(mask_index_kernel, dim3(1), dim3(MI_NT), lds ? (size_t)words * 4 : 0, s, mask, p.views, wpv, p.TX,
                     p.TY, w.wpre, list, w.vfirst, w.tab, count_out, lds, skip_if_zero);
}

// Lists one slab of the depth order (order = valA after the 32-bit depth sort):
// counts, offsets, capacity check, emission (into `mask`'s tiles, whose index
// w.wpre / `mlist` is built), tile sort, ranges.
hipError_t list_slab(const BinPlan& p, const clsp_projected& proj, const clsp_bins& bins, const WsPtrs& w, int which,
                     int use_mask, const uint32_t* mask, const uint32_t* mlist, uint32_t* ranges, hipStream_t s,
                     bool recount_first = false) {
  const int V = p.views;
  const int64_t n = p.n, E = p.entries;
  const int wpv = (p.T + 31) / 32;
  const uint2* rect = reinterpret_cast<const uint2*>(proj.rect);
  uint32_t* counters = bins.counters;
  uint32_t* order = w.valA;
  hipError_t err;
  const int epb = which == 1 ? EMIT_EPB_NEAR : EMIT_EPB;
  // the most entries the slab can hold (the first slab of depth-sliced lists holds at
  // most max(E/16, 16384)); blocks loop beyond their grids
  const int64_t slab_max = (which == 1 && bins.mode != CLSP_BINS_COMPLETE)
                               ? std::min<int64_t>(E, std::max<int64_t>(E >> 4, 16384))
                               : E;
  // counts and per-chunk pair counts, then the chunks' offsets (relative to the slab's
  // first pair) and the capacity check
  const int sliced = bins.mode != CLSP_BINS_COMPLETE ? 1 : 0;
  // counting placement (the first slab, and the second of CLSP_BINS_DEPTH_SLICED_LOCAL
  // lists) when the count matrix fits: count, column scan, emission straight into tile
  // order (with the first slab's ranges); no tile sort, no range scan
  const int64_t gt = (int64_t)V * p.T;
  const int64_t nq_bound = (slab_max + CM_EPB - 1) / CM_EPB;
  if (use_mask && p.cm_words > 0 && nq_bound * gt <= p.cm_words &&
      (which == 1 || bins.mode == CLSP_BINS_DEPTH_SLICED_LOCAL)) {
    const int gq = (int)std::min<int64_t>(std::max<int64_t>(nq_bound, 1), 2048);
    const uint32_t tab_words = (uint32_t)(V * (p.TY + 1) * (p.TX + 1));
    const size_t lds_count = cm_count_lds(gt, tab_words), lds_emit = cm_emit_lds(gt, tab_words);
    const int slab_sliced = which == 1 ? sliced : 1;
    // the tile masks pass from the count to the emission when the slab's fit
    unsigned long long* cmask = w.cmask;
    const uint64_t cmw = (uint64_t)p.cmask_words;
    hipLaunchKernelGGL(cm_count_kernel, dim3(gq), dim3(NT), lds_count, s, order, rect, w.tab, w.vfirst, counters,
                       which, slab_sliced, (uint32_t)n, p.TX, p.TY, tab_words, w.cm, cmask, cmw);
    hipLaunchKernelGGL(cm_scan_kernel, dim3((unsigned)((gt + CS_COLS - 1) / CS_COLS)), dim3(CS_NT), 0, s, w.cm,
                       counters, which, w.ctot);
    hipLaunchKernelGGL(cm_emit_kernel, dim3(gq), dim3(NT), lds_emit, s, order, rect, w.tab, w.vfirst, mlist, w.cm,
                       w.ctot, counters, which, (uint32_t)n, p.TX, p.TY, tab_words, (uint64_t)p.capacity, bins.keys,
                       bins.values, reinterpret_cast<uint2*>(ranges), cmask, cmw);
    return hipGetLastError();
  }
  if (which == 1 && !recount_first)
    hipLaunchKernelGGL(gather_counts_kernel, dim3(grid_for(slab_max)), dim3(NT), 0, s, order, w.cnt, rect, counters,
                       sliced, epb, w.tmp, w.rsort, w.blk);
  else
    hipLaunchKernelGGL(recount_kernel, dim3(grid_for(slab_max)), dim3(NT), 0, s, order, rect, w.tab, counters,
                       (uint32_t)n, p.TX, p.TY, which, which == 1 ? sliced : 1, epb, w.tmp, w.rsort, w.blk);
  const int tpasses = passes_for(p.tile_bits);
  uint32_t* ek = (tpasses % 2 == 0) ? bins.keys : w.pairK;
  uint32_t* ev = (tpasses % 2 == 0) ? bins.values : w.pairV;
  // at most four blocks per CU: each block's copy of the mask index serves many groups
  const int eg = (int)std::min<int64_t>(std::max<int64_t>((slab_max + epb - 1) / epb, 1), 1024);
  const int64_t tab_words = (int64_t)V * (p.TY + 1) * (p.TX + 1) + (int64_t)V * p.T;
  if (which == 1 && !use_mask) {
    hipLaunchKernelGGL((emit_kernel<false, false>), dim3(eg), dim3(NT), 0, s, order, w.tmp, w.blk, w.rsort, w.tab, w.vfirst,
                       mlist, counters, n, p.TX, p.TY, V, epb, which, (uint64_t)p.capacity, ek, ev);
  } else if (tab_words <= EMIT_TAB_WORDS) {
    hipLaunchKernelGGL((emit_kernel<true, true>), dim3(eg), dim3(NT), (size_t)tab_words * 4, s, order, w.tmp, w.blk, w.rsort,
                       w.tab, w.vfirst, mlist, counters, n, p.TX, p.TY, V, epb, which, (uint64_t)p.capacity, ek, ev);
  } else {
    hipLaunchKernelGGL((emit_kernel<true, false>), dim3(eg), dim3(NT), 0, s, order, w.tmp, w.blk, w.rsort, w.tab, w.vfirst,
                       mlist, counters, n, p.TX, p.TY, V, epb, which, (uint64_t)p.capacity, ek, ev);
  }
  if (tpasses > 0) {
    uint32_t *k1 = (ek == bins.keys) ? w.pairK : bins.keys, *v1 = (ev == bins.values) ? w.pairV : bins.values;
    radix_sort(ek, ev, k1, v1, counters + C_SLAB_PAIRS, counters + C_SLAB_BASE, p.capacity, p.tile_bits, w.hist,
               w.dtot, s);
  }
  // the second slab's runs are found by the second forward phase itself (only its tiles
  // read them), which saves a launch
  if (which == 1)
    hipLaunchKernelGGL(ranges_kernel, dim3(grid_for(p.capacity, 1 << 14)), dim3(NT), 0, s, bins.keys, counters,
                       reinterpret_cast<uint2*>(ranges));
  return hipGetLastError();
}

}  // namespace

hipError_t launch_fill_u32(uint32_t* p, uint32_t value, int64_t count, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(fill_u32_kernel, dim3(grid_for(count, 4096)), dim3(NT), 0, s, p, value, count);
  return hipGetLastError();
}

BinPlan make_bin_plan(int64_t n, int views, int W, int H, int64_t capacity) {
  BinPlan p{};
  p.n = n;
  p.views = views;
  p.TX = (W + TILE - 1) / TILE;
  p.TY = (H + TILE - 1) / TILE;
  p.T = p.TX * p.TY;
  p.capacity = capacity;
  const int64_t gt = (int64_t)views * p.T;
  int bits = 0;
  while (((int64_t)1 << bits) < gt) ++bits;
  p.tile_bits = bits;
  p.entries = (int64_t)views * n;
  const int64_t E = p.entries > 0 ? p.entries : 1;
  p.scan_blocks = MAX_SCAN_BLOCKS;
  p.sort_blocks_gauss = sort_blocks(E);
  p.sort_blocks_pairs = sort_blocks(capacity);
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off += align256(bytes);
    return o;
  };
  p.off_cnt = take(E * 4);
  p.off_flag = take(E * 4);
  p.off_keyA = take(E * 4);
  p.off_valA = take(E * 4);
  p.off_keyB = take(E * 4);
  p.off_valB = take(E * 4);
  // partial sums: the count pass's blocks, or a slab's emission chunks (EMIT_EPB_NEAR
  // entries or more each)
  p.off_scanBlk = take((size_t)std::max<int64_t>(MAX_SCAN_BLOCKS, E / EMIT_EPB_NEAR + 1) * 4);
  p.off_hist = take((size_t)256 * MAX_SORT_BLOCKS * 4);
  p.off_digit = take(256 * 4);
  const bool need_pair_buf = passes_for(bits) > 0;
  p.off_pairK = take(need_pair_buf ? (size_t)(capacity > 0 ? capacity : 1) * 4 : 4);
  p.off_pairV = take(need_pair_buf ? (size_t)(capacity > 0 ? capacity : 1) * 4 : 4);
  p.off_tflag = take((gt + 1) * 4 * 2);
  p.off_vfirst = take((size_t)views * 4);
  p.off_tab = take((size_t)views * (p.TY + 1) * (p.TX + 1) * 4);
  p.off_rsort = take(E * 8);
  // the count matrix of the slabs' counting placement (and its column totals): sized
  // for a slab of every entry when that fits the budget (then both slabs and complete
  // lists use it), else for the depth-sliced first slab, else not at all
  {
    const int64_t slab1 = std::min<int64_t>(E, std::max<int64_t>(E >> 4, 16384));
    const int64_t w1 = (slab1 + CM_EPB - 1) / CM_EPB * gt, w2 = (E + CM_EPB - 1) / CM_EPB * gt;
    p.cm_words = gt > CM_MAX_SLOTS ? 0 : (w2 <= CM_MAX_WORDS ? w2 : (w1 <= CM_MAX_WORDS ? w1 : 0));
    p.off_cm = take(p.cm_words > 0 ? (size_t)(p.cm_words + gt) * 4 : 4);
    // the count pass's tile masks, kept for the emission when a slab's chunks x slots
    // fit (decided on the device by both kernels alike)
    p.cmask_words = p.cm_words > 0 ? std::min<int64_t>(p.cm_words, CM_MASK_WORDS) : 0;
    p.off_cmask = take(p.cmask_words > 0 ? (size_t)p.cmask_words * 8 : 8);
  }
  // per rendered tile slot: alive flag, and per pixel the carried compositing state
  p.off_alive = take(gt * 4);
  p.off_carry = take((size_t)gt * TILE_PIX * CARRY_FIELDS * 4);
  p.total = off;
  return p;
}

namespace {

// Clears the outputs, builds the render mask (the rectangles of the visible entries of
// rows [a0, a1), or every tile) and its index.
hipError_t mask_and_index(const BinPlan& p, const clsp_projected& proj, int64_t a0, int64_t a1, int use_mask,
                          const clsp_bins& bins, const WsPtrs& w, hipStream_t s) {
  const int V = p.views;
  const int64_t n = p.n, gt = (int64_t)V * p.T;
  const int wpv = (p.T + 31) / 32;
  const uint2* rect = reinterpret_cast<const uint2*>(proj.rect);
  uint32_t* counters = bins.counters;
  // clear outputs (counters[C_STICKY] is left alone: it remembers any overflow)
  {
    ClearList c{};
    bool full = false;
    auto add = [&](uint32_t* ptr, int64_t cnt) {
      if (c.k == CLEAR_SEGS) {
        full = true;
        return;
      }
      c.p[c.k] = ptr;
      c.n[c.k++] = cnt;
    };
    add(counters, C_STICKY);
    add(counters + C_STICKY + 1, CLSP_COUNTERS - C_STICKY - 1);
    add(bins.ranges, gt * 2);
    add(bins.ranges2, gt * 2);
    add(bins.alive_mask, (int64_t)V * wpv);
    if (use_mask) add(bins.tile_mask, (int64_t)V * wpv);
    if (full) return hipErrorInvalidValue;  // more buffers than the clear kernel's list holds
    int64_t total = 0;
    for (int i = 0; i < c.k; ++i) total += c.n[i];
    hipLaunchKernelGGL(clear_kernel, dim3(grid_for(total, 2048)), dim3(NT), 0, s, c);
  }
  // the mask, and its index: the sorted list of tiles to render (all tiles in full mode)
  if (use_mask) {
    if (a1 > a0) {
      hipLaunchKernelGGL(mask_kernel, dim3(ceil_div(a1 - a0, NT), V), dim3(NT), wpv * 4, s, rect, proj.flags, n, a0,
                         a1, p.TX, wpv, bins.tile_mask);
    }
  } else {
    hipLaunchKernelGGL(mask_all_kernel, dim3(grid_for((int64_t)V * wpv, 1 << 20)), dim3(NT), 0, s, bins.tile_mask, V,
                       p.T, wpv);
  }
  index_mask(p, bins.tile_mask, w, bins.tile_list, counters + C_TILES, s);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_bin_and_sort(const BinPlan& p, const clsp_projected& proj, int64_t a0, int64_t a1, int use_mask,
                               const clsp_bins& bins, char* ws, hipStream_t s) {
  const int64_t n = p.n, E = p.entries;
  const WsPtrs w = carve(p, ws);
  const uint2* rect = reinterpret_cast<const uint2*>(proj.rect);
  uint32_t* counters = bins.counters;
  hipError_t err;
  // 1. mask and index
  if ((err = mask_and_index(p, proj, a0, a1, use_mask, bins, w, s)) != hipSuccess) return err;
  if (E > 0) {
    // 2-3. counts (with the block sums of the has-pairs flags), then the compaction of
    // entries with pairs, keyed by depth
    {
      const int G = count_blocks(E);
      hipLaunchKernelGGL(count_kernel, dim3(G), dim3(NT), 0, s, rect, proj.flags, w.tab, (uint32_t)n, (uint32_t)E, G,
                         p.TX, p.TY, use_mask, (uint32_t)n, w.cnt, w.blk);
      hipLaunchKernelGGL(scan_compact_kernel, dim3(G), dim3(NT), 0, s, w.cnt, (uint32_t)E, w.blk, G, proj.depth,
                         w.keyA, w.valA, counters + C_ENTRIES);
    }
    // 4. depth order: 32 key bits, 4 passes, the result back in (keyA, valA)
    radix_sort(w.keyA, w.valA, w.keyB, w.valB, counters + C_ENTRIES, nullptr, E, 32, w.hist, w.dtot, s);
    // 5-7 for the first slab (the whole order for complete lists)
    if ((err = list_slab(p, proj, bins, w, 1, use_mask, bins.tile_mask, bins.tile_list, bins.ranges, s)) != hipSuccess)
      return err;
  }
  return hipGetLastError();
}

size_t frozen_order_bytes(int64_t views, int64_t a0) {
  const uint64_t cap = (uint64_t)views * (uint64_t)a0;
  return (size_t)(ord_rect_word(cap) * 4 + cap * 8);
}

hipError_t launch_frozen_order(const BinPlan& p, const clsp_projected& proj, int64_t a0, uint32_t* ord, char* ws,
                               hipStream_t s) {
  const int64_t n = p.n, E = p.entries, cap = (int64_t)p.views * a0;
  if (cap == 0) return launch_fill_u32(ord, 0u, 1, s);
  const WsPtrs w = carve(p, ws);
  const uint2* rect = reinterpret_cast<const uint2*>(proj.rect);
  // the entries of rows [0, a0) with a visible nonempty rectangle, in entry order, then
  // sorted by depth (stable: (depth key, entry) order), stored with their rectangles
  const int G = count_blocks(E);
  hipLaunchKernelGGL(count_kernel, dim3(G), dim3(NT), 0, s, rect, proj.flags, nullptr, (uint32_t)n, (uint32_t)E, G,
                     p.TX, p.TY, 0, (uint32_t)a0, w.cnt, w.blk);
  hipLaunchKernelGGL(scan_compact_kernel, dim3(G), dim3(NT), 0, s, w.cnt, (uint32_t)E, w.blk, G, proj.depth, w.keyA,
                     w.valA, ord);
  radix_sort(w.keyA, w.valA, w.keyB, w.valB, ord, nullptr, cap, 32, w.hist, w.dtot, s);
  hipLaunchKernelGGL(order_store_kernel, dim3(grid_for(cap)), dim3(NT), 0, s, w.keyA, w.valA, rect, (uint32_t)cap,
                     ord);
  return hipGetLastError();
}

hipError_t launch_bin_and_sort_frozen(const BinPlan& p, const clsp_projected& proj, int64_t a0, const uint32_t* ord,
                                      const clsp_bins& bins, char* ws, hipStream_t s) {
  const int64_t n = p.n, E = p.entries, cap = (int64_t)p.views * a0, nact = (int64_t)p.views * (n - a0);
  const WsPtrs w = carve(p, ws);
  const uint2* rect = reinterpret_cast<const uint2*>(proj.rect);
  uint32_t* counters = bins.counters;
  hipError_t err;
  // 1. the mask of the changed rows [a0, n), and its index
  if ((err = mask_and_index(p, proj, a0, n, 1, bins, w, s)) != hipSuccess) return err;
  if (E > 0) {
    // 2-3. counts and compaction over the stored order, then the changed entries:
    // (keyB, valB) = [stored entries with pairs, in depth order | changed ones]
    const int G = count_blocks(E);
    hipLaunchKernelGGL(count_frozen_kernel, dim3(G), dim3(NT), 0, s, ord, (uint32_t)cap, rect, proj.flags, w.tab,
                       (uint32_t)n, (uint32_t)a0, (uint32_t)E, G, p.TX, p.TY, w.cnt, w.blk, w.tmp);
    hipLaunchKernelGGL(scan_compact_frozen_kernel, dim3(G), dim3(NT), 0, s, w.cnt, (uint32_t)E, w.blk, w.tmp, G, ord,
                       (uint32_t)cap, proj.depth, (uint32_t)n, (uint32_t)a0, w.keyB, w.valB, counters);
    // 4. depth order: the changed entries sorted in place (4 passes return to (keyB,
    // valB)), then both runs merged into valA
    if (nact > 0 && radix_sort(w.keyB, w.valB, w.keyA, w.valA, counters + C_NACT, counters + C_FSPLIT, nact, 32,
                               w.hist, w.dtot, s) != 0)
      return hipErrorInvalidValue;
    hipLaunchKernelGGL(merge_runs_kernel, dim3(grid_for((E + MG_ITEMS - 1) / MG_ITEMS, 4096)), dim3(NT), 0, s, w.keyB,
                       w.valB, counters, w.valA);
    // 5-7 for the first slab; its counts come from the rectangles again
    if ((err = list_slab(p, proj, bins, w, 1, 1, bins.tile_mask, bins.tile_list, bins.ranges, s, true)) != hipSuccess)
      return err;
  }
  return hipGetLastError();
}

hipError_t launch_list_second_slab(const BinPlan& p, const clsp_projected& proj, const clsp_bins& bins, char* ws,
                                   hipStream_t s) {
  if (p.entries == 0) return hipSuccess;
  const WsPtrs w = carve(p, ws);
  index_mask(p, bins.alive_mask, w, w.tlist, nullptr, s, bins.counters + C_ALIVE);
  return list_slab(p, proj, bins, w, 2, 1, bins.alive_mask, w.tlist, bins.ranges2, s);
}

uint32_t* bin_alive_flags(const BinPlan& p, char* ws) { return reinterpret_cast<uint32_t*>(ws + p.off_alive); }
float* bin_carry(const BinPlan& p, char* ws) { return reinterpret_cast<float*>(ws + p.off_carry); }

}  // namespace clsp
