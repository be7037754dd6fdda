// Tile rasteriser: forward compositing, L1 loss gradient, and reverse compositing with
// per-Gaussian gradient reduction (Supp. "Local Optimization Kernel", item 2: only the
// tiles of the render mask are launched; Table tab:timings "Forward::Render" and
// "Backward::Render").
//
// One 256-thread workgroup (four wave64s) per 16x16 tile, one pixel per thread.  The
// tile's depth-ordered records are staged through LDS 256 at a time; every lane reads
// the same LDS record, so the reads are broadcasts.  In the backward each wave sums its
// 64 pixels' partials with DPP row operations, the four wave sums meet in LDS, and one
// global float atomic per (record, component) is issued, only for changed Gaussians.
#include <algorithm>

#include "internal.hpp"

namespace clsp {
namespace {

constexpr int NT = TILE_PIX;
constexpr int C_OVERFLOW = 1, C_TILES = 2, C_ALIVE = 8, C_SLAB_PAIRS = 11, C_SLAB_BASE = 12;

// Opacity of a record at a pixel centre, evaluated with explicitly rounded operations
// so the forward and the backward take the same decisions bit for bit.
// Returns false when the record is skipped (positive exponent or alpha < 1/255).
// Pixel of thread t in its 16x16 tile: each wave64 takes an 8x8 quadrant (t bits 0-2:
// x, 3-5: y, 6: quadrant x, 7: quadrant y), so a wave's pixels are compact and tend to
// finish compositing together.  Every kernel that keeps per-thread state of a tile
// (compositing chunks, carries) uses this same map.
__device__ __forceinline__ int pixel_x(uint32_t t) { return (int)((((t >> 6) & 1u) << 3) | (t & 7u)); }
__device__ __forceinline__ int pixel_y(uint32_t t) { return (int)((((t >> 7) & 1u) << 3) | ((t >> 3) & 7u)); }

// Records are staged in LDS with the conic in base-2 exponent units:
// a = (u, v, A2, B2), b = (C2, o, r, g) with A2 = -A log2(e)/2, B2 = -B log2(e),
// C2 = -C log2(e)/2, so that the Gaussian's exponent (A dx^2 + 2B dx dy + C dy^2)(-1/2)
// is p2 / log2(e) with p2 = A2 dx^2 + B2 dx dy + C2 dy^2, and G = 2^p2.
constexpr float LOG2E = 1.4426950408889634f;
constexpr float K_AC = -0.5f * LOG2E;
constexpr float K_B = -LOG2E;

__device__ __forceinline__ void stage_record(const float* __restrict__ splat, uint32_t e, float4& a, float4& b,
                                             float& c) {
  const float4* sp = reinterpret_cast<const float4*>(splat + (size_t)e * SPLAT_STRIDE);
  const float4 r0 = sp[0], r1 = sp[1];
  a = make_float4(r0.x, r0.y, r0.z * K_AC, r0.w * K_B);
  b = make_float4(r1.x * K_AC, r1.y, r1.z, r1.w);
  c = sp[2].x;
}

// Weight of a staged record at pixel centre (fx, fy): false if the exponent is positive
// or alpha = min(0.99, o G) < 1/255 (branch-free, so that the weights of neighbouring
// records can be computed together).
__device__ __forceinline__ bool splat_alpha(const float4 a, const float4 b, float fx, float fy, float& dx, float& dy,
                                            float& G, float& alpha, bool& clamped) {
  dx = __fsub_rn(fx, a.x);
  dy = __fsub_rn(fy, a.y);
  const float p2 = __fmaf_rn(__fmul_rn(a.z, dx), dx, __fmaf_rn(__fmul_rn(a.w, dx), dy, __fmul_rn(__fmul_rn(b.x, dy), dy)));
  G = __builtin_amdgcn_exp2f(p2);
  const float oG = __fmul_rn(b.y, G);
  clamped = !(oG < ALPHA_MAX);
  alpha = clamped ? ALPHA_MAX : oG;
  return !(p2 > 0.0f) && alpha >= ALPHA_MIN;
}

// Compositing state per rendered tile slot: the largest contributor count of its pixels
// and the tile's chunk length, then per (chunk, pixel) the transmittance after the chunk
// and the chunk's colour.
struct StateView {
  uint32_t* maxlast;   // [slots]
  uint32_t* chunk_len; // [slots]
  float4* chunks;      // [slots][CHUNKS][256]
};

__host__ __device__ inline size_t state_header_bytes(int64_t slots) { return ((size_t)slots * 8 + 255) & ~(size_t)255; }

__device__ __forceinline__ StateView state_view(void* base, int64_t slots) {
  StateView v;
  v.maxlast = reinterpret_cast<uint32_t*>(base);
  v.chunk_len = v.maxlast + slots;
  v.chunks = reinterpret_cast<float4*>(reinterpret_cast<char*>(base) + state_header_bytes(slots));
  return v;
}

// A tile's list is cut into chunks of CH entries; when a list reaches CHUNKS of them,
// neighbouring chunks are merged pairwise and the chunk length doubles, so every chunk
// holds at most max(CH, 2L/CHUNKS) entries of a list of L and no chunk is unbounded.
constexpr int CH = CLSP_STATE_CHUNK;
constexpr int CHUNKS = CLSP_STATE_CHUNKS;

// The chunk length of a tile after compositing the first `len` entries of its list.
__device__ __forceinline__ int chunk_len_after(int len) {
  int c = CH;
  while (len >= CHUNKS * c) c *= 2;
  return c;
}

// First positions i in [0, n) with keys[i] >= x and with keys[i] > x in ascending
// keys (every thread of the block calls it and gets both): 256-ary searches run
// together, one probe per thread per round, so n = 16M takes three rounds.
__device__ __forceinline__ void block_equal_range(const uint32_t* __restrict__ keys, uint32_t n, uint32_t x,
                                                  uint32_t& first, uint32_t& last) {
  uint32_t lo_a = 0, hi_a = n, lo_b = 0, hi_b = n;  // each answer lies in [lo, hi]
  while (hi_a > lo_a || hi_b > lo_b) {
    const uint32_t span_a = hi_a - lo_a, span_b = hi_b - lo_b;
    // probes lo + span * t / NT (span >= NT: strictly increasing in t, the first at lo),
    // or every position lo + t when the span is shorter
    const uint32_t qa = lo_a + (span_a < NT ? threadIdx.x : (uint32_t)(((uint64_t)span_a * threadIdx.x) / NT));
    const uint32_t qb = lo_b + (span_b < NT ? threadIdx.x : (uint32_t)(((uint64_t)span_b * threadIdx.x) / NT));
    const bool below_a = span_a > 0 && (span_a >= NT || threadIdx.x < span_a) && keys[qa] < x;
    const bool below_b = span_b > 0 && (span_b >= NT || threadIdx.x < span_b) && keys[qb] <= x;
    const uint32_t ca = (uint32_t)__syncthreads_count(below_a);
    const uint32_t cb = (uint32_t)__syncthreads_count(below_b);
    // the answer is past the last probe below x and at or before the first one not below
    auto narrow = [&](uint32_t& lo, uint32_t& hi, uint32_t span, uint32_t c) {
      if (span == 0) return;
      if (span < NT) {  // every position was probed
        lo = hi = lo + c;
        return;
      }
      const uint32_t l = lo;
      if (c > 0) lo = l + (uint32_t)(((uint64_t)span * (c - 1)) / NT) + 1;
      if (c < NT) hi = l + (uint32_t)(((uint64_t)span * c) / NT);
    };
    narrow(lo_a, hi_a, span_a, ca);
    narrow(lo_b, hi_b, span_b, cb);
  }
  first = lo_a;
  last = lo_b;
}

// Entry of list position k of a tile whose list is [r1.x, r1.y) followed by [r2.x, r2.y).
__device__ __forceinline__ uint32_t list_entry(const uint32_t* __restrict__ values, uint2 r1, uint2 r2, int k) {
  const int len1 = (int)(r1.y - r1.x);
  return k < len1 ? values[r1.x + k] : values[r2.x + (k - len1)];
}

// Optional L1 loss gradient computed by the forward itself (dL NULL: none).
struct L1Out {
  const float* target;
  float* dL;
  float* loss_sum;
};

// PHASE 1 composites each rendered tile's first list (the whole list for complete
// bins).  With `sliced`, tiles in which a pixel is still compositing at the end are
// marked alive and their per-pixel state is saved in `carry`; PHASE 2 continues the
// alive tiles with their second lists from that state.  Chunk boundaries (every CH
// list positions) and all arithmetic are the same as in one pass over the whole list,
// so the outputs are identical bit for bit.
// Records whose weights the forward computes together: 8, or 16 for the lists of the
// optimiser's local steps, where few tiles are rendered and each wave's own
// instruction-level parallelism sets the pace (the larger group costs registers, and so
// occupancy, which full renders need).
constexpr int FW_GROUP = 8, FW_GROUP_LOCAL = 16;

template <int PHASE, int FW_UNROLL>
__global__ void __launch_bounds__(NT) render_forward_kernel(
    const float* __restrict__ splat, const uint32_t* __restrict__ values, const uint32_t* __restrict__ pair_keys,
    const uint2* __restrict__ ranges, uint2* __restrict__ ranges2, const uint32_t* __restrict__ tile_list,
    uint32_t* __restrict__ counters, int T,
    int TX, int W, int H, float bg0, float bg1, float bg2, float* __restrict__ image, float* __restrict__ T_final,
    uint32_t* __restrict__ n_contrib, void* state, int64_t slots, int sliced, uint32_t* __restrict__ alive,
    uint32_t* __restrict__ alive_mask, int wpv, float* __restrict__ carry, L1Out l1) {
  const uint32_t slot = blockIdx.x;
  if (slot >= counters[C_TILES]) return;
  if (PHASE == 2 && (counters[C_OVERFLOW] || !alive[slot])) return;
  __shared__ float4 s_a[NT];
  __shared__ float4 s_b[NT];
  __shared__ float s_c[NT];
  __shared__ uint32_t s_max;
  const uint32_t gt = tile_list[slot];
  const int v = gt / T, t = gt % T;
  const int px = (t % TX) * TILE + pixel_x(threadIdx.x);
  const int py = (t / TX) * TILE + pixel_y(threadIdx.x);
  const bool inside = px < W && py < H;
  const float fx = (float)px + 0.5f, fy = (float)py + 0.5f;
  const uint2 r1 = ranges[gt];
  uint2 r2 = make_uint2(0u, 0u);
  if (PHASE == 2) {
    // this tile's run among the second slab's pairs (sorted by global tile), recorded
    // in ranges2 for the backward
    const uint32_t base = counters[C_SLAB_BASE], P2 = counters[C_SLAB_PAIRS];
    uint32_t first, last;
    block_equal_range(pair_keys + base, P2, gt, first, last);
    if (last > first) r2 = make_uint2(base + first, base + last);
    if (threadIdx.x == 0) ranges2[gt] = r2;
  }
  const int len1 = (int)(r1.y - r1.x);
  const int k_begin = PHASE == 1 ? 0 : len1;
  const int k_end = PHASE == 1 ? len1 : len1 + (int)(r2.y - r2.x);
  const bool keep = state != nullptr;
  StateView sv;
  if (keep) sv = state_view(state, slots);
  float4* my_chunks = keep ? sv.chunks + (size_t)slot * CHUNKS * NT + threadIdx.x : nullptr;
  float* my_carry = carry + (size_t)slot * CARRY_FIELDS * NT + threadIdx.x;

  float Tr = 1.0f, cr = 0.0f, cg = 0.0f, cb = 0.0f;   // colour of the flushed chunks
  float dr = 0.0f, dg = 0.0f, db = 0.0f;              // colour of the current chunk
  uint32_t last = 0;
  // transmittance for blending: Tr while the pixel composites, 0 once it has stopped
  float Tb = inside ? 1.0f : 0.0f;
  int chunk = 0;
  int chl = CH;  // the tile's current chunk length (uniform over the workgroup)
  if (PHASE == 2) {
    Tr = my_carry[0 * NT];
    cr = my_carry[1 * NT];
    cg = my_carry[2 * NT];
    cb = my_carry[3 * NT];
    dr = my_carry[4 * NT];
    dg = my_carry[5 * NT];
    db = my_carry[6 * NT];
    last = __float_as_uint(my_carry[7 * NT]);
    Tb = my_carry[8 * NT] != 0.0f ? 0.0f : Tr;
    // the first phase composited the whole first list (the tile was still alive)
    chl = chunk_len_after(len1);
    chunk = len1 / chl;
  }
  for (int kb = k_begin; kb < k_end; kb += NT) {
    if (__syncthreads_count(Tb == 0.0f) == NT) break;
    const int k = kb + threadIdx.x;
    if (k < k_end) {
      const uint32_t e = list_entry(values, r1, r2, k);
      stage_record(splat, e, s_a[threadIdx.x], s_b[threadIdx.x], s_c[threadIdx.x]);
    }
    __syncthreads();
    const int cnt = min(NT, k_end - kb);
    // segments of the batch between chunk boundaries of the list
    for (int j = 0; j < cnt;) {
      const int next_b = ((kb + j) / chl + 1) * chl;
      const int jhi = min(cnt, next_b - kb);
      // Branch-free blending, FW_UNROLL records per iteration: their weights are
      // computed first, then applied in order.  The per-lane state is kept in floats so
      // that no lane-mask logic is needed: a skipped record has weight 0 (then
      // Tb * (1 - 0) = Tb exactly), and a record that would take the transmittance below
      // T_STOP is not blended and sets Tb to 0, which blends nothing more (0 * x = 0 and
      // 0 < T_STOP), while Tr keeps the transmittance after the last blended record; this
      // is the same arithmetic, and gives the same bits, as blending with branches.  A
      // group that reaches past the segment's end (chunk boundaries of the second list,
      // which starts anywhere, and the list's end) gives the records past it weight 0;
      // whole groups need no check.  The wave leaves the segment once all its lanes have
      // stopped.
      auto group = [&](int jj, int lim) {
        float ae[FW_UNROLL], cq[FW_UNROLL];
        float4 bq[FW_UNROLL];
#pragma unroll
        for (int u = 0; u < FW_UNROLL; ++u) {
          const int ju = jj + (u < lim ? u : lim - 1);   // uniform; lim = FW_UNROLL: jj + u
          const float4 aq = s_a[ju];
          bq[u] = s_b[ju];
          cq[u] = s_c[ju];
          float dx, dy, G, al;
          bool cl;
          ae[u] = (splat_alpha(aq, bq[u], fx, fy, dx, dy, G, al, cl) && u < lim) ? al : 0.0f;
        }
        uint32_t lastu = 0;   // 1 + the group's last blended record, 0 if none
#pragma unroll
        for (int u = 0; u < FW_UNROLL; ++u) {
          const float Tn = Tb * (1.0f - ae[u]);
          // (written as the condition to go on, which selects with the short encoding)
          const bool go = Tn >= T_STOP;          // false only when ae > 0 or Tb = 0
          const float w = go ? ae[u] * Tb : 0.0f;   // colours are finite and >= 0: adding 0*c is exact
          dr = fmaf(w, bq[u].z, dr);
          dg = fmaf(w, bq[u].w, dg);
          db = fmaf(w, cq[u], db);
          Tb = go ? Tn : 0.0f;
          Tr = go ? Tn : Tr;
          lastu = w > 0.0f ? (uint32_t)(u + 1) : lastu;
        }
        last = lastu ? (uint32_t)(kb + jj) + lastu : last;
      };
      for (int jj = j; jj < jhi; jj += FW_UNROLL) {
        if (__ballot(Tb != 0.0f) == 0ull) break;
        if (jj + FW_UNROLL <= jhi)
          group(jj, FW_UNROLL);
        else
          group(jj, jhi - jj);
      }
      // a chunk boundary of the tile's list: record this pixel's state
      if (kb + jhi == next_b) {
        if (keep) my_chunks[(size_t)chunk * NT] = make_float4(Tr, dr, dg, db);
        cr += dr;
        cg += dg;
        cb += db;
        dr = dg = db = 0.0f;
        if (++chunk == CHUNKS) {
          // every chunk is full: merge neighbours pairwise (the transmittance after the
          // second, the sum of the colours) and double the chunk length
          if (keep) {
            for (int c = 0; c < CHUNKS / 2; ++c) {
              const float4 x = my_chunks[(size_t)(2 * c) * NT], y = my_chunks[(size_t)(2 * c + 1) * NT];
              my_chunks[(size_t)c * NT] = make_float4(y.x, x.y + y.y, x.z + y.z, x.w + y.w);
            }
          }
          chunk = CHUNKS / 2;
          chl *= 2;
        }
      }
      j = jhi;
    }
  }
  bool more = false;  // the second phase continues this tile
  if (PHASE == 1 && sliced) {
    more = __syncthreads_count(Tb == 0.0f) < NT;
    if (more) {
      // save the state; the second list continues this tile
      my_carry[0 * NT] = Tr;
      my_carry[1 * NT] = cr;
      my_carry[2 * NT] = cg;
      my_carry[3 * NT] = cb;
      my_carry[4 * NT] = dr;
      my_carry[5 * NT] = dg;
      my_carry[6 * NT] = db;
      my_carry[7 * NT] = __uint_as_float(last);
      my_carry[8 * NT] = Tb == 0.0f ? 1.0f : 0.0f;
    }
    if (threadIdx.x == 0) {
      alive[slot] = more ? 1u : 0u;
      if (more) {
        atomicOr(&alive_mask[(int64_t)v * wpv + (t >> 5)], 1u << (t & 31));
        atomicAdd(&counters[C_ALIVE], 1u);
      }
    }
  }
  if (keep) my_chunks[(size_t)chunk * NT] = make_float4(Tr, dr, dg, db);
  cr += dr;
  cg += dg;
  cb += db;
  if (keep) {
    if (threadIdx.x == 0) s_max = 0;
    __syncthreads();
    atomicMax(&s_max, last);
    __syncthreads();
    if (threadIdx.x == 0) {
      sv.maxlast[slot] = s_max;
      sv.chunk_len[slot] = (uint32_t)chl;
    }
  }
  const size_t hw = (size_t)H * W;
  const size_t pix = (size_t)py * W + px;
  const float col[3] = {fmaf(Tr, bg0, cr), fmaf(Tr, bg1, cg), fmaf(Tr, bg2, cb)};
  if (inside) {
    for (int c = 0; c < 3; ++c) image[((size_t)v * 3 + c) * hw + pix] = col[c];
    T_final[(size_t)v * hw + pix] = Tr;
    n_contrib[(size_t)v * hw + pix] = last;
  }
  // L1 gradient of the finished pixels (the same arithmetic as l1_loss_grad_kernel on
  // the stored image); a tile the second phase continues is finished there
  if (l1.dL && !more) {
    const float norm = 1.0f / (3.0f * (float)W * (float)H);
    float acc = 0.0f;
    if (inside) {
      for (int c = 0; c < 3; ++c) {
        const size_t idx = ((size_t)v * 3 + c) * hw + pix;
        const float d = col[c] - l1.target[idx];
        l1.dL[idx] = d > 0.0f ? norm : (d < 0.0f ? -norm : 0.0f);
        acc += fabsf(d);
      }
    }
    if (l1.loss_sum) {
      for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
      __syncthreads();  // s_c is free: the blending is over
      if ((threadIdx.x & 63) == 0) s_c[threadIdx.x >> 6] = acc;
      __syncthreads();
      if (threadIdx.x == 0) atomicAdd(l1.loss_sum, (s_c[0] + s_c[1] + s_c[2] + s_c[3]) * norm);
    }
  }
}

// Blocks loop over the rendered tiles (at most L1_BLOCKS of them), so that the loss
// sum costs one float atomic per block rather than per tile: atomics on one address
// serialise.
constexpr int L1_BLOCKS = 512;
// Workgroups of the backward, which loop over the (tile, chunk) items.
constexpr int64_t BWD_BLOCKS = 16384;

__global__ void __launch_bounds__(NT) l1_loss_grad_kernel(const float* __restrict__ image,
                                                          const float* __restrict__ target,
                                                          const uint32_t* __restrict__ tile_list,
                                                          const uint32_t* __restrict__ counters, int T, int TX, int W,
                                                          int H, float* __restrict__ dL, float* __restrict__ loss_sum) {
  __shared__ float s_sum[4];
  const uint32_t tiles = counters[C_TILES];
  if (blockIdx.x >= tiles) return;
  const float norm = 1.0f / (3.0f * (float)W * (float)H);
  const size_t hw = (size_t)H * W;
  float acc = 0.0f;
  for (uint32_t slot = blockIdx.x; slot < tiles; slot += gridDim.x) {
    const uint32_t gt = tile_list[slot];
    const int v = gt / T, t = gt % T;
    // row-major within the tile: each wave reads four 64-byte row segments
    const int px = (t % TX) * TILE + (int)(threadIdx.x & 15u);
    const int py = (t / TX) * TILE + (int)(threadIdx.x >> 4);
    if (px < W && py < H) {
      for (int c = 0; c < 3; ++c) {
        const size_t idx = ((size_t)v * 3 + c) * hw + (size_t)py * W + px;
        const float d = image[idx] - target[idx];
        dL[idx] = d > 0.0f ? norm : (d < 0.0f ? -norm : 0.0f);
        acc += fabsf(d);
      }
    }
  }
  if (loss_sum) {
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
    if ((threadIdx.x & 63) == 0) s_sum[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) atomicAdd(loss_sum, (s_sum[0] + s_sum[1] + s_sum[2] + s_sum[3]) * norm);
  }
}

template <int CTRL, int ROW_MASK>
__device__ __forceinline__ float dpp_f(float x) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, ROW_MASK, 0xf, false));
}

// Sums over the 64 lanes of a wave of each of N values per lane, scattered over the
// lanes (a butterfly reduce-scatter): at each of six levels, lane distance 32, 16, ... 1,
// a lane keeps one half of its values (the lower lane of a pair the first half) and
// adds the partner's copy of that half, so a level of m values costs about m/2
// exchanges and adds instead of the 6 m of separate reductions.  Afterwards the lane
// with bfly_index >= 0 holds the sum of that value index in x[0].  Every lane of the
// wave must be active.
template <int D> __device__ __forceinline__ float lane_xor(float v);
template <> __device__ __forceinline__ float lane_xor<16>(float v) {
  return __int_as_float(__builtin_amdgcn_ds_swizzle(__float_as_int(v), 0x401F));  // lane ^ 16 within 32
}
template <> __device__ __forceinline__ float lane_xor<8>(float v) { return dpp_f<0x128, 0xf>(v); }  // row_ror:8
template <> __device__ __forceinline__ float lane_xor<4>(float v) {
  return __int_as_float(__builtin_amdgcn_ds_swizzle(__float_as_int(v), 0x101F));  // lane ^ 4 within 32
}
template <> __device__ __forceinline__ float lane_xor<2>(float v) { return dpp_f<0x4e, 0xf>(v); }  // quad_perm [2,3,0,1]
template <> __device__ __forceinline__ float lane_xor<1>(float v) { return dpp_f<0xb1, 0xf>(v); }  // quad_perm [1,0,3,2]

// One level over the first M values (an odd count is padded with a zero).
template <int M, int D>
__device__ __forceinline__ void bfly_level(float* x, bool upper) {
  constexpr int H = (M + 1) / 2;
  if (M & 1) x[M] = 0.0f;
#pragma unroll
  for (int i = 0; i < H; ++i) {
    const float send = upper ? x[i] : x[H + i];
    const float keep = upper ? x[H + i] : x[i];
    x[i] = keep + lane_xor<D>(send);
  }
}

template <int N>
__device__ __forceinline__ void bfly_reduce(float (&x)[N], uint32_t lane) {
  static_assert(N % 2 == 0, "the first level takes pairs (i, N/2 + i)");
  constexpr int H1 = N / 2;
  // distance 32: one lane-half swap (v_permlane32_swap) moves both halves of a pair
#pragma unroll
  for (int i = 0; i < H1; ++i) {
    const auto sw = __builtin_amdgcn_permlane32_swap(__float_as_uint(x[i]), __float_as_uint(x[H1 + i]), false, false);
    x[i] = __uint_as_float(sw[0]) + __uint_as_float(sw[1]);
  }
  constexpr int M2 = H1, M3 = (M2 + 1) / 2, M4 = (M3 + 1) / 2, M5 = (M4 + 1) / 2, M6 = (M5 + 1) / 2;
  bfly_level<M2, 16>(x, (lane & 16u) != 0);
  bfly_level<M3, 8>(x, (lane & 8u) != 0);
  bfly_level<M4, 4>(x, (lane & 4u) != 0);
  bfly_level<M5, 2>(x, (lane & 2u) != 0);
  bfly_level<M6, 1>(x, (lane & 1u) != 0);
}

// The value index whose sum bfly_reduce leaves in this lane, or -1 (a padding zero).
template <int N>
__device__ __forceinline__ int bfly_index(uint32_t lane) {
  constexpr int M2 = N / 2, M3 = (M2 + 1) / 2, M4 = (M3 + 1) / 2, M5 = (M4 + 1) / 2, M6 = (M5 + 1) / 2;
  const int m[6] = {N, M2, M3, M4, M5, M6};
  const int h[6] = {N / 2, (M2 + 1) / 2, (M3 + 1) / 2, (M4 + 1) / 2, (M5 + 1) / 2, (M6 + 1) / 2};
  int pos = 0;
  bool ok = true;
  for (int k = 5; k >= 0; --k) {
    pos += (lane & (32u >> k)) ? h[k] : 0;
    ok = ok && pos < m[k];
  }
  return ok ? pos : -1;
}

// Records whose gradient terms are reduced together (BW_GROUP * 9 values).
constexpr int BW_GROUP = 4;

// One workgroup per (rendered tile, chunk of its list): reverse traversal of the
// chunk's entries from the chunk's stored end state.
__global__ void __launch_bounds__(NT) render_backward_kernel(
    const float* __restrict__ splat, const uint32_t* __restrict__ values, const uint2* __restrict__ ranges,
    const uint2* __restrict__ ranges2, const uint32_t* __restrict__ tile_list, const uint32_t* __restrict__ counters,
    int T, int TX, int W, int H, int64_t n, float bg0, float bg1, float bg2, int64_t a0, int64_t a1,
    const float* __restrict__ T_final, const uint32_t* __restrict__ n_contrib, void* state, int64_t slots,
    const float* __restrict__ dL, float* __restrict__ grad2d) {
  __shared__ float4 s_a[NT];
  __shared__ float4 s_b[NT];
  __shared__ float s_c[NT];
  __shared__ uint32_t s_e[NT];
  __shared__ uint32_t s_act[NT];  // the record's Gaussian is in the active range
  __shared__ float s_g[NT][9];
  // One (rendered tile, chunk) work item per iteration: the grid is capped and loops
  // over the items, chunk-major, so that no workgroup is launched for the slots past
  // the rendered tiles.
  auto item = [&](uint32_t slot, int chunk) {
    const StateView sv = state_view(state, slots);
    const int maxlast = (int)sv.maxlast[slot];
    if (maxlast == 0) return;
    const int chl = (int)sv.chunk_len[slot];
    const int k0 = chunk * chl;
    if (k0 >= maxlast) return;
    const int last_chunk = (maxlast - 1) / chl;   // < CHUNKS: the forward keeps it so
    const int k1 = (chunk == last_chunk) ? maxlast : (chunk + 1) * chl;

    const uint32_t gt = tile_list[slot];
    const uint2 r1 = ranges[gt], r2 = ranges2[gt];
    if (a0 > 0 || a1 < n) {
      // A chunk without a record of the active range adds nothing to any gradient: its
      // frozen records only un-blend, and no other chunk starts from where it ends.  (The
      // block-wide OR goes through s_act, which is rewritten before its first use below.)
      const int64_t vb = (int64_t)(gt / T) * n;
      bool any = false;
      for (int k = k0 + (int)threadIdx.x; k < k1; k += NT) {
        const int64_t gid = (int64_t)list_entry(values, r1, r2, k) - vb;
        any = any || (gid >= a0 && gid < a1);
      }
      const bool wave_any = __ballot(any) != 0ull;
      if ((threadIdx.x & 63u) == 0) s_act[threadIdx.x >> 6] = wave_any ? 1u : 0u;
      __syncthreads();
      const bool block_any = (s_act[0] | s_act[1] | s_act[2] | s_act[3]) != 0u;
      __syncthreads();
      if (!block_any) return;
    }

    const int v = gt / T, t = gt % T;
    const int px = (t % TX) * TILE + pixel_x(threadIdx.x);
    const int py = (t / TX) * TILE + pixel_y(threadIdx.x);
    const bool inside = px < W && py < H;
    const float fx = (float)px + 0.5f, fy = (float)py + 0.5f;
    const size_t hw = (size_t)H * W;
    const size_t pix = (size_t)py * W + px;

    float Tr = 1.0f, g0 = 0.f, g1 = 0.f, g2 = 0.f;
    uint32_t last = 0;
    float Tfin = 1.0f;
    if (inside) {
      Tfin = T_final[(size_t)v * hw + pix];
      last = n_contrib[(size_t)v * hw + pix];
      g0 = dL[((size_t)v * 3 + 0) * hw + pix];
      g1 = dL[((size_t)v * 3 + 1) * hw + pix];
      g2 = dL[((size_t)v * 3 + 2) * hw + pix];
    }
    // state at the end of this chunk: transmittance, and the colour of everything behind
    // it (later chunks plus the background)
    const float4* my_chunks = sv.chunks + (size_t)slot * CHUNKS * NT + threadIdx.x;
    float S0 = Tfin * bg0, S1 = Tfin * bg1, S2 = Tfin * bg2;
    for (int c = last_chunk; c > chunk; --c) {
      const float4 st = my_chunks[(size_t)c * NT];
      S0 += st.y;
      S1 += st.z;
      S2 += st.w;
    }
    Tr = (chunk == last_chunk) ? Tfin : my_chunks[(size_t)chunk * NT].x;

    const int64_t na = a1 - a0;
    const int64_t vbase = (int64_t)v * n;
    const uint32_t lane = threadIdx.x & 63;
    const int bidx = bfly_index<BW_GROUP * 9>(lane);

    for (int end = k1; end > k0; end -= NT) {
      const int beg = max(k0, end - NT);
      const int cnt = end - beg;
      __syncthreads();
      if ((int)threadIdx.x < cnt) {
        const uint32_t e = list_entry(values, r1, r2, beg + (int)threadIdx.x);
        stage_record(splat, e, s_a[threadIdx.x], s_b[threadIdx.x], s_c[threadIdx.x]);
        s_e[threadIdx.x] = e;
        const int64_t gid = (int64_t)e - vbase;
        s_act[threadIdx.x] = (gid >= a0 && gid < a1) ? 1u : 0u;
      }
#pragma unroll
      for (int c = 0; c < 9; ++c) s_g[threadIdx.x][c] = 0.0f;
      __syncthreads();
      // a frozen Gaussian's record: only the transmittance and the colour behind move on
      auto unblend = [&](bool ok, float alpha, float4 b, float c) {
        if (!ok) return;
        // 1 - alpha is in [0.01, 1]: the hardware reciprocal (about 1 ulp) in place of a
        // division
        const float Tj = Tr * __builtin_amdgcn_rcpf(1.0f - alpha);
        const float w = alpha * Tj;
        S0 = fmaf(w, b.z, S0);
        S1 = fmaf(w, b.w, S1);
        S2 = fmaf(w, c, S2);
        Tr = Tj;
      };
      // BW_GROUP records at a time: their weights first (independent), then in order the
      // frozen ones un-blend and the active ones give their gradient terms (every lane
      // evaluates the record's weight; if some lane of the wave is touched, the terms are
      // computed branch-free, masked by 0/1 factors: exact, the unmasked terms are
      // multiplied by 1, the masked ones add zeros); the group's terms are summed over the
      // wave in one reduce-scatter.
      for (int jb = cnt - 1; jb >= 0; jb -= BW_GROUP) {
        float4 aq[BW_GROUP], bq[BW_GROUP];
        float cq[BW_GROUP], dxq[BW_GROUP], dyq[BW_GROUP], Gq[BW_GROUP], alq[BW_GROUP];
        bool okq[BW_GROUP], clq[BW_GROUP], actq[BW_GROUP];
#pragma unroll
        for (int q = 0; q < BW_GROUP; ++q) {
          const int j = jb - q;
          const int js = j >= 0 ? j : 0;
          aq[q] = s_a[js];
          bq[q] = s_b[js];
          cq[q] = s_c[js];
          actq[q] = j >= 0 && s_act[js] != 0u;
          okq[q] = splat_alpha(aq[q], bq[q], fx, fy, dxq[q], dyq[q], Gq[q], alq[q], clq[q]) && j >= 0 &&
                   beg + j < (int)last;
        }
        float P[BW_GROUP * 9];
        bool any = false;  // some record of the group touched a lane of the wave (uniform)
#pragma unroll
        for (int q = 0; q < BW_GROUP; ++q) {
#pragma unroll
          for (int c = 0; c < 9; ++c) P[q * 9 + c] = 0.0f;
          if (!actq[q]) {  // (uniform: one record for the whole wave)
            unblend(okq[q], alq[q], bq[q], cq[q]);
            continue;
          }
          const float4 a = aq[q], b = bq[q];
          const float cb = cq[q], dx = dxq[q], dy = dyq[q], G = Gq[q], alpha = alq[q];
          const bool contrib = okq[q], clamped = clq[q];
          if (__ballot(contrib)) {
            any = true;
            const float om = 1.0f - alpha;
            const float io = __builtin_amdgcn_rcpf(om);  // om in [0.01, 1]
            const float Tj = Tr * io;
            const float w = alpha * Tj;
            const float dLda = g0 * (Tj * b.z - S0 * io) + g1 * (Tj * b.w - S1 * io) + g2 * (Tj * cb - S2 * io);
            S0 = contrib ? fmaf(w, b.z, S0) : S0;
            S1 = contrib ? fmaf(w, b.w, S1) : S1;
            S2 = contrib ? fmaf(w, cb, S2) : S2;
            Tr = contrib ? Tj : Tr;
            const float cf = contrib ? 1.0f : 0.0f;
            const float gf = (contrib && !clamped) ? 1.0f : 0.0f;  // the 0.99 clamp has zero derivative
            const float gp = alpha * dLda * gf;                     // dL/dpower
            // dL/du = gp (A dx + B dy), dL/dv = gp (B dx + C dy); in staged units A = A2 / K_AC,
            // B = B2 / K_B = B2 / (2 K_AC), C = C2 / K_AC
            const float gk = gp * (1.0f / K_AC);
            P[q * 9 + 0] = gk * (a.z * dx + 0.5f * a.w * dy);
            P[q * 9 + 1] = gk * (0.5f * a.w * dx + b.x * dy);
            P[q * 9 + 2] = -0.5f * gp * dx * dx;
            P[q * 9 + 3] = -gp * dx * dy;
            P[q * 9 + 4] = -0.5f * gp * dy * dy;
            P[q * 9 + 5] = G * dLda * gf;  // dL/dopacity
            P[q * 9 + 6] = w * g0 * cf;
            P[q * 9 + 7] = w * g1 * cf;
            P[q * 9 + 8] = w * g2 * cf;
          }
        }
        if (any) {
          bfly_reduce(P, lane);
          const int q = bidx / 9, c = bidx % 9;
          if (bidx >= 0 && jb - q >= 0 && P[0] != 0.0f) atomicAdd(&s_g[jb - q][c], P[0]);
        }
      }
      __syncthreads();
      if ((int)threadIdx.x < cnt) {
        const int64_t gid = (int64_t)s_e[threadIdx.x] - vbase;
        if (s_act[threadIdx.x]) {
          float* dst = grad2d + ((int64_t)v * na + (gid - a0)) * G2D_STRIDE;
#pragma unroll
          for (int c = 0; c < 9; ++c) {
            const float val = s_g[threadIdx.x][c];
            if (val != 0.0f) atomicAdd(dst + c, val);
          }
        }
      }
    }
  };
  // lists that ran out of pair capacity were not rendered completely: no gradient
  if (counters[C_OVERFLOW]) return;
  const uint32_t tiles = counters[C_TILES];
  const uint32_t items = tiles * (uint32_t)CHUNKS;
  for (uint32_t w = blockIdx.x; w < items; w += gridDim.x) {
    __syncthreads();  // the previous item's LDS is free
    item(w % tiles, (int)(w / tiles));
  }
}

}  // namespace

size_t render_state_bytes(int views, int TX, int TY) {
  const int64_t slots = (int64_t)views * TX * TY;
  return state_header_bytes(slots) + (size_t)slots * CHUNKS * NT * sizeof(float4);
}

hipError_t launch_render_forward(const clsp_projected& proj, const clsp_bins& bins, int views, int W, int H, int TX,
                                 int TY, const float bg[3], float* image, float* T_final, uint32_t* n_contrib,
                                 void* state, hipStream_t s, const float* target, float* dL, float* loss_sum) {
  const L1Out l1{target, dL, loss_sum};
  const int T = TX * TY;
  const int blocks = views * T;
  const int sliced = bins.mode != CLSP_BINS_COMPLETE;
  const BinPlan plan = make_bin_plan(bins.n, views, W, H, bins.capacity);
  char* ws = static_cast<char*>(bins.ws);
  uint32_t* alive = bin_alive_flags(plan, ws);
  float* carry = bin_carry(plan, ws);
  const int wpv = (T + 31) / 32;
  auto phase = [&](auto kernel) {
    hipLaunchKernelGGL(kernel, dim3(blocks), dim3(NT), 0, s, proj.splat, bins.values, bins.keys,
                       reinterpret_cast<const uint2*>(bins.ranges), reinterpret_cast<uint2*>(bins.ranges2),
                       bins.tile_list, bins.counters, T, TX, W, H, bg[0], bg[1], bg[2], image, T_final, n_contrib,
                       state, (int64_t)blocks, sliced, alive, bins.alive_mask, wpv, carry, l1);
  };
  const bool local = bins.mode == CLSP_BINS_DEPTH_SLICED_LOCAL;
  if (local)
    phase(render_forward_kernel<1, FW_GROUP_LOCAL>);
  else
    phase(render_forward_kernel<1, FW_GROUP>);
  if (!sliced) return hipGetLastError();
  hipError_t err = launch_list_second_slab(plan, proj, bins, ws, s);
  if (err != hipSuccess) return err;
  if (local)
    phase(render_forward_kernel<2, FW_GROUP_LOCAL>);
  else
    phase(render_forward_kernel<2, FW_GROUP>);
  return hipGetLastError();
}

hipError_t launch_l1_loss_grad(const float* image, const float* target, const clsp_bins& bins, int views, int W, int H,
                               int TX, int TY, float* dL, float* loss_sum, hipStream_t s) {
  const int T = TX * TY;
  hipLaunchKernelGGL(l1_loss_grad_kernel, dim3(std::min(views * T, L1_BLOCKS)), dim3(NT), 0, s, image, target,
                     bins.tile_list, bins.counters, T, TX, W, H, dL, loss_sum);
  return hipGetLastError();
}

hipError_t launch_render_backward(const clsp_projected& proj, const clsp_bins& bins, int views, int64_t n, int W,
                                  int H, int TX, int TY, const float bg[3], int64_t a0, int64_t a1,
                                  const float* T_final, const uint32_t* n_contrib, void* state, const float* dL,
                                  float* grad2d, hipStream_t s, bool clear) {
  const int T = TX * TY;
  if (clear) {
    const hipError_t err = launch_fill_u32(reinterpret_cast<uint32_t*>(grad2d), 0u, (a1 - a0) * views * G2D_STRIDE, s);
    if (err != hipSuccess) return err;
  }
  const int grid = (int)std::min<int64_t>((int64_t)views * T * CHUNKS, BWD_BLOCKS);
  hipLaunchKernelGGL(render_backward_kernel, dim3(grid), dim3(NT), 0, s, proj.splat, bins.values,
                     reinterpret_cast<const uint2*>(bins.ranges), reinterpret_cast<const uint2*>(bins.ranges2),
                     bins.tile_list, bins.counters, T, TX, W, H, n,
                     bg[0], bg[1], bg[2], a0, a1, T_final, n_contrib, state, (int64_t)views * T, dL, grad2d);
  return hipGetLastError();
}

}  // namespace clsp
