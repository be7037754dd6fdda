// History operations on the resident Gaussians (Supp. "History Recovery", alg:example;
// Supp. "Batched Updates").
//
//   reorder: before optimising a step, the unchanged Gaussians (indicator 0) are moved
//            first and the changed ones after them, both in their order, so the change
//            set is the contiguous suffix and G^t[:#static] is the static part of G^{t-1};
//   recover: G^{k-1} from G^k, I^k and O^k: O^k where I^k is 1, the first #static rows of
//            G^k, in order, where it is 0;
//   merge:   two concurrent updates: the rows of G^{t-1} neither update changed, then
//            O_1, then O_2.
//
// All three are row copies whose positions are exclusive ranks of a 0/1 indicator:
// per-block counts of the ones, then each block adds the counts of the blocks before it
// to its own block scan.  Every parameter component is copied (component-major rows, so
// neighbouring threads touch neighbouring addresses of each component).
#include <algorithm>

#include "internal.hpp"

namespace clsp {
namespace {

constexpr int NT = 256;
constexpr int MAX_BLOCKS = 1024;

__device__ __forceinline__ void span_of(int64_t n, int G, int b, int64_t& beg, int64_t& end) {
  const int64_t per = (n + G - 1) / G;
  beg = min(n, (int64_t)b * per);
  end = min(n, beg + per);
}

__device__ __forceinline__ bool flag_at(const uint8_t* f1, const uint8_t* f2, int64_t i) {
  return f1[i] != 0 || (f2 && f2[i] != 0);
}

__device__ __forceinline__ void copy_row(const MutParams& src, int64_t from, const MutParams& dst, int64_t to,
                                         int comps) {
  for (int c = 0; c < comps; ++c) component(dst, c)[to] = component(src, c)[from];
}

// blk[b] = ones of f1 | f2 in block b's span of [0, n)
__global__ void __launch_bounds__(NT) ones_count_kernel(const uint8_t* __restrict__ f1, const uint8_t* __restrict__ f2,
                                                        int64_t n, int G, uint32_t* __restrict__ blk) {
  int64_t beg, end;
  span_of(n, G, blockIdx.x, beg, end);
  uint32_t c = 0;
  for (int64_t i = beg + threadIdx.x; i < end; i += NT) c += flag_at(f1, f2, i) ? 1u : 0u;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o, 64);
  __shared__ uint32_t s4[4];
  if ((threadIdx.x & 63u) == 0) s4[threadIdx.x >> 6] = c;
  __syncthreads();
  if (threadIdx.x == 0) blk[blockIdx.x] = s4[0] + s4[1] + s4[2] + s4[3];
}

// Ones before block b and over all blocks.
__device__ __forceinline__ void block_bases(const uint32_t* __restrict__ blk, int G, uint32_t& before,
                                            uint32_t& total) {
  __shared__ uint32_t s_b[2];
  if (threadIdx.x == 0) {
    uint32_t a = 0, t = 0;
    for (int j = 0; j < G; ++j) {
      if (j == (int)blockIdx.x) a = t;
      t += blk[j];
    }
    s_b[0] = a;
    s_b[1] = t;
  }
  __syncthreads();
  before = s_b[0];
  total = s_b[1];
  __syncthreads();
}

// Exclusive scan of k (0/1) over the block; returns the rank and adds the block's total
// to `tot`.
__device__ __forceinline__ uint32_t block_rank(uint32_t k, uint32_t& tot) {
  __shared__ uint32_t s4[4];
  uint32_t inc = k;
  const uint32_t lane = threadIdx.x & 63u;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t y = __shfl_up(inc, o, 64);
    if (lane >= (uint32_t)o) inc += y;
  }
  const int w = threadIdx.x >> 6;
  if (lane == 63) s4[w] = inc;
  __syncthreads();
  uint32_t off = 0;
  for (int j = 0; j < w; ++j) off += s4[j];
  tot = s4[0] + s4[1] + s4[2] + s4[3];
  __syncthreads();
  return off + inc - k;
}

enum { REORDER = 0, RECOVER = 1, MERGE = 2 };

// REORDER: src row i -> dst row (ind ? zeros + rank1 : rank0).
// RECOVER: dst row i <- ind ? b[rank1] : a[rank0].
// MERGE:   src row i with neither flag -> dst row rank0.
template <int MODE>
__global__ void __launch_bounds__(NT) rank_copy_kernel(MutParams a, MutParams b, MutParams dst, int comps,
                                                       const uint8_t* __restrict__ f1, const uint8_t* __restrict__ f2,
                                                       int64_t n, int G, const uint32_t* __restrict__ blk,
                                                       uint32_t* __restrict__ zeros_out) {
  uint32_t ones_before, ones_total;
  block_bases(blk, G, ones_before, ones_total);
  int64_t beg, end;
  span_of(n, G, blockIdx.x, beg, end);
  const uint32_t zeros_total = (uint32_t)(n - ones_total);
  if (blockIdx.x == 0 && threadIdx.x == 0 && zeros_out) *zeros_out = zeros_total;
  uint32_t r1 = ones_before;                         // ones before this round
  uint32_t r0 = (uint32_t)beg - ones_before;         // zeros before this round
  for (int64_t i0 = beg; i0 < end; i0 += NT) {
    const int64_t i = i0 + threadIdx.x;
    const bool in = i < end;
    const bool one = in && flag_at(f1, f2, i);
    uint32_t t1;
    const uint32_t k1 = block_rank(one ? 1u : 0u, t1);
    const uint32_t k0 = (uint32_t)threadIdx.x - k1;   // zeros before this thread in the round
    if (in) {
      if (MODE == REORDER) {
        const int64_t to = one ? (int64_t)zeros_total + r1 + k1 : (int64_t)r0 + k0;
        if (to < dst.n) copy_row(a, i, dst, to, comps);
      } else if (MODE == RECOVER) {
        if (i < dst.n) {
          if (one) {
            const int64_t from = (int64_t)r1 + k1;
            if (from < b.n) copy_row(b, from, dst, i, comps);
          } else {
            const int64_t from = (int64_t)r0 + k0;
            if (from < a.n) copy_row(a, from, dst, i, comps);
          }
        }
      } else {
        const int64_t to = (int64_t)r0 + k0;
        if (!one && to < dst.n) copy_row(a, i, dst, to, comps);
      }
    }
    const uint32_t cnt = min((int64_t)NT, end - i0);
    r1 += t1;
    r0 += cnt - t1;
  }
}

// dst rows zeros + offset + j <- src row j (the merge's appended updates), zeros from the
// block counts.
__global__ void __launch_bounds__(NT) append_kernel(MutParams src, MutParams dst, int comps, int64_t offset,
                                                    int64_t n_prev, int G, const uint32_t* __restrict__ blk) {
  __shared__ uint32_t s_t;
  if (threadIdx.x == 0) {
    uint32_t t = 0;
    for (int j = 0; j < G; ++j) t += blk[j];
    s_t = t;
  }
  __syncthreads();
  const int64_t zeros = n_prev - s_t;
  for (int64_t j = (int64_t)blockIdx.x * NT + threadIdx.x; j < src.n; j += (int64_t)gridDim.x * NT) {
    const int64_t to = zeros + offset + j;
    if (to < dst.n) copy_row(src, j, dst, to, comps);
  }
}

int blocks_for(int64_t n) { return (int)std::max<int64_t>(1, std::min<int64_t>(MAX_BLOCKS, ceil_div(n, 4 * NT))); }
int comps_of(const MutParams& p) { return 11 + 3 * (p.sh_degree + 1) * (p.sh_degree + 1); }

}  // namespace

size_t history_workspace_bytes() { return (size_t)MAX_BLOCKS * 4; }

hipError_t launch_reorder_static_first(const MutParams& src, const uint8_t* changed, const MutParams& dst,
                                       uint32_t* n_static, void* ws, hipStream_t s) {
  hipError_t e = launch_fill_u32(n_static, (uint32_t)src.n, 1, s);
  if (e != hipSuccess || src.n == 0) return e;
  const int G = blocks_for(src.n);
  uint32_t* blk = static_cast<uint32_t*>(ws);
  hipLaunchKernelGGL(ones_count_kernel, dim3(G), dim3(NT), 0, s, changed, nullptr, src.n, G, blk);
  hipLaunchKernelGGL(rank_copy_kernel<REORDER>, dim3(G), dim3(NT), 0, s, src, src, dst, comps_of(src), changed,
                     nullptr, src.n, G, blk, n_static);
  return hipGetLastError();
}

hipError_t launch_recover_previous(const MutParams& latest, const uint8_t* ind, const MutParams& older,
                                   const MutParams& dst, void* ws, hipStream_t s) {
  if (dst.n == 0) return hipSuccess;
  const int G = blocks_for(dst.n);
  uint32_t* blk = static_cast<uint32_t*>(ws);
  hipLaunchKernelGGL(ones_count_kernel, dim3(G), dim3(NT), 0, s, ind, nullptr, dst.n, G, blk);
  hipLaunchKernelGGL(rank_copy_kernel<RECOVER>, dim3(G), dim3(NT), 0, s, latest, older, dst, comps_of(dst), ind,
                     nullptr, dst.n, G, blk, nullptr);
  return hipGetLastError();
}

hipError_t launch_merge_updates(const MutParams& prev, const uint8_t* ind1, const uint8_t* ind2, const MutParams& o1,
                                const MutParams& o2, const MutParams& dst, void* ws, hipStream_t s) {
  const int G = blocks_for(prev.n);
  uint32_t* blk = static_cast<uint32_t*>(ws);
  const int comps = comps_of(dst);
  if (prev.n > 0) {
    hipLaunchKernelGGL(ones_count_kernel, dim3(G), dim3(NT), 0, s, ind1, ind2, prev.n, G, blk);
    hipLaunchKernelGGL(rank_copy_kernel<MERGE>, dim3(G), dim3(NT), 0, s, prev, prev, dst, comps, ind1, ind2, prev.n, G,
                       blk, nullptr);
  } else {
    hipError_t e = launch_fill_u32(blk, 0u, G, s);
    if (e != hipSuccess) return e;
  }
  if (o1.n > 0)
    hipLaunchKernelGGL(append_kernel, dim3((unsigned)std::min<int64_t>(ceil_div(o1.n, NT), 1024)), dim3(NT), 0, s, o1,
                       dst, comps, (int64_t)0, prev.n, G, blk);
  if (o2.n > 0)
    hipLaunchKernelGGL(append_kernel, dim3((unsigned)std::min<int64_t>(ceil_div(o2.n, NT), 1024)), dim3(NT), 0, s, o2,
                       dst, comps, o1.n, prev.n, G, blk);
  return hipGetLastError();
}

}  // namespace clsp
