// Change-region spheres: fit, membership and compaction of the change set.
//
// The changed Gaussians O^t are clustered (outside this library) and one sphere is
// fitted per cluster: centre = mean of the cluster's centres, radius = 1.1 x the 98th
// percentile of their distances to it (Supp. "Identifying Changed 3D Regions via
// Majority Voting").  During local optimisation the changed Gaussians whose centre has
// left every sphere are removed (Sec. 3.3 "Sphere Pruning"; Supp. "3DGS Optimization in
// Changed Regions": a check every 15 iterations), and the change set is compacted so it
// stays the contiguous suffix after the static prefix (Supp. "History Recovery").
//
// fit:      one workgroup per sphere.  The mean is a block reduction in double over the
//           change set in a fixed order (deterministic); the two order statistics around
//           the percentile are found by 8-bit radix selection over the float32 distances
//           (four histogram passes each, recomputing the distances), so nothing is sorted
//           or stored per point.
// keep:     one thread per changed row, the spheres in LDS.
// compact:  per-block counts of the kept rows, then each block scans its rows and copies
//           the kept ones (every parameter component, and the Adam moments) to their
//           place in the destination; the static prefix is copied as it is.
#include "internal.hpp"

namespace clsp {
namespace {

constexpr int NT = 256;
constexpr int MAX_COMPACT_BLOCKS = 1024;

// Distance of a centre to a sphere centre, float32, no contraction (the order of the
// oracle's float32 evaluation of the same quantities).
__device__ __forceinline__ float dist2(float x, float y, float z, float cx, float cy, float cz) {
#pragma clang fp contract(off)
  const float dx = x - cx, dy = y - cy, dz = z - cz;
  return (dx * dx + dy * dy) + dz * dz;
}

__device__ __forceinline__ double block_sum_double(double x, double* s4) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
  __syncthreads();
  if ((threadIdx.x & 63u) == 0) s4[threadIdx.x >> 6] = x;
  __syncthreads();
  return (s4[0] + s4[1]) + (s4[2] + s4[3]);
}

// The k-th smallest (0-based) distance of sphere s's points, by radix selection over the
// distances' bit patterns (non-negative floats order like their bits).
__device__ uint32_t select_distance(const float* __restrict__ means, int64_t nr, int64_t a0, int64_t a1,
                                    const int32_t* __restrict__ labels, int s, float cx, float cy, float cz,
                                    uint32_t k, uint32_t* hist, uint32_t* s_pick) {
  uint32_t prefix = 0, mask = 0, rank = k;
  for (int shift = 24; shift >= 0; shift -= 8) {
    for (int b = threadIdx.x; b < 256; b += NT) hist[b] = 0;
    __syncthreads();
    for (int64_t i = a0 + threadIdx.x; i < a1; i += NT) {
      if (labels[i - a0] != s) continue;
      const float d = sqrtf(dist2(means[i], means[nr + i], means[2 * nr + i], cx, cy, cz));
      const uint32_t bits = __float_as_uint(d);
      if ((bits & mask) == prefix) atomicAdd(&hist[(bits >> shift) & 255u], 1u);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      uint32_t acc = 0, digit = 255;
      for (uint32_t b = 0; b < 256; ++b) {
        if (acc + hist[b] > rank) {
          digit = b;
          break;
        }
        acc += hist[b];
      }
      s_pick[0] = digit;
      s_pick[1] = acc;
    }
    __syncthreads();
    prefix |= s_pick[0] << shift;
    mask |= 255u << shift;
    rank -= s_pick[1];
    __syncthreads();
  }
  return prefix;
}

__global__ void __launch_bounds__(NT) fit_spheres_kernel(const float* __restrict__ means, int64_t nr, int64_t a0,
                                                         int64_t a1, const int32_t* __restrict__ labels,
                                                         float* __restrict__ centers, float* __restrict__ radii) {
  __shared__ double s4[4];
  __shared__ uint32_t hist[256];
  __shared__ uint32_t s_pick[2];
  const int s = blockIdx.x;
  double sx = 0.0, sy = 0.0, sz = 0.0, sc = 0.0;
  for (int64_t i = a0 + threadIdx.x; i < a1; i += NT) {
    if (labels[i - a0] != s) continue;
    sx += (double)means[i];
    sy += (double)means[nr + i];
    sz += (double)means[2 * nr + i];
    sc += 1.0;
  }
  sx = block_sum_double(sx, s4);
  sy = block_sum_double(sy, s4);
  sz = block_sum_double(sz, s4);
  const uint32_t c = (uint32_t)block_sum_double(sc, s4);
  if (c == 0) {
    if (threadIdx.x == 0) {
      centers[3 * s] = centers[3 * s + 1] = centers[3 * s + 2] = 0.0f;
      radii[s] = -1.0f;
    }
    return;
  }
  const float cx = (float)(sx / c), cy = (float)(sy / c), cz = (float)(sz / c);
  // q = 0.98 (c - 1): the percentile between the order statistics floor(q) and floor(q) + 1
  const double q = (double)CLSP_SPHERE_QUANTILE * (double)(c - 1);
  const uint32_t lo = (uint32_t)floor(q);
  const double frac = q - (double)lo;
  const float d_lo = __uint_as_float(select_distance(means, nr, a0, a1, labels, s, cx, cy, cz, lo, hist, s_pick));
  float d_hi = d_lo;
  if (lo + 1 < c && frac > 0.0)
    d_hi = __uint_as_float(select_distance(means, nr, a0, a1, labels, s, cx, cy, cz, lo + 1, hist, s_pick));
  if (threadIdx.x == 0) {
    centers[3 * s] = cx;
    centers[3 * s + 1] = cy;
    centers[3 * s + 2] = cz;
    radii[s] = (float)((double)CLSP_SPHERE_SCALE * ((double)d_lo + frac * ((double)d_hi - (double)d_lo)));
  }
}

__global__ void __launch_bounds__(NT) sphere_keep_kernel(const float* __restrict__ means, int64_t nr, int64_t a0,
                                                         int64_t a1, const float* __restrict__ centers,
                                                         const float* __restrict__ radii, int ns,
                                                         uint8_t* __restrict__ keep, uint32_t* __restrict__ kept) {
  extern __shared__ float s_sph[];   // [ns][4]: centre, r^2 (negative: contains nothing)
  for (int j = threadIdx.x; j < ns; j += NT) {
#pragma clang fp contract(off)
    const float r = radii[j];
    s_sph[4 * j] = centers[3 * j];
    s_sph[4 * j + 1] = centers[3 * j + 1];
    s_sph[4 * j + 2] = centers[3 * j + 2];
    s_sph[4 * j + 3] = r < 0.0f ? -1.0f : r * r;
  }
  __syncthreads();
  const int64_t i = a0 + (int64_t)blockIdx.x * NT + threadIdx.x;
  bool in = false;
  if (i < a1) {
    const float x = means[i], y = means[nr + i], z = means[2 * nr + i];
    for (int j = 0; j < ns && !in; ++j) {
      const float r2 = s_sph[4 * j + 3];
      in = r2 >= 0.0f && dist2(x, y, z, s_sph[4 * j], s_sph[4 * j + 1], s_sph[4 * j + 2]) <= r2;
    }
    keep[i - a0] = in ? 1 : 0;
  }
  const uint32_t cnt = (uint32_t)__syncthreads_count(in);
  if (threadIdx.x == 0 && cnt) atomicAdd(kept, cnt);
}

struct CompactSets {
  MutParams src[3], dst[3];
  int sets;        // 1: parameters only; 3: with both Adam moments
  int comps;       // components per row
};

__device__ __forceinline__ void copy_row(const CompactSets& cs, int64_t from, int64_t to) {
  for (int k = 0; k < cs.sets; ++k)
    for (int c = 0; c < cs.comps; ++c) component(cs.dst[k], c)[to] = component(cs.src[k], c)[from];
}

__device__ __forceinline__ void span_of(int64_t n, int G, int b, int64_t& beg, int64_t& end) {
  const int64_t per = (n + G - 1) / G;
  beg = min(n, (int64_t)b * per);
  end = min(n, beg + per);
}

__global__ void __launch_bounds__(NT) compact_count_kernel(const uint8_t* __restrict__ keep, int64_t na, int G,
                                                           uint32_t* __restrict__ blk) {
  int64_t beg, end;
  span_of(na, G, blockIdx.x, beg, end);
  uint32_t c = 0;
  for (int64_t i = beg + threadIdx.x; i < end; i += NT) c += keep[i] ? 1u : 0u;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o, 64);
  __shared__ uint32_t s4[4];
  if ((threadIdx.x & 63u) == 0) s4[threadIdx.x >> 6] = c;
  __syncthreads();
  if (threadIdx.x == 0) blk[blockIdx.x] = s4[0] + s4[1] + s4[2] + s4[3];
}

// Block b copies its kept rows to a0 + (kept rows before it) + (their rank in it); rows
// at or past dst_n are not written.
__global__ void __launch_bounds__(NT) compact_scatter_kernel(CompactSets cs, const uint8_t* __restrict__ keep,
                                                             int64_t a0, int64_t na, int G,
                                                             const uint32_t* __restrict__ blk, int64_t dst_n) {
  __shared__ uint32_t s4[4];
  __shared__ uint32_t s_base;
  if (threadIdx.x == 0) {
    uint32_t b = 0;
    for (int j = 0; j < (int)blockIdx.x; ++j) b += blk[j];
    s_base = b;
  }
  __syncthreads();
  uint32_t base = s_base;
  int64_t beg, end;
  span_of(na, G, blockIdx.x, beg, end);
  for (int64_t i0 = beg; i0 < end; i0 += NT) {
    const int64_t i = i0 + threadIdx.x;
    const uint32_t k = (i < end && keep[i]) ? 1u : 0u;
    // exclusive scan of k over the block
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
    const uint32_t tot = s4[0] + s4[1] + s4[2] + s4[3];
    __syncthreads();
    if (k) {
      const int64_t to = a0 + base + off + inc - 1;
      if (to < dst_n) copy_row(cs, a0 + i, to);
    }
    base += tot;
  }
}

__global__ void __launch_bounds__(NT) copy_prefix_kernel(CompactSets cs, int64_t a0) {
  for (int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x; i < a0; i += (int64_t)gridDim.x * NT) copy_row(cs, i, i);
}

}  // namespace

hipError_t launch_fit_spheres(const float* means, int64_t nr, int64_t a0, int64_t a1, const int32_t* labels, int ns,
                              float* centers, float* radii, hipStream_t s) {
  if (ns <= 0) return hipSuccess;
  hipLaunchKernelGGL(fit_spheres_kernel, dim3(ns), dim3(NT), 0, s, means, nr, a0, a1, labels, centers, radii);
  return hipGetLastError();
}

hipError_t launch_sphere_keep(const float* means, int64_t nr, int64_t a0, int64_t a1, const float* centers,
                              const float* radii, int ns, uint8_t* keep, uint32_t* kept, hipStream_t s) {
  hipError_t e = launch_fill_u32(kept, 0u, 1, s);
  if (e != hipSuccess || a1 <= a0) return e;
  hipLaunchKernelGGL(sphere_keep_kernel, dim3(ceil_div(a1 - a0, NT)), dim3(NT), (size_t)ns * 16, s, means, nr, a0, a1,
                     centers, radii, ns, keep, kept);
  return hipGetLastError();
}

size_t compact_workspace_bytes(int64_t na) {
  (void)na;
  return (size_t)MAX_COMPACT_BLOCKS * 4;
}

hipError_t launch_compact_rows(const MutParams src[3], const MutParams dst[3], int sets, int64_t a0, int64_t a1,
                               const uint8_t* keep, void* ws, hipStream_t s) {
  CompactSets cs;
  for (int k = 0; k < 3; ++k) {
    cs.src[k] = src[k];
    cs.dst[k] = dst[k];
  }
  cs.sets = sets;
  cs.comps = 11 + 3 * (src[0].sh_degree + 1) * (src[0].sh_degree + 1);
  if (a0 > 0) {
    hipLaunchKernelGGL(copy_prefix_kernel, dim3((unsigned)std::min<int64_t>(ceil_div(a0, NT), 2048)), dim3(NT), 0, s,
                       cs, a0);
  }
  const int64_t na = a1 - a0;
  if (na > 0) {
    const int G = (int)std::min<int64_t>(MAX_COMPACT_BLOCKS, ceil_div(na, 4 * NT));
    uint32_t* blk = static_cast<uint32_t*>(ws);
    hipLaunchKernelGGL(compact_count_kernel, dim3(G), dim3(NT), 0, s, keep, na, G, blk);
    hipLaunchKernelGGL(compact_scatter_kernel, dim3(G), dim3(NT), 0, s, cs, keep, a0, na, G, blk, dst[0].n);
  }
  return hipGetLastError();
}

}  // namespace clsp
