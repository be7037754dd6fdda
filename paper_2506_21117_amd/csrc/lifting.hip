// Lifting 2D change masks to the 3D change set: mask dilation (Supp. "Detecting Changes
// in 2D": dilate by 2% of the image width with a kernel of ones, threshold at 0) and the
// majority vote over the views (Supp. "Identifying Changed 3D Regions via Majority
// Voting": g_i is changed iff 4/3 o_i < |I| < 2 c_i, c_i the views whose mask holds the
// projected centre, o_i those whose image it falls outside).
//
// Dilation is separable for a square kernel: "some 1 in the square" = "some row of the
// square holds a 1".  Pass 1, one workgroup per image row: the row's prefix counts in
// LDS, each pixel tests its window [x - r, x + r] with two reads.  Pass 2, one thread
// per (column, run of 32 rows): a window count over [y - r, y + r] slid down the run,
// the loads of neighbouring threads coalesced along the row.
//
// Vote: one thread per Gaussian, up to VOTE_VIEWS cameras per launch (passed by value);
// the counts accumulate over launches and the last one decides.
#include "internal.hpp"

namespace clsp {
namespace {

constexpr int NT = 256;
constexpr int RUN = 32;          // rows per thread in the vertical pass
constexpr int VOTE_VIEWS = 16;   // cameras per vote launch

__global__ void __launch_bounds__(NT) dilate_rows_kernel(const uint8_t* __restrict__ m, int W, int H, int r,
                                                        uint8_t* __restrict__ out) {
  extern __shared__ uint16_t pre[];   // [W + 1] prefix counts of the row
  __shared__ uint32_t s_wave[NT / 64];
  const int y = blockIdx.x, v = blockIdx.y;
  const uint8_t* row = m + ((size_t)v * H + y) * W;
  uint8_t* orow = out + ((size_t)v * H + y) * W;
  // each thread sums a contiguous piece of the row, then an exclusive scan over threads
  const int per = (W + NT - 1) / NT;
  const int x0 = min(W, (int)threadIdx.x * per), x1 = min(W, x0 + per);
  uint32_t sum = 0;
  for (int x = x0; x < x1; ++x) sum += row[x] ? 1u : 0u;
  uint32_t inc = sum;
  const uint32_t lane = threadIdx.x & 63u;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t t = __shfl_up(inc, o, 64);
    if (lane >= (uint32_t)o) inc += t;
  }
  if (lane == 63) s_wave[threadIdx.x >> 6] = inc;
  __syncthreads();
  uint32_t base = 0;
  for (int w = 0; w < (int)(threadIdx.x >> 6); ++w) base += s_wave[w];
  uint32_t acc = base + inc - sum;
  for (int x = x0; x < x1; ++x) {
    pre[x] = (uint16_t)acc;
    acc += row[x] ? 1u : 0u;
  }
  if (threadIdx.x == NT - 1) pre[W] = (uint16_t)acc;   // the last thread's running count is the row total
  __syncthreads();
  for (int x = threadIdx.x; x < W; x += NT) {
    const int a = max(0, x - r), b = min(W, x + r + 1);
    orow[x] = pre[b] != pre[a] ? 1 : 0;
  }
}

__global__ void __launch_bounds__(NT) dilate_cols_kernel(const uint8_t* __restrict__ m, int W, int H, int r,
                                                        uint8_t* __restrict__ out) {
  const int64_t t = (int64_t)blockIdx.x * NT + threadIdx.x;
  const int runs = (H + RUN - 1) / RUN;
  const int v = blockIdx.y;
  if (t >= (int64_t)W * runs) return;
  const int x = (int)(t % W), y0 = (int)(t / W) * RUN;
  const uint8_t* col = m + (size_t)v * H * W + x;
  uint8_t* ocol = out + (size_t)v * H * W + x;
  int cnt = 0;
  for (int y = max(0, y0 - r); y <= min(H - 1, y0 + r); ++y) cnt += col[(size_t)y * W] ? 1 : 0;
  const int y1 = min(H, y0 + RUN);
  for (int y = y0; y < y1; ++y) {
    ocol[(size_t)y * W] = cnt > 0 ? 1 : 0;
    const int ya = y + r + 1, yb = y - r;
    if (ya < H) cnt += col[(size_t)ya * W] ? 1 : 0;
    if (yb >= 0) cnt -= col[(size_t)yb * W] ? 1 : 0;
  }
}

struct VoteCams {
  float R[VOTE_VIEWS][9];
  float t[VOTE_VIEWS][3];
  float f[VOTE_VIEWS][4];    // fx, fy, cx, cy
  int count;                 // cameras in this launch
  int first;                 // index of the first (its mask is masks[first])
  int W, H;
};

__global__ void __launch_bounds__(NT) vote_kernel(const float* __restrict__ means, int64_t nr, int64_t n, VoteCams vc,
                                                  const uint8_t* __restrict__ masks, uint8_t* __restrict__ c_in,
                                                  uint8_t* __restrict__ c_out, uint8_t* __restrict__ changed,
                                                  uint32_t* __restrict__ n_changed, int total_views, int last) {
  const int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x;
  bool ch = false;
  if (i < n) {
    const float x = means[i], y = means[nr + i], z = means[2 * nr + i];
    int cin = vc.first == 0 ? 0 : c_in[i];
    int cout = vc.first == 0 ? 0 : c_out[i];
    for (int k = 0; k < vc.count; ++k) {
#pragma clang fp contract(off)
      const float* R = vc.R[k];
      const float X = ((R[0] * x + R[1] * y) + R[2] * z) + vc.t[k][0];
      const float Y = ((R[3] * x + R[4] * y) + R[5] * z) + vc.t[k][1];
      const float Z = ((R[6] * x + R[7] * y) + R[8] * z) + vc.t[k][2];
      bool inside = Z > NEAR_Z;
      float u = 0.0f, v = 0.0f;
      if (inside) {
        u = (vc.f[k][0] * X) / Z + vc.f[k][2];
        v = (vc.f[k][1] * Y) / Z + vc.f[k][3];
        inside = u >= 0.0f && u < (float)vc.W && v >= 0.0f && v < (float)vc.H;
      }
      if (!inside) {
        ++cout;
      } else {
        const int px = (int)floorf(u), py = (int)floorf(v);
        if (masks[((size_t)(vc.first + k) * vc.H + py) * vc.W + px]) ++cin;
      }
    }
    c_in[i] = (uint8_t)cin;
    c_out[i] = (uint8_t)cout;
    if (last) {
      ch = 4 * cout < 3 * total_views && total_views < 2 * cin;
      changed[i] = ch ? 1 : 0;
    }
  }
  if (last) {
    const uint32_t k = (uint32_t)__syncthreads_count(ch);
    if (threadIdx.x == 0 && k) atomicAdd(n_changed, k);
  }
}

}  // namespace

size_t dilate_workspace_bytes(int views, int W, int H) { return (size_t)views * W * H; }

hipError_t launch_dilate_masks(const uint8_t* masks, int views, int W, int H, int r, uint8_t* out, void* ws,
                               hipStream_t s) {
  uint8_t* mid = static_cast<uint8_t*>(ws);
  hipLaunchKernelGGL(dilate_rows_kernel, dim3(H, views), dim3(NT), (size_t)(W + 1) * 2, s, masks, W, H, r, mid);
  const int64_t threads = (int64_t)W * ((H + RUN - 1) / RUN);
  hipLaunchKernelGGL(dilate_cols_kernel, dim3(ceil_div(threads, NT), views), dim3(NT), 0, s, mid, W, H, r, out);
  return hipGetLastError();
}

hipError_t launch_majority_vote(const float* means, int64_t nr, int64_t n, const DevCam* cams, int views,
                                const uint8_t* masks, uint8_t* c_in, uint8_t* c_out, uint8_t* changed,
                                uint32_t* n_changed, hipStream_t s) {
  hipError_t e = launch_fill_u32(n_changed, 0u, 1, s);
  if (e != hipSuccess || n == 0) return e;
  for (int first = 0; first < views; first += VOTE_VIEWS) {
    VoteCams vc;
    vc.count = std::min(VOTE_VIEWS, views - first);
    vc.first = first;
    vc.W = cams[0].W;
    vc.H = cams[0].H;
    for (int k = 0; k < vc.count; ++k) {
      const DevCam& c = cams[first + k];
      for (int j = 0; j < 9; ++j) vc.R[k][j] = c.R[j];
      for (int j = 0; j < 3; ++j) vc.t[k][j] = c.t[j];
      vc.f[k][0] = c.fx;
      vc.f[k][1] = c.fy;
      vc.f[k][2] = c.cx;
      vc.f[k][3] = c.cy;
    }
    const int last = first + VOTE_VIEWS >= views;
    hipLaunchKernelGGL(vote_kernel, dim3(ceil_div(n, NT)), dim3(NT), 0, s, means, nr, n, vc, masks, c_in, c_out,
                       changed, n_changed, views, last);
  }
  return hipGetLastError();
}

}  // namespace clsp
