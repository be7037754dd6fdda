// L1 + D-SSIM loss gradient on the rendered tiles: the default 3D Gaussian Splatting
// loss (1 - lambda) L1 + lambda (1 - SSIM) that the paper trains with (Supp.
// "Implementation Details"), SSIM with an 11 x 11 Gaussian window (sigma 1.5), C1 =
// 0.01^2, C2 = 0.03^2, zero padding at the image border, averaged over channels and
// pixels of the whole image.
//
// One 256-thread workgroup per rendered tile and, in turn, per channel.  The gradient at
// a pixel q is the window sum over p of SSIM(p)'s partials in (mu_x, E[xx], E[xy]), and
// those need the window sums at p, so a tile needs its pixels +- 10: the 36 x 36 region
// is staged in LDS (pixels of unrendered tiles come from the caller's render of the
// frozen Gaussians in local steps: outside the render mask no changed Gaussian reaches,
// so the frozen render is the current image there), the five window sums over the
// 26 x 26 region +- 5 are separable (11 rows, then 11 columns), then the three partial
// maps, then their window sums over the tile.  The sums and partials are in double:
// gfx950 runs FP64 vector arithmetic at the FP32 (non-packed) rate, and the variances
// E[xx] - mu^2 cancel in float32 on flat image regions.
#include "internal.hpp"

namespace clsp {
namespace {

constexpr int NT = TILE_PIX;
constexpr int RW = 5;                 // window radius
constexpr int WS = 2 * RW + 1;        // window size
constexpr int R2 = TILE + 4 * RW;     // 36: tile +- 10 (pixels whose values are read)
constexpr int R1 = TILE + 2 * RW;     // 26: tile +- 5 (pixels whose SSIM is differentiated)
constexpr int C_TILES = 2;

struct SsimConst {
  double g[WS];      // normalised 1D Gaussian window
  double c1, c2;
  double lam;        // weight of the D-SSIM term
  double inv_n;      // 1 / (3 H W)
};

__device__ __forceinline__ bool tile_rendered(const uint32_t* __restrict__ mask_v, int x, int y, int TX) {
  const int t = (y >> 4) * TX + (x >> 4);
  return (mask_v[t >> 5] >> (t & 31)) & 1u;
}

__global__ void __launch_bounds__(NT) l1_dssim_kernel(const float* __restrict__ image, const float* __restrict__ target,
                                                      const float* __restrict__ frozen,
                                                      const uint32_t* __restrict__ tile_list,
                                                      const uint32_t* __restrict__ tile_mask,
                                                      const uint32_t* __restrict__ counters, int T, int TX, int W,
                                                      int H, int wpv, SsimConst k, float* __restrict__ dL,
                                                      float* __restrict__ loss_sum) {
  const uint32_t slot = blockIdx.x;
  if (slot >= counters[C_TILES]) return;
  __shared__ float xs[R2 * R2], ys[R2 * R2];
  __shared__ double h[R2 * R1];          // one quantity's row sums; then the partials' row sums
  __shared__ double st[5 * R1 * R1];     // mu_x, mu_y, E[xx], E[yy], E[xy]; then row sums of the partials
  __shared__ double gm[3 * R1 * R1];     // partials of SSIM(p) in mu_x, E[xx], E[xy]
  __shared__ double s_red[NT / 64];
  const uint32_t gt = tile_list[slot];
  const int v = gt / T, t = gt % T;
  const int X0 = (t % TX) * TILE, Y0 = (t / TX) * TILE;
  const uint32_t* mask_v = tile_mask + (size_t)v * wpv;
  const size_t hw = (size_t)H * W;
  const int qx = X0 + (int)(threadIdx.x & 15u), qy = Y0 + (int)(threadIdx.x >> 4);
  const bool q_in = qx < W && qy < H;
  double loss = 0.0;
  for (int c = 0; c < 3; ++c) {
    const float* img = image + ((size_t)v * 3 + c) * hw;
    const float* tgt = target + ((size_t)v * 3 + c) * hw;
    const float* frz = frozen ? frozen + ((size_t)v * 3 + c) * hw : nullptr;
    for (int e = threadIdx.x; e < R2 * R2; e += NT) {
      const int x = X0 - 2 * RW + e % R2, y = Y0 - 2 * RW + e / R2;
      float xv = 0.0f, yv = 0.0f;
      if (x >= 0 && y >= 0 && x < W && y < H) {
        const size_t o = (size_t)y * W + x;
        xv = (frz && !tile_rendered(mask_v, x, y, TX)) ? frz[o] : img[o];
        yv = tgt[o];
      }
      xs[e] = xv;
      ys[e] = yv;
    }
    __syncthreads();
    // window sums of x, y, xx, yy, xy over the 26 x 26 region
    for (int qi = 0; qi < 5; ++qi) {
      for (int e = threadIdx.x; e < R2 * R1; e += NT) {
        const int r = e / R1, j = e % R1;
        double acc = 0.0;
        for (int m = 0; m < WS; ++m) {
          const double a = xs[r * R2 + j + m], b = ys[r * R2 + j + m];
          const double f = qi == 0 ? a : qi == 1 ? b : qi == 2 ? a * a : qi == 3 ? b * b : a * b;
          acc = fma(k.g[m], f, acc);
        }
        h[e] = acc;
      }
      __syncthreads();
      for (int e = threadIdx.x; e < R1 * R1; e += NT) {
        const int i = e / R1, j = e % R1;
        double acc = 0.0;
        for (int m = 0; m < WS; ++m) acc = fma(k.g[m], h[(i + m) * R1 + j], acc);
        st[qi * R1 * R1 + e] = acc;
      }
      __syncthreads();
    }
    // SSIM(p) and its partials; zero outside the image (the mean runs over image pixels)
    for (int e = threadIdx.x; e < R1 * R1; e += NT) {
      const int px = X0 - RW + e % R1, py = Y0 - RW + e / R1;
      double d_mx = 0.0, d_exx = 0.0, d_exy = 0.0;
      if (px >= 0 && py >= 0 && px < W && py < H) {
        const double mx = st[e], my = st[R1 * R1 + e], exx = st[2 * R1 * R1 + e], eyy = st[3 * R1 * R1 + e],
                     exy = st[4 * R1 * R1 + e];
        const double A = 2.0 * mx * my + k.c1;
        const double B = 2.0 * (exy - mx * my) + k.c2;
        const double C = mx * mx + my * my + k.c1;
        const double D = (exx - mx * mx) + (eyy - my * my) + k.c2;
        const double s = A * B / (C * D);
        d_mx = (2.0 * my * B - 2.0 * my * A) / (C * D) - s * (2.0 * mx / C - 2.0 * mx / D);
        d_exx = -s / D;
        d_exy = 2.0 * A / (C * D);
        const int ti = e / R1 - RW, tj = e % R1 - RW;   // a pixel of this tile: its loss
        if (ti >= 0 && tj >= 0 && ti < TILE && tj < TILE) loss += k.lam * (1.0 - s);
      }
      gm[e] = d_mx;
      gm[R1 * R1 + e] = d_exx;
      gm[2 * R1 * R1 + e] = d_exy;
    }
    __syncthreads();
    // window sums of the partial maps over the tile: rows, then columns
    for (int e = threadIdx.x; e < 3 * R1 * TILE; e += NT) {
      const int map = e / (R1 * TILE), r = (e / TILE) % R1, j = e % TILE;
      double acc = 0.0;
      for (int m = 0; m < WS; ++m) acc = fma(k.g[m], gm[map * R1 * R1 + r * R1 + j + m], acc);
      st[e] = acc;
    }
    __syncthreads();
    if (q_in) {
      const int i = threadIdx.x >> 4, j = threadIdx.x & 15;
      double sm = 0.0, sxx = 0.0, sxy = 0.0;
      for (int m = 0; m < WS; ++m) {
        sm = fma(k.g[m], st[(i + m) * TILE + j], sm);
        sxx = fma(k.g[m], st[R1 * TILE + (i + m) * TILE + j], sxx);
        sxy = fma(k.g[m], st[2 * R1 * TILE + (i + m) * TILE + j], sxy);
      }
      const double x = xs[(i + 2 * RW) * R2 + j + 2 * RW], y = ys[(i + 2 * RW) * R2 + j + 2 * RW];
      const double g_ssim = sm + 2.0 * x * sxx + y * sxy;
      const double sgn = x > y ? 1.0 : (x < y ? -1.0 : 0.0);
      const double g = ((1.0 - k.lam) * sgn - k.lam * g_ssim) * k.inv_n;
      dL[((size_t)v * 3 + c) * hw + (size_t)qy * W + qx] = (float)g;
      loss += (1.0 - k.lam) * fabs(x - y);
    }
    __syncthreads();
  }
  if (loss_sum) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) loss += __shfl_xor(loss, o, 64);
    if ((threadIdx.x & 63u) == 0) s_red[threadIdx.x >> 6] = loss;
    __syncthreads();
    if (threadIdx.x == 0) atomicAdd(loss_sum, (float)((s_red[0] + s_red[1] + s_red[2] + s_red[3]) * k.inv_n));
  }
}

}  // namespace

hipError_t launch_l1_dssim(const float* image, const float* target, const float* frozen, const clsp_bins& bins,
                           int views, int W, int H, int TX, int TY, float lam, float* dL, float* loss_sum,
                           hipStream_t s) {
  SsimConst k;
  double sum = 0.0;
  for (int m = 0; m < WS; ++m) {
    const double i = m - RW;
    k.g[m] = exp(-(i * i) / (2.0 * CLSP_SSIM_SIGMA * CLSP_SSIM_SIGMA));
    sum += k.g[m];
  }
  for (int m = 0; m < WS; ++m) k.g[m] /= sum;
  k.c1 = CLSP_SSIM_C1;
  k.c2 = CLSP_SSIM_C2;
  k.lam = lam;
  k.inv_n = 1.0 / (3.0 * (double)W * (double)H);
  const int T = TX * TY;
  hipLaunchKernelGGL(l1_dssim_kernel, dim3(views * T), dim3(NT), 0, s, image, target, frozen, bins.tile_list,
                     bins.tile_mask, bins.counters, T, TX, W, H, (T + 31) / 32, k, dL, loss_sum);
  return hipGetLastError();
}

}  // namespace clsp
