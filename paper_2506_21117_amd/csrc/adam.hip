// Masked Adam and gradient clearing over the rows of the change set (Supp. "3DGS
// Optimization in Changed Regions": only Gaussians of O^t receive gradients and
// optimiser updates, so their first and second moments cannot move the others).
//
// One thread per row; every parameter component is a separate coalesced stream over the
// contiguous row range, so frozen rows are never read or written.
#include "internal.hpp"

namespace clsp {
namespace {

struct AdamConst {
  float lr[6];
  float b1, b2, eps;
  float bc1, bc2;             // 1 - beta^step (host step count)
  const int32_t* step_dev;    // device step count, or null
  int zero_grads;             // clear the gradient rows after use
  const uint32_t* skip;       // device flag: nonzero leaves every buffer unchanged, or null
};

__device__ __forceinline__ void adam_one(float* p, float* g, float* m, float* v, float lr, const AdamConst& h) {
  const float gg = *g;
  if (h.zero_grads) *g = 0.0f;
  const float mm = h.b1 * (*m) + (1.0f - h.b1) * gg;
  const float vv = h.b2 * (*v) + (1.0f - h.b2) * gg * gg;
  *m = mm;
  *v = vv;
  *p -= lr * (mm / h.bc1) / (sqrtf(vv / h.bc2) + h.eps);
}

__global__ void __launch_bounds__(256) adam_kernel(MutParams P, MutParams Gr, MutParams M, MutParams V, int64_t a0,
                                                   int64_t a1, const uint8_t* __restrict__ row_mask, AdamConst h) {
  const int64_t i = a0 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a1 || (h.skip && *h.skip)) return;
  if (row_mask && !row_mask[i]) {
    if (h.zero_grads) {
      const int64_t n = Gr.n;
      for (int c = 0; c < 3; ++c) Gr.means[c * n + i] = 0.0f;
      for (int c = 0; c < 3; ++c) Gr.log_scales[c * n + i] = 0.0f;
      for (int c = 0; c < 4; ++c) Gr.quats[c * n + i] = 0.0f;
      Gr.opac[i] = 0.0f;
      const int K3 = 3 * (Gr.sh_degree + 1) * (Gr.sh_degree + 1);
      for (int c = 0; c < K3; ++c) Gr.sh[(int64_t)c * n + i] = 0.0f;
    }
    return;
  }
  if (h.step_dev) {
    const float t = (float)max(*h.step_dev, 1);
    h.bc1 = 1.0f - powf(h.b1, t);
    h.bc2 = 1.0f - powf(h.b2, t);
  }
  const int64_t n = P.n;
  for (int c = 0; c < 3; ++c) adam_one(P.means + c * n + i, Gr.means + c * n + i, M.means + c * n + i, V.means + c * n + i, h.lr[0], h);
  for (int c = 0; c < 3; ++c)
    adam_one(P.log_scales + c * n + i, Gr.log_scales + c * n + i, M.log_scales + c * n + i, V.log_scales + c * n + i,
             h.lr[1], h);
  for (int c = 0; c < 4; ++c) adam_one(P.quats + c * n + i, Gr.quats + c * n + i, M.quats + c * n + i, V.quats + c * n + i, h.lr[2], h);
  adam_one(P.opac + i, Gr.opac + i, M.opac + i, V.opac + i, h.lr[3], h);
  const int K3 = 3 * (P.sh_degree + 1) * (P.sh_degree + 1);
  for (int c = 0; c < K3; ++c) {
    const int64_t o = (int64_t)c * n + i;
    adam_one(P.sh + o, Gr.sh + o, M.sh + o, V.sh + o, c < 3 ? h.lr[4] : h.lr[5], h);
  }
}

__global__ void __launch_bounds__(256) zero_rows_kernel(MutParams G, int64_t a0, int64_t a1) {
  const int64_t i = a0 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a1) return;
  const int64_t n = G.n;
  for (int c = 0; c < 3; ++c) G.means[c * n + i] = 0.0f;
  for (int c = 0; c < 3; ++c) G.log_scales[c * n + i] = 0.0f;
  for (int c = 0; c < 4; ++c) G.quats[c * n + i] = 0.0f;
  G.opac[i] = 0.0f;
  const int K3 = 3 * (G.sh_degree + 1) * (G.sh_degree + 1);
  for (int c = 0; c < K3; ++c) G.sh[(int64_t)c * n + i] = 0.0f;
}

}  // namespace

hipError_t launch_adam(const MutParams& p, const MutParams& g, const MutParams& m, const MutParams& v, int64_t a0,
                       int64_t a1, const uint8_t* row_mask, const clsp_adam_hparams& hp, hipStream_t s) {
  if (a1 <= a0) return hipSuccess;
  AdamConst h;
  for (int k = 0; k < 6; ++k) h.lr[k] = hp.lr[k];
  h.b1 = hp.beta1;
  h.b2 = hp.beta2;
  h.eps = hp.eps;
  h.bc1 = (float)(1.0 - pow((double)hp.beta1, (double)hp.step));
  h.bc2 = (float)(1.0 - pow((double)hp.beta2, (double)hp.step));
  h.step_dev = hp.step_device;
  h.zero_grads = hp.zero_grads;
  h.skip = hp.skip_flag;
  hipLaunchKernelGGL(adam_kernel, dim3(ceil_div(a1 - a0, 256)), dim3(256), 0, s, p, g, m, v, a0, a1, row_mask, h);
  return hipGetLastError();
}

hipError_t launch_zero_rows(const MutParams& g, int64_t a0, int64_t a1, hipStream_t s) {
  if (a1 <= a0) return hipSuccess;
  hipLaunchKernelGGL(zero_rows_kernel, dim3(ceil_div(a1 - a0, 256)), dim3(256), 0, s, g, a0, a1);
  return hipGetLastError();
}

}  // namespace clsp
