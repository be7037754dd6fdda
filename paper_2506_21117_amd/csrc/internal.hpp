// Internal declarations of the gfx950 kernels behind the clsplat C-ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "clsplat.h"

namespace clsp {

constexpr int TILE = CLSP_TILE;
constexpr int TILE_PIX = TILE * TILE;  // 256 pixels = one workgroup of four wave64s
constexpr int SPLAT_STRIDE = 12;       // floats per projected record
constexpr int G2D_STRIDE = 12;         // floats per screen-space gradient row (9 used)

// Compositing constants of the forward model.
constexpr float ALPHA_MIN = 1.0f / 255.0f;
constexpr float ALPHA_MAX = 0.99f;
constexpr float T_STOP = 1e-4f;
constexpr float NEAR_Z = 0.2f;
constexpr float LOWPASS = 0.3f;
constexpr float EXTENT_MARGIN = 1.0f + 1.0f / 4096.0f;
// Per-pixel compositing state carried from the first to the second depth slab:
// T, colour of the flushed chunks (3), colour of the current chunk (3), last, done.
constexpr int CARRY_FIELDS = 9;

// Camera as the kernels take it (by value): the C-ABI camera plus derived constants.
struct DevCam {
  float R[9];
  float t[3];
  float fx, fy, cx, cy;
  float limx, limy;      // 1.3 x half-image tangent
  float campos[3];       // camera centre in world space
  int W, H, TX, TY;
};

struct RawParams {
  const float* means;
  const float* log_scales;
  const float* quats;
  const float* opac;
  const float* sh;
  const int32_t* gather;
  int64_t n;
  int64_t n_rows;
  int sh_degree;
};

struct MutParams {
  float* means;
  float* log_scales;
  float* quats;
  float* opac;
  float* sh;
  int64_t n;
  int sh_degree;
};

inline int ceil_div(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }

// Pointer to component c of a parameter set (means 0-2, log_scales 3-5, quats 6-9,
// opacity 10, sh 11..); a row has 11 + 3 (sh_degree + 1)^2 components.
__device__ __forceinline__ float* component(const MutParams& p, int c) {
  if (c < 3) return p.means + (int64_t)c * p.n;
  if (c < 6) return p.log_scales + (int64_t)(c - 3) * p.n;
  if (c < 10) return p.quats + (int64_t)(c - 6) * p.n;
  if (c == 10) return p.opac;
  return p.sh + (int64_t)(c - 11) * p.n;
}

// ---------------------------------------------------------------- launchers
// preprocess.hip
// Projects entries [r0, r1) of view `view` (all n: r0 = 0, r1 = g.n).
hipError_t launch_preprocess(const RawParams& g, const DevCam& cam, int view, int64_t r0, int64_t r1, float* splat,
                             float* depth, uint32_t* rect, uint32_t* flags, hipStream_t s);
// skip (device, nullable): nonzero leaves everything unchanged.
hipError_t launch_preprocess_backward(const RawParams& g, const DevCam& cam, int view, int64_t a0, int64_t a1,
                                      const uint32_t* flags, const float* grad2d, const MutParams& grads,
                                      const uint32_t* skip, hipStream_t s);
// One view's preprocess backward followed by one Adam step of rows [a0, a1).
struct FusedAdam {
  MutParams P, M, V;
  float lr[6];
  float b1, b2, eps;
  float bc1, bc2;            // 1 - beta^step (host step count)
  const int32_t* step_dev;   // device step count, or null
  const uint32_t* skip;      // device flag: nonzero leaves everything unchanged, or null
};
hipError_t launch_preprocess_backward_adam(const RawParams& g, const DevCam& cam, int64_t a0, int64_t a1,
                                           const uint32_t* flags, const float* grad2d, const FusedAdam& A,
                                           hipStream_t s);

// binning.hip
struct BinPlan {
  int64_t n;          // Gaussians per view
  int views;
  int TX, TY, T;      // tiles per view
  int64_t capacity;
  int tile_bits;      // bits of the global tile index
  int64_t entries;    // views * n
  // workspace carve-up (byte offsets)
  size_t off_cnt, off_flag, off_keyA, off_valA, off_keyB, off_valB, off_scanBlk, off_hist, off_digit,
      off_pairK, off_pairV, off_tflag, off_vfirst, off_tab, off_rsort, off_cm, off_alive, off_carry, total;
  int64_t cm_words;   // count matrix of the first slab's counting placement (0: not used)
  size_t off_cmask;
  int64_t cmask_words;  // the depth-sliced first slab's tile masks per (chunk, slot), 64-bit (0: not kept)
  int scan_blocks;
  int sort_blocks_gauss, sort_blocks_pairs;
};
BinPlan make_bin_plan(int64_t n, int views, int W, int H, int64_t capacity);
hipError_t launch_bin_and_sort(const BinPlan& p, const clsp_projected& proj, int64_t a0, int64_t a1, int use_mask,
                               const clsp_bins& bins, char* ws, hipStream_t s);
// Stored depth order of the unchanged rows [0, a0) (see binning.hip), and lists of the
// changed rows [a0, n) built from it.
size_t frozen_order_bytes(int64_t views, int64_t a0);
hipError_t launch_frozen_order(const BinPlan& p, const clsp_projected& proj, int64_t a0, uint32_t* ord, char* ws,
                               hipStream_t s);
hipError_t launch_bin_and_sort_frozen(const BinPlan& p, const clsp_projected& proj, int64_t a0, const uint32_t* ord,
                                      const clsp_bins& bins, char* ws, hipStream_t s);
// Depth-sliced lists: list the second slab into the alive tiles (bins.alive_mask).
hipError_t launch_list_second_slab(const BinPlan& p, const clsp_projected& proj, const clsp_bins& bins, char* ws,
                                   hipStream_t s);
uint32_t* bin_alive_flags(const BinPlan& p, char* ws);
float* bin_carry(const BinPlan& p, char* ws);

// render.hip
size_t render_state_bytes(int views, int TX, int TY);
// With dL given (target too) it also writes the L1 gradient of the rendered pixels and
// adds their loss to *loss_sum (if given), as launch_l1_loss_grad would.
hipError_t launch_render_forward(const clsp_projected& proj, const clsp_bins& bins, int views, int W, int H,
                                 int TX, int TY, const float bg[3], float* image, float* T_final,
                                 uint32_t* n_contrib, void* state, hipStream_t s, const float* target = nullptr,
                                 float* dL = nullptr, float* loss_sum = nullptr);
hipError_t launch_l1_loss_grad(const float* image, const float* target, const clsp_bins& bins, int views, int W,
                               int H, int TX, int TY, float* dL, float* loss_sum, hipStream_t s);
hipError_t launch_render_backward(const clsp_projected& proj, const clsp_bins& bins, int views, int64_t n, int W,
                                  int H, int TX, int TY, const float bg[3], int64_t a0, int64_t a1,
                                  const float* T_final, const uint32_t* n_contrib, void* state, const float* dL,
                                  float* grad2d, hipStream_t s, bool clear = true);
hipError_t launch_fill_u32(uint32_t* p, uint32_t value, int64_t count, hipStream_t s);

// spheres.hip
hipError_t launch_fit_spheres(const float* means, int64_t nr, int64_t a0, int64_t a1, const int32_t* labels, int ns,
                              float* centers, float* radii, hipStream_t s);
hipError_t launch_sphere_keep(const float* means, int64_t nr, int64_t a0, int64_t a1, const float* centers,
                              const float* radii, int ns, uint8_t* keep, uint32_t* kept, hipStream_t s);
size_t compact_workspace_bytes(int64_t na);
// src/dst[0] parameters, [1], [2] the Adam moments (used when sets == 3)
hipError_t launch_compact_rows(const MutParams src[3], const MutParams dst[3], int sets, int64_t a0, int64_t a1,
                               const uint8_t* keep, void* ws, hipStream_t s);

// lifting.hip
size_t dilate_workspace_bytes(int views, int W, int H);
hipError_t launch_dilate_masks(const uint8_t* masks, int views, int W, int H, int r, uint8_t* out, void* ws,
                               hipStream_t s);
hipError_t launch_majority_vote(const float* means, int64_t nr, int64_t n, const DevCam* cams, int views,
                                const uint8_t* masks, uint8_t* c_in, uint8_t* c_out, uint8_t* changed,
                                uint32_t* n_changed, hipStream_t s);

// history.hip
size_t history_workspace_bytes();
// dst = rows of src with changed = 0, then those with 1 (both in order); *n_static = zeros
hipError_t launch_reorder_static_first(const MutParams& src, const uint8_t* changed, const MutParams& dst,
                                       uint32_t* n_static, void* ws, hipStream_t s);
// dst[i] = ind[i] ? older[rank among ones] : latest[rank among zeros], i < dst.n
hipError_t launch_recover_previous(const MutParams& latest, const uint8_t* ind, const MutParams& older,
                                   const MutParams& dst, void* ws, hipStream_t s);
// dst = prev rows with ind1 = ind2 = 0, then o1, then o2
hipError_t launch_merge_updates(const MutParams& prev, const uint8_t* ind1, const uint8_t* ind2, const MutParams& o1,
                                const MutParams& o2, const MutParams& dst, void* ws, hipStream_t s);

// ssim.hip
hipError_t launch_l1_dssim(const float* image, const float* target, const float* frozen, const clsp_bins& bins,
                           int views, int W, int H, int TX, int TY, float lam, float* dL, float* loss_sum,
                           hipStream_t s);

// adam.hip
hipError_t launch_adam(const MutParams& p, const MutParams& g, const MutParams& m, const MutParams& v, int64_t a0,
                       int64_t a1, const uint8_t* row_mask, const clsp_adam_hparams& hp, hipStream_t s);
hipError_t launch_zero_rows(const MutParams& g, int64_t a0, int64_t a1, hipStream_t s);

}  // namespace clsp
