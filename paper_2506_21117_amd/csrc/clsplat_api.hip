// extern "C" entry points of libclsplat: argument validation on the host, derived
// camera constants, workspace carve-up, and launches on the caller's stream.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>

#include <mutex>

#include "internal.hpp"

// Screen-space gradient scratch of clsp_render_backward_noalloc, one copy per GPU.  In
// host code this name stands for the variable, not for its device address: host code
// passes only the address hipGetSymbolAddress returned for the current device.
static __device__ __align__(256) float scratch[CLSP_NOALLOC_SCRATCH_BYTES / sizeof(float)];

namespace {

thread_local char g_err[512] = "";

clsp_status fail(clsp_status code, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof g_err, fmt, ap);
  va_end(ap);
  return code;
}

clsp_status hip_status(hipError_t e, const char* where) {
  if (e == hipSuccess) return CLSP_OK;
  return fail(CLSP_ERR_HIP, "%s: %s", where, hipGetErrorString(e));
}

constexpr int64_t MAX_ENTRIES = 0xffffffffLL;
constexpr int MAX_TILES_PER_VIEW = 65536;

clsp_status check_cams(const clsp_camera* cams, int32_t n_views) {
  if (!cams) return fail(CLSP_ERR_INVALID_ARG, "cams is NULL");
  if (n_views < 1 || n_views > CLSP_MAX_VIEWS) return fail(CLSP_ERR_INVALID_ARG, "n_views=%d not in 1..%d", n_views, CLSP_MAX_VIEWS);
  const int W = cams[0].width, H = cams[0].height;
  if (W < 1 || H < 1 || W > CLSP_MAX_SIDE || H > CLSP_MAX_SIDE)
    return fail(CLSP_ERR_INVALID_ARG, "image size %dx%d not in 1..%d", W, H, CLSP_MAX_SIDE);
  const int TX = (W + CLSP_TILE - 1) / CLSP_TILE, TY = (H + CLSP_TILE - 1) / CLSP_TILE;
  if (TX * TY > MAX_TILES_PER_VIEW) return fail(CLSP_ERR_INVALID_ARG, "more than %d tiles per view", MAX_TILES_PER_VIEW);
  for (int v = 0; v < n_views; ++v) {
    const clsp_camera& c = cams[v];
    if (c.width != W || c.height != H) return fail(CLSP_ERR_INVALID_ARG, "view %d size differs from view 0", v);
    if (!(c.fx > 0.f) || !(c.fy > 0.f) || !isfinite(c.fx) || !isfinite(c.fy) || !isfinite(c.cx) || !isfinite(c.cy))
      return fail(CLSP_ERR_INVALID_ARG, "view %d has invalid intrinsics", v);
    for (int k = 0; k < 9; ++k)
      if (!isfinite(c.R[k])) return fail(CLSP_ERR_INVALID_ARG, "view %d rotation not finite", v);
    for (int k = 0; k < 3; ++k)
      if (!isfinite(c.t[k])) return fail(CLSP_ERR_INVALID_ARG, "view %d translation not finite", v);
  }
  return CLSP_OK;
}

clsp::DevCam dev_cam(const clsp_camera& c) {
  clsp::DevCam d;
  for (int k = 0; k < 9; ++k) d.R[k] = c.R[k];
  for (int k = 0; k < 3; ++k) d.t[k] = c.t[k];
  d.fx = c.fx;
  d.fy = c.fy;
  d.cx = c.cx;
  d.cy = c.cy;
  d.W = c.width;
  d.H = c.height;
  d.TX = (c.width + CLSP_TILE - 1) / CLSP_TILE;
  d.TY = (c.height + CLSP_TILE - 1) / CLSP_TILE;
  d.limx = 1.3f * (0.5f * (float)c.width) / c.fx;
  d.limy = 1.3f * (0.5f * (float)c.height) / c.fy;
  for (int k = 0; k < 3; ++k) d.campos[k] = -(c.R[k] * c.t[0] + c.R[3 + k] * c.t[1] + c.R[6 + k] * c.t[2]);
  return d;
}

clsp_status check_gaussians(const clsp_gaussians* g) {
  if (!g) return fail(CLSP_ERR_INVALID_ARG, "gaussians is NULL");
  if (g->n < 0) return fail(CLSP_ERR_INVALID_ARG, "n=%lld < 0", (long long)g->n);
  if (g->sh_degree < 0 || g->sh_degree > 3) return fail(CLSP_ERR_INVALID_ARG, "sh_degree=%d not in 0..3", g->sh_degree);
  if (g->n > 0) {
    if (!g->means || !g->log_scales || !g->quats || !g->opacity_logit || !g->sh)
      return fail(CLSP_ERR_INVALID_ARG, "a Gaussian parameter pointer is NULL");
    if (!g->gather && g->n_rows < g->n) return fail(CLSP_ERR_INVALID_ARG, "n_rows < n without gather");
    if (g->gather && g->n_rows < 1) return fail(CLSP_ERR_INVALID_ARG, "n_rows < 1 with gather");
  }
  return CLSP_OK;
}

clsp::RawParams raw_params(const clsp_gaussians* g) {
  clsp::RawParams r;
  r.means = g->means;
  r.log_scales = g->log_scales;
  r.quats = g->quats;
  r.opac = g->opacity_logit;
  r.sh = g->sh;
  r.gather = g->gather;
  r.n = g->n;
  r.n_rows = g->n_rows;
  r.sh_degree = g->sh_degree;
  return r;
}

clsp_status check_params(const clsp_params* p, const char* what) {
  if (!p) return fail(CLSP_ERR_INVALID_ARG, "%s is NULL", what);
  if (p->n < 0) return fail(CLSP_ERR_INVALID_ARG, "%s: n < 0", what);
  if (p->sh_degree < 0 || p->sh_degree > 3) return fail(CLSP_ERR_INVALID_ARG, "%s: sh_degree not in 0..3", what);
  if (p->n > 0 && (!p->means || !p->log_scales || !p->quats || !p->opacity_logit || !p->sh))
    return fail(CLSP_ERR_INVALID_ARG, "%s: a pointer is NULL", what);
  return CLSP_OK;
}

clsp::MutParams mut_params(const clsp_params* p) {
  clsp::MutParams m;
  m.means = p->means;
  m.log_scales = p->log_scales;
  m.quats = p->quats;
  m.opac = p->opacity_logit;
  m.sh = p->sh;
  m.n = p->n;
  m.sh_degree = p->sh_degree;
  return m;
}

clsp_status check_range(clsp_range r, int64_t n) {
  if (r.begin < 0 || r.end < r.begin || r.end > n)
    return fail(CLSP_ERR_INVALID_ARG, "active range [%lld, %lld) not inside [0, %lld]", (long long)r.begin,
                (long long)r.end, (long long)n);
  return CLSP_OK;
}

clsp_status check_projected(const clsp_projected* p) {
  if (!p || !p->splat || !p->depth || !p->rect || !p->flags) return fail(CLSP_ERR_INVALID_ARG, "projected buffers missing");
  return CLSP_OK;
}

clsp_status check_bins(const clsp_bins* b) {
  if (!b || !b->values || !b->keys || !b->ranges || !b->ranges2 || !b->tile_mask || !b->alive_mask || !b->tile_list ||
      !b->counters)
    return fail(CLSP_ERR_INVALID_ARG, "bins buffers missing");
  if (b->capacity < 0 || b->capacity > MAX_ENTRIES) return fail(CLSP_ERR_INVALID_ARG, "capacity not in 0..2^32-1");
  if (b->mode != CLSP_BINS_COMPLETE && b->mode != CLSP_BINS_DEPTH_SLICED && b->mode != CLSP_BINS_DEPTH_SLICED_LOCAL)
    return fail(CLSP_ERR_INVALID_ARG, "unknown bins mode %d", b->mode);
  if (b->n < 0) return fail(CLSP_ERR_INVALID_ARG, "bins n < 0");
  return CLSP_OK;
}

// The bins' workspace must hold the plan for these views and this capacity.
clsp_status check_bins_ws(const clsp_bins* b, const clsp::BinPlan& plan) {
  if (!b->ws || b->ws_bytes < plan.total)
    return fail(CLSP_ERR_INVALID_ARG, "bins workspace of %zu bytes is smaller than the %zu needed", b->ws_bytes,
                plan.total);
  return CLSP_OK;
}

#define CHECK(x)                        \
  do {                                  \
    clsp_status _s = (x);               \
    if (_s != CLSP_OK) return _s;       \
  } while (0)

// Device address of `scratch` on each GPU, looked up on the first call made with that
// GPU current.
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
float* g_scratch_ptr[MAX_DEVICES] = {};

clsp_status scratch_for_stream(hipStream_t s, float** out) {
  int dev = -1;
  CHECK(hip_status(hipGetDevice(&dev), "hipGetDevice"));
  if (dev < 0 || dev >= MAX_DEVICES) return fail(CLSP_ERR_UNSUPPORTED, "device %d beyond the %d supported", dev, MAX_DEVICES);
  if (s) {
    hipDevice_t sdev = -1;
    CHECK(hip_status(hipStreamGetDevice(s, &sdev), "hipStreamGetDevice"));
    if (sdev != dev)
      return fail(CLSP_ERR_INVALID_ARG, "stream belongs to device %d but device %d is current", (int)sdev, dev);
  }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    CHECK(hip_status(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)"));
    if (!p) return fail(CLSP_ERR_HIP, "hipGetSymbolAddress(scratch) returned NULL");
    g_scratch_ptr[dev] = static_cast<float*>(p);
  }
  *out = g_scratch_ptr[dev];
  return CLSP_OK;
}

// Validation shared by clsp_render_backward and clsp_render_backward_noalloc.
clsp_status check_render_backward(const clsp_gaussians* g, const clsp_projected* proj, const clsp_bins* bins,
                                  const clsp_camera* cams, int32_t n_views, const float* bg, clsp_range active,
                                  const float* T_final, const uint32_t* n_contrib, const void* state,
                                  size_t state_bytes, const float* dL_dimage, const clsp_params* grads) {
  CHECK(check_gaussians(g));
  if (g->gather) return fail(CLSP_ERR_INVALID_ARG, "render_backward needs un-gathered parameters");
  CHECK(check_projected(proj));
  CHECK(check_bins(bins));
  CHECK(check_cams(cams, n_views));
  CHECK(check_params(grads, "grads"));
  CHECK(check_range(active, g->n));
  if (grads->n != g->n || grads->sh_degree != g->sh_degree)
    return fail(CLSP_ERR_INVALID_ARG, "grads layout differs from the parameters");
  if (!bg || !T_final || !n_contrib || !dL_dimage) return fail(CLSP_ERR_INVALID_ARG, "render_backward input is NULL");
  if (!state || state_bytes < clsp_render_state_bytes(n_views, cams[0].width, cams[0].height))
    return fail(CLSP_ERR_INVALID_ARG, "render_backward needs the forward's state (%zu bytes)",
                clsp_render_state_bytes(n_views, cams[0].width, cams[0].height));
  return CLSP_OK;
}

// The raster backward into g2d (cleared first), then the preprocess backward per view.
clsp_status run_render_backward(const clsp_gaussians* g, const clsp_projected* proj, const clsp_bins* bins,
                                const clsp_camera* cams, int32_t n_views, const float* bg, clsp_range active,
                                const float* T_final, const uint32_t* n_contrib, const void* state,
                                const float* dL_dimage, const clsp_params* grads, float* g2d, hipStream_t s,
                                const char* what) {
  const int W = cams[0].width, H = cams[0].height;
  const int TX = (W + CLSP_TILE - 1) / CLSP_TILE, TY = (H + CLSP_TILE - 1) / CLSP_TILE;
  CHECK(hip_status(clsp::launch_render_backward(*proj, *bins, n_views, g->n, W, H, TX, TY, bg, active.begin,
                                                active.end, T_final, n_contrib, const_cast<void*>(state), dL_dimage,
                                                g2d, s),
                   what));
  const clsp::RawParams rp = raw_params(g);
  const clsp::MutParams gm = mut_params(grads);
  for (int v = 0; v < n_views; ++v)
    CHECK(hip_status(clsp::launch_preprocess_backward(rp, dev_cam(cams[v]), v, active.begin, active.end, proj->flags,
                                                      g2d, gm, bins->counters + 1, s),
                     what));
  return CLSP_OK;
}

}  // namespace

extern "C" {

const char* clsp_version(void) { return "clsplat 0.1 gfx950"; }

const char* clsp_last_error(void) { return g_err; }

clsp_status clsp_project_preprocess(const clsp_gaussians* g, const clsp_camera* cams, int32_t n_views,
                                    const clsp_projected* out, clsp_stream stream) {
  CHECK(check_gaussians(g));
  CHECK(check_cams(cams, n_views));
  CHECK(check_projected(out));
  if ((int64_t)n_views * g->n > MAX_ENTRIES) return fail(CLSP_ERR_INVALID_ARG, "n_views * n >= 2^32");
  const clsp::RawParams rp = raw_params(g);
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  for (int v = 0; v < n_views; ++v)
    CHECK(hip_status(clsp::launch_preprocess(rp, dev_cam(cams[v]), v, 0, g->n, out->splat, out->depth, out->rect,
                                             out->flags, s),
                     "project_preprocess"));
  return CLSP_OK;
}

clsp_status clsp_project_preprocess_rows(const clsp_gaussians* g, const clsp_camera* cams, int32_t n_views,
                                         clsp_range rows, const clsp_projected* out, clsp_stream stream) {
  CHECK(check_gaussians(g));
  CHECK(check_cams(cams, n_views));
  CHECK(check_projected(out));
  if ((int64_t)n_views * g->n > MAX_ENTRIES) return fail(CLSP_ERR_INVALID_ARG, "n_views * n >= 2^32");
  if (rows.begin < 0 || rows.end < rows.begin || rows.end > g->n)
    return fail(CLSP_ERR_INVALID_ARG, "rows [%lld, %lld) not within [0, %lld]", (long long)rows.begin,
                (long long)rows.end, (long long)g->n);
  const clsp::RawParams rp = raw_params(g);
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  for (int v = 0; v < n_views; ++v)
    CHECK(hip_status(clsp::launch_preprocess(rp, dev_cam(cams[v]), v, rows.begin, rows.end, out->splat, out->depth,
                                             out->rect, out->flags, s),
                     "project_preprocess_rows"));
  return CLSP_OK;
}

size_t clsp_bin_and_sort_workspace_bytes(int64_t n, int32_t n_views, int32_t width, int32_t height, int64_t capacity) {
  if (n < 0 || n_views < 1 || width < 1 || height < 1 || capacity < 0) return 0;
  return clsp::make_bin_plan(n, n_views, width, height, capacity).total;
}

clsp_status clsp_bin_and_sort(const clsp_projected* proj, const clsp_camera* cams, int32_t n_views, clsp_range active,
                              int32_t use_mask, const clsp_bins* bins, clsp_stream stream) {
  CHECK(check_projected(proj));
  CHECK(check_cams(cams, n_views));
  CHECK(check_bins(bins));
  const int64_t n = bins->n;
  if ((int64_t)n_views * n > MAX_ENTRIES) return fail(CLSP_ERR_INVALID_ARG, "n_views * n >= 2^32");
  CHECK(check_range(active, n));
  const clsp::BinPlan plan = clsp::make_bin_plan(n, n_views, cams[0].width, cams[0].height, bins->capacity);
  CHECK(check_bins_ws(bins, plan));
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  return hip_status(clsp::launch_bin_and_sort(plan, *proj, active.begin, active.end, use_mask ? 1 : 0, *bins,
                                              static_cast<char*>(bins->ws), s),
                    "bin_and_sort");
}

size_t clsp_frozen_order_bytes(int64_t n, int32_t n_views, int64_t a0) {
  if (n < 0 || n_views < 1 || a0 < 0 || a0 > n || (int64_t)n_views * n > MAX_ENTRIES) return 0;
  return clsp::frozen_order_bytes(n_views, a0);
}

clsp_status clsp_frozen_order(const clsp_projected* proj, const clsp_camera* cams, int32_t n_views, int64_t n,
                              int64_t a0, void* order, size_t order_bytes, void* ws, size_t ws_bytes,
                              clsp_stream stream) {
  CHECK(check_projected(proj));
  CHECK(check_cams(cams, n_views));
  if (n < 0 || (int64_t)n_views * n > MAX_ENTRIES) return fail(CLSP_ERR_INVALID_ARG, "n < 0 or n_views * n >= 2^32");
  if (a0 < 0 || a0 > n) return fail(CLSP_ERR_INVALID_ARG, "a0 = %lld not in [0, %lld]", (long long)a0, (long long)n);
  if (!order || order_bytes < clsp::frozen_order_bytes(n_views, a0))
    return fail(CLSP_ERR_INVALID_ARG, "order buffer of %zu bytes is smaller than the %zu needed", order_bytes,
                clsp::frozen_order_bytes(n_views, a0));
  const clsp::BinPlan plan = clsp::make_bin_plan(n, n_views, cams[0].width, cams[0].height, 0);
  if (!ws || ws_bytes < plan.total)
    return fail(CLSP_ERR_INVALID_ARG, "workspace of %zu bytes is smaller than the %zu needed", ws_bytes, plan.total);
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  return hip_status(clsp::launch_frozen_order(plan, *proj, a0, static_cast<uint32_t*>(order), static_cast<char*>(ws), s),
                    "frozen_order");
}

clsp_status clsp_bin_and_sort_frozen(const clsp_projected* proj, const clsp_camera* cams, int32_t n_views, int64_t a0,
                                     const void* order, size_t order_bytes, const clsp_bins* bins,
                                     clsp_stream stream) {
  CHECK(check_projected(proj));
  CHECK(check_cams(cams, n_views));
  CHECK(check_bins(bins));
  const int64_t n = bins->n;
  if ((int64_t)n_views * n > MAX_ENTRIES) return fail(CLSP_ERR_INVALID_ARG, "n_views * n >= 2^32");
  if (a0 < 0 || a0 > n) return fail(CLSP_ERR_INVALID_ARG, "a0 = %lld not in [0, %lld]", (long long)a0, (long long)n);
  if (!order || order_bytes < clsp::frozen_order_bytes(n_views, a0))
    return fail(CLSP_ERR_INVALID_ARG, "order buffer of %zu bytes is smaller than the %zu needed", order_bytes,
                clsp::frozen_order_bytes(n_views, a0));
  const clsp::BinPlan plan = clsp::make_bin_plan(n, n_views, cams[0].width, cams[0].height, bins->capacity);
  CHECK(check_bins_ws(bins, plan));
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  return hip_status(clsp::launch_bin_and_sort_frozen(plan, *proj, a0, static_cast<const uint32_t*>(order), *bins,
                                                     static_cast<char*>(bins->ws), s),
                    "bin_and_sort_frozen");
}

size_t clsp_render_state_bytes(int32_t n_views, int32_t width, int32_t height) {
  if (n_views < 1 || width < 1 || height < 1) return 0;
  return clsp::render_state_bytes(n_views, (width + CLSP_TILE - 1) / CLSP_TILE, (height + CLSP_TILE - 1) / CLSP_TILE);
}

clsp_status clsp_render_forward(const clsp_projected* proj, const clsp_bins* bins, const clsp_camera* cams,
                                int32_t n_views, const float* bg, float* image, float* T_final, uint32_t* n_contrib,
                                void* state, size_t state_bytes, clsp_stream stream) {
  CHECK(check_projected(proj));
  CHECK(check_bins(bins));
  CHECK(check_cams(cams, n_views));
  if (!bg || !image || !T_final || !n_contrib) return fail(CLSP_ERR_INVALID_ARG, "render_forward output or bg is NULL");
  const int W = cams[0].width, H = cams[0].height;
  if (state && state_bytes < clsp_render_state_bytes(n_views, W, H))
    return fail(CLSP_ERR_INVALID_ARG, "state of %zu bytes is smaller than the %zu needed", state_bytes,
                clsp_render_state_bytes(n_views, W, H));
  CHECK(check_bins_ws(bins, clsp::make_bin_plan(bins->n, n_views, W, H, bins->capacity)));
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  return hip_status(clsp::launch_render_forward(*proj, *bins, n_views, W, H, (W + CLSP_TILE - 1) / CLSP_TILE,
                                                (H + CLSP_TILE - 1) / CLSP_TILE, bg, image, T_final, n_contrib,
                                                state, s),
                    "render_forward");
}

clsp_status clsp_render_forward_l1(const clsp_projected* proj, const clsp_bins* bins, const clsp_camera* cams,
                                   int32_t n_views, const float* bg, const float* target, float* image, float* T_final,
                                   uint32_t* n_contrib, void* state, size_t state_bytes, float* dL_dimage,
                                   float* loss_sum, clsp_stream stream) {
  CHECK(check_projected(proj));
  CHECK(check_bins(bins));
  CHECK(check_cams(cams, n_views));
  if (!bg || !image || !T_final || !n_contrib || !target || !dL_dimage)
    return fail(CLSP_ERR_INVALID_ARG, "render_forward_l1 input, output or bg is NULL");
  const int W = cams[0].width, H = cams[0].height;
  if (state && state_bytes < clsp_render_state_bytes(n_views, W, H))
    return fail(CLSP_ERR_INVALID_ARG, "state of %zu bytes is smaller than the %zu needed", state_bytes,
                clsp_render_state_bytes(n_views, W, H));
  CHECK(check_bins_ws(bins, clsp::make_bin_plan(bins->n, n_views, W, H, bins->capacity)));
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  return hip_status(clsp::launch_render_forward(*proj, *bins, n_views, W, H, (W + CLSP_TILE - 1) / CLSP_TILE,
                                                (H + CLSP_TILE - 1) / CLSP_TILE, bg, image, T_final, n_contrib,
                                                state, s, target, dL_dimage, loss_sum),
                    "render_forward_l1");
}

clsp_status clsp_l1_loss_grad(const float* image, const float* target, const clsp_bins* bins, const clsp_camera* cams,
                              int32_t n_views, float* dL_dimage, float* loss_sum, clsp_stream stream) {
  CHECK(check_bins(bins));
  CHECK(check_cams(cams, n_views));
  if (!image || !target || !dL_dimage) return fail(CLSP_ERR_INVALID_ARG, "l1_loss_grad pointer is NULL");
  const int W = cams[0].width, H = cams[0].height;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  return hip_status(clsp::launch_l1_loss_grad(image, target, *bins, n_views, W, H, (W + CLSP_TILE - 1) / CLSP_TILE,
                                              (H + CLSP_TILE - 1) / CLSP_TILE, dL_dimage, loss_sum, s),
                    "l1_loss_grad");
}

clsp_status clsp_l1_dssim_loss_grad(const float* image, const float* target, const float* frozen_image,
                                    const clsp_bins* bins, const clsp_camera* cams, int32_t n_views, float lambda,
                                    float* dL_dimage, float* loss_sum, clsp_stream stream) {
  CHECK(check_bins(bins));
  CHECK(check_cams(cams, n_views));
  if (!image || !target || !dL_dimage) return fail(CLSP_ERR_INVALID_ARG, "l1_dssim_loss_grad pointer is NULL");
  if (!(lambda >= 0.0f && lambda <= 1.0f)) return fail(CLSP_ERR_INVALID_ARG, "lambda not in [0, 1]");
  const int W = cams[0].width, H = cams[0].height;
  return hip_status(clsp::launch_l1_dssim(image, target, frozen_image, *bins, n_views, W, H,
                                          (W + CLSP_TILE - 1) / CLSP_TILE, (H + CLSP_TILE - 1) / CLSP_TILE, lambda,
                                          dL_dimage, loss_sum, reinterpret_cast<hipStream_t>(stream)),
                    "l1_dssim_loss_grad");
}

size_t clsp_render_backward_workspace_bytes(int64_t n_active, int32_t n_views) {
  if (n_active < 0 || n_views < 1) return 0;
  return (size_t)n_active * n_views * clsp::G2D_STRIDE * sizeof(float);
}

clsp_status clsp_render_backward(const clsp_gaussians* g, const clsp_projected* proj, const clsp_bins* bins,
                                 const clsp_camera* cams, int32_t n_views, const float* bg, clsp_range active,
                                 const float* T_final, const uint32_t* n_contrib, const void* state,
                                 size_t state_bytes, const float* dL_dimage, const clsp_params* grads, void* ws,
                                 size_t ws_bytes, clsp_stream stream) {
  CHECK(check_render_backward(g, proj, bins, cams, n_views, bg, active, T_final, n_contrib, state, state_bytes,
                              dL_dimage, grads));
  const int64_t na = active.end - active.begin;
  const size_t need = clsp_render_backward_workspace_bytes(na, n_views);
  if (na > 0 && (!ws || ws_bytes < need))
    return fail(CLSP_ERR_INVALID_ARG, "workspace of %zu bytes is smaller than the %zu needed", ws_bytes, need);
  if (na == 0) return CLSP_OK;
  return run_render_backward(g, proj, bins, cams, n_views, bg, active, T_final, n_contrib, state, dL_dimage, grads,
                             static_cast<float*>(ws), reinterpret_cast<hipStream_t>(stream), "render_backward");
}

clsp_status clsp_render_backward_noalloc(const clsp_gaussians* g, const clsp_projected* proj, const clsp_bins* bins,
                                         const clsp_camera* cams, int32_t n_views, const float* bg, clsp_range active,
                                         const float* T_final, const uint32_t* n_contrib, const void* state,
                                         size_t state_bytes, const float* dL_dimage, const clsp_params* grads,
                                         clsp_stream stream) {
  CHECK(check_render_backward(g, proj, bins, cams, n_views, bg, active, T_final, n_contrib, state, state_bytes,
                              dL_dimage, grads));
  const int64_t na = active.end - active.begin;
  const size_t need = clsp_render_backward_workspace_bytes(na, n_views);
  if (need > CLSP_NOALLOC_SCRATCH_BYTES)
    return fail(CLSP_ERR_INVALID_ARG,
                "render_backward_noalloc: %lld active Gaussians x %d views need %zu bytes of scratch, more than its "
                "%zu (at most %lld active Gaussian-views)",
                (long long)na, n_views, need, (size_t)CLSP_NOALLOC_SCRATCH_BYTES,
                (long long)(CLSP_NOALLOC_SCRATCH_BYTES / clsp_render_backward_workspace_bytes(1, 1)));
  if (na == 0) return CLSP_OK;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  float* g2d = nullptr;
  CHECK(scratch_for_stream(s, &g2d));
  return run_render_backward(g, proj, bins, cams, n_views, bg, active, T_final, n_contrib, state, dL_dimage, grads,
                             g2d, s, "render_backward_noalloc");
}

clsp_status clsp_masked_adam_step(const clsp_params* params, const clsp_params* grads, const clsp_params* exp_avg,
                                  const clsp_params* exp_avg_sq, clsp_range active, const uint8_t* row_mask,
                                  const clsp_adam_hparams* hp, clsp_stream stream) {
  CHECK(check_params(params, "params"));
  CHECK(check_params(grads, "grads"));
  CHECK(check_params(exp_avg, "exp_avg"));
  CHECK(check_params(exp_avg_sq, "exp_avg_sq"));
  if (!hp) return fail(CLSP_ERR_INVALID_ARG, "hparams is NULL");
  const int64_t n = params->n;
  if (grads->n != n || exp_avg->n != n || exp_avg_sq->n != n || grads->sh_degree != params->sh_degree ||
      exp_avg->sh_degree != params->sh_degree || exp_avg_sq->sh_degree != params->sh_degree)
    return fail(CLSP_ERR_INVALID_ARG, "params, grads and moments differ in layout");
  CHECK(check_range(active, n));
  if (!hp->step_device && hp->step < 1) return fail(CLSP_ERR_INVALID_ARG, "step must be >= 1");
  if (!(hp->beta1 >= 0.f && hp->beta1 < 1.f && hp->beta2 >= 0.f && hp->beta2 < 1.f && hp->eps >= 0.f))
    return fail(CLSP_ERR_INVALID_ARG, "invalid Adam betas or eps");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  return hip_status(clsp::launch_adam(mut_params(params), mut_params(grads), mut_params(exp_avg), mut_params(exp_avg_sq),
                                      active.begin, active.end, row_mask, *hp, s),
                    "masked_adam_step");
}

clsp_status clsp_render_backward_adam(const clsp_gaussians* g, const clsp_projected* proj, const clsp_bins* bins,
                                      const clsp_camera* cams, int32_t n_views, const float* bg, clsp_range active,
                                      const float* T_final, const uint32_t* n_contrib, const void* state,
                                      size_t state_bytes, const float* dL_dimage, const clsp_params* params,
                                      const clsp_params* exp_avg, const clsp_params* exp_avg_sq,
                                      const clsp_adam_hparams* hp, void* ws, size_t ws_bytes, clsp_stream stream) {
  CHECK(check_gaussians(g));
  if (g->gather) return fail(CLSP_ERR_INVALID_ARG, "render_backward_adam needs un-gathered parameters");
  CHECK(check_projected(proj));
  CHECK(check_bins(bins));
  CHECK(check_cams(cams, n_views));
  if (n_views != 1) return fail(CLSP_ERR_INVALID_ARG, "render_backward_adam takes one view (n_views=%d)", n_views);
  CHECK(check_params(params, "params"));
  CHECK(check_params(exp_avg, "exp_avg"));
  CHECK(check_params(exp_avg_sq, "exp_avg_sq"));
  CHECK(check_range(active, g->n));
  if (params->n != g->n || params->sh_degree != g->sh_degree || exp_avg->n != g->n || exp_avg_sq->n != g->n ||
      exp_avg->sh_degree != g->sh_degree || exp_avg_sq->sh_degree != g->sh_degree)
    return fail(CLSP_ERR_INVALID_ARG, "params and moments differ in layout from the parameters");
  if (!hp) return fail(CLSP_ERR_INVALID_ARG, "hparams is NULL");
  if (!hp->step_device && hp->step < 1) return fail(CLSP_ERR_INVALID_ARG, "step must be >= 1");
  if (!(hp->beta1 >= 0.f && hp->beta1 < 1.f && hp->beta2 >= 0.f && hp->beta2 < 1.f && hp->eps >= 0.f))
    return fail(CLSP_ERR_INVALID_ARG, "invalid Adam betas or eps");
  if (!bg || !T_final || !n_contrib || !dL_dimage)
    return fail(CLSP_ERR_INVALID_ARG, "render_backward_adam input is NULL");
  if (!state || state_bytes < clsp_render_state_bytes(n_views, cams[0].width, cams[0].height))
    return fail(CLSP_ERR_INVALID_ARG, "render_backward_adam needs the forward's state (%zu bytes)",
                clsp_render_state_bytes(n_views, cams[0].width, cams[0].height));
  const int64_t na = active.end - active.begin;
  const size_t need = clsp_render_backward_workspace_bytes(na, n_views);
  if (na > 0 && (!ws || ws_bytes < need))
    return fail(CLSP_ERR_INVALID_ARG, "workspace of %zu bytes is smaller than the %zu needed", ws_bytes, need);
  if (na == 0) return CLSP_OK;
  const int W = cams[0].width, H = cams[0].height;
  const int TX = (W + CLSP_TILE - 1) / CLSP_TILE, TY = (H + CLSP_TILE - 1) / CLSP_TILE;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  float* g2d = static_cast<float*>(ws);
  // the workspace is zero on entry (and left zero below): no clearing launch
  CHECK(hip_status(clsp::launch_render_backward(*proj, *bins, n_views, g->n, W, H, TX, TY, bg, active.begin,
                                                active.end, T_final, n_contrib, const_cast<void*>(state), dL_dimage,
                                                g2d, s, false),
                   "render_backward_adam"));
  clsp::FusedAdam A;
  A.P = mut_params(params);
  A.M = mut_params(exp_avg);
  A.V = mut_params(exp_avg_sq);
  for (int k = 0; k < 6; ++k) A.lr[k] = hp->lr[k];
  A.b1 = hp->beta1;
  A.b2 = hp->beta2;
  A.eps = hp->eps;
  A.bc1 = (float)(1.0 - pow((double)hp->beta1, (double)hp->step));
  A.bc2 = (float)(1.0 - pow((double)hp->beta2, (double)hp->step));
  A.step_dev = hp->step_device;
  A.skip = bins->counters + 1;   // pair-capacity overflow of the step's lists
  return hip_status(clsp::launch_preprocess_backward_adam(raw_params(g), dev_cam(cams[0]), active.begin, active.end,
                                                          proj->flags, g2d, A, s),
                    "render_backward_adam");
}

size_t clsp_dilate_masks_workspace_bytes(int32_t n_views, int32_t width, int32_t height) {
  if (n_views < 1 || width < 1 || height < 1) return 0;
  return clsp::dilate_workspace_bytes(n_views, width, height);
}

clsp_status clsp_dilate_masks(const uint8_t* masks, int32_t n_views, int32_t width, int32_t height, int32_t radius,
                              uint8_t* out, void* ws, size_t ws_bytes, clsp_stream stream) {
  if (!masks || !out) return fail(CLSP_ERR_INVALID_ARG, "dilate_masks pointer is NULL");
  if (n_views < 1 || n_views > CLSP_MAX_VIEWS) return fail(CLSP_ERR_INVALID_ARG, "n_views=%d not in 1..%d", n_views, CLSP_MAX_VIEWS);
  if (width < 1 || height < 1 || width > CLSP_MAX_SIDE || height > CLSP_MAX_SIDE)
    return fail(CLSP_ERR_INVALID_ARG, "image size %dx%d not in 1..%d", width, height, CLSP_MAX_SIDE);
  if (radius < 0) return fail(CLSP_ERR_INVALID_ARG, "radius < 0");
  const size_t need = clsp_dilate_masks_workspace_bytes(n_views, width, height);
  if (!ws || ws_bytes < need)
    return fail(CLSP_ERR_INVALID_ARG, "workspace of %zu bytes is smaller than the %zu needed", ws_bytes, need);
  return hip_status(clsp::launch_dilate_masks(masks, n_views, width, height, radius, out, ws,
                                              reinterpret_cast<hipStream_t>(stream)),
                    "dilate_masks");
}

clsp_status clsp_majority_vote(const float* means, int64_t n_rows, int64_t n, const clsp_camera* cams,
                               int32_t n_views, const uint8_t* masks, uint8_t* in_count, uint8_t* out_count,
                               uint8_t* changed, uint32_t* n_changed, clsp_stream stream) {
  if (!means || !masks || !in_count || !out_count || !changed || !n_changed)
    return fail(CLSP_ERR_INVALID_ARG, "majority_vote pointer is NULL");
  if (n < 0 || n > n_rows) return fail(CLSP_ERR_INVALID_ARG, "n=%lld not in 0..n_rows", (long long)n);
  CHECK(check_cams(cams, n_views));
  clsp::DevCam dc[CLSP_MAX_VIEWS];
  for (int v = 0; v < n_views; ++v) dc[v] = dev_cam(cams[v]);
  return hip_status(clsp::launch_majority_vote(means, n_rows, n, dc, n_views, masks, in_count, out_count, changed,
                                               n_changed, reinterpret_cast<hipStream_t>(stream)),
                    "majority_vote");
}

clsp_status clsp_fit_spheres(const float* means, int64_t n_rows, clsp_range rows, const int32_t* labels,
                             int32_t n_spheres, float* centers, float* radii, clsp_stream stream) {
  if (!means || !labels || !centers || !radii) return fail(CLSP_ERR_INVALID_ARG, "fit_spheres pointer is NULL");
  if (n_spheres < 1 || n_spheres > CLSP_MAX_SPHERES)
    return fail(CLSP_ERR_INVALID_ARG, "n_spheres=%d not in 1..%d", n_spheres, CLSP_MAX_SPHERES);
  CHECK(check_range(rows, n_rows));
  return hip_status(clsp::launch_fit_spheres(means, n_rows, rows.begin, rows.end, labels, n_spheres, centers, radii,
                                             reinterpret_cast<hipStream_t>(stream)),
                    "fit_spheres");
}

clsp_status clsp_sphere_keep(const float* means, int64_t n_rows, clsp_range rows, const float* centers,
                             const float* radii, int32_t n_spheres, uint8_t* keep, uint32_t* kept,
                             clsp_stream stream) {
  if (!means || !centers || !radii || !keep || !kept) return fail(CLSP_ERR_INVALID_ARG, "sphere_keep pointer is NULL");
  if (n_spheres < 1 || n_spheres > CLSP_MAX_SPHERES)
    return fail(CLSP_ERR_INVALID_ARG, "n_spheres=%d not in 1..%d", n_spheres, CLSP_MAX_SPHERES);
  CHECK(check_range(rows, n_rows));
  return hip_status(clsp::launch_sphere_keep(means, n_rows, rows.begin, rows.end, centers, radii, n_spheres, keep,
                                             kept, reinterpret_cast<hipStream_t>(stream)),
                    "sphere_keep");
}

size_t clsp_compact_rows_workspace_bytes(int64_t n_changed) {
  if (n_changed < 0) return 0;
  return clsp::compact_workspace_bytes(n_changed);
}

clsp_status clsp_compact_rows(const clsp_params* src, const clsp_params* src_m, const clsp_params* src_v,
                              clsp_range rows, const uint8_t* keep, const clsp_params* dst, const clsp_params* dst_m,
                              const clsp_params* dst_v, void* ws, size_t ws_bytes, clsp_stream stream) {
  CHECK(check_params(src, "src"));
  CHECK(check_params(dst, "dst"));
  const bool moments = src_m || src_v || dst_m || dst_v;
  if (moments) {
    if (!src_m || !src_v || !dst_m || !dst_v)
      return fail(CLSP_ERR_INVALID_ARG, "compact_rows: give all four moment sets or none");
    CHECK(check_params(src_m, "src_m"));
    CHECK(check_params(src_v, "src_v"));
    CHECK(check_params(dst_m, "dst_m"));
    CHECK(check_params(dst_v, "dst_v"));
    if (src_m->n != src->n || src_v->n != src->n || dst_m->n != dst->n || dst_v->n != dst->n)
      return fail(CLSP_ERR_INVALID_ARG, "compact_rows: moments sized differently from their parameters");
  }
  const clsp_params* all[6] = {src, src_m, src_v, dst, dst_m, dst_v};
  for (const clsp_params* q : all)
    if (q && q->sh_degree != src->sh_degree) return fail(CLSP_ERR_INVALID_ARG, "compact_rows: sh degrees differ");
  CHECK(check_range(rows, src->n));
  if (rows.end != src->n) return fail(CLSP_ERR_INVALID_ARG, "compact_rows: rows.end must equal src->n");
  if (dst->n < rows.begin || dst->n > src->n)
    return fail(CLSP_ERR_INVALID_ARG, "compact_rows: dst->n=%lld not in [%lld, %lld]", (long long)dst->n,
                (long long)rows.begin, (long long)src->n);
  if (rows.end > rows.begin && !keep) return fail(CLSP_ERR_INVALID_ARG, "compact_rows: keep is NULL");
  const size_t need = clsp_compact_rows_workspace_bytes(rows.end - rows.begin);
  if (!ws || ws_bytes < need)
    return fail(CLSP_ERR_INVALID_ARG, "workspace of %zu bytes is smaller than the %zu needed", ws_bytes, need);
  clsp::MutParams s3[3] = {mut_params(src), moments ? mut_params(src_m) : mut_params(src),
                           moments ? mut_params(src_v) : mut_params(src)};
  clsp::MutParams d3[3] = {mut_params(dst), moments ? mut_params(dst_m) : mut_params(dst),
                           moments ? mut_params(dst_v) : mut_params(dst)};
  return hip_status(clsp::launch_compact_rows(s3, d3, moments ? 3 : 1, rows.begin, rows.end, keep, ws,
                                              reinterpret_cast<hipStream_t>(stream)),
                    "compact_rows");
}

size_t clsp_history_workspace_bytes(void) { return clsp::history_workspace_bytes(); }

namespace {
clsp_status check_history_ws(void* ws, size_t ws_bytes) {
  if (!ws || ws_bytes < clsp::history_workspace_bytes())
    return fail(CLSP_ERR_INVALID_ARG, "workspace of %zu bytes is smaller than the %zu needed", ws_bytes,
                clsp::history_workspace_bytes());
  return CLSP_OK;
}
clsp_status same_degree(const clsp_params* a, const clsp_params* b) {
  if (a->sh_degree != b->sh_degree) return fail(CLSP_ERR_INVALID_ARG, "parameter sets of different sh degree");
  return CLSP_OK;
}
}  // namespace

clsp_status clsp_reorder_static_first(const clsp_params* src, const uint8_t* changed, const clsp_params* dst,
                                      uint32_t* n_static, void* ws, size_t ws_bytes, clsp_stream stream) {
  CHECK(check_params(src, "src"));
  CHECK(check_params(dst, "dst"));
  CHECK(same_degree(src, dst));
  if (dst->n != src->n) return fail(CLSP_ERR_INVALID_ARG, "reorder_static_first: dst->n != src->n");
  if (!n_static || (src->n > 0 && !changed)) return fail(CLSP_ERR_INVALID_ARG, "reorder_static_first pointer is NULL");
  CHECK(check_history_ws(ws, ws_bytes));
  return hip_status(clsp::launch_reorder_static_first(mut_params(src), changed, mut_params(dst), n_static, ws,
                                                      reinterpret_cast<hipStream_t>(stream)),
                    "reorder_static_first");
}

clsp_status clsp_recover_previous(const clsp_params* latest, const uint8_t* indicator,
                                  const clsp_params* changed_before, const clsp_params* dst, void* ws,
                                  size_t ws_bytes, clsp_stream stream) {
  CHECK(check_params(latest, "latest"));
  CHECK(check_params(changed_before, "changed_before"));
  CHECK(check_params(dst, "dst"));
  CHECK(same_degree(latest, dst));
  CHECK(same_degree(changed_before, dst));
  if (dst->n > 0 && !indicator) return fail(CLSP_ERR_INVALID_ARG, "recover_previous: indicator is NULL");
  if (latest->n + changed_before->n < dst->n)
    return fail(CLSP_ERR_INVALID_ARG, "recover_previous: %lld + %lld source rows cannot fill %lld",
                (long long)latest->n, (long long)changed_before->n, (long long)dst->n);
  CHECK(check_history_ws(ws, ws_bytes));
  return hip_status(clsp::launch_recover_previous(mut_params(latest), indicator, mut_params(changed_before),
                                                  mut_params(dst), ws, reinterpret_cast<hipStream_t>(stream)),
                    "recover_previous");
}

clsp_status clsp_merge_updates(const clsp_params* prev, const uint8_t* ind1, const uint8_t* ind2,
                               const clsp_params* o1, const clsp_params* o2, const clsp_params* dst, void* ws,
                               size_t ws_bytes, clsp_stream stream) {
  CHECK(check_params(prev, "prev"));
  CHECK(check_params(o1, "o1"));
  CHECK(check_params(o2, "o2"));
  CHECK(check_params(dst, "dst"));
  CHECK(same_degree(prev, dst));
  CHECK(same_degree(o1, dst));
  CHECK(same_degree(o2, dst));
  if (prev->n > 0 && (!ind1 || !ind2)) return fail(CLSP_ERR_INVALID_ARG, "merge_updates: an indicator is NULL");
  if (dst->n > prev->n + o1->n + o2->n)
    return fail(CLSP_ERR_INVALID_ARG, "merge_updates: dst->n larger than the rows merged");
  CHECK(check_history_ws(ws, ws_bytes));
  return hip_status(clsp::launch_merge_updates(mut_params(prev), ind1, ind2, mut_params(o1), mut_params(o2),
                                               mut_params(dst), ws, reinterpret_cast<hipStream_t>(stream)),
                    "merge_updates");
}

clsp_status clsp_zero_grads(const clsp_params* grads, clsp_range active, clsp_stream stream) {
  CHECK(check_params(grads, "grads"));
  CHECK(check_range(active, grads->n));
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  return hip_status(clsp::launch_zero_rows(mut_params(grads), active.begin, active.end, s), "zero_grads");
}

}  // extern "C"
