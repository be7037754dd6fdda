/*
 * clsplat — C-ABI of the MI355X (gfx950) hot path of CL-Splats' local optimisation.
 *
 * The paper (CL-Splats, Sec. 3 problem statement) updates an existing 3D Gaussian
 * reconstruction G^{t-1} from new posed images I^t, optimising only the changed
 * Gaussians O^t (Sec. 3.2 "Mask Majority Voting") with a local kernel (Sec. 3.3 "Local
 * Optimization Kernel"; Supp. "Local Optimization Kernel", items 1-3) and a masked Adam
 * step (Supp. "3DGS Optimization in Changed Regions").  The calls below are one
 * optimisation step of that loop:
 *
 *   clsp_project_preprocess  per-Gaussian projection, colour, extent, tile rectangle
 *                            (Table tab:timings "Forward::Preprocess")
 *   clsp_bin_and_sort        tile render mask from O^t (item 1), per-tile depth order
 *                            restricted to masked tiles
 *   clsp_render_forward      front-to-back compositing of masked tiles (item 2;
 *                            "Forward::Render")
 *   clsp_l1_loss_grad        dL/dimage of the L1 photometric loss on masked tiles
 *   clsp_render_backward     reverse compositing of masked tiles with gradients only for
 *                            O^t (item 2; "Backward::Render"), then the preprocess
 *                            backward for O^t only (item 3; "Backward::Preprocess")
 *   clsp_masked_adam_step    Adam on the rows of O^t only; other rows and their moments
 *                            are not touched
 *   clsp_zero_grads          clear the gradient rows of O^t
 *   clsp_render_forward_l1, clsp_render_backward_adam, clsp_project_preprocess_rows
 *                            fused or partial forms of the calls above, for the
 *                            optimisation step
 *
 * Conventions shared by every call
 * --------------------------------
 * - Every data pointer is a DEVICE pointer owned by the caller, except `cams`, `bg`
 *   and `hp`, which are HOST pointers read before the call returns.  The library never
 *   allocates device memory; scratch space is a caller-provided workspace whose size
 *   the *_workspace_bytes() queries return (clsp_render_backward_noalloc instead uses a
 *   fixed static device array of the library).
 * - Every call enqueues work on `stream` (a hipStream_t; NULL is the default stream)
 *   and returns without synchronising.  Inputs must stay valid until that work is done.
 * - Arguments are validated on the host before anything is enqueued.  On error nothing
 *   is enqueued and a negative status is returned; clsp_last_error() gives a message
 *   (per host thread).  CLSP_ERR_HIP reports a failed launch.
 * - Floating point is IEEE float32 throughout.
 * - Gaussian parameters are raw (pre-activation) and component-major (SoA):
 *   component c of Gaussian i is at [c * n_rows + row(i)], row(i) = gather ? gather[i] : i.
 *   means[3], log_scales[3], quats[4] (w, x, y, z; normalised inside), opacity_logit[1],
 *   sh[K][3] with K = (D+1)^2 real spherical-harmonic coefficients per colour channel.
 * - The change set O^t is the contiguous index range [active.begin, active.end): the
 *   paper stores the unchanged Gaussians first and the changed ones last (Supp.
 *   "History Recovery"), so O^t is a suffix.  A full-scene step uses {0, n}.
 * - Views: one call handles n_views cameras of equal width and height.  Per-view
 *   outputs are stacked: Gaussian i of view v is entry v*n + i; tile t of view v is the
 *   global tile v*T + t with T = TX*TY, TX = ceil(W/16), TY = ceil(H/16), t = ty*TX + tx.
 * - Images are planar: image[v][c][y][x], T_final[v][y][x], n_contrib[v][y][x].
 *
 * The forward model (the paper builds on standard 3D Gaussian Splatting, Supp.
 * "Implementation Details"): pixel (x, y) samples (x + 0.5, y + 0.5); a Gaussian is
 * projected with p = R mu + t, u = fx X/Z + cx, v = fy Y/Z + cy, screen covariance
 * J R Sigma R^T J^T + 0.3 I (J with X/Z, Y/Z clamped to 1.3 (W/2)/fx, 1.3 (H/2)/fy);
 * colour = max(0, sum_k f_k Y_k(dir) + 0.5) with real SH (no Condon-Shortley phase,
 * k = l^2 + l + m) of the direction from the camera centre; per pixel, Gaussians are
 * composited front to back in order of the float32 depth key
 * z32 = fmaf(R[6], x, fmaf(R[7], y, fmaf(R[8], z, t[2]))) (ties: lower index first), with
 * alpha = min(0.99, o exp(-d^T conic d / 2)), alpha < 1/255 skipped, and compositing
 * stopped before the Gaussian that would take the transmittance below 1e-4.
 * Gaussians are culled when z32 <= 0.2, the quaternion is zero, or the opacity is
 * below 1/255.  The tile rectangle covers every pixel centre within (u +- rx, v +- ry)
 * where rx, ry bound the ellipse alpha >= 1/255 with a relative margin of 2^-12 for
 * float32 rounding (rx = sqrt(2 ln(255 o) a) (1 + 2^-12), a, c the diagonal of the
 * screen covariance):
 * x0 = clamp(floor((u - rx - 0.5) * 0.0625), 0, TX), x1 = clamp(floor((u + rx - 0.5) *
 * 0.0625) + 1, 0, TX), evaluated in float32 in that order; y likewise.
 */
#ifndef CLSPLAT_H
#define CLSPLAT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t clsp_status;
#define CLSP_OK 0
#define CLSP_ERR_INVALID_ARG (-1)
#define CLSP_ERR_HIP (-3)
#define CLSP_ERR_UNSUPPORTED (-4)

#define CLSP_TILE 16
#define CLSP_MAX_VIEWS 64
#define CLSP_MAX_SIDE 16384

/* hipStream_t; NULL selects the default stream. */
typedef void *clsp_stream;

/* Pinhole camera, world to camera: p = R x + t (row-major R), OpenCV axes. */
typedef struct clsp_camera {
  float R[9];
  float t[3];
  float fx, fy, cx, cy;
  int32_t width, height;
} clsp_camera;

/* Raw Gaussian parameters (device, SoA, see above).  n Gaussians; the arrays hold
 * n_rows rows; gather (nullable, int32[n]) selects row gather[i] for Gaussian i, which
 * lets one resident pool serve several stored scene states. */
typedef struct clsp_gaussians {
  const float *means;
  const float *log_scales;
  const float *quats;
  const float *opacity_logit;
  const float *sh;
  const int32_t *gather;
  int64_t n;
  int64_t n_rows;
  int32_t sh_degree;
  int32_t reserved;
} clsp_gaussians;

/* Writable views of the same arrays (Adam updates them in place; gradients use the
 * same layout with n_rows = n and no gather). */
typedef struct clsp_params {
  float *means;
  float *log_scales;
  float *quats;
  float *opacity_logit;
  float *sh;
  int64_t n;
  int32_t sh_degree;
  int32_t reserved;
} clsp_params;

typedef struct clsp_range {
  int64_t begin;
  int64_t end;
} clsp_range;

/* Output of clsp_project_preprocess (device), [n_views * n] entries each.
 *   splat  float[12] per entry: u, v, A, B | C, opacity, r, g | b, rx, ry, 0
 *          (A, B, C: the inverse screen covariance [[A, B], [B, C]])
 *   depth  float z32 depth key
 *   rect   uint32[2] per entry: x0 | x1 << 16, y0 | y1 << 16 (tiles [x0,x1) x [y0,y1));
 *          empty for culled Gaussians
 *   flags  uint32: bit 0 visible, 1 x-ratio clamped, 2 y-ratio clamped,
 *          3..5 colour channel r, g, b clamped at 0 */
typedef struct clsp_projected {
  float *splat;
  float *depth;
  uint32_t *rect;
  uint32_t *flags;
} clsp_projected;

#define CLSP_FLAG_VISIBLE 1u
#define CLSP_FLAG_CLAMP_X 2u
#define CLSP_FLAG_CLAMP_Y 4u
#define CLSP_FLAG_SHCLAMP_R 8u

/* Per-tile depth-ordered lists (device buffers owned by the caller, plus host fields).
 *
 * A tile's list is every visible Gaussian whose tile rectangle contains the tile, in
 * ascending (depth key, index) order.  Two ways to build it (`mode`):
 *   CLSP_BINS_COMPLETE      clsp_bin_and_sort builds every rendered tile's full list.
 *   CLSP_BINS_DEPTH_SLICED  clsp_bin_and_sort builds the lists of a first depth slab
 *                           (the nearest 1/16 of the Gaussians that have pairs, at least
 *                           16384 of them); clsp_render_forward renders it, then lists
 *                           the remaining Gaussians only for tiles in which some pixel is
 *                           still compositing, and continues those tiles.  Each list is
 *                           then a prefix of the complete one that reaches at least as
 *                           far as any pixel of the tile composites, so images and
 *                           gradients are the same as with complete lists.
 *   CLSP_BINS_DEPTH_SLICED_LOCAL  the same lists as CLSP_BINS_DEPTH_SLICED, for steps in
 *                           which few tiles need the second slab (local optimisation):
 *                           the second slab's pairs are placed by counting per tile
 *                           (work that grows with the tiles still compositing) instead
 *                           of by a sort of its pairs (launches that cost the same when
 *                           no tile needs it).
 *   values    uint32[capacity]: entry index v*n + i of each (tile, Gaussian) pair
 *   keys      uint32[capacity]: the global tile of each pair
 *             Pairs [0, counters[7]) hold the first lists sorted by (global tile, depth,
 *             index); in depth-sliced mode pairs [counters[7], counters[3]) hold the
 *             second lists sorted the same way.
 *   ranges    uint32[n_views*T][2]: [start, end) of each tile's first list
 *   ranges2   uint32[n_views*T][2]: [start, end) of each tile's second list ([0, 0) in
 *             complete mode); a tile's list is its first list followed by its second
 *   tile_mask uint32[n_views][ceil(T/32)]: bit (t % 32) of word t/32 of view v is set
 *             when tile t of view v is rendered
 *   alive_mask uint32[n_views][ceil(T/32)]: tiles that needed the second list
 *   tile_list uint32[n_views*T]: the rendered global tiles, ascending
 *   counters  uint32[16]: [0] pairs needed P, [1] overflow (1 when P > capacity; then
 *             the lists are not valid, tiles are not rendered or not finished, and the
 *             caller must grow `capacity` and redo the binning and the forward),
 *             [2] number of rendered tiles, [3] pairs written (P, or 0 on overflow),
 *             [4] entries with at least one pair, [5] sticky overflow: set to 1 on
 *             overflow and never cleared by the library, so a caller can check once after
 *             many steps, [6] entries in the first slab, [7] pairs of the first lists,
 *             [8] tiles that needed the second list; [9..15] reserved.  Slots other than
 *             [5] are rewritten by every clsp_bin_and_sort call.
 *   ws, ws_bytes: device workspace of clsp_bin_and_sort_workspace_bytes(...) bytes; it
 *             belongs to these lists (the depth-sliced forward uses it too)
 *   capacity: pairs the value and key buffers (and the workspace) hold
 *   n:        Gaussians per view of the projection the lists are built from */
#define CLSP_BINS_COMPLETE 0
#define CLSP_BINS_DEPTH_SLICED 1
#define CLSP_BINS_DEPTH_SLICED_LOCAL 2
#define CLSP_COUNTERS 16
typedef struct clsp_bins {
  uint32_t *values;
  uint32_t *keys;
  uint32_t *ranges;
  uint32_t *ranges2;
  uint32_t *tile_mask;
  uint32_t *alive_mask;
  uint32_t *tile_list;
  uint32_t *counters;
  void *ws;
  size_t ws_bytes;
  int64_t capacity;
  int64_t n;
  int32_t mode;
  int32_t reserved;
} clsp_bins;

/* Adam hyper-parameters (host).  lr per group: 0 means, 1 log_scales, 2 quats,
 * 3 opacity_logit, 4 sh degree-0 rows (k = 0), 5 higher sh rows (k >= 1).  step is the
 * 1-based step count used in the bias corrections.  When step_device (device int32[1])
 * is not NULL the kernel reads the step count from there instead (and `step` is
 * ignored), so a captured graph can replay the call while the caller advances the
 * counter on the device.  With zero_grads != 0 the call also sets the gradient rows of
 * `active` to zero after using them (all of them, row_mask or not), which replaces a
 * separate clsp_zero_grads before the next step's backward.  skip_flag (device
 * uint32[1], nullable): when it holds a nonzero value at the time the update runs, the
 * call leaves params, gradients and moments unchanged; pass &bins->counters[1] (the
 * pair-capacity overflow of the step's lists) so that a step whose lists did not fit
 * updates nothing (clsp_render_backward_adam checks its bins' flag by itself). */
typedef struct clsp_adam_hparams {
  float lr[6];
  float beta1, beta2, eps;
  int32_t step;
  const int32_t *step_device;
  int32_t zero_grads;
  int32_t reserved;
  const uint32_t *skip_flag;
} clsp_adam_hparams;

/* Library version string and the last error message of the calling host thread. */
const char *clsp_version(void);
const char *clsp_last_error(void);

/* ---------------------------------------------------------------------------------
 * Forward preprocess (Table tab:timings "Forward::Preprocess"; Sec. 3.3 step 1 reuses
 * this projection for the render mask and the depth order).
 * g: raw parameters; cams[n_views] (host); out: [n_views*n] entries as documented for
 * clsp_projected.  All n Gaussians are projected in every mode: unchanged Gaussians
 * still occlude and colour the masked tiles.
 * Errors: null pointers, n < 0, sh_degree not in 0..3, n_views not in 1..64, sizes
 * not in 1..16384 or differing between views, n_views*n >= 2^32. */
clsp_status clsp_project_preprocess(const clsp_gaussians *g, const clsp_camera *cams, int32_t n_views,
                                    const clsp_projected *out, clsp_stream stream);

/* The same projection for the entries of rows [rows.begin, rows.end) of every view only
 * (entry v*n + i, i in the range); every other entry of `out` is left as it was.  A
 * caller that keeps one projection per view re-projects only the rows whose parameters
 * changed (during local optimisation, the change set O^t; Sec. 3.3 freezes the rest),
 * and the result is the full projection bit for bit.
 * Errors: as clsp_project_preprocess, plus rows not within [0, n]. */
clsp_status clsp_project_preprocess_rows(const clsp_gaussians *g, const clsp_camera *cams, int32_t n_views,
                                         clsp_range rows, const clsp_projected *out, clsp_stream stream);

/* ---------------------------------------------------------------------------------
 * Render mask and per-tile depth order (Supp. "Local Optimization Kernel", item 1: a
 * boolean ceil(w/16) x ceil(h/16) mask that is true where at least one changed
 * Gaussian projects, reusing the projection for the per-tile depth ordering).
 * With use_mask != 0 the mask is the union of the tile rectangles of the visible
 * Gaussians in `active` and pairs are emitted only into masked tiles; with use_mask == 0
 * every tile is rendered.  bins->mode selects complete or depth-sliced lists (see
 * clsp_bins); bins->n must equal the projection's n.  Capacity overflow is reported on
 * the device (counters[1]); nothing is read back.
 * Errors: as above, plus capacity not in 0..2^32-1, active outside [0, n], workspace
 * smaller than clsp_bin_and_sort_workspace_bytes(n, n_views, width, height, capacity),
 * unknown mode. */
size_t clsp_bin_and_sort_workspace_bytes(int64_t n, int32_t n_views, int32_t width, int32_t height,
                                         int64_t capacity);
clsp_status clsp_bin_and_sort(const clsp_projected *proj, const clsp_camera *cams, int32_t n_views, clsp_range active,
                              int32_t use_mask, const clsp_bins *bins, clsp_stream stream);

/* ---------------------------------------------------------------------------------
 * Lists of local optimisation from a stored depth order of the unchanged Gaussians
 * (Supp. "Local Optimization Kernel", item 1: the projection, and with it the depth
 * order, of the Gaussians outside the change set is reused).  During local
 * optimisation of the change set [a0, n) (the suffix after the unchanged rows, Supp.
 * "3DGS Optimization in Changed Regions"), rows [0, a0) do not change, so for fixed
 * cameras their entries' depth order does not either.
 *
 * clsp_frozen_order stores that order once: the entries v*n + i, i < a0, that are visible
 * with a nonempty tile rectangle, in ascending (depth key, entry) order, with their
 * rectangles.  order: device buffer of clsp_frozen_order_bytes(n, n_views, a0) bytes
 * (16 bytes per entry plus a header; the call writes it, the caller owns it); ws:
 * device scratch of at least clsp_bin_and_sort_workspace_bytes(n, n_views, width,
 * height, 0) bytes (any bins' workspace for this n, views and size qualifies).
 *
 * clsp_bin_and_sort_frozen then builds exactly the lists clsp_bin_and_sort builds with
 * use_mask = 1 and active = [a0, n): the mask comes from the changed rows, the unchanged
 * entries with pairs are taken in the stored order, and only the changed entries are
 * sorted and merged in.  `order` must come from clsp_frozen_order with the same a0,
 * n_views and image size, on a projection whose rows [0, a0) equal `proj`'s (the call
 * cannot check this: other contents give wrong lists).
 * Errors: as clsp_bin_and_sort, plus a0 not in [0, n], an order buffer or workspace
 * smaller than stated. */
size_t clsp_frozen_order_bytes(int64_t n, int32_t n_views, int64_t a0);
clsp_status clsp_frozen_order(const clsp_projected *proj, const clsp_camera *cams, int32_t n_views, int64_t n,
                              int64_t a0, void *order, size_t order_bytes, void *ws, size_t ws_bytes,
                              clsp_stream stream);
clsp_status clsp_bin_and_sort_frozen(const clsp_projected *proj, const clsp_camera *cams, int32_t n_views, int64_t a0,
                                     const void *order, size_t order_bytes, const clsp_bins *bins,
                                     clsp_stream stream);

/* ---------------------------------------------------------------------------------
 * Forward rendering of the rendered tiles (Sec. 3.3 step 2; Supp. item 2: threads of
 * unmasked tiles do no work).  bg: host float[3] background colour.  Writes image,
 * T_final and n_contrib (1 + position, within the tile's list, of the last Gaussian
 * blended at the pixel; 0 if none) for the pixels of rendered tiles only; other pixels
 * are left as they were.
 * state (nullable, device, clsp_render_state_bytes(n_views, width, height) bytes)
 * receives the compositing state the backward needs: for each rendered tile (in
 * tile_list order) the largest n_contrib of its pixels, the tile's chunk length and,
 * per pixel, the transmittance and the colour added by each chunk of consecutive list
 * entries.  Chunks start CLSP_STATE_CHUNK entries long; when a tile's list fills
 * CLSP_STATE_CHUNKS of them, neighbouring chunks are merged pairwise and the length
 * doubles, so a list of L entries has chunks of at most max(CLSP_STATE_CHUNK,
 * 2 L / CLSP_STATE_CHUNKS) entries.  It lets the backward process the chunks of a tile
 * in parallel, each from its own stored transmittance.  Pass NULL when no
 * backward follows.  With depth-sliced bins this call also lists the second slab for
 * the tiles that need it (using the bins' workspace) and finishes those tiles; `proj`
 * must be the projection the bins were built from. */
#define CLSP_STATE_CHUNK 96
#define CLSP_STATE_CHUNKS 16
size_t clsp_render_state_bytes(int32_t n_views, int32_t width, int32_t height);
clsp_status clsp_render_forward(const clsp_projected *proj, const clsp_bins *bins, const clsp_camera *cams,
                                int32_t n_views, const float *bg, float *image, float *T_final, uint32_t *n_contrib,
                                void *state, size_t state_bytes, clsp_stream stream);

/* clsp_render_forward followed by clsp_l1_loss_grad (below) in one pass: the forward
 * also writes dL_dimage for the pixels it renders, from the colour it stores, and adds
 * their loss to loss_sum (device float[1], accumulated +=; may be NULL).  image,
 * T_final, n_contrib, state and dL_dimage get the same values as from the two calls
 * (loss_sum up to float summation order); it saves the second call's launch and its
 * read of the image.  target: planar [n_views][3][H][W] like image.
 * Errors: as clsp_render_forward, plus target or dL_dimage NULL. */
clsp_status clsp_render_forward_l1(const clsp_projected *proj, const clsp_bins *bins, const clsp_camera *cams,
                                   int32_t n_views, const float *bg, const float *target, float *image,
                                   float *T_final, uint32_t *n_contrib, void *state, size_t state_bytes,
                                   float *dL_dimage, float *loss_sum, clsp_stream stream);

/* ---------------------------------------------------------------------------------
 * L1 photometric loss gradient on the rendered tiles: dL_dimage = sign(image - target)
 * / (3 H W) (sign(0) = 0, full-image normalisation in every mode), zero elsewhere is NOT
 * written (pixels outside rendered tiles are left as they were).  loss_sum (device
 * float[1], accumulated +=) receives sum |image - target| / (3 H W) over rendered
 * pixels; it may be NULL. */
clsp_status clsp_l1_loss_grad(const float *image, const float *target, const clsp_bins *bins,
                              const clsp_camera *cams, int32_t n_views, float *dL_dimage, float *loss_sum,
                              clsp_stream stream);

/* ---------------------------------------------------------------------------------
 * The default 3D Gaussian Splatting loss, which the paper trains with (Supp.
 * "Implementation Details"): L = (1 - lambda) L1 + lambda (1 - SSIM), SSIM per channel
 * with an 11 x 11 Gaussian window of standard deviation CLSP_SSIM_SIGMA, constants
 * CLSP_SSIM_C1, CLSP_SSIM_C2, zero padding at the image border, L1 and SSIM averaged
 * over the 3 H W values of the whole image (lambda = CLSP_LAMBDA_DSSIM by default).
 * Writes dL_dimage for the pixels of rendered tiles (others are not written) and adds
 * the loss of those pixels to loss_sum (device float[1], may be NULL).  The gradient at
 * a pixel reads the image within 10 pixels of it; pixels of tiles that were not
 * rendered are read from frozen_image (device, like image; nullable), which local steps
 * set to a render of the unchanged Gaussians alone: outside the render mask no changed
 * Gaussian reaches, so that render is the current image there and the gradient on the
 * masked tiles is the full-image gradient.  With frozen_image NULL every pixel is read
 * from image (full steps render every tile).  Sums and SSIM partials are evaluated in
 * double; dL_dimage is rounded to float once.
 * Errors: as clsp_l1_loss_grad, plus lambda not in [0, 1]. */
#define CLSP_SSIM_SIGMA 1.5
#define CLSP_SSIM_C1 (0.01 * 0.01)
#define CLSP_SSIM_C2 (0.03 * 0.03)
#define CLSP_LAMBDA_DSSIM 0.2f
clsp_status clsp_l1_dssim_loss_grad(const float *image, const float *target, const float *frozen_image,
                                    const clsp_bins *bins, const clsp_camera *cams, int32_t n_views, float lambda,
                                    float *dL_dimage, float *loss_sum, clsp_stream stream);

/* ---------------------------------------------------------------------------------
 * Backward (Table tab:timings "Backward::Render" and "Backward::Preprocess"; Supp.
 * items 2-3).  Reverse compositing over the rendered tiles accumulates screen-space
 * gradients for the Gaussians in `active` only, then the chain rule to raw parameters
 * runs for `active` only.  Gradients are ADDED to `grads` (layout of clsp_params,
 * n_rows = n, rows outside `active` never written).  g must be the parameters the
 * projection was made from; T_final, n_contrib and state (required here) come from the
 * clsp_render_forward call on the same bins.  Each tile's list is split into the
 * chunks of the forward's state and every (tile, chunk) is processed by its own
 * workgroup, back to front from that chunk's stored transmittance and the colour of
 * the chunks behind it.  If counters[1] of the bins is set (the lists ran out of pair
 * capacity, so the forward did not render every tile completely) the call writes no
 * gradient at all.
 * ws: device workspace of clsp_render_backward_workspace_bytes(active.end -
 * active.begin, n_views) bytes. */
size_t clsp_render_backward_workspace_bytes(int64_t n_active, int32_t n_views);
clsp_status clsp_render_backward(const clsp_gaussians *g, const clsp_projected *proj, const clsp_bins *bins,
                                 const clsp_camera *cams, int32_t n_views, const float *bg, clsp_range active,
                                 const float *T_final, const uint32_t *n_contrib, const void *state,
                                 size_t state_bytes, const float *dL_dimage, const clsp_params *grads, void *ws,
                                 size_t ws_bytes, clsp_stream stream);

/* ---------------------------------------------------------------------------------
 * clsp_render_backward without a workspace argument, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving or training loops, hosts
 * that forbid allocation).  Same arguments, results and errors as clsp_render_backward
 * minus ws/ws_bytes: the screen-space gradients live in a static device array of
 * CLSP_NOALLOC_SCRATCH_BYTES that the library holds on each GPU it runs on until the
 * process ends, so the call allocates nothing (no hipMalloc, hipFree or allocating
 * library routine).  The array's address on the current device is looked up on the
 * first call made with that device current.  The call clears the part it uses before
 * use (by a kernel on `stream`), so nothing carries over from an earlier call.
 * Every call on a GPU shares that GPU's array: calls that overlap on one GPU (on
 * different streams, or from different host threads, without ordering between them)
 * race and give wrong gradients.
 * Errors: as clsp_render_backward, plus (active.end - active.begin) * n_views *
 * clsp_render_backward_workspace_bytes(1, 1) > CLSP_NOALLOC_SCRATCH_BYTES, and a non-NULL
 * stream that belongs to another device than the current one (CLSP_ERR_INVALID_ARG). */
#define CLSP_NOALLOC_SCRATCH_BYTES ((size_t)32 << 20)
clsp_status clsp_render_backward_noalloc(const clsp_gaussians *g, const clsp_projected *proj, const clsp_bins *bins,
                                         const clsp_camera *cams, int32_t n_views, const float *bg, clsp_range active,
                                         const float *T_final, const uint32_t *n_contrib, const void *state,
                                         size_t state_bytes, const float *dL_dimage, const clsp_params *grads,
                                         clsp_stream stream);

/* ---------------------------------------------------------------------------------
 * Masked Adam (Supp. "3DGS Optimization in Changed Regions": gradients and optimiser
 * updates only for O^t, so the first and second moments cannot move frozen
 * Gaussians).  For every row in `active` (and, when row_mask is not NULL, with
 * row_mask[row] != 0): m = b1 m + (1-b1) g; v = b2 v + (1-b2) g^2;
 * theta -= lr * (m / (1 - b1^step)) / (sqrt(v / (1 - b2^step)) + eps).  Other rows of
 * params, m and v are not read or written. */
clsp_status clsp_masked_adam_step(const clsp_params *params, const clsp_params *grads, const clsp_params *exp_avg,
                                  const clsp_params *exp_avg_sq, clsp_range active, const uint8_t *row_mask,
                                  const clsp_adam_hparams *hp, clsp_stream stream);

/* Set the gradient rows in `active` to zero. */
clsp_status clsp_zero_grads(const clsp_params *grads, clsp_range active, clsp_stream stream);

/* One optimisation step's backward and Adam update for a single view in one call:
 * clsp_zero_grads + clsp_render_backward (n_views = 1) + clsp_masked_adam_step
 * (row_mask NULL) on the same rows, with no gradient buffer: the preprocess backward
 * applies each row's Adam update from the gradients it has just computed, and rows
 * and components without a gradient get Adam's update for a zero gradient.  params
 * must describe the same arrays as g (which is read, then written); exp_avg and
 * exp_avg_sq as for clsp_masked_adam_step (hp->zero_grads is ignored).  The results
 * equal the three calls' up to the summation order of the raster backward's float
 * atomics; it saves the Adam launch and the gradient buffer's writes and reads.
 * ws (clsp_render_backward_workspace_bytes(active.end - active.begin, 1) bytes) must be
 * all zero on entry, e.g. zero-filled once when allocated: the call leaves it all zero,
 * so it needs no clearing launch of its own (a workspace last used by
 * clsp_render_backward must be cleared first).  If counters[1] of the bins is set
 * (pair-capacity overflow) the call changes nothing: params, exp_avg and exp_avg_sq
 * keep their values bit for bit.
 * Errors: as clsp_render_backward and clsp_masked_adam_step, plus n_views != 1. */
clsp_status clsp_render_backward_adam(const clsp_gaussians *g, const clsp_projected *proj, const clsp_bins *bins,
                                      const clsp_camera *cams, int32_t n_views, const float *bg, clsp_range active,
                                      const float *T_final, const uint32_t *n_contrib, const void *state,
                                      size_t state_bytes, const float *dL_dimage, const clsp_params *params,
                                      const clsp_params *exp_avg, const clsp_params *exp_avg_sq,
                                      const clsp_adam_hparams *hp, void *ws, size_t ws_bytes, clsp_stream stream);

/* ---------------------------------------------------------------------------------
 * Lifting 2D change masks to the change set (the steps before local optimisation).
 *
 * clsp_dilate_masks (Supp. "Detecting Changes in 2D": the binary change masks are
 * dilated by 2% of the image width, by a convolution with a kernel of ones and a
 * threshold at 0): out[v][y][x] = 1 when masks[v] (uint8, nonzero = changed,
 * [n_views][height][width]) holds a nonzero pixel in the (2 radius + 1)^2 square around
 * (x, y), pixels outside the image counting as 0; else 0.  The paper's radius is
 * round(CLSP_DILATE_FRACTION width), halves up.  out must not overlap masks.
 * ws: device workspace of clsp_dilate_masks_workspace_bytes(n_views, width, height).
 * Errors: NULL pointers, n_views not in 1..64, sizes not in 1..16384, radius < 0,
 * workspace too small. */
#define CLSP_DILATE_FRACTION 0.02
size_t clsp_dilate_masks_workspace_bytes(int32_t n_views, int32_t width, int32_t height);
clsp_status clsp_dilate_masks(const uint8_t *masks, int32_t n_views, int32_t width, int32_t height, int32_t radius,
                              uint8_t *out, void *ws, size_t ws_bytes, clsp_stream stream);

/* clsp_majority_vote (Supp. "Identifying Changed 3D Regions via Majority Voting"): the
 * centre of Gaussian i < n (means: device float[3][n_rows], component-major) is
 * projected into every view of cams (host, equal sizes) in float32, every operation
 * rounded, in this order: X = ((R0 x + R1 y) + R2 z) + t0 (Y, Z alike), u = (fx X) / Z +
 * cx, v = (fy Y) / Z + cy.  It is outside view k when Z <= 0.2 or (u, v) is not in
 * [0, W) x [0, H); otherwise it falls in pixel (floor(u), floor(v)).  in_count[i] (device
 * uint8[n]) = views whose mask (masks: device uint8 [n_views][H][W], nonzero = changed)
 * holds it there, out_count[i] (uint8[n]) = views it is outside, changed[i] (uint8[n]) =
 * 1 iff 4 out_count < 3 n_views and n_views < 2 in_count (the paper's
 * 4/3 o_i < |I| < 2 c_i), n_changed (device uint32[1], overwritten) = the number of 1s.
 * The changed Gaussians become O^t once the rows are reordered static-first.
 * Errors: NULL pointers, n < 0 or n > n_rows, invalid cameras (as for
 * clsp_project_preprocess). */
clsp_status clsp_majority_vote(const float *means, int64_t n_rows, int64_t n, const clsp_camera *cams,
                               int32_t n_views, const uint8_t *masks, uint8_t *in_count, uint8_t *out_count,
                               uint8_t *changed, uint32_t *n_changed, clsp_stream stream);

/* ---------------------------------------------------------------------------------
 * Change-region spheres (Supp. "Identifying Changed 3D Regions via Majority Voting";
 * Sec. 3.3 "Sphere Pruning"; Supp. "3DGS Optimization in Changed Regions").  The change
 * set O^t is clustered outside this library; each cluster gets one sphere, and during
 * local optimisation the changed Gaussians whose centre has left every sphere are
 * removed (the paper checks every 15 iterations), keeping O^t the contiguous suffix.
 *
 * clsp_fit_spheres: means (device float[3][n_rows], component-major) of rows
 * [rows.begin, rows.end); labels (device int32[rows.end - rows.begin]) give each row's
 * cluster in 0..n_spheres-1, or -1 for none.  Writes centers (device float[n_spheres][3])
 * = the cluster's mean (summed in double, rounded to float) and radii (device
 * float[n_spheres]) = CLSP_SPHERE_SCALE x the CLSP_SPHERE_QUANTILE percentile of the
 * float32 distances to that centre, interpolated linearly between the order statistics
 * floor(q) and floor(q) + 1, q = CLSP_SPHERE_QUANTILE (c - 1) for c points (computed in
 * double, rounded to float).  An empty cluster gets centre 0 and radius -1.
 * Errors: NULL pointers, n_spheres not in 1..CLSP_MAX_SPHERES, rows not within
 * [0, n_rows]. */
#define CLSP_SPHERE_QUANTILE 0.98
#define CLSP_SPHERE_SCALE 1.1
#define CLSP_MAX_SPHERES 4096
clsp_status clsp_fit_spheres(const float *means, int64_t n_rows, clsp_range rows, const int32_t *labels,
                             int32_t n_spheres, float *centers, float *radii, clsp_stream stream);

/* clsp_sphere_keep: keep[i - rows.begin] = 1 when the centre of row i lies in some
 * sphere (|mu - m| <= r, the boundary inside; spheres with a negative radius contain
 * nothing), else 0; kept (device uint32[1], overwritten) = the number of 1s.  The
 * decision is taken in float32 in this order, every operation rounded: d = mu - m per
 * axis, d2 = (dx dx + dy dy) + dz dz, inside iff d2 <= r r.
 * Errors: NULL pointers, n_spheres not in 1..CLSP_MAX_SPHERES, rows not within
 * [0, n_rows]. */
clsp_status clsp_sphere_keep(const float *means, int64_t n_rows, clsp_range rows, const float *centers,
                             const float *radii, int32_t n_spheres, uint8_t *keep, uint32_t *kept,
                             clsp_stream stream);

/* clsp_compact_rows: copies src (and, when both are given, the Adam moments src_m, src_v)
 * to dst (dst_m, dst_v) without the rows of [rows.begin, src->n) whose keep (as written
 * by clsp_sphere_keep) is 0: rows before rows.begin stay where they are, the kept rows
 * follow in their order.  rows.end must equal src->n (the change set is the suffix).
 * dst->n should be rows.begin + kept; no row at or past dst->n is written.  Source and
 * destination must not overlap; every set uses its own n as its row stride.
 * ws: device workspace of clsp_compact_rows_workspace_bytes(rows.end - rows.begin).
 * Errors: NULL or mismatched parameter sets (sh degree), rows.end != src->n,
 * dst->n < rows.begin or > src->n, workspace too small. */
size_t clsp_compact_rows_workspace_bytes(int64_t n_changed);
clsp_status clsp_compact_rows(const clsp_params *src, const clsp_params *src_m, const clsp_params *src_v,
                              clsp_range rows, const uint8_t *keep, const clsp_params *dst, const clsp_params *dst_m,
                              const clsp_params *dst_v, void *ws, size_t ws_bytes, clsp_stream stream);

/* ---------------------------------------------------------------------------------
 * History of the reconstruction (Supp. "History Recovery", Alg. alg:example; Supp.
 * "Batched Updates").  Row copies of whole Gaussians (every parameter component; each
 * set uses its own n as its row stride); source and destination must not overlap.
 * ws: device workspace of clsp_history_workspace_bytes() bytes.
 *
 * clsp_reorder_static_first: before step t is optimised, dst = the rows of src whose
 * changed (uint8[src->n], e.g. from clsp_majority_vote: I^t) is 0, in order, then those
 * whose changed is 1, in order, so that O^t is the suffix and dst[:#static] is the
 * static part of G^{t-1}; n_static (device uint32[1]) = #static.  dst->n must equal
 * src->n.  The caller keeps I^t and O^t (dst's suffix at this moment) for recovery.
 *
 * clsp_recover_previous: G^{k-1} from G^k (latest), I^k (indicator, uint8[dst->n], over
 * G^{k-1}) and O^k (changed_before, the changed Gaussians' values before step k):
 * dst[i] = O^k[j] where indicator[i] is the j-th 1, latest[j] where it is the j-th 0.
 * Sizes must agree (latest->n >= zeros of I^k, changed_before->n = ones of I^k); a row
 * whose source is missing is not written.  Repeating it recovers any earlier state.
 *
 * clsp_merge_updates: two concurrent updates of G^{t-1} (prev): dst = the rows of prev
 * that neither ind1 nor ind2 (uint8[prev->n]) marks, in order, then o1's rows, then
 * o2's (the paper's merge, read so that every unchanged Gaussian is kept).  dst->n should
 * be that total; no row at or past dst->n is written.
 * Errors: NULL or mismatched parameter sets (sh degree), size mismatches stated above
 * that the host can check, workspace too small. */
size_t clsp_history_workspace_bytes(void);
clsp_status clsp_reorder_static_first(const clsp_params *src, const uint8_t *changed, const clsp_params *dst,
                                      uint32_t *n_static, void *ws, size_t ws_bytes, clsp_stream stream);
clsp_status clsp_recover_previous(const clsp_params *latest, const uint8_t *indicator,
                                  const clsp_params *changed_before, const clsp_params *dst, void *ws,
                                  size_t ws_bytes, clsp_stream stream);
clsp_status clsp_merge_updates(const clsp_params *prev, const uint8_t *ind1, const uint8_t *ind2,
                               const clsp_params *o1, const clsp_params *o2, const clsp_params *dst, void *ws,
                               size_t ws_bytes, clsp_stream stream);

#ifdef __cplusplus
}
#endif

#endif /* CLSPLAT_H */
