/*
 * sss.h -- C-ABI of the MI355X (gfx950) hot path of 3D Student Splatting and
 * Scooping (arXiv 2503.10148): a differentiable 16x16-tile rasterizer for
 * signed Student's t mixture components, followed by an SGHMC step.
 *
 * The five calls of one training step, in order:
 *   sss_project     per (view, component): 3D t -> 2D t (Sec. 3.2 eq. t_2D)
 *   sss_bin_sort    tile binning + depth order (the rasterizer's list build)
 *   sss_render_fwd  signed front-to-back compositing (Sec. 3.4 eq. SSS_color)
 *   sss_render_bwd  closed-form gradients (SM "Backward Pass")
 *   sss_sghmc_step  SGHMC on the means (Sec. 3.4 eq. sigmoidUpdate)
 *
 * General rules for every call:
 *  - Pointers named "device" point to device memory of the current HIP
 *    device; the caller allocates and owns them.  Structs passed by pointer
 *    (sss_scene_t, sss_camera_t, ...) live in host memory and are read during
 *    the call only.
 *  - `stream` is a hipStream_t (NULL = the default stream).  All device work
 *    is enqueued on it.  sss_bin_sort waits for the stream once unless its
 *    no_wait flag is set (it reads two counts back); every other call
 *    returns without waiting (sss_relocate when asked for its count).
 *  - Return value: SSS_OK or a negative SSS_ERR_* code.  On error nothing
 *    has been enqueued unless stated otherwise, and sss_last_error() returns
 *    a message for the calling thread.
 *  - All arithmetic of the raster kernels is FP32; the per-component
 *    projection (forward and backward) computes in FP64 and stores FP32.
 *  - Workspaces (`ws`) are device buffers of at least the size the matching
 *    *_workspace() call returns, 256-byte aligned (hipMalloc and torch
 *    allocations are); a misaligned ws is rejected with SSS_ERR_INVALID.
 *  - Cameras of one call may have different sizes.  Images of all views are
 *    concatenated: view v occupies pixels [P_v, P_v + W_v H_v) with
 *    P_v = sum_{u<v} W_u H_u, row-major, 3 channels (HWC) where noted.
 *    Tiles likewise: view v owns global tile ids [T_v, T_v + tx_v ty_v),
 *    tx = ceil(W/16), ty = ceil(H/16), row-major inside the view.
 */
#ifndef SSS_H
#define SSS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SSS_VERSION 106
#define SSS_TILE 16           /* tile edge in pixels                            */
#define SSS_MAX_VIEWS 16      /* views per call                                 */
#define SSS_RECORD_BYTES 64   /* size of one projected record                  */

enum {
  SSS_OK = 0,
  SSS_ERR_INVALID = -1,      /* bad argument (null pointer, size, degree ...)   */
  SSS_ERR_CAPACITY = -2,     /* pair buffer too small; see sss_bins_t.n_pairs  */
  SSS_ERR_HIP = -3,          /* a HIP runtime call failed                       */
  SSS_ERR_UNSUPPORTED = -4,  /* valid request outside what this build supports */
};

/* Components (Sec. 3.2): mean mu, covariance Sigma = R S S^T R^T, degrees of
 * freedom nu, signed opacity o (Sec. 3.3) and SH colour.  Activated values:
 *   means   [n][3]                 device, FP32
 *   scales  [n][3]   S diagonal, > 0
 *   quats   [n][4]   R as a quaternion (w, x, y, z), any non-zero norm
 *                    (normalised inside; gradients flow through it)
 *   nu      [n]      clamped to [nu_min, nu_max] inside
 *   opacity [n]      o in [-1, 1] (the caller applies tanh)
 *   sh      [n][(d+1)^2][3]  real SH coefficients, degree d in 0..3, basis
 *                    ordered k = l*l + l + m with the Condon-Shortley phase;
 *                    colour = max(0, sum_k Y_k(dir) sh[k] + 1/2) with dir the
 *                    unit vector from the camera centre to the mean.
 * quats and sh must be 16-byte aligned (any device allocation is);
 * otherwise calls taking a scene return SSS_ERR_INVALID. */
typedef struct {
  int64_t n;
  int32_t sh_degree;
  int32_t reserved;
  const float* means;
  const float* scales;
  const float* quats;
  const float* nu;
  const float* opacity;
  const float* sh;
} sss_scene_t;

/* Gradients with the same layout as sss_scene_t (device, FP32).  With
 * overwrite = 0 calls ADD into them (+=; the caller zeroes them first); with
 * overwrite = 1 every element is written, components that no view sees get 0.
 * A NULL array is skipped. */
typedef struct {
  float* means;
  float* scales;
  float* quats;
  float* nu;
  float* opacity;
  float* sh;
  int32_t overwrite;
  int32_t reserved;
} sss_grads_t;

/* Pinhole camera, OpenCV axes (x right, y down, z forward).  viewmat is the
 * 3x4 row-major world->camera transform [R | t]; pixel (x, y) is sampled at
 * (x + 1/2, y + 1/2). */
typedef struct {
  float viewmat[12];
  float fx, fy, cx, cy;
  int32_t width, height;
} sss_camera_t;

/* Rendering conventions.  Defaults from sss_default_render_opts():
 *   alpha_min 1/255  a component is skipped at a pixel where |o T2D| < alpha_min
 *   alpha_max 0.99   |alpha| is clamped to alpha_max (no gradient when clamped);
 *                    must lie in (0, 1)
 *   t_min     1e-4   a pixel stops before the component that would bring its
 *                    transmittance below t_min (that component is not added);
 *                    values below the smallest normal float (1.18e-38), 0
 *                    included, act as that value
 *   z_near    0.2    components with depth <= z_near are culled
 *   nu_min, nu_max   1, 1e4 (SM "Implementation Details")
 *   lowpass   0      added to the diagonal of the 2D covariance (the paper's
 *                    final model uses none; 0.3 in its ablation setting 1)
 *   bg        0,0,0  background colour, weighted by the final transmittance
 *   family    SSS_FAMILY_STUDENT_T; SSS_FAMILY_GAUSSIAN renders every component
 *                    with the Gaussian kernel exp(-h/2) (the nu -> infinity limit,
 *                    Sec. 3.2; the paper's SGHMC-with-Gaussians ablation), nu
 *                    is ignored and gets no gradient.  The projected records
 *                    carry the family, and the raster calls are compiled per
 *                    family: sss_render_fwd / sss_render_bwd must get the
 *                    family the entries were projected with
 *   trunc_mode SSS_TRUNC_ALPHA: a component's tile rectangle bounds its alpha
 *                    level set h <= h* (lossless: outside it every pixel
 *                    fails the alpha test).  SSS_TRUNC_COVERAGE: the paper's
 *                    truncation by a t critical value (Sec. 3.2, SM
 *                    "Implementation Details"), read as the ellipse h <= q
 *                    holding the probability mass of the Gaussian 3-sigma
 *                    ellipse, 1 - exp(-9/2): P(h <= q) = 1 - (1 + q/nu)^(-nu/2)
 *                    gives q = nu (exp(9/nu) - 1) (9 for the Gaussian
 *                    family); the rectangle bounds h <= min(q, h*), so heavy
 *                    tails (small nu) are unchanged and light ones are cut. */
enum { SSS_FAMILY_STUDENT_T = 0, SSS_FAMILY_GAUSSIAN = 1 };
enum { SSS_TRUNC_ALPHA = 0, SSS_TRUNC_COVERAGE = 1 };

typedef struct {
  float alpha_min, alpha_max, t_min, z_near, nu_min, nu_max, lowpass;
  float bg[3];
  int32_t family;
  int32_t trunc_mode;
} sss_render_opts_t;

void sss_default_render_opts(sss_render_opts_t* opts);

/* ------------------------------------------------------------------------
 * sss_project -- Sec. 3.2 eq. (t_2D) and SM "Forward Pass".
 * For every view v and component i (entry e = v*n + i): camera-space
 * position, 2D mean, 2D covariance J W Sigma W^T J^T (local affine
 * approximation; x/z and y/z clamped to 1.3 half-fov for J), its inverse
 * (the conic), colour from SH, clamped nu, and the truncation ellipse
 * h <= h* with h* = nu ((|o|/alpha_min)^(2/(nu+2)) - 1), outside of which
 * |o T2D| < alpha_min (SSS_TRUNC_COVERAGE: h <= min(q, h*), see
 * sss_render_opts_t).  The rectangle is the range of tiles of its
 * axis-aligned box;
 * the entry is listed in the tiles of that range whose box of pixel centres
 * meets the ellipse (row by row: the ellipse's x-extent over the band of
 * pixel-centre rows), and tiles_touched counts those tiles.
 * Depth key = bits of the FP32 depth fmaf(W20, x, fmaf(W21, y, fmaf(W22, z, t2))).
 * Culled (tiles_touched = 0): depth key <= z_near, |o| < alpha_min, degenerate
 * 2D covariance, or a rectangle entirely off screen.
 * Outputs (device, caller-allocated, n_views*n entries each):
 *   entries        SSS_ENTRY_BYTES (128) per entry, 16-byte aligned:
 *                    bytes   0..63   the raster record (opaque to the caller)
 *                    bytes  64..95   the FP64 ellipse: 2D covariance A, B, D
 *                                    and the level of the listed ellipse
 *                    bytes  96..103  the tile rectangle x0, y0, x1, y1
 *                                    (uint16, inclusive)
 *                    bytes 104..127  unused
 *                  (valid where tiles_touched > 0).  One line per entry, so
 *                  sss_bin_sort gathers each visible entry's data in depth
 *                  order with one 128-byte read.
 *   depth_key      uint32
 *   tiles_touched  uint32, number of listed tiles, 0 = culled
 * Errors: INVALID for n <= 0, sh_degree outside 0..3, n_views outside
 * 1..SSS_MAX_VIEWS, a NULL array, a camera with width/height <= 0 or
 * non-positive focal lengths, entries not 16-byte aligned. */
#define SSS_ENTRY_BYTES 128   /* size of one projected entry                  */

typedef struct {
  void* entries;
  uint32_t* depth_key;
  uint32_t* tiles_touched;
} sss_proj_t;

int sss_project(const sss_scene_t* scene, const sss_camera_t* cams, int n_views,
                const sss_render_opts_t* opts, const sss_proj_t* out, void* stream);

/* ------------------------------------------------------------------------
 * sss_bin_sort -- per-tile component lists in ascending (depth key,
 * component index) order (the list build of the tile rasterizer the paper
 * modifies, SM "Implementation Details").
 * Visible entries are sorted once by depth key (stable radix sort, ties by
 * entry index), giving each a rank; every (tile, rank) pair of a visible
 * entry's rectangle is emitted and stably radix-sorted by tile.
 * Inputs: proj (from sss_project), the same cameras, n_entries = n_views*n.
 * Outputs (device, caller-allocated):
 *   order          [n_entries]   rank -> entry; the first n_visible are valid
 *   sorted_records [n_entries] x 64 B, record of rank r at position r
 *   tile_start     [n_tiles + 1] pairs of global tile t are
 *                  pair_rank[tile_start[t] .. tile_start[t+1])
 *   pair_rank      [pair_capacity] ranks, ascending within each tile
 *   rank_offset    [n_entries] (nullable) first pair of rank r in emission
 *                  order: rank r emitted its rectangle's tiles row-major at
 *                  positions rank_offset[r] + k, k < tiles_touched.  Needed
 *                  by the deterministic backward pass.
 *   tile_order     [n_tiles] (nullable) a permutation of the global tiles,
 *                  longest list first (coarse buckets of the list length;
 *                  order within a bucket unspecified).  The raster kernels
 *                  render a tile as 1, 2 or 4 workgroups (units of 16, 8 or
 *                  4 pixel rows) and launch the units of tile tile_order[b]
 *                  after those of tile_order[b - 1], so the tiles with the
 *                  most work start first; NULL launches them in row-major
 *                  order.  Only the schedule changes: every pixel's and
 *                  every pair's result is the same.
 *   tile_work      [n_tiles][4] (nullable) not written here: sss_render_fwd
 *                  stores, per 16x4 pixel strip s (tile rows 4s..4s+3), the
 *                  largest n_contrib of its pixels (the list prefix the
 *                  backward pass walks), and the stored-mode backward
 *                  launches its units in decreasing order of it.
 * A non-NULL tile_order must hold what sss_bin_sort wrote (tiles outside
 * the grid are skipped, so another permutation only reorders work and
 * anything else leaves tiles unrendered).
 * Counts: the number of visible entries and the number of pairs the lists
 * need (which may exceed pair_capacity).  The kernels read them on the
 * device, so the work is enqueued without waiting for them:
 *   no_wait = 0  the call waits once for the counts and writes n_visible and
 *                n_pairs (host fields, also on SSS_ERR_CAPACITY); on
 *                CAPACITY nothing after the count is enqueued.
 *   no_wait = 1  the call never waits; n_visible and n_pairs are set to -1.
 *                If the pairs exceed pair_capacity the lists hold only the
 *                first pair_capacity emitted pairs (no write leaves the
 *                buffers) and must not be used: the caller checks counts[1]
 *                and calls again with a larger pair_rank and workspace.
 *   counts       (nullable) receives (n_visible, required pairs) as two
 *                uint64, written by a kernel of the call, in either mode:
 *                device memory, or pinned host memory the device can write
 *                (hipHostMalloc), which the host may read once the call's
 *                work has completed (no copy needed).
 * The deterministic backward pass needs the host counts (no_wait = 0).
 * Workspace: ws of ws_bytes >= sss_bin_sort_workspace(n_entries, pair_capacity).
 * Errors: CAPACITY (no_wait = 0) when n_pairs > pair_capacity (re-allocate
 * pair_rank and the workspace for n_pairs and call again); INVALID for NULL
 * pointers or a short workspace; UNSUPPORTED for pair_capacity >= 2^32. */
typedef struct {
  uint32_t* order;
  void* sorted_records;
  uint32_t* tile_start;
  uint32_t* pair_rank;
  uint32_t* rank_offset;
  uint32_t* tile_order;
  uint32_t* tile_work;
  int64_t pair_capacity;
  int64_t n_visible;   /* out (host; -1 with no_wait) */
  int64_t n_pairs;     /* out (host; -1 with no_wait) */
  uint64_t* counts;    /* nullable [2], device or pinned host: n_visible, required pairs */
  int32_t no_wait;     /* 1: enqueue everything without waiting for the counts */
  int32_t reserved;
} sss_bins_t;

size_t sss_bin_sort_workspace(int64_t n_entries, int64_t pair_capacity);
int64_t sss_total_tiles(const sss_camera_t* cams, int n_views);
int64_t sss_total_pixels(const sss_camera_t* cams, int n_views);

int sss_bin_sort(const sss_proj_t* proj, const sss_camera_t* cams, int n_views, int64_t n,
                 sss_bins_t* bins, void* ws, size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------------
 * sss_render_fwd -- Sec. 3.4 eq. (SSS_color): per pixel, over its tile's
 * list front to back: h = d^T Q d (d = pixel - mean2d), T2D = (1 + h/nu)^(-(nu+2)/2),
 * alpha = o T2D (skip if |alpha| < alpha_min, clamp |alpha| <= alpha_max),
 * stop before T(1 - alpha) < t_min, C += colour alpha T, T *= 1 - alpha.
 * Outputs (device, P = sss_total_pixels):
 *   image     [P][3]  C + T bg
 *   t_final   [P]     final transmittance T
 *   n_contrib [P]     list position after the last added component
 *   bins->tile_work   (if not NULL) per 16x4 strip, the largest n_contrib of its pixels
 * Tiles are launched in bins->tile_order when it is not NULL.
 * Errors: INVALID for NULL pointers / bad views. */
int sss_render_fwd(const sss_bins_t* bins, const sss_camera_t* cams, int n_views,
                   const sss_render_opts_t* opts, float* image, float* t_final,
                   uint32_t* n_contrib, void* stream);

/* ------------------------------------------------------------------------
 * sss_render_bwd -- SM "Backward Pass": gradients of a loss L(image) with
 * respect to means, scales, quats, nu, opacity and sh, through alpha, T2D,
 * h, the 2D mean and conic, the projection and the SH colour.  dT2D/dnu is
 * the complete derivative T/2 [(nu+2) h/(nu (nu+h)) - log(1 + h/nu)].
 *   mode SSS_BWD_STORED     uses image and n_contrib from sss_render_fwd
 *   mode SSS_BWD_RECOMPUTE  recomputes the forward pass per tile (image,
 *                           t_final, n_contrib ignored; image_out, if not
 *                           NULL, receives the forward image)
 *   | SSS_BWD_DETERMINISTIC (flag OR-ed into either mode): no float
 *                           atomics; each (tile, component) pair's per-tile
 *                           sums go to their own slot, then every entry sums
 *                           its slots in emission order, so gradients and
 *                           loss_out are bit-identical run to run.  Needs
 *                           bins->order and bins->rank_offset, proj->entries
 *                           and the larger workspace
 *                           sss_render_bwd_workspace_det(n_entries,
 *                           bins->n_pairs, n_tiles).
 *   loss SSS_LOSS_GRAD      dl_or_target = dL/dimage [P][3]
 *   loss SSS_LOSS_L1        dl_or_target = target [P][3]; L = mean |image - target|
 *                           over all 3P values; loss_out (device float,
 *                           nullable) receives += L
 * grads: += or = (see sss_grads_t).  Workspace: ws_bytes >=
 * sss_render_bwd_workspace(n_views*n, n_tiles) (per-entry screen-space
 * gradients, 12 FP64 each, one loss value per tile and the tiles' launch
 * order; the L1 loss is summed over tiles in a fixed order, so loss_out
 * gets the same value on every run).  Schedule: in stored mode with
 * bins->tile_work set (by sss_render_fwd), the units with the longest walks
 * start first; otherwise bins->tile_order (or row-major) as in the forward
 * pass.  The schedule never changes a unit's own sums.
 * Errors: INVALID for NULL pointers, a short workspace, unknown mode/loss. */
enum { SSS_BWD_STORED = 0, SSS_BWD_RECOMPUTE = 1, SSS_BWD_DETERMINISTIC = 4 };
enum { SSS_LOSS_GRAD = 0, SSS_LOSS_L1 = 1 };

size_t sss_render_bwd_workspace(int64_t n_entries, int64_t n_tiles);
size_t sss_render_bwd_workspace_det(int64_t n_entries, int64_t n_pairs, int64_t n_tiles);

int sss_render_bwd(const sss_scene_t* scene, const sss_proj_t* proj, const sss_bins_t* bins,
                   const sss_camera_t* cams, int n_views, const sss_render_opts_t* opts,
                   int mode, int loss, const float* dl_or_target, const float* image,
                   const uint32_t* n_contrib, float* image_out, float* loss_out,
                   const sss_grads_t* grads, void* ws, size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------------
 * sss_render_bwd_noalloc -- for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): sss_render_bwd with the same arguments, modes and results,
 * minus the workspace, which the library holds itself as a device array of
 * SSS_NOALLOC_WORKSPACE_BYTES (128 MiB; about 1.3M entries at 1080p in the
 * atomic modes) per GPU it runs on, kept until the process ends.  The call
 * allocates nothing (no hipMalloc/hipFree, no library allocator).
 * The first call on a device looks up that device's copy of the array.
 * Calls that overlap on one GPU share the array and race: serialise them
 * (one stream, or events between streams).  Each call clears what it needs
 * zeroed with a kernel of its own (no memset node under graph capture).
 * Errors: as sss_render_bwd, plus INVALID (with the needed size in the
 * message) when sss_render_bwd_workspace / _workspace_det of the call
 * exceeds SSS_NOALLOC_WORKSPACE_BYTES; HIP if the array's address cannot be
 * looked up. */
#define SSS_NOALLOC_WORKSPACE_BYTES ((size_t)128 << 20)

int sss_render_bwd_noalloc(const sss_scene_t* scene, const sss_proj_t* proj, const sss_bins_t* bins,
                           const sss_camera_t* cams, int n_views, const sss_render_opts_t* opts,
                           int mode, int loss, const float* dl_or_target, const float* image,
                           const uint32_t* n_contrib, float* image_out, float* loss_out,
                           const sss_grads_t* grads, void* stream);

/* ------------------------------------------------------------------------
 * sss_sghmc_step -- Sec. 3.4 eq. (sigmoidUpdate) / SM eq. (SGHMC), per mean
 * element, eps = lr, C = friction, switch s = sigmoid(k ((1 - |o|) - t)) (on
 * for |o| below 1 - t), n ~ N(0, 2 eps C) per axis:
 *   F  = s eps (1 - eps C) r        (F = 0 when burn_in)
 *   mu <- mu - eps^2 G + F + s eps n  (burn_in: s eps Sigma n, Sigma = R S S^T R^T)
 *   r  <- (1 - eps C) r - eps G + n
 * G = grad_means.  Noise: Philox4x32-10 with key (seed lo, seed hi) and
 * counter (i lo, step lo, step hi, i hi); uniforms ((x >> 9) + 1/2) 2^-23;
 * Box-Muller on words (0, 1) for x, y and (2, 3) for z.  noise = 0 turns it off.
 * adam (nullable): Adam (beta1, beta2, eps, step t >= 1) on up to 6 further
 * arrays (the paper's non-mean parameters), each clamped to [lo, hi]; one
 * launch for all arrays (an array of count 0 is skipped).
 * Arrays: device FP32; means, momentum, grad_means [n][3]; opacity [n];
 * scales [n][3] and quats [n][4] (read only for burn_in; quats 16-byte aligned).
 * Errors: INVALID for n <= 0, NULL arrays, lr < 0, adam->t < 1. */
typedef struct {
  float lr, friction, k, t;
  int32_t burn_in, noise;
  uint64_t seed, step;
} sss_sghmc_opts_t;

typedef struct {
  float* param;
  const float* grad;
  float* m;
  float* v;
  int64_t count;
  float lr, lo, hi;
} sss_adam_array_t;

typedef struct {
  float beta1, beta2, eps;
  int32_t n_arrays;
  int64_t t;
  sss_adam_array_t arrays[6];
} sss_adam_t;

int sss_sghmc_step(float* means, float* momentum, const float* grad_means, const float* opacity,
                   const float* scales, const float* quats, int64_t n,
                   const sss_sghmc_opts_t* opts, const sss_adam_t* adam, void* stream);

/* ------------------------------------------------------------------------
 * sss_render_bwd_step -- sss_render_bwd followed by sss_sghmc_step with Adam
 * on the other parameters, in one call: the projection backward applies the
 * update to each component while its gradient (summed over the views) is
 * still in registers, so the parameter gradients never go through memory.
 * The result is that of the two calls in sequence: SGHMC on the means with
 * the old opacity (and, with burn_in, the old scales and rotation), then
 * Adam (bias-corrected with t) on scales, quats, nu, opacity and sh, each
 * clamped to [lo, hi].
 *   scene    read for the gradients; its six arrays are the ones updated,
 *            given again, writable, in step->params (means, scales, quats,
 *            nu, opacity, sh; each must equal the scene's pointer)
 *   step     momentum [n][3] of the means; sghmc options (as
 *            sss_sghmc_step); Adam beta1, beta2, eps, t >= 1 and per array
 *            (scales, quats, nu, opacity, sh) the moments m, v of the
 *            array's shape, lr, lo, hi; adam = 0 leaves those arrays as
 *            they are
 *   grads    nullable: when given, also receives the gradients (overwrite)
 * Other arguments, modes, workspace and errors as sss_render_bwd
 * (INVALID also for a NULL step, momentum or moment array, pointers that
 * differ from the scene's, lr < 0 or t < 1). */
typedef struct {
  float* params[6];
  float* momentum;
  sss_sghmc_opts_t sghmc;
  float beta1, beta2, eps;
  int32_t adam;
  int64_t t;
  float* m[5];
  float* v[5];
  float lr[5], lo[5], hi[5];
} sss_step_t;

int sss_render_bwd_step(const sss_scene_t* scene, const sss_proj_t* proj, const sss_bins_t* bins,
                        const sss_camera_t* cams, int n_views, const sss_render_opts_t* opts, int mode, int loss,
                        const float* dl_or_target, const float* image, const uint32_t* n_contrib,
                        float* image_out, float* loss_out, const sss_grads_t* grads, const sss_step_t* step,
                        void* ws, size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------------
 * sss_loss -- the photometric loss of Sec. 3.4,
 *   L = (1 - lambda) L1 + lambda (1 - SSIM),
 * and dL/dimage, to feed sss_render_bwd (SSS_LOSS_GRAD).  L1 and SSIM are
 * means over all 3P values of all views; SSIM uses an 11x11 Gaussian window
 * (sigma 1.5), C1 = 0.01^2, C2 = 0.03^2 and zero padding, each view filtered
 * on its own.  (The paper's opacity and scale regularisers are sums over
 * parameters and do not enter dL/dimage: see sss_regularise.)
 *   image, target [P][3]  device; dl_dimage [P][3] written;
 *   loss_out (device float, nullable) receives += L;
 *   ws of ws_bytes >= sss_loss_workspace(P) (per-pixel SSIM partials).
 * Errors: INVALID for null pointers, lambda outside [0, 1], short workspace. */
size_t sss_loss_workspace(int64_t total_pixels);
int sss_loss(const float* image, const float* target, const sss_camera_t* cams, int n_views, float lambda_dssim,
             float* dl_dimage, float* loss_out, void* ws, size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------------
 * sss_regularise -- the two regularisers of the Sec. 3.4 loss,
 *   eps_opacity sum_i |o_i| + eps_sigma sum_i sum_j sqrt(lambda_ij),
 * lambda_ij the eigenvalues of Sigma_i = R S S^T R^T, so sqrt(lambda_ij) =
 * |s_ij|.  Adds the gradient eps sign(x) (0 at x = 0) into d_opacity [n] and
 * d_scales [n][3] (device, nullable: skipped) and, when loss_out (device
 * float) is given, adds the value to it.  opacity [n], scales [n][3] device.
 * Errors: INVALID for null inputs, n <= 0, negative weights. */
int sss_regularise(const float* opacity, const float* scales, int64_t n, float eps_opacity, float eps_sigma,
                   float* d_opacity, float* d_scales, float* loss_out, void* stream);

/* ------------------------------------------------------------------------
 * sss_relocate -- recycling of low-opacity components (Sec. 3.4 "Adding and
 * Recycling Components", eq. relocation; SM "Component Recycling").
 * Dead components (|o| <= dead_opacity), in index order and at most
 * floor(n * max_fraction) of them, are moved onto live targets drawn from a
 * multinomial over |o| (integer weights floor(|o| 2^24); draw j: Philox4x32-10,
 * key (seed lo, seed hi), counter (j lo, step lo, step hi, 2^31 | j hi),
 * position floor(((x1 << 32) | x0) W / 2^64) in the weight prefix sum W).
 * A target drawn m times ends with N = m + 1 components at its mean: the
 * moved ones copy its mean, rotation, nu and SH; all N get the opacity from
 * (1 - o_new)^N = 1 - |o| (sign of the target's o) and scales multiplied by
 * |o| beta(1/2, (nu+2)/2) / K with
 * K = sum_{i=1..N} sum_{k<i} C(i-1,k) (-1)^k o_new^(k+1) beta(1/2, ((k+1)(nu+3)-1)/2)
 * (nu unchanged, clamped to [1, 1e4] in the rule), beta through ln Gamma.
 * Every listed state array (width floats per component: SGHMC momentum, Adam
 * moments ...) gets the moved components' rows zeroed.  Components to add
 * are appended by the caller with opacity 0 before the call (they are dead).
 * The scene's arrays are modified in place (device, caller-owned).
 * n_moved (host, nullable): when given, the call waits for the stream and
 * writes the number of components moved.
 * Errors: INVALID for null arrays, n < 1, max_fraction outside [0, 1],
 * a short workspace or more than 8 state arrays. */
typedef struct {
  float dead_opacity;   /* 0.005 */
  float max_fraction;   /* 0.05 */
  uint64_t seed, step;
} sss_relocate_opts_t;

typedef struct {
  float* ptr;           /* [n][width] device */
  int32_t width;
  int32_t reserved;
} sss_state_t;

size_t sss_relocate_workspace(int64_t n, float max_fraction);
int sss_relocate(const sss_scene_t* scene, const sss_state_t* state, int n_state,
                 const sss_relocate_opts_t* opts, void* ws, size_t ws_bytes, int64_t* n_moved,
                 void* stream);

/* ------------------------------------------------------------------------
 * sss_stream_copy -- a measurement aid, not a step of the method.  Copies
 * `bytes` from src to dst (device pointers, 16-byte aligned, not
 * overlapping; bytes a multiple of 16) with the access pattern of the
 * library's streaming kernels at their best: 16-byte non-temporal loads and
 * stores, four in flight per thread, up to 32768 workgroups.  Its rate is
 * the HBM rate such kernels reach on the device, against which the
 * memory-bound stages are read (the runtime's own device copy moves less).
 * Ownership stays with the caller; the call is asynchronous on `stream`.
 * Errors: INVALID for a NULL or misaligned pointer or a size that is not a
 * multiple of 16 (nothing launched); HIP for a launch error.  bytes = 0
 * launches nothing. */
int sss_stream_copy(const void* src, void* dst, size_t bytes, void* stream);

/* ------------------------------------------------------------------------
 * Kernel timing (tracing).  When enabled, every kernel the library launches
 * is bracketed by two HIP events on its own stream; sss_timing_read waits
 * for the recorded events and returns, per kernel name, the number of
 * launches and their summed duration in milliseconds since the last reset.
 * Off by default; the events cost a few microseconds per launch.
 * sss_timing_read returns the number of entries written (<= max_entries) or
 * a negative error code. */
typedef struct {
  char name[48];
  int64_t launches;
  double total_ms;
} sss_kernel_time_t;

int sss_timing_enable(int on);
void sss_timing_reset(void);
int sss_timing_read(sss_kernel_time_t* out, int max_entries);

/* ------------------------------------------------------------------------ */
const char* sss_last_error(void);   /* message of the last failed call on this thread */
int sss_version(void);              /* SSS_VERSION */

#ifdef __cplusplus
}
#endif
#endif /* SSS_H */
