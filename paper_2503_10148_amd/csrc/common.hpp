// Internal definitions shared by the HIP translation units of libsss.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sss.h"

namespace sss {

constexpr int kTile = SSS_TILE;
constexpr int kBlock = 256;               // threads per workgroup (4 waves of 64)

// Per-view camera constants, passed by value in the kernel argument segment.
struct CamDev {
  float R[9];          // world->camera rotation, row-major
  float t[3];
  float fx, fy, cx, cy;
  int32_t W, H, tiles_x, tiles_y;
  int32_t tile_offset;  // first global tile id of the view
  int32_t pad;
  int64_t pix_offset;   // first pixel of the view
};

struct CamBatch {
  CamDev v[SSS_MAX_VIEWS];
  int32_t n_views;
  int32_t total_tiles;
};

struct OptsDev {
  float alpha_min, alpha_max, t_min, z_near, nu_min, nu_max, lowpass;
  float bg[3];
  int32_t family, trunc_mode;
};

// Projected record of one (view, component) entry, 64 bytes.
// The 2D mean is kept in FP64 so that pixel offsets are exact to well below
// 1e-6 px at 1080p; everything a pixel evaluation needs follows.
struct __align__(16) Rec {
  double mx, my;       // 2D mean (pixels)
  float l11, l21, l22; // the conic Q = L L^T by its Cholesky factor L = [[l11, 0], [l21, l22]]:
                       // h = d^T Q d = (l11 dx + l21 dy)^2 + (l22 dy)^2
  float cr, cg, cb;    // colour
  float o;             // signed opacity
  float inv_nu;        // 1 / nu; 0 for the Gaussian family
  float nb;            // -(nu + 2) / 2; -log2(e) / 2 for the Gaussian family
  float hs;            // truncation level h*
  uint32_t entry;      // v * n + i
  float ey;            // half extent in y of the ellipse h <= h*: sqrt(h* Sigma2D_yy)
};
static_assert(sizeof(Rec) == SSS_RECORD_BYTES, "record size");

// Number of slots per entry in the screen-space gradient buffer:
// d/d(mx, my), d/d(qa, qb, qc), d/d(cr, cg, cb), d/do, d/dnu (+2 pad).  The
// per-entry buffer holds FP64 (it sums the partial sums of every tile the
// entry is listed in, often with cancellation); the deterministic mode's
// per-pair slots hold FP32.
constexpr int kG2 = 12;

// Brackets one kernel launch with HIP events when timing is enabled.
class KernelTimer {
 public:
  KernelTimer(const char* name, hipStream_t st);
  ~KernelTimer();

 private:
  const char* name_;
  hipStream_t st_;
  hipEvent_t a_ = nullptr, b_ = nullptr;
};

// Launch with optional event timing under the kernel's short name.
#define SSS_LAUNCH(label, kernel, grid, block, shmem, stream, ...)         \
  do {                                                                     \
    ::sss::KernelTimer sss_kt_(label, stream);                             \
    hipLaunchKernelGGL(kernel, grid, block, shmem, stream, __VA_ARGS__);   \
  } while (0)

void set_error(const char* fmt, ...);
bool hip_ok(hipError_t e, const char* what);
int make_cam_batch(const sss_camera_t* cams, int n_views, CamBatch* out);
OptsDev make_opts(const sss_render_opts_t* o);

// launchers (stream is hipStream_t)
void launch_project(const CamBatch& cb, const OptsDev& op, const sss_scene_t& s,
                    const sss_proj_t& out, hipStream_t st);
struct StepArgs;
void launch_project_bwd(const CamBatch& cb, const OptsDev& op, const sss_scene_t& s,
                        const uint32_t* touched, double* g2, const sss_grads_t& g, const StepArgs& sa,
                        hipStream_t st);
int run_bin_sort(const CamBatch& cb, const sss_proj_t& proj, int64_t n, sss_bins_t* bins,
                 void* ws, size_t ws_bytes, hipStream_t st);
size_t bin_sort_workspace(int64_t n_entries, int64_t pair_capacity);
void launch_render_fwd(const CamBatch& cb, const OptsDev& op, const sss_bins_t& b,
                       float* image, float* t_final, uint32_t* n_contrib, hipStream_t st);
// Per-entry FP64 ellipse written by the projection: 2D covariance
// [[A, B], [B, D]] and the level hr of the listed ellipse
// {d : d^T Sigma^-1 d <= hr} (see tiles.hpp).
struct Ellipse {
  double A, B, D, hr;
};

// One projected entry (the layout sss.h states): the raster record, the
// FP64 ellipse and the tile rectangle in one 128-byte line.
struct __align__(16) Entry {
  Rec rec;
  Ellipse ell;
  ushort4 rect;
  uint32_t pad[6];
};
static_assert(sizeof(Entry) == SSS_ENTRY_BYTES, "entry size");

// Buffers of the deterministic backward pass (see raster.hip).
struct DetArgs {
  const uint32_t* order;      // rank -> entry
  const uint32_t* rank_off;   // first emission position of each rank
  const Entry* ent;           // projected entries (tile rectangles and ellipses)
  float* part;                // [n_pairs][kG2] per-pair sums
  uint32_t* lastp1;           // [n_tiles] last visited rank + 1
  float* loss_part;           // [n_tiles] per-tile loss (both modes)
  uint32_t* order_ws;         // [4 n_tiles] the backward's own unit order (both modes)
  const uint32_t* tile_order; // launch order (nullable: row-major) of tiles, or of units if unit_order
  int32_t unit_order;
  uint32_t n_pairs;           // bound of the slots (part has n_pairs rows)
  uint32_t* queue;            // work counter of the persistent backward (zeroed before the launch)
  uint32_t n_units;           // launch slots of the backward
};
// Items (tiles or units) sorted by a coarse bucket of their cost, most
// expensive first.  The cost of item t is the largest of
// strip_cost[k*t .. k*t + k) (k = strips_per_item) or, when strip_cost is
// NULL, the list length of tile t from tile_start.
void launch_tile_order(const uint32_t* strip_cost, int strips_per_item, const uint32_t* tile_start, int64_t n_items,
                       uint32_t* order, hipStream_t st);
size_t render_bwd_det_workspace(int64_t n_entries, int64_t n_pairs, int64_t n_tiles);
size_t render_bwd_workspace(int64_t n_entries, int64_t n_tiles);
DetArgs carve_bwd(void* ws, int64_t n_entries, int64_t n_tiles, double** g2);
DetArgs carve_det(void* ws, int64_t n_entries, int64_t n_pairs, int64_t n_tiles, double** g2);
void launch_render_bwd(const CamBatch& cb, const OptsDev& op, const sss_bins_t& b, int mode,
                       int loss, const float* dl_or_target, const float* image,
                       const uint32_t* n_contrib, float* image_out, float* loss_out, double* g2,
                       int64_t total_pixels, bool det_mode, const DetArgs& dargs, int64_t n, hipStream_t st);
void launch_zero(float* p, int64_t count, hipStream_t st);
// Argument checks and launches of sss_render_bwd (api.hip); ws == nullptr
// checks only and returns the workspace size in *need_out.
int render_bwd_impl(const char* fn, const sss_scene_t* scene, const sss_proj_t* proj, const sss_bins_t* bins,
                    const sss_camera_t* cams, int n_views, const sss_render_opts_t* opts, int mode, int loss,
                    const float* dl_or_target, const float* image, const uint32_t* n_contrib, float* image_out,
                    float* loss_out, const sss_grads_t* grads, const sss_step_t* step, void* ws, size_t ws_bytes,
                    size_t* need_out, hipStream_t st);
size_t relocate_workspace(int64_t n, double max_fraction);
size_t loss_workspace(int64_t total_pixels);
void launch_loss(const CamBatch& cb, const float* img, const float* tgt, float lam, float* dl, float* loss_out,
                 float* partial, int64_t total_pixels, hipStream_t st);
int run_relocate(const sss_scene_t& s, float* const* state, const int32_t* widths, int n_state,
                 const sss_relocate_opts_t& o, void* ws, size_t ws_bytes, int64_t* n_moved, hipStream_t st);
void launch_sghmc(float* means, float* mom, const float* g, const float* opac, const float* scales,
                  const float* quats, int64_t n, const sss_sghmc_opts_t& o, hipStream_t st);
void launch_adam(const sss_adam_t& ad, hipStream_t st);
void launch_regularise(const float* opac, const float* scales, int64_t n, float eps_o, float eps_s, float* d_opac,
                       float* d_scales, float* loss_out, hipStream_t st);

}  // namespace sss
