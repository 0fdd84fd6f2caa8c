// C-ABI entry points (include/sss.h): argument validation, camera and option
// marshalling, workspace carving and kernel launches.
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include "common.hpp"
#include "step.hpp"

namespace sss {

static thread_local char g_err[512] = "";

void set_error(const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
}

bool hip_ok(hipError_t e, const char* what) {
  if (e == hipSuccess) return true;
  set_error("%s: %s", what, hipGetErrorString(e));
  return false;
}

int make_cam_batch(const sss_camera_t* cams, int n_views, CamBatch* out) {
  if (!cams || n_views < 1 || n_views > SSS_MAX_VIEWS) {
    set_error("n_views must be in 1..%d and cams non-null", SSS_MAX_VIEWS);
    return SSS_ERR_INVALID;
  }
  memset(out, 0, sizeof(*out));
  int64_t tiles = 0, pix = 0;
  for (int v = 0; v < n_views; ++v) {
    const sss_camera_t& c = cams[v];
    if (c.width <= 0 || c.height <= 0 || c.width > 65535 * kTile || c.height > 65535 * kTile ||
        !(c.fx > 0.0f) || !(c.fy > 0.0f)) {
      set_error("camera %d: width/height must be positive and focal lengths > 0", v);
      return SSS_ERR_INVALID;
    }
    CamDev& d = out->v[v];
    for (int r = 0; r < 3; ++r) {
      for (int k = 0; k < 3; ++k) d.R[3 * r + k] = c.viewmat[4 * r + k];
      d.t[r] = c.viewmat[4 * r + 3];
    }
    d.fx = c.fx; d.fy = c.fy; d.cx = c.cx; d.cy = c.cy;
    d.W = c.width; d.H = c.height;
    d.tiles_x = (c.width + kTile - 1) / kTile;
    d.tiles_y = (c.height + kTile - 1) / kTile;
    d.tile_offset = (int32_t)tiles;
    d.pix_offset = pix;
    tiles += (int64_t)d.tiles_x * d.tiles_y;
    pix += (int64_t)c.width * c.height;
  }
  if (tiles > (int64_t)0x7FFFFFFF) {
    set_error("too many tiles");
    return SSS_ERR_UNSUPPORTED;
  }
  out->n_views = n_views;
  out->total_tiles = (int32_t)tiles;
  return SSS_OK;
}

OptsDev make_opts(const sss_render_opts_t* o) {
  sss_render_opts_t d;
  if (!o) {
    sss_default_render_opts(&d);
    o = &d;
  }
  OptsDev r;
  // a t_min below the smallest normal float acts as that value, so a
  // compositing pixel's transmittance stays positive and a finished one's
  // (negated) stays below it whatever it is multiplied by
  r.alpha_min = o->alpha_min; r.alpha_max = o->alpha_max; r.t_min = fmaxf(o->t_min, 1.17549435e-38f);
  r.z_near = o->z_near;
  r.nu_min = o->nu_min; r.nu_max = o->nu_max; r.lowpass = o->lowpass;
  r.bg[0] = o->bg[0]; r.bg[1] = o->bg[1]; r.bg[2] = o->bg[2];
  r.family = o->family;
  r.trunc_mode = o->trunc_mode;
  return r;
}

static int check_scene(const sss_scene_t* s, const char* fn) {
  if (!s || s->n <= 0 || s->n > (int64_t)0xFFFFFFFF / SSS_MAX_VIEWS || s->sh_degree < 0 || s->sh_degree > 3 ||
      !s->means || !s->scales || !s->quats || !s->nu || !s->opacity || !s->sh) {
    set_error("%s: scene needs n in 1..%lld, sh_degree in 0..3 and six non-null arrays", fn,
              (long long)(0xFFFFFFFFll / SSS_MAX_VIEWS));
    return SSS_ERR_INVALID;
  }
  // quaternions and SH rows are read with 16-byte loads
  if (((uintptr_t)s->quats | (uintptr_t)s->sh) & 15) {
    set_error("%s: scene quats and sh must be 16-byte aligned", fn);
    return SSS_ERR_INVALID;
  }
  return SSS_OK;
}

static int check_opts(const sss_render_opts_t* o, const char* fn) {
  if (!o) return SSS_OK;
  if (!(o->alpha_min >= 0.0f) || !(o->alpha_max > 0.0f && o->alpha_max < 1.0f) || !(o->t_min >= 0.0f) ||
      !(o->nu_min >= 1.0f) ||
      !(o->nu_max >= o->nu_min) || !(o->lowpass >= 0.0f) ||
      (o->family != SSS_FAMILY_STUDENT_T && o->family != SSS_FAMILY_GAUSSIAN) ||
      (o->trunc_mode != SSS_TRUNC_ALPHA && o->trunc_mode != SSS_TRUNC_COVERAGE)) {
    set_error("%s: options out of range (alpha_min >= 0, 0 < alpha_max < 1, t_min >= 0, 1 <= nu_min <= nu_max, "
              "lowpass >= 0, known family and truncation mode)", fn);
    return SSS_ERR_INVALID;
  }
  return SSS_OK;
}

static int64_t total_pixels(const CamBatch& cb) {
  int64_t p = 0;
  for (int v = 0; v < cb.n_views; ++v) p += (int64_t)cb.v[v].W * cb.v[v].H;
  return p;
}

}  // namespace sss

using namespace sss;

extern "C" {

void sss_default_render_opts(sss_render_opts_t* o) {
  if (!o) return;
  o->alpha_min = 1.0f / 255.0f;
  o->alpha_max = 0.99f;
  o->t_min = 1e-4f;
  o->z_near = 0.2f;
  o->nu_min = 1.0f;
  o->nu_max = 1e4f;
  o->lowpass = 0.0f;
  o->bg[0] = o->bg[1] = o->bg[2] = 0.0f;
  o->family = SSS_FAMILY_STUDENT_T;
  o->trunc_mode = SSS_TRUNC_ALPHA;
}

const char* sss_last_error(void) { return g_err; }
int sss_version(void) { return SSS_VERSION; }

int64_t sss_total_tiles(const sss_camera_t* cams, int n_views) {
  CamBatch cb;
  if (make_cam_batch(cams, n_views, &cb) != SSS_OK) return -1;
  return cb.total_tiles;
}

int64_t sss_total_pixels(const sss_camera_t* cams, int n_views) {
  CamBatch cb;
  if (make_cam_batch(cams, n_views, &cb) != SSS_OK) return -1;
  return total_pixels(cb);
}

size_t sss_bin_sort_workspace(int64_t n_entries, int64_t pair_capacity) {
  if (n_entries < 0 || pair_capacity < 0) return 0;
  return bin_sort_workspace(n_entries, pair_capacity);
}

size_t sss_render_bwd_workspace(int64_t n_entries, int64_t n_tiles) {
  if (n_entries < 0 || n_tiles < 0) return 0;
  return render_bwd_workspace(n_entries, n_tiles);
}

int sss_project(const sss_scene_t* scene, const sss_camera_t* cams, int n_views, const sss_render_opts_t* opts,
                const sss_proj_t* out, void* stream) {
  int rc = check_scene(scene, "sss_project");
  if (rc) return rc;
  if ((rc = check_opts(opts, "sss_project"))) return rc;
  CamBatch cb;
  if ((rc = make_cam_batch(cams, n_views, &cb))) return rc;
  if (!out || !out->entries || !out->depth_key || !out->tiles_touched) {
    set_error("sss_project: output arrays must be non-null");
    return SSS_ERR_INVALID;
  }
  if ((uintptr_t)out->entries & 15) {
    set_error("sss_project: entries must be 16-byte aligned");
    return SSS_ERR_INVALID;
  }
  hipStream_t st = (hipStream_t)stream;
  launch_project(cb, make_opts(opts), *scene, *out, st);
  return hip_ok(hipGetLastError(), "sss_project launch") ? SSS_OK : SSS_ERR_HIP;
}

// Workspaces are carved into 256-byte aligned parts, read with 16-byte loads.
static bool ws_aligned(const void* ws, const char* fn) {
  if (((uintptr_t)ws & 255) == 0) return true;
  set_error("%s: workspace must be 256-byte aligned", fn);
  return false;
}

int sss_bin_sort(const sss_proj_t* proj, const sss_camera_t* cams, int n_views, int64_t n, sss_bins_t* bins,
                 void* ws, size_t ws_bytes, void* stream) {
  CamBatch cb;
  int rc = make_cam_batch(cams, n_views, &cb);
  if (rc) return rc;
  if (!proj || !proj->entries || !proj->depth_key || !proj->tiles_touched || !bins ||
      !bins->order || !bins->sorted_records || !bins->tile_start || !bins->pair_rank || !ws || n <= 0 ||
      bins->pair_capacity < 0 || n > (int64_t)0xFFFFFFFF / SSS_MAX_VIEWS) {
    set_error("sss_bin_sort: null pointer, n <= 0 or negative pair capacity");
    return SSS_ERR_INVALID;
  }
  if (!ws_aligned(ws, "sss_bin_sort")) return SSS_ERR_INVALID;
  return run_bin_sort(cb, *proj, n, bins, ws, ws_bytes, (hipStream_t)stream);
}

int sss_render_fwd(const sss_bins_t* bins, const sss_camera_t* cams, int n_views, const sss_render_opts_t* opts,
                   float* image, float* t_final, uint32_t* n_contrib, void* stream) {
  CamBatch cb;
  int rc = make_cam_batch(cams, n_views, &cb);
  if (rc) return rc;
  if ((rc = check_opts(opts, "sss_render_fwd"))) return rc;
  if (!bins || !bins->sorted_records || !bins->tile_start || !bins->pair_rank || !image) {
    set_error("sss_render_fwd: bins arrays and image must be non-null");
    return SSS_ERR_INVALID;
  }
  launch_render_fwd(cb, make_opts(opts), *bins, image, t_final, n_contrib, (hipStream_t)stream);
  return hip_ok(hipGetLastError(), "sss_render_fwd launch") ? SSS_OK : SSS_ERR_HIP;
}

}  // extern "C"

namespace sss {

// The body of sss_render_bwd and of its variant with a library-held
// workspace (noalloc.hip).  ws == nullptr asks for the size check only:
// on success *need is the workspace size and nothing is enqueued; with a
// workspace, the check and the launches.
// Checks the fused update's arguments and fills its kernel arguments.
static int make_step_args(const char* fn, const sss_scene_t* scene, const sss_step_t* step, StepArgs* sa) {
  *sa = StepArgs{};
  if (!step) return SSS_OK;
  const float* want[6] = {scene->means, scene->scales, scene->quats, scene->nu, scene->opacity, scene->sh};
  for (int k = 0; k < 6; ++k)
    if (step->params[k] != want[k]) {
      set_error("%s: step->params[%d] must be the scene's array", fn, k);
      return SSS_ERR_INVALID;
    }
  if (!step->momentum || !(step->sghmc.lr >= 0.0f)) {
    set_error("%s: step needs the momentum array and lr >= 0", fn);
    return SSS_ERR_INVALID;
  }
  if (step->adam) {
    if (step->t < 1) {
      set_error("%s: Adam needs t >= 1", fn);
      return SSS_ERR_INVALID;
    }
    for (int k = 0; k < 5; ++k)
      if (!step->m[k] || !step->v[k]) {
        set_error("%s: Adam moments of array %d are NULL", fn, k);
        return SSS_ERR_INVALID;
      }
  }
  sa->on = 1;
  sa->means = step->params[0];
  sa->scales = step->params[1];
  sa->quats = step->params[2];
  sa->nu = step->params[3];
  sa->opac = step->params[4];
  sa->sh = step->params[5];
  sa->mom = step->momentum;
  sa->sg = sghmc_args(step->sghmc);
  sa->adam = step->adam ? 1 : 0;
  if (step->adam) sa->ac = adam_const(step->beta1, step->beta2, step->eps, step->t);
  for (int k = 0; k < 5; ++k) {
    sa->m[k] = step->m[k];
    sa->v[k] = step->v[k];
    sa->lr[k] = step->lr[k];
    sa->lo[k] = step->lo[k];
    sa->hi[k] = step->hi[k];
  }
  return SSS_OK;
}

int render_bwd_impl(const char* fn, const sss_scene_t* scene, const sss_proj_t* proj, const sss_bins_t* bins,
                    const sss_camera_t* cams, int n_views, const sss_render_opts_t* opts, int mode, int loss,
                    const float* dl_or_target, const float* image, const uint32_t* n_contrib, float* image_out,
                    float* loss_out, const sss_grads_t* grads, const sss_step_t* step, void* ws, size_t ws_bytes,
                    size_t* need_out, hipStream_t st) {
  int rc = check_scene(scene, fn);
  if (rc) return rc;
  if ((rc = check_opts(opts, fn))) return rc;
  CamBatch cb;
  if ((rc = make_cam_batch(cams, n_views, &cb))) return rc;
  const bool det = (mode & SSS_BWD_DETERMINISTIC) != 0;
  mode &= ~SSS_BWD_DETERMINISTIC;
  if (mode != SSS_BWD_STORED && mode != SSS_BWD_RECOMPUTE) {
    set_error("%s: unknown mode %d", fn, mode);
    return SSS_ERR_INVALID;
  }
  if (loss != SSS_LOSS_GRAD && loss != SSS_LOSS_L1) {
    set_error("%s: unknown loss %d", fn, loss);
    return SSS_ERR_INVALID;
  }
  if (!proj || !proj->tiles_touched || !bins || !bins->sorted_records || !bins->tile_start || !bins->pair_rank ||
      !dl_or_target || (!grads && !step)) {
    set_error("%s: null pointer", fn);
    return SSS_ERR_INVALID;
  }
  StepArgs sa;
  if ((rc = make_step_args(fn, scene, step, &sa))) return rc;
  // with the fused update the gradients are optional, and written whole
  sss_grads_t gr{};
  if (grads) gr = *grads;
  if (step) gr.overwrite = 1;
  if (mode == SSS_BWD_STORED && (!image || !n_contrib)) {
    set_error("%s: STORED mode needs image and n_contrib", fn);
    return SSS_ERR_INVALID;
  }
  const int64_t n_entries = scene->n * n_views;
  if (det && (!bins->order || !bins->rank_offset || !proj->entries || bins->n_pairs < 0 ||
              bins->n_visible < 0 || bins->n_visible > n_entries)) {
    set_error("%s: the deterministic mode needs bins->order, bins->rank_offset, proj->entries and the "
              "host counts of an sss_bin_sort call that waited for them (no_wait = 0)", fn);
    return SSS_ERR_INVALID;
  }
  const size_t need = det ? render_bwd_det_workspace(n_entries, bins->n_pairs, cb.total_tiles)
                          : render_bwd_workspace(n_entries, cb.total_tiles);
  if (need_out) *need_out = need;
  if (!ws) return SSS_OK;
  if (ws_bytes < need) {
    set_error("%s: workspace of %zu bytes, %zu needed", fn, ws_bytes, need);
    return SSS_ERR_INVALID;
  }
  if (!ws_aligned(ws, fn)) return SSS_ERR_INVALID;
  const OptsDev op = make_opts(opts);
  double* g2 = (double*)ws;
  DetArgs da{};
  if (!det) da = carve_bwd(ws, n_entries, cb.total_tiles, &g2);
  if (det) {
    da = carve_det(ws, n_entries, bins->n_pairs, cb.total_tiles, &g2);
    da.order = bins->order;
    da.rank_off = bins->rank_offset;
    da.ent = (const Entry*)proj->entries;
    da.n_pairs = (uint32_t)bins->n_pairs;
  }
  launch_zero((float*)g2, n_entries * kG2 * 2, st);
  launch_render_bwd(cb, op, *bins, mode, loss, dl_or_target, image, n_contrib, image_out, loss_out, g2,
                    total_pixels(cb), det, da, scene->n, st);
  launch_project_bwd(cb, op, *scene, proj->tiles_touched, g2, gr, sa, st);
  return hip_ok(hipGetLastError(), fn) ? SSS_OK : SSS_ERR_HIP;
}


}  // namespace sss

extern "C" {

int sss_render_bwd(const sss_scene_t* scene, const sss_proj_t* proj, const sss_bins_t* bins,
                   const sss_camera_t* cams, int n_views, const sss_render_opts_t* opts, int mode, int loss,
                   const float* dl_or_target, const float* image, const uint32_t* n_contrib, float* image_out,
                   float* loss_out, const sss_grads_t* grads, void* ws, size_t ws_bytes, void* stream) {
  if (!ws) {
    set_error("sss_render_bwd: null workspace");
    return SSS_ERR_INVALID;
  }
  return render_bwd_impl("sss_render_bwd", scene, proj, bins, cams, n_views, opts, mode, loss, dl_or_target, image,
                         n_contrib, image_out, loss_out, grads, nullptr, ws, ws_bytes, nullptr, (hipStream_t)stream);
}

int sss_render_bwd_step(const sss_scene_t* scene, const sss_proj_t* proj, const sss_bins_t* bins,
                        const sss_camera_t* cams, int n_views, const sss_render_opts_t* opts, int mode, int loss,
                        const float* dl_or_target, const float* image, const uint32_t* n_contrib,
                        float* image_out, float* loss_out, const sss_grads_t* grads, const sss_step_t* step,
                        void* ws, size_t ws_bytes, void* stream) {
  if (!ws || !step) {
    set_error("sss_render_bwd_step: null workspace or step");
    return SSS_ERR_INVALID;
  }
  return render_bwd_impl("sss_render_bwd_step", scene, proj, bins, cams, n_views, opts, mode, loss, dl_or_target,
                         image, n_contrib, image_out, loss_out, grads, step, ws, ws_bytes, nullptr,
                         (hipStream_t)stream);
}

size_t sss_render_bwd_workspace_det(int64_t n_entries, int64_t n_pairs, int64_t n_tiles) {
  if (n_entries < 0 || n_pairs < 0 || n_tiles < 0) return 0;
  return render_bwd_det_workspace(n_entries, n_pairs, n_tiles);
}

int sss_sghmc_step(float* means, float* momentum, const float* grad_means, const float* opacity,
                   const float* scales, const float* quats, int64_t n, const sss_sghmc_opts_t* opts,
                   const sss_adam_t* adam, void* stream) {
  if (!means || !momentum || !grad_means || !opacity || !opts || n <= 0 || !(opts->lr >= 0.0f) ||
      (opts->burn_in && (!scales || !quats))) {
    set_error("sss_sghmc_step: null array, n <= 0 or lr < 0 (burn-in needs scales and quats)");
    return SSS_ERR_INVALID;
  }
  if (opts->burn_in && ((uintptr_t)quats & 15)) {
    set_error("sss_sghmc_step: quats must be 16-byte aligned");
    return SSS_ERR_INVALID;
  }
  if (adam) {
    if (adam->t < 1 || adam->n_arrays < 0 || adam->n_arrays > 6) {
      set_error("sss_sghmc_step: adam needs t >= 1 and 0..6 arrays");
      return SSS_ERR_INVALID;
    }
    for (int k = 0; k < adam->n_arrays; ++k) {
      const sss_adam_array_t& a = adam->arrays[k];
      if (a.count < 0 || (a.count > 0 && (!a.param || !a.grad || !a.m || !a.v))) {
        set_error("sss_sghmc_step: adam array %d has a null pointer or a negative count", k);
        return SSS_ERR_INVALID;
      }
    }
  }
  hipStream_t st = (hipStream_t)stream;
  launch_sghmc(means, momentum, grad_means, opacity, scales, quats, n, *opts, st);
  if (adam) launch_adam(*adam, st);
  return hip_ok(hipGetLastError(), "sss_sghmc_step launch") ? SSS_OK : SSS_ERR_HIP;
}

size_t sss_loss_workspace(int64_t total_pixels) {
  if (total_pixels < 0) return 0;
  return loss_workspace(total_pixels);
}

int sss_loss(const float* image, const float* target, const sss_camera_t* cams, int n_views, float lambda_dssim,
             float* dl_dimage, float* loss_out, void* ws, size_t ws_bytes, void* stream) {
  CamBatch cb;
  int rc = make_cam_batch(cams, n_views, &cb);
  if (rc) return rc;
  if (!image || !target || !dl_dimage || !ws || !(lambda_dssim >= 0.0f && lambda_dssim <= 1.0f)) {
    set_error("sss_loss: null pointer or lambda outside [0, 1]");
    return SSS_ERR_INVALID;
  }
  const int64_t P = total_pixels(cb);
  if (ws_bytes < loss_workspace(P)) {
    set_error("sss_loss: workspace of %zu bytes, %zu needed", ws_bytes, loss_workspace(P));
    return SSS_ERR_INVALID;
  }
  if (!ws_aligned(ws, "sss_loss")) return SSS_ERR_INVALID;
  launch_loss(cb, image, target, lambda_dssim, dl_dimage, loss_out, (float*)ws, P, (hipStream_t)stream);
  return hip_ok(hipGetLastError(), "sss_loss launch") ? SSS_OK : SSS_ERR_HIP;
}

int sss_regularise(const float* opacity, const float* scales, int64_t n, float eps_opacity, float eps_sigma,
                   float* d_opacity, float* d_scales, float* loss_out, void* stream) {
  if (!opacity || !scales || n <= 0 || n > (int64_t)0x7FFFFFFF * kBlock || !(eps_opacity >= 0.0f) ||
      !(eps_sigma >= 0.0f)) {
    set_error("sss_regularise: null array, n <= 0 or a negative weight");
    return SSS_ERR_INVALID;
  }
  launch_regularise(opacity, scales, n, eps_opacity, eps_sigma, d_opacity, d_scales, loss_out, (hipStream_t)stream);
  return hip_ok(hipGetLastError(), "sss_regularise launch") ? SSS_OK : SSS_ERR_HIP;
}

size_t sss_relocate_workspace(int64_t n, float max_fraction) {
  if (n < 1 || !(max_fraction >= 0.0f && max_fraction <= 1.0f)) return 0;
  return relocate_workspace(n, (double)max_fraction);
}

int sss_relocate(const sss_scene_t* scene, const sss_state_t* state, int n_state, const sss_relocate_opts_t* opts,
                 void* ws, size_t ws_bytes, int64_t* n_moved, void* stream) {
  int rc = check_scene(scene, "sss_relocate");
  if (rc) return rc;
  if (!opts || !(opts->max_fraction >= 0.0f && opts->max_fraction <= 1.0f) || !ws || n_state < 0 || n_state > 8 ||
      (n_state > 0 && !state)) {
    set_error("sss_relocate: options, workspace or state list invalid (max_fraction in [0,1], <= 8 states)");
    return SSS_ERR_INVALID;
  }
  if (!ws_aligned(ws, "sss_relocate")) return SSS_ERR_INVALID;
  float* ptrs[8];
  int32_t widths[8];
  for (int k = 0; k < n_state; ++k) {
    if (!state[k].ptr || state[k].width < 1) {
      set_error("sss_relocate: state array %d is null or has width < 1", k);
      return SSS_ERR_INVALID;
    }
    ptrs[k] = state[k].ptr;
    widths[k] = state[k].width;
  }
  return run_relocate(*scene, ptrs, widths, n_state, *opts, ws, ws_bytes, n_moved, (hipStream_t)stream);
}

}  // extern "C"
