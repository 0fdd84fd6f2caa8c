// sss_render_bwd_noalloc: sss_render_bwd with its workspace held by the
// library, for callers that cannot allocate device memory.
//
// The workspace is the file-scope device array `scratch` below.  Every GPU
// the library runs on holds its own copy, at its own address, for the life
// of the process.  In host code the name `scratch` is only a host-side
// handle: its device address comes from hipGetSymbolAddress, looked up once
// per device (with that device current) on the first call there and kept in
// g_ptr[device].  Only that address is handed to the kernels.
//
// Calls that overlap on one GPU share the one array and race; the caller
// serialises them (one stream, or events between streams).  Every part of
// the array that must start at zero is cleared by a kernel of the call.
#include <mutex>

#include "common.hpp"

namespace sss {
namespace {

constexpr size_t kScratchBytes = SSS_NOALLOC_WORKSPACE_BYTES;
__device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

// Device address of the current device's copy of `scratch`.
int scratch_address(void** out) {
  int dev = -1;
  if (!hip_ok(hipGetDevice(&dev), "sss_render_bwd_noalloc: hipGetDevice")) return SSS_ERR_HIP;
  if (dev < 0 || dev >= kMaxDevices) {
    set_error("sss_render_bwd_noalloc: device %d outside 0..%d", dev, kMaxDevices - 1);
    return SSS_ERR_UNSUPPORTED;
  }
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_ptr[dev]) {
    void* p = nullptr;
    if (!hip_ok(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "sss_render_bwd_noalloc: hipGetSymbolAddress"))
      return SSS_ERR_HIP;
    if (!p) {
      set_error("sss_render_bwd_noalloc: hipGetSymbolAddress returned a null address");
      return SSS_ERR_HIP;
    }
    g_ptr[dev] = p;
  }
  *out = g_ptr[dev];
  return SSS_OK;
}

}  // namespace
}  // namespace sss

using namespace sss;

extern "C" int sss_render_bwd_noalloc(const sss_scene_t* scene, const sss_proj_t* proj, const sss_bins_t* bins,
                                      const sss_camera_t* cams, int n_views, const sss_render_opts_t* opts,
                                      int mode, int loss, const float* dl_or_target, const float* image,
                                      const uint32_t* n_contrib, float* image_out, float* loss_out,
                                      const sss_grads_t* grads, void* stream) {
  static const char* fn = "sss_render_bwd_noalloc";
  const hipStream_t st = (hipStream_t)stream;
  // arguments and the workspace size first: nothing is enqueued
  size_t need = 0;
  int rc = render_bwd_impl(fn, scene, proj, bins, cams, n_views, opts, mode, loss, dl_or_target, image, n_contrib,
                           image_out, loss_out, grads, nullptr, nullptr, 0, &need, st);
  if (rc) return rc;
  if (need > kScratchBytes) {
    set_error("%s: the call needs a workspace of %zu bytes and the library holds %zu (SSS_NOALLOC_WORKSPACE_BYTES); "
              "call sss_render_bwd with a workspace of its own", fn, need, kScratchBytes);
    return SSS_ERR_INVALID;
  }
  void* ws = nullptr;
  if ((rc = scratch_address(&ws))) return rc;
  return render_bwd_impl(fn, scene, proj, bins, cams, n_views, opts, mode, loss, dl_or_target, image, n_contrib,
                         image_out, loss_out, grads, nullptr, ws, kScratchBytes, nullptr, st);
}
