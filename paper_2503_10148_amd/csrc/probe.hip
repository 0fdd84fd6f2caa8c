// Streaming copy: a measurement aid, not a step of the method.  Timing it
// gives the HBM rate that a kernel built the way the library's streaming
// kernels are (16-byte non-temporal loads and stores, several in flight per
// thread, many workgroups) reaches on the device; the memory-bound stages'
// rates are read against it.
#include "common.hpp"

namespace sss {
namespace {

typedef float f4 __attribute__((ext_vector_type(4)));
constexpr int kCopyThreads = 256;
constexpr int kCopyRuns = 4;              // 16-byte runs in flight per thread
constexpr int64_t kCopyGrid = 32768;      // workgroups (grid-stride beyond)

__global__ __launch_bounds__(kCopyThreads) void stream_copy_kernel(const f4* __restrict__ src, f4* __restrict__ dst,
                                                                   int64_t n4) {
  const int64_t stride = (int64_t)gridDim.x * kCopyThreads * kCopyRuns;
  for (int64_t i = (int64_t)blockIdx.x * kCopyThreads * kCopyRuns + threadIdx.x; i < n4; i += stride) {
    f4 v[kCopyRuns];
#pragma unroll
    for (int u = 0; u < kCopyRuns; ++u)
      if (i + (int64_t)u * kCopyThreads < n4) v[u] = __builtin_nontemporal_load(src + i + (int64_t)u * kCopyThreads);
#pragma unroll
    for (int u = 0; u < kCopyRuns; ++u)
      if (i + (int64_t)u * kCopyThreads < n4) __builtin_nontemporal_store(v[u], dst + i + (int64_t)u * kCopyThreads);
  }
}

}  // namespace
}  // namespace sss

extern "C" int sss_stream_copy(const void* src, void* dst, size_t bytes, void* stream) {
  using namespace sss;
  if (!src || !dst || ((uintptr_t)src & 15u) || ((uintptr_t)dst & 15u) || (bytes & 15u)) {
    set_error("sss_stream_copy: NULL or not 16-byte aligned pointer, or a size that is not a multiple of 16");
    return SSS_ERR_INVALID;
  }
  const int64_t n4 = (int64_t)(bytes / 16);
  if (n4 == 0) return SSS_OK;
  const int64_t per = (int64_t)kCopyThreads * kCopyRuns;
  const int64_t blocks = (n4 + per - 1) / per;
  const dim3 grid((unsigned)(blocks < kCopyGrid ? blocks : kCopyGrid));
  hipStream_t st = (hipStream_t)stream;
  SSS_LAUNCH("stream_copy", stream_copy_kernel, grid, dim3(kCopyThreads), 0, st, (const f4*)src, (f4*)dst, n4);
  return hip_ok(hipGetLastError(), "sss_stream_copy launch") ? SSS_OK : SSS_ERR_HIP;
}
