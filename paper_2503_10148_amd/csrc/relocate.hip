// Recycling of low-opacity components (Sec. 3.4 "Adding and Recycling
// Components", eq. relocation; SM "Component Recycling").
//
//  1. dead components (|o| <= dead_opacity) are listed in index order and at
//     most floor(n * max_fraction) of them move;
//  2. live components get integer weights floor(|o| 2^24) (exact in FP32);
//     a 64-bit exclusive scan gives their intervals, so drawing a target is
//     exact integer arithmetic: draw j takes Philox4x32-10 words (x0, x1) at
//     counter (j, step lo, step hi, 2^31 | j hi), position
//     floor(((x1 << 32) | x0) * W / 2^64), and a binary search;
//  3. a target drawn m times ends with N = m + 1 components at its mean: the
//     moved ones copy it, all N take (1 - o_new)^N = 1 - |o| (sign kept) and
//     the covariance factor o^2 (beta(1/2, (nu+2)/2) / K)^2, with nu unchanged
//     and K the binomial sum of beta functions, evaluated through ln Gamma in
//     FP64; the moved components' optimiser state rows are zeroed.
// Every count stays on the device; grids are sized by the cap.
#include "common.hpp"
#include "step.hpp"
#include "scan.hpp"

namespace sss {
namespace {

__global__ __launch_bounds__(kBlock) void rl_weights_kernel(const float* __restrict__ opac, int64_t n, float dead,
                                                            uint32_t* __restrict__ flag,
                                                            unsigned long long* __restrict__ w) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const float a = fabsf(opac[i]);
  const bool d = a <= dead;
  flag[i] = d ? 1u : 0u;
  w[i] = d ? 0ull : (unsigned long long)floorf(a * 16777216.0f);
}

// counts[0] = number moved, counts[1] = total weight W
__global__ void rl_counts_kernel(const uint32_t* __restrict__ flag, const uint32_t* __restrict__ pos,
                                 const unsigned long long* __restrict__ w, const unsigned long long* __restrict__ excl,
                                 int64_t n, int64_t cap, unsigned long long* __restrict__ counts) {
  const unsigned long long nd = (unsigned long long)pos[n - 1] + flag[n - 1];
  counts[0] = nd < (unsigned long long)cap ? nd : (unsigned long long)cap;
  counts[1] = excl[n - 1] + w[n - 1];
}

__global__ __launch_bounds__(kBlock) void rl_dead_list_kernel(const uint32_t* __restrict__ flag,
                                                              const uint32_t* __restrict__ pos, int64_t n, int64_t cap,
                                                              uint32_t* __restrict__ dead) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < n && flag[i] && (int64_t)pos[i] < cap) dead[pos[i]] = (uint32_t)i;
}

__global__ __launch_bounds__(kBlock) void rl_draw_kernel(const unsigned long long* __restrict__ excl, int64_t n,
                                                         const unsigned long long* __restrict__ counts, int64_t cap,
                                                         uint64_t seed, uint64_t step, uint32_t* __restrict__ target,
                                                         uint32_t* __restrict__ hits) {
  const int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (j >= cap || j >= (int64_t)counts[0] || counts[1] == 0) return;
  const uint4 x = philox4x32_10(make_uint4((uint32_t)j, (uint32_t)step, (uint32_t)(step >> 32), 0x80000000u | (uint32_t)(j >> 32)),
                         make_uint2((uint32_t)seed, (uint32_t)(seed >> 32)));
  const unsigned long long r = ((unsigned long long)x.y << 32) | x.x;
  const unsigned long long pos = __umul64hi(r, counts[1]);
  int64_t lo = 0, hi = n;                 // last t with excl[t] <= pos
  while (hi - lo > 1) {
    const int64_t mid = (lo + hi) >> 1;
    if (excl[mid] <= pos) lo = mid;
    else hi = mid;
  }
  target[j] = (uint32_t)lo;
  atomicAdd(hits + lo, 1u);
}

// New opacity and covariance factor for N components replacing one of
// opacity o and degrees of freedom nu (nu unchanged).
__device__ void relocation_rule(float o, float nu_raw, int N, float* o_new, float* scale_mul) {
  const double a = fabs((double)o);
  const double nu = fmin(fmax((double)nu_raw, 1.0), 1e4);
  const double on = 1.0 - pow(1.0 - a, 1.0 / (double)N);
  double K = 0.0;
  for (int i = 1; i <= N; ++i) {
    double binom = 1.0;
    for (int k = 0; k < i; ++k) {
      const double y = ((k + 1) * (nu + 3.0) - 1.0) * 0.5;
      const double lb = lgamma(0.5) + lgamma(y) - lgamma(0.5 + y);
      K += ((k & 1) ? -binom : binom) * pow(on, (double)(k + 1)) * exp(lb);
      binom = binom * (double)(i - 1 - k) / (double)(k + 1);
    }
  }
  const double yo = (nu + 2.0) * 0.5;
  const double bo = exp(lgamma(0.5) + lgamma(yo) - lgamma(0.5 + yo));
  const double ratio = bo / K;
  *o_new = (float)(o < 0.0f ? -on : on);
  *scale_mul = (float)sqrt(a * a * ratio * ratio);
}

struct StateRows {
  float* ptr[8];
  int32_t width[8];
  int32_t count;
};

__global__ __launch_bounds__(kBlock) void rl_move_kernel(
    const unsigned long long* __restrict__ counts, int64_t cap, const uint32_t* __restrict__ dead,
    const uint32_t* __restrict__ target, const uint32_t* __restrict__ hits, int kc, float* __restrict__ means,
    float* __restrict__ scales, float* __restrict__ quats, float* __restrict__ nu, float* __restrict__ opac,
    float* __restrict__ sh, StateRows st) {
  const int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (j >= cap || j >= (int64_t)counts[0] || counts[1] == 0) return;
  const int64_t d = dead[j], t = target[j];
  float on, mul;
  relocation_rule(opac[t], nu[t], (int)hits[t] + 1, &on, &mul);
  for (int a = 0; a < 3; ++a) {
    means[3 * d + a] = means[3 * t + a];
    scales[3 * d + a] = scales[3 * t + a] * mul;
  }
  for (int a = 0; a < 4; ++a) quats[4 * d + a] = quats[4 * t + a];
  nu[d] = nu[t];
  opac[d] = on;
  for (int a = 0; a < kc; ++a) sh[(size_t)d * kc + a] = sh[(size_t)t * kc + a];
  for (int s = 0; s < st.count; ++s)
    for (int a = 0; a < st.width[s]; ++a) st.ptr[s][(size_t)d * st.width[s] + a] = 0.0f;
}

__global__ __launch_bounds__(kBlock) void rl_targets_kernel(const uint32_t* __restrict__ hits, int64_t n,
                                                            float* __restrict__ scales, const float* __restrict__ nu,
                                                            float* __restrict__ opac) {
  const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (t >= n || hits[t] == 0) return;
  float on, mul;
  relocation_rule(opac[t], nu[t], (int)hits[t] + 1, &on, &mul);
  opac[t] = on;
  for (int a = 0; a < 3; ++a) scales[3 * t + a] *= mul;
}

struct RlWs {
  uint32_t *flag, *pos, *dead, *target, *hits, *scan32;
  unsigned long long *w, *excl, *scan64, *counts;
  size_t bytes;
};

RlWs rl_carve(void* base, int64_t n, int64_t cap) {
  RlWs w;
  char* p = (char*)base;
  size_t off = 0;
  auto take = [&](size_t b) { char* q = p ? p + off : nullptr; off += (b + 255) & ~(size_t)255; return q; };
  w.counts = (unsigned long long*)take(4 * sizeof(unsigned long long));
  w.flag = (uint32_t*)take(4 * (size_t)n);
  w.pos = (uint32_t*)take(4 * (size_t)n);
  w.hits = (uint32_t*)take(4 * (size_t)n);
  w.dead = (uint32_t*)take(4 * (size_t)(cap > 0 ? cap : 1));
  w.target = (uint32_t*)take(4 * (size_t)(cap > 0 ? cap : 1));
  w.w = (unsigned long long*)take(8 * (size_t)n);
  w.excl = (unsigned long long*)take(8 * (size_t)n);
  w.scan32 = (uint32_t*)take(4 * (size_t)scan_ws_words(n));
  w.scan64 = (unsigned long long*)take(8 * (size_t)scan_ws_words(n));
  w.bytes = off;
  return w;
}

__global__ __launch_bounds__(kBlock) void rl_zero_kernel(uint32_t* __restrict__ p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < n) p[i] = 0u;
}

}  // namespace

size_t relocate_workspace(int64_t n, double max_fraction) {
  const int64_t cap = (int64_t)floor((double)n * max_fraction);
  return rl_carve(nullptr, n, cap).bytes;
}

int run_relocate(const sss_scene_t& s, float* const* state, const int32_t* widths, int n_state,
                 const sss_relocate_opts_t& o, void* ws, size_t ws_bytes, int64_t* n_moved, hipStream_t st) {
  const int64_t n = s.n;
  const int64_t cap = (int64_t)floor((double)n * (double)o.max_fraction);
  RlWs w = rl_carve(ws, n, cap);
  if (ws_bytes < w.bytes) {
    set_error("sss_relocate: workspace of %zu bytes, %zu needed", ws_bytes, w.bytes);
    return SSS_ERR_INVALID;
  }
  StateRows sr;
  sr.count = n_state;
  for (int k = 0; k < 8; ++k) {
    sr.ptr[k] = k < n_state ? state[k] : nullptr;
    sr.width[k] = k < n_state ? widths[k] : 0;
  }
  float* means = const_cast<float*>(s.means);
  float* scales = const_cast<float*>(s.scales);
  float* quats = const_cast<float*>(s.quats);
  float* nu = const_cast<float*>(s.nu);
  float* opac = const_cast<float*>(s.opacity);
  float* sh = const_cast<float*>(s.sh);
  const int kc = 3 * (s.sh_degree + 1) * (s.sh_degree + 1);
  const unsigned gn = (unsigned)((n + kBlock - 1) / kBlock);
  const unsigned gc = (unsigned)((cap + kBlock - 1) / kBlock);
  SSS_LAUNCH("rl_zero", rl_zero_kernel, dim3(gn), dim3(kBlock), 0, st, w.hits, n);
  SSS_LAUNCH("rl_weights", rl_weights_kernel, dim3(gn), dim3(kBlock), 0, st, s.opacity, n, o.dead_opacity, w.flag, w.w);
  scan_excl<uint32_t>(w.flag, w.pos, n, w.scan32, st);
  scan_excl<unsigned long long>(w.w, w.excl, n, w.scan64, st);
  SSS_LAUNCH("rl_counts", rl_counts_kernel, dim3(1), dim3(1), 0, st, w.flag, w.pos, w.w, w.excl, n, cap, w.counts);
  if (cap > 0) {
    SSS_LAUNCH("rl_dead_list", rl_dead_list_kernel, dim3(gn), dim3(kBlock), 0, st, w.flag, w.pos, n, cap, w.dead);
    SSS_LAUNCH("rl_draw", rl_draw_kernel, dim3(gc), dim3(kBlock), 0, st, w.excl, n, w.counts, cap, o.seed, o.step,
               w.target, w.hits);
    SSS_LAUNCH("rl_move", rl_move_kernel, dim3(gc), dim3(kBlock), 0, st, w.counts, cap, w.dead, w.target, w.hits, kc,
               means, scales, quats, nu, opac, sh, sr);
    SSS_LAUNCH("rl_targets", rl_targets_kernel, dim3(gn), dim3(kBlock), 0, st, w.hits, n, scales, nu, opac);
  }
  if (!hip_ok(hipGetLastError(), "sss_relocate launch")) return SSS_ERR_HIP;
  if (n_moved) {
    unsigned long long c[2];
    if (!hip_ok(hipMemcpyAsync(c, w.counts, sizeof(c), hipMemcpyDeviceToHost, st), "count readback")) return SSS_ERR_HIP;
    if (!hip_ok(hipStreamSynchronize(st), "count sync")) return SSS_ERR_HIP;
    *n_moved = c[1] == 0 ? 0 : (int64_t)c[0];
  }
  return SSS_OK;
}

}  // namespace sss
