// SGHMC on the component means (Sec. 3.4 eq. sigmoidUpdate, SM eq. SGHMC)
// and Adam on the other parameters (the per-element arithmetic is in
// step.hpp).  Elementwise and HBM-bound: one thread per component reads 40
// bytes (mean, momentum, gradient, opacity) and writes 24; the noise is
// generated in registers from a counter-based generator, so a step is
// reproducible from (seed, step) alone.
#include "common.hpp"
#include "step.hpp"

namespace sss {
namespace {

__global__ __launch_bounds__(kBlock) void sghmc_kernel(float* __restrict__ means, float* __restrict__ mom,
                                                       const float* __restrict__ grad, const float* __restrict__ opac,
                                                       const float* __restrict__ scales, const float* __restrict__ quats,
                                                       int64_t n, SghmcArgs a) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  float mu[3], r[3], G[3], s[3] = {0.0f, 0.0f, 0.0f};
  float4 q = make_float4(1.0f, 0.0f, 0.0f, 0.0f);
  for (int c = 0; c < 3; ++c) {
    mu[c] = means[3 * i + c];
    r[c] = mom[3 * i + c];
    G[c] = grad[3 * i + c];
  }
  if (a.burn_in) {
    q = *reinterpret_cast<const float4*>(quats + 4 * i);
    for (int c = 0; c < 3; ++c) s[c] = scales[3 * i + c];
  }
  sghmc_one(i, mu, r, G, opac[i], q, s, a);
  for (int c = 0; c < 3; ++c) {
    means[3 * i + c] = mu[c];
    mom[3 * i + c] = r[c];
  }
}

// Adam on up to six arrays in one launch: array a owns the workgroups
// [first_block[a], first_block[a+1]), so the array (and its pointers) is
// uniform over a workgroup and is picked on scalar registers.
struct AdamBatch {
  float* p[6];
  const float* g[6];
  float* m[6];
  float* v[6];
  int64_t count[6];
  uint32_t first_block[7];
  float lr[6], lo[6], hi[6];
  int32_t n;
};

// Elements per thread in the Adam kernel, 256 apart (each round of loads
// coalesced), all loaded before any is updated: 2-3% faster than one per
// thread; eight measured 13% slower.
constexpr int kAdamIt = 4;

__global__ __launch_bounds__(kBlock) void adam_kernel(AdamBatch ab, AdamConst ac) {
  int a = 0;
  for (int k = 1; k < ab.n; ++k)
    if (blockIdx.x >= ab.first_block[k]) a = k;
  a = __builtin_amdgcn_readfirstlane(a);
  const int64_t i0 = (int64_t)(blockIdx.x - ab.first_block[a]) * (kBlock * kAdamIt) + threadIdx.x;
  const int64_t cnt = ab.count[a];
  float* __restrict__ p = ab.p[a];
  float* __restrict__ m = ab.m[a];
  float* __restrict__ v = ab.v[a];
  const float* __restrict__ g = ab.g[a];
  // every element is touched once per step: streaming (non-temporal) loads
  // and stores keep the caches out of the way (measured 6% faster)
  float pi[kAdamIt], mi[kAdamIt], vi[kAdamIt], gi[kAdamIt];
#pragma unroll
  for (int k = 0; k < kAdamIt; ++k) {
    const int64_t i = i0 + (int64_t)k * kBlock;
    if (i < cnt) {
      pi[k] = __builtin_nontemporal_load(p + i); mi[k] = __builtin_nontemporal_load(m + i);
      vi[k] = __builtin_nontemporal_load(v + i); gi[k] = __builtin_nontemporal_load(g + i);
    }
  }
#pragma unroll
  for (int k = 0; k < kAdamIt; ++k) {
    const int64_t i = i0 + (int64_t)k * kBlock;
    if (i < cnt) {
      adam_one(pi[k], gi[k], mi[k], vi[k], ab.lr[a], ab.lo[a], ab.hi[a], ac);
      __builtin_nontemporal_store(pi[k], p + i);
      __builtin_nontemporal_store(mi[k], m + i);
      __builtin_nontemporal_store(vi[k], v + i);
    }
  }
}

// Regularisers of the Sec. 3.4 loss: eps_o sum_i |o_i| + eps_s sum_ij sqrt(lambda_ij)
// with lambda_ij the eigenvalues of Sigma_i = R S S^T R^T, i.e. |s_ij| (R is
// orthogonal).  Adds the (sub)gradient sign(x) eps to the opacity and scale
// gradients and accumulates the value.  HBM-bound: 16 B read, 16 B read +
// written per component.
__global__ __launch_bounds__(kBlock) void regularise_kernel(const float* __restrict__ opac,
                                                            const float* __restrict__ scales, int64_t n, float eps_o,
                                                            float eps_s, float* __restrict__ d_opac,
                                                            float* __restrict__ d_scales, float* __restrict__ loss_out) {
  __shared__ float red[kBlock / 64];
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  float acc = 0.0f;
  if (i < n) {
    const float o = opac[i];
    acc = eps_o * fabsf(o);
    if (d_opac) d_opac[i] += o > 0.0f ? eps_o : (o < 0.0f ? -eps_o : 0.0f);
    for (int a = 0; a < 3; ++a) {
      const float s = scales[3 * i + a];
      acc += eps_s * fabsf(s);
      if (d_scales) d_scales[3 * i + a] += s > 0.0f ? eps_s : (s < 0.0f ? -eps_s : 0.0f);
    }
  }
  if (loss_out) {
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) atomicAdd(loss_out, red[0] + red[1] + red[2] + red[3]);
  }
}

}  // namespace

void launch_regularise(const float* opac, const float* scales, int64_t n, float eps_o, float eps_s, float* d_opac,
                       float* d_scales, float* loss_out, hipStream_t st) {
  SSS_LAUNCH("regularise", regularise_kernel, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, st, opac,
             scales, n, eps_o, eps_s, d_opac, d_scales, loss_out);
}

void launch_sghmc(float* means, float* mom, const float* g, const float* opac, const float* scales,
                  const float* quats, int64_t n, const sss_sghmc_opts_t& o, hipStream_t st) {
  SSS_LAUNCH("sghmc", sghmc_kernel, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, st, means, mom, g,
             opac, scales, quats, n, sghmc_args(o));
}

void launch_adam(const sss_adam_t& ad, hipStream_t st) {
  AdamBatch ab{};
  ab.first_block[0] = 0;
  int k = 0;
  for (int a = 0; a < ad.n_arrays; ++a) {
    const sss_adam_array_t& x = ad.arrays[a];
    if (x.count <= 0) continue;
    ab.p[k] = x.param; ab.g[k] = x.grad; ab.m[k] = x.m; ab.v[k] = x.v;
    ab.lr[k] = x.lr; ab.lo[k] = x.lo; ab.hi[k] = x.hi;
    ab.count[k] = x.count;
    ab.first_block[k + 1] = ab.first_block[k] + (uint32_t)((x.count + kBlock * kAdamIt - 1) / (kBlock * kAdamIt));
    ++k;
  }
  ab.n = k;
  const uint32_t blocks = ab.first_block[k];
  if (blocks == 0) return;
  SSS_LAUNCH("adam", adam_kernel, dim3(blocks), dim3(kBlock), 0, st, ab, adam_const(ad.beta1, ad.beta2, ad.eps, ad.t));
}

}  // namespace sss
