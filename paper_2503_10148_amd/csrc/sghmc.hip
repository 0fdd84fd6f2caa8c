// SGHMC on the component means (Sec. 3.4 eq. sigmoidUpdate, SM eq. SGHMC)
// and Adam on the other parameters.  Elementwise and HBM-bound: one thread
// per component reads 40 bytes (mean, momentum, gradient, opacity) and writes
// 24; the noise is generated in registers from a counter-based generator, so
// a step is reproducible from (seed, step) alone.
#include "common.hpp"

namespace sss {
namespace {

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two
// 32x32->64 multiplies with the published multipliers and Weyl key schedule.
__device__ __forceinline__ uint4 philox4x32_10(uint4 c, uint2 k) {
  for (int r = 0; r < 10; ++r) {
    const uint32_t lo0 = 0xD2511F53u * c.x, hi0 = __umulhi(0xD2511F53u, c.x);
    const uint32_t lo1 = 0xCD9E8D57u * c.z, hi1 = __umulhi(0xCD9E8D57u, c.z);
    c = make_uint4(hi1 ^ c.y ^ k.x, lo1, hi0 ^ c.w ^ k.y, lo0);
    k.x += 0x9E3779B9u;
    k.y += 0xBB67AE85u;
  }
  return c;
}

// (0, 1) uniform from the top 23 bits, exact in FP32.
__device__ __forceinline__ float unit_open(uint32_t x) { return ((float)(x >> 9) + 0.5f) * (1.0f / 8388608.0f); }

__global__ __launch_bounds__(kBlock) void sghmc_kernel(float* __restrict__ means, float* __restrict__ mom,
                                                       const float* __restrict__ grad, const float* __restrict__ opac,
                                                       const float* __restrict__ scales, const float* __restrict__ quats,
                                                       int64_t n, float lr, float friction, float k, float t,
                                                       int burn_in, int noise, uint64_t seed, uint64_t step) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const float sw = 1.0f / (1.0f + expf(-k * ((1.0f - fabsf(opac[i])) - t)));
  float z0 = 0.0f, z1 = 0.0f, z2 = 0.0f;
  if (noise) {
    const uint4 x = philox4x32_10(make_uint4((uint32_t)i, (uint32_t)step, (uint32_t)(step >> 32), (uint32_t)(i >> 32)),
                                  make_uint2((uint32_t)seed, (uint32_t)(seed >> 32)));
    const float r0 = sqrtf(-2.0f * logf(unit_open(x.x)));
    const float r1 = sqrtf(-2.0f * logf(unit_open(x.z)));
    const float a0 = 2.0f * unit_open(x.y), a1 = 2.0f * unit_open(x.w);
    z0 = r0 * cospif(a0);
    z1 = r0 * sinpif(a0);
    z2 = r1 * cospif(a1);
  }
  const float sd = sqrtf(2.0f * lr * friction);
  const float n0 = sd * z0, n1 = sd * z1, n2 = sd * z2;
  float k0 = n0, k1 = n1, k2 = n2;
  if (burn_in) {
    // Sigma n with Sigma = R diag(s^2) R^T
    const float4 q = *reinterpret_cast<const float4*>(quats + 4 * i);
    const float inv = rsqrtf(q.x * q.x + q.y * q.y + q.z * q.z + q.w * q.w);
    const float w = q.x * inv, x = q.y * inv, y = q.z * inv, z = q.w * inv;
    const float R[9] = {1.0f - 2.0f * (y * y + z * z), 2.0f * (x * y - w * z), 2.0f * (x * z + w * y),
                        2.0f * (x * y + w * z), 1.0f - 2.0f * (x * x + z * z), 2.0f * (y * z - w * x),
                        2.0f * (x * z - w * y), 2.0f * (y * z + w * x), 1.0f - 2.0f * (x * x + y * y)};
    const float s0 = scales[3 * i], s1 = scales[3 * i + 1], s2 = scales[3 * i + 2];
    const float sq[3] = {s0 * s0, s1 * s1, s2 * s2};
    // u = diag(s^2) R^T n
    float u[3];
    for (int c = 0; c < 3; ++c) u[c] = sq[c] * (R[c] * n0 + R[3 + c] * n1 + R[6 + c] * n2);
    k0 = R[0] * u[0] + R[1] * u[1] + R[2] * u[2];
    k1 = R[3] * u[0] + R[4] * u[1] + R[5] * u[2];
    k2 = R[6] * u[0] + R[7] * u[1] + R[8] * u[2];
  }
  const float decay = 1.0f - lr * friction;
  const float fsc = burn_in ? 0.0f : sw * lr * decay;
  const float lr2 = lr * lr;
  const float kick[3] = {k0, k1, k2};
  const float nz[3] = {n0, n1, n2};
  for (int a = 0; a < 3; ++a) {
    const float r = mom[3 * i + a], G = grad[3 * i + a];
    means[3 * i + a] = means[3 * i + a] - lr2 * G + fsc * r + sw * lr * kick[a];
    mom[3 * i + a] = decay * r - lr * G + nz[a];
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

__device__ __forceinline__ void adam_one(float& p, float g, float& m, float& v, float lr, float lo, float hi, float b1,
                                         float b2, float omb1, float omb2, float eps, float c1, float c2) {
  m = b1 * m + omb1 * g;
  v = b2 * v + omb2 * g * g;
  const float upd = lr * (m / c1) / (sqrtf(v / c2) + eps);
  p = fminf(fmaxf(p - upd, lo), hi);
}

__global__ __launch_bounds__(kBlock) void adam_kernel(AdamBatch ab, float b1, float b2, float omb1, float omb2,
                                                      float eps, float c1, float c2) {
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
      adam_one(pi[k], gi[k], mi[k], vi[k], ab.lr[a], ab.lo[a], ab.hi[a], b1, b2, omb1, omb2, eps, c1, c2);
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
                     opac, scales, quats, n, o.lr, o.friction, o.k, o.t, (int)o.burn_in, (int)o.noise, o.seed, o.step);
}

void launch_adam(const sss_adam_t& ad, hipStream_t st) {
  // 1 - beta and the bias corrections on the host, in FP64
  const float c1 = (float)(1.0 - pow((double)ad.beta1, (double)ad.t));
  const float c2 = (float)(1.0 - pow((double)ad.beta2, (double)ad.t));
  const float omb1 = (float)(1.0 - (double)ad.beta1), omb2 = (float)(1.0 - (double)ad.beta2);
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
  SSS_LAUNCH("adam", adam_kernel, dim3(blocks), dim3(kBlock), 0, st, ab,
             ad.beta1, ad.beta2, omb1, omb2, ad.eps, c1, c2);
}

}  // namespace sss
