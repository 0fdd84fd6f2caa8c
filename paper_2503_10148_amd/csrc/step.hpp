// Per-component update of one sampler step (Sec. 3.4 eq. sigmoidUpdate, SM
// eq. SGHMC) and the per-element Adam update, shared by sss_sghmc_step's
// kernels and by the projection backward of sss_render_bwd_step, so that the
// fused and the separate calls compute the same values.
#pragma once

#include "common.hpp"

namespace sss {

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

// SGHMC settings of one step, as kernel arguments.
struct SghmcArgs {
  float lr, friction, k, t;
  int burn_in, noise;
  uint64_t seed, step;
};

inline SghmcArgs sghmc_args(const sss_sghmc_opts_t& o) {
  return SghmcArgs{o.lr, o.friction, o.k, o.t, (int)o.burn_in, (int)o.noise, o.seed, o.step};
}

// One component's mean and momentum: switch s = sigmoid(k((1 - |o|) - t)),
// noise n ~ N(0, 2 eps C) per axis (Philox counter (i, step), Box-Muller),
// F = s eps (1 - eps C) r (0 in burn-in), mu <- mu - eps^2 G + F + s eps kick
// with kick = n (burn-in: Sigma n), r <- (1 - eps C) r - eps G + n.
// q (w, x, y, z) and s are read only in burn-in.
__device__ __forceinline__ void sghmc_one(int64_t i, float* mu, float* r, const float* G, float o, const float4& q,
                                          const float* s, const SghmcArgs& a) {
  const float sw = 1.0f / (1.0f + expf(-a.k * ((1.0f - fabsf(o)) - a.t)));
  float z0 = 0.0f, z1 = 0.0f, z2 = 0.0f;
  if (a.noise) {
    const uint4 x = philox4x32_10(make_uint4((uint32_t)i, (uint32_t)a.step, (uint32_t)(a.step >> 32), (uint32_t)(i >> 32)),
                                  make_uint2((uint32_t)a.seed, (uint32_t)(a.seed >> 32)));
    const float r0 = sqrtf(-2.0f * logf(unit_open(x.x)));
    const float r1 = sqrtf(-2.0f * logf(unit_open(x.z)));
    const float a0 = 2.0f * unit_open(x.y), a1 = 2.0f * unit_open(x.w);
    z0 = r0 * cospif(a0);
    z1 = r0 * sinpif(a0);
    z2 = r1 * cospif(a1);
  }
  const float sd = sqrtf(2.0f * a.lr * a.friction);
  const float n0 = sd * z0, n1 = sd * z1, n2 = sd * z2;
  float k0 = n0, k1 = n1, k2 = n2;
  if (a.burn_in) {
    // Sigma n with Sigma = R diag(s^2) R^T
    const float inv = rsqrtf(q.x * q.x + q.y * q.y + q.z * q.z + q.w * q.w);
    const float w = q.x * inv, x = q.y * inv, y = q.z * inv, z = q.w * inv;
    const float R[9] = {1.0f - 2.0f * (y * y + z * z), 2.0f * (x * y - w * z), 2.0f * (x * z + w * y),
                        2.0f * (x * y + w * z), 1.0f - 2.0f * (x * x + z * z), 2.0f * (y * z - w * x),
                        2.0f * (x * z - w * y), 2.0f * (y * z + w * x), 1.0f - 2.0f * (x * x + y * y)};
    const float sq[3] = {s[0] * s[0], s[1] * s[1], s[2] * s[2]};
    // u = diag(s^2) R^T n
    float u[3];
    for (int c = 0; c < 3; ++c) u[c] = sq[c] * (R[c] * n0 + R[3 + c] * n1 + R[6 + c] * n2);
    k0 = R[0] * u[0] + R[1] * u[1] + R[2] * u[2];
    k1 = R[3] * u[0] + R[4] * u[1] + R[5] * u[2];
    k2 = R[6] * u[0] + R[7] * u[1] + R[8] * u[2];
  }
  const float decay = 1.0f - a.lr * a.friction;
  const float fsc = a.burn_in ? 0.0f : sw * a.lr * decay;
  const float lr2 = a.lr * a.lr;
  const float kick[3] = {k0, k1, k2};
  const float nz[3] = {n0, n1, n2};
  for (int c = 0; c < 3; ++c) {
    const float rc = r[c];
    mu[c] = mu[c] - lr2 * G[c] + fsc * rc + sw * a.lr * kick[c];
    r[c] = decay * rc - a.lr * G[c] + nz[c];
  }
}

// Adam hyper-parameters of one step: 1 - beta and the bias corrections
// 1 - beta^t are formed on the host in FP64.
struct AdamConst {
  float b1, b2, omb1, omb2, eps, c1, c2;
};

inline AdamConst adam_const(float beta1, float beta2, float eps, int64_t t) {
  AdamConst c;
  c.b1 = beta1;
  c.b2 = beta2;
  c.omb1 = (float)(1.0 - (double)beta1);
  c.omb2 = (float)(1.0 - (double)beta2);
  c.eps = eps;
  c.c1 = (float)(1.0 - pow((double)beta1, (double)t));
  c.c2 = (float)(1.0 - pow((double)beta2, (double)t));
  return c;
}

__device__ __forceinline__ void adam_one(float& p, float g, float& m, float& v, float lr, float lo, float hi,
                                         const AdamConst& a) {
  m = a.b1 * m + a.omb1 * g;
  v = a.b2 * v + a.omb2 * g * g;
  const float upd = lr * (m / a.c1) / (sqrtf(v / a.c2) + a.eps);
  p = fminf(fmaxf(p - upd, lo), hi);
}

// The update sss_render_bwd_step applies in the projection backward.
struct StepArgs {
  int on;                                        // 0: gradients only
  float *means, *scales, *quats, *nu, *opac, *sh;
  float* mom;
  SghmcArgs sg;
  int adam;
  AdamConst ac;
  float* m[5];                                   // scales, quats, nu, opacity, sh
  float* v[5];
  float lr[5], lo[5], hi[5];
};

}  // namespace sss
