// Projection of 3D Student's t components to 2D (Sec. 3.2 eq. t_2D, SM
// "Forward Pass") and its backward pass (SM "Backward Pass").
//
// One thread per (view, component).  The grid's y dimension is the view, so
// the camera constants are wave-uniform scalar loads from the kernel
// argument segment.  Geometry is evaluated in FP64 (full rate on CDNA4's
// vector ALUs, and these kernels are HBM-bound) so that the stored 2D mean
// is exact to far below a pixel's 1e-6; results are stored in FP32 except the
// mean, which the record keeps in FP64.
#include "common.hpp"
#include "step.hpp"
#include "tiles.hpp"

namespace sss {
namespace {

// Real SH basis, degree <= 3, Condon-Shortley phase, k = l*l + l + m.
constexpr double kY0 = 0.28209479177387814;
constexpr double kY1 = 0.4886025119029199;
constexpr double kY2a = 1.0925484305920792;   // xy, yz, xz terms
constexpr double kY2b = 0.31539156525252005;  // 2zz - xx - yy
constexpr double kY2c = 0.5462742152960396;   // xx - yy
constexpr double kY3a = 0.5900435899266435;   // y(3xx - yy), x(xx - 3yy)
constexpr double kY3b = 2.890611442640554;    // xyz
constexpr double kY3c = 0.4570457994644658;   // y(4zz - xx - yy), x(4zz - xx - yy)
constexpr double kY3d = 0.3731763325901154;   // z(2zz - 3xx - 3yy)
constexpr double kY3e = 1.445305721320277;    // z(xx - yy)

template <typename F>
__device__ __forceinline__ void sh_basis(int deg, F x, F y, F z, F* Y) {
  Y[0] = F(kY0);
  if (deg < 1) return;
  Y[1] = -F(kY1) * y;
  Y[2] = F(kY1) * z;
  Y[3] = -F(kY1) * x;
  if (deg < 2) return;
  const F xx = x * x, yy = y * y, zz = z * z;
  Y[4] = F(kY2a) * x * y;
  Y[5] = -F(kY2a) * y * z;
  Y[6] = F(kY2b) * (F(2.0) * zz - xx - yy);
  Y[7] = -F(kY2a) * x * z;
  Y[8] = F(kY2c) * (xx - yy);
  if (deg < 3) return;
  Y[9] = -F(kY3a) * y * (F(3.0) * xx - yy);
  Y[10] = F(kY3b) * x * y * z;
  Y[11] = -F(kY3c) * y * (F(4.0) * zz - xx - yy);
  Y[12] = F(kY3d) * z * (F(2.0) * zz - F(3.0) * xx - F(3.0) * yy);
  Y[13] = -F(kY3c) * x * (F(4.0) * zz - xx - yy);
  Y[14] = F(kY3e) * z * (xx - yy);
  Y[15] = -F(kY3a) * x * (xx - F(3.0) * yy);
}

// Gradient of sum_k w[k] Y_k(x, y, z) (polynomial extension) w.r.t. (x, y, z).
template <typename F>
__device__ __forceinline__ void sh_basis_grad(int deg, F x, F y, F z, const F* w, F* gx, F* gy, F* gz) {
  F ax = 0, ay = 0, az = 0;
  if (deg >= 1) {
    ay += -F(kY1) * w[1];
    az += F(kY1) * w[2];
    ax += -F(kY1) * w[3];
  }
  if (deg >= 2) {
    ax += F(kY2a) * y * w[4];             ay += F(kY2a) * x * w[4];
    ay += -F(kY2a) * z * w[5];            az += -F(kY2a) * y * w[5];
    ax += -F(2.0) * F(kY2b) * x * w[6];      ay += -F(2.0) * F(kY2b) * y * w[6];  az += F(4.0) * F(kY2b) * z * w[6];
    ax += -F(kY2a) * z * w[7];            az += -F(kY2a) * x * w[7];
    ax += F(2.0) * F(kY2c) * x * w[8];       ay += -F(2.0) * F(kY2c) * y * w[8];
  }
  if (deg >= 3) {
    const F xx = x * x, yy = y * y, zz = z * z;
    // Y9 = -a (3 xx y - y^3)
    ax += -F(kY3a) * F(6.0) * x * y * w[9];
    ay += -F(kY3a) * (F(3.0) * xx - F(3.0) * yy) * w[9];
    // Y10 = b x y z
    ax += F(kY3b) * y * z * w[10];  ay += F(kY3b) * x * z * w[10];  az += F(kY3b) * x * y * w[10];
    // Y11 = -c (4 y zz - xx y - y^3)
    ax += F(kY3c) * F(2.0) * x * y * w[11];
    ay += -F(kY3c) * (F(4.0) * zz - xx - F(3.0) * yy) * w[11];
    az += -F(kY3c) * F(8.0) * y * z * w[11];
    // Y12 = d (2 z^3 - 3 xx z - 3 yy z)
    ax += -F(kY3d) * F(6.0) * x * z * w[12];
    ay += -F(kY3d) * F(6.0) * y * z * w[12];
    az += F(kY3d) * (F(6.0) * zz - F(3.0) * xx - F(3.0) * yy) * w[12];
    // Y13 = -c (4 x zz - x^3 - x yy)
    ax += -F(kY3c) * (F(4.0) * zz - F(3.0) * xx - yy) * w[13];
    ay += F(kY3c) * F(2.0) * x * y * w[13];
    az += -F(kY3c) * F(8.0) * x * z * w[13];
    // Y14 = e (xx z - yy z)
    ax += F(kY3e) * F(2.0) * x * z * w[14];
    ay += -F(kY3e) * F(2.0) * y * z * w[14];
    az += F(kY3e) * (xx - yy) * w[14];
    // Y15 = -a (x^3 - 3 x yy)
    ax += -F(kY3a) * (F(3.0) * xx - F(3.0) * yy) * w[15];
    ay += F(kY3a) * F(6.0) * x * y * w[15];
  }
  *gx = ax; *gy = ay; *gz = az;
}

// Rotation of a unit quaternion (w, x, y, z), row-major.
template <typename F>
__device__ __forceinline__ void rotation(const F* q, F* R) {
  const F w = q[0], x = q[1], y = q[2], z = q[3];
  R[0] = F(1.0) - F(2.0) * (y * y + z * z); R[1] = F(2.0) * (x * y - w * z);       R[2] = F(2.0) * (x * z + w * y);
  R[3] = F(2.0) * (x * y + w * z);       R[4] = F(1.0) - F(2.0) * (x * x + z * z); R[5] = F(2.0) * (y * z - w * x);
  R[6] = F(2.0) * (x * z - w * y);       R[7] = F(2.0) * (y * z + w * x);       R[8] = F(1.0) - F(2.0) * (x * x + y * y);
}

// Forward intermediates of one entry, shared by the forward and backward kernels.
template <typename F>
struct Geo {
  F X, Y, Z;        // camera-space position
  F qn, q[4];       // quaternion norm and unit quaternion
  F Rq[9];          // component rotation
  F S[6];           // Sigma (xx, xy, xz, yy, yz, zz)
  F xz, yz, txz, tyz;
  bool clx, cly;         // EWA clamp active
  F M[6];           // J * Rview (2x3)
  F A, B, D, det;   // 2D covariance (+lowpass) and determinant
};

template <typename F>
__device__ __forceinline__ void geometry(const CamDev& c, const OptsDev& op, const float* mu, const float* s,
                                         const float* qraw, Geo<F>& g) {
  const F m0 = mu[0], m1 = mu[1], m2 = mu[2];
  g.X = (F)c.R[0] * m0 + (F)c.R[1] * m1 + (F)c.R[2] * m2 + (F)c.t[0];
  g.Y = (F)c.R[3] * m0 + (F)c.R[4] * m1 + (F)c.R[5] * m2 + (F)c.t[1];
  g.Z = (F)c.R[6] * m0 + (F)c.R[7] * m1 + (F)c.R[8] * m2 + (F)c.t[2];
  const F q0 = qraw[0], q1 = qraw[1], q2 = qraw[2], q3 = qraw[3];
  g.qn = sqrt(q0 * q0 + q1 * q1 + q2 * q2 + q3 * q3);
  const F iq = F(1.0) / g.qn;
  g.q[0] = q0 * iq; g.q[1] = q1 * iq; g.q[2] = q2 * iq; g.q[3] = q3 * iq;
  rotation(g.q, g.Rq);
  const F s0 = (F)s[0] * s[0], s1 = (F)s[1] * s[1], s2 = (F)s[2] * s[2];
  const F* R = g.Rq;
  g.S[0] = R[0] * R[0] * s0 + R[1] * R[1] * s1 + R[2] * R[2] * s2;
  g.S[1] = R[0] * R[3] * s0 + R[1] * R[4] * s1 + R[2] * R[5] * s2;
  g.S[2] = R[0] * R[6] * s0 + R[1] * R[7] * s1 + R[2] * R[8] * s2;
  g.S[3] = R[3] * R[3] * s0 + R[4] * R[4] * s1 + R[5] * R[5] * s2;
  g.S[4] = R[3] * R[6] * s0 + R[4] * R[7] * s1 + R[5] * R[8] * s2;
  g.S[5] = R[6] * R[6] * s0 + R[7] * R[7] * s1 + R[8] * R[8] * s2;
  const F limx = F(1.3) * (F)c.W / (F(2.0) * (F)c.fx);
  const F limy = F(1.3) * (F)c.H / (F(2.0) * (F)c.fy);
  const F iz = F(1.0) / g.Z;
  g.xz = g.X * iz;
  g.yz = g.Y * iz;
  g.clx = g.xz < -limx || g.xz > limx;
  g.cly = g.yz < -limy || g.yz > limy;
  g.txz = fmin(fmax(g.xz, -limx), limx);
  g.tyz = fmin(fmax(g.yz, -limy), limy);
  const F j00 = c.fx * iz, j02 = -c.fx * g.txz * iz;
  const F j11 = c.fy * iz, j12 = -c.fy * g.tyz * iz;
  for (int k = 0; k < 3; ++k) {
    g.M[k] = j00 * c.R[k] + j02 * c.R[6 + k];
    g.M[3 + k] = j11 * c.R[3 + k] + j12 * c.R[6 + k];
  }
  // Sigma2 = M S M^T with S symmetric
  F t0[3], t1[3];
  const F* S = g.S;
  for (int r = 0; r < 2; ++r) {
    const F* m = g.M + 3 * r;
    F* t = r ? t1 : t0;
    t[0] = m[0] * S[0] + m[1] * S[1] + m[2] * S[2];
    t[1] = m[0] * S[1] + m[1] * S[3] + m[2] * S[4];
    t[2] = m[0] * S[2] + m[1] * S[4] + m[2] * S[5];
  }
  g.A = t0[0] * g.M[0] + t0[1] * g.M[1] + t0[2] * g.M[2] + op.lowpass;
  g.B = t0[0] * g.M[3] + t0[1] * g.M[4] + t0[2] * g.M[5];
  g.D = t1[0] * g.M[3] + t1[1] * g.M[4] + t1[2] * g.M[5] + op.lowpass;
  g.det = g.A * g.D - g.B * g.B;
}

template <typename F>
__device__ __forceinline__ void view_dir(const CamDev& c, const float* mu, F* dir, F* vn) {
  // camera centre = -R^T t
  const F px = -((F)c.R[0] * c.t[0] + (F)c.R[3] * c.t[1] + (F)c.R[6] * c.t[2]);
  const F py = -((F)c.R[1] * c.t[0] + (F)c.R[4] * c.t[1] + (F)c.R[7] * c.t[2]);
  const F pz = -((F)c.R[2] * c.t[0] + (F)c.R[5] * c.t[1] + (F)c.R[8] * c.t[2]);
  const F vx = mu[0] - px, vy = mu[1] - py, vz = mu[2] - pz;
  *vn = sqrt(vx * vx + vy * vy + vz * vz);
  const F inv = F(1.0) / *vn;
  dir[0] = vx * inv; dir[1] = vy * inv; dir[2] = vz * inv;
}

// Coalesced copy of the SH coefficients of components [i0, i0 + cnt) into LDS
// with a padded stride (3K + 1 floats), so that each thread afterwards reads
// its own coefficients without bank conflicts.
template <int DEG, int B>
__device__ __forceinline__ void stage_sh(const float* __restrict__ sh, int64_t i0, int cnt, float* lds) {
  constexpr int KC = 3 * (DEG + 1) * (DEG + 1), STR = KC + 1;
  const float* src = sh + (size_t)i0 * KC;
  // every load of the thread is issued before the first LDS store, so the
  // memory latencies overlap instead of adding up
  if constexpr (KC % 4 == 0) {
    constexpr int PER = KC / 4;                 // float4 loads per thread for a full block
    const float4* s4 = reinterpret_cast<const float4*>(src);
    const int total = cnt * KC / 4;
    // read once per step: streaming (non-temporal) loads, measured 13% faster
    typedef float f4v __attribute__((ext_vector_type(4)));
    float4 q[PER];
#pragma unroll
    for (int it = 0; it < PER; ++it) {
      const int g = threadIdx.x + it * B;
      q[it] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
      if (g < total) {
        const f4v t = __builtin_nontemporal_load(reinterpret_cast<const f4v*>(s4 + g));
        q[it] = make_float4(t.x, t.y, t.z, t.w);
      }
    }
#pragma unroll
    for (int it = 0; it < PER; ++it) {
      const int g = threadIdx.x + it * B;
      if (g < total) {
        const int f = 4 * g, c = f / KC, j = f - c * KC;
        float* d = lds + c * STR + j;
        d[0] = q[it].x; d[1] = q[it].y; d[2] = q[it].z; d[3] = q[it].w;
      }
    }
  } else {
    constexpr int PER = KC;                     // loads per thread for a full block
    const int total = cnt * KC;
    float q[PER];
#pragma unroll
    for (int it = 0; it < PER; ++it) {
      const int g = threadIdx.x + it * B;
      q[it] = g < total ? src[g] : 0.0f;
    }
#pragma unroll
    for (int it = 0; it < PER; ++it) {
      const int g = threadIdx.x + it * B;
      if (g < total) {
        const int c = g / KC, j = g - c * KC;
        lds[c * STR + j] = q[it];
      }
    }
  }
}

// One entry: writes its depth key and (0 when culled) tile count, and
// returns true with the entry's line in `out` when it is listed anywhere.
template <int DEG>
__device__ __forceinline__ bool project_entry(const CamDev& c, const OptsDev& op, int64_t i, int64_t e,
                                              const float* __restrict__ means, const float* __restrict__ scales,
                                              const float* __restrict__ quats, const float* __restrict__ nu,
                                              const float* __restrict__ opac, const float* __restrict__ sh,
                                              uint32_t* __restrict__ keys, uint32_t* __restrict__ touched,
                                              Entry& out) {
  constexpr int K = (DEG + 1) * (DEG + 1);
  const float* mu = means + 3 * i;

  const float zf = fmaf(c.R[6], mu[0], fmaf(c.R[7], mu[1], fmaf(c.R[8], mu[2], c.t[2])));
  keys[e] = __float_as_uint(zf);
  touched[e] = 0;
  const float o = opac[i];
  if (!(zf > op.z_near) || !(fabsf(o) >= op.alpha_min)) return false;

  Geo<double> g;
  geometry<double>(c, op, mu, scales + 3 * i, quats + 4 * i, g);
  if (!(g.qn > 0.0) || !(g.det > 0.0)) return false;

  const double mx = c.fx * g.xz + c.cx, my = c.fy * g.yz + c.cy;
  const double nuc = fmin(fmax((double)nu[i], (double)op.nu_min), (double)op.nu_max);
  double hs, ey, hr;
  int x0, x1, y0, y1;
  const bool gauss = op.family == SSS_FAMILY_GAUSSIAN;
  if (op.alpha_min > 0.0f) {
    // alpha level set |o| T2D(h*) = alpha_min
    const double lr = log(fabs((double)o) / (double)op.alpha_min);
    hs = gauss ? 2.0 * lr : nuc * expm1(2.0 / (nuc + 2.0) * lr);
    ey = sqrt(hs * g.D);   // row extent of the pixels that can pass the alpha test
    // coverage rule: the ellipse with the Gaussian 3-sigma probability mass,
    // P(h <= q) = 1 - (1 + q/nu)^(-nu/2) = 1 - exp(-9/2); never beyond h*
    hr = op.trunc_mode == SSS_TRUNC_COVERAGE ? fmin(hs, gauss ? 9.0 : nuc * expm1(9.0 / nuc)) : hs;
    const double erx = sqrt(hr * g.A), ery = sqrt(hr * g.D);
    const double lx = (mx - erx) * (1.0 / kTile), hx = (mx + erx) * (1.0 / kTile);
    const double ly = (my - ery) * (1.0 / kTile), hy = (my + ery) * (1.0 / kTile);
    if (hx < 0.0 || lx >= c.tiles_x || hy < 0.0 || ly >= c.tiles_y) return false;
    x0 = (int)fmax(0.0, floor(lx)); x1 = (int)fmin((double)(c.tiles_x - 1), floor(hx));
    y0 = (int)fmax(0.0, floor(ly)); y1 = (int)fmin((double)(c.tiles_y - 1), floor(hy));
  } else {
    hs = hr = __builtin_inf();
    ey = __builtin_inf();
    x0 = 0; x1 = c.tiles_x - 1; y0 = 0; y1 = c.tiles_y - 1;
  }
  // the rectangle's rows, each cut to the ellipse's extent
  const Ellipse el{g.A, g.B, g.D, hr};
  const RowGeo rg = make_row_geo(mx, my, el);
  int count = 0;
  for (int ty = y0; ty <= y1; ++ty) {
    int t0;
    count += row_run(rg, ty, x0, x1, &t0);
  }
  if (count == 0) return false;

  double dir[3], vn;
  view_dir<double>(c, mu, dir, &vn);
  double Y[16];
  sh_basis<double>(DEG, dir[0], dir[1], dir[2], Y);
  // Each thread reads its own coefficients (16-byte loads when the row is a
  // multiple of 4 floats): without a staging array in LDS the kernel keeps 4
  // waves per SIMD instead of 3, and only entries that reach a tile read them.
  float shi[3 * K];
  if constexpr ((3 * K) % 4 == 0) {
    const float4* s4 = reinterpret_cast<const float4*>(sh + (size_t)i * 3 * K);
#pragma unroll
    for (int q = 0; q < 3 * K / 4; ++q) {
      const float4 t = s4[q];
      shi[4 * q] = t.x; shi[4 * q + 1] = t.y; shi[4 * q + 2] = t.z; shi[4 * q + 3] = t.w;
    }
  } else {
#pragma unroll
    for (int q = 0; q < 3 * K; ++q) shi[q] = sh[(size_t)i * 3 * K + q];
  }
  double col[3] = {0.5, 0.5, 0.5};
#pragma unroll
  for (int k = 0; k < K; ++k) {
    col[0] += Y[k] * shi[3 * k + 0];
    col[1] += Y[k] * shi[3 * k + 1];
    col[2] += Y[k] * shi[3 * k + 2];
  }

  const double idet = 1.0 / g.det;
  Rec r;
  r.mx = mx;
  r.my = my;
  // the conic (D, -B, A) / det as its Cholesky factor, from the covariance
  // in FP64 (det = A D - B^2 makes l22 = 1/sqrt(D)): h as a sum of two
  // squares keeps its precision in FP32 near an elongated ellipse's major
  // axis, where the three conic entries cancel about 2 log2(axis ratio) bits
  const double sD = sqrt(g.D);
  r.l11 = (float)(sD * sqrt(idet));
  r.l21 = (float)(-g.B * sqrt(idet) / sD);
  r.l22 = (float)(1.0 / sD);
  r.cr = (float)fmax(col[0], 0.0);
  r.cg = (float)fmax(col[1], 0.0);
  r.cb = (float)fmax(col[2], 0.0);
  r.o = o;
  r.inv_nu = gauss ? 0.0f : (float)(1.0 / nuc);
  r.nb = gauss ? (float)(-0.5 * 1.4426950408889634) : (float)(-0.5 * (nuc + 2.0));
  r.hs = (float)hs;
  r.entry = (uint32_t)e;
  r.ey = (float)ey;
  out.rec = r;
  out.ell = el;
  out.rect = make_ushort4((unsigned short)x0, (unsigned short)y0, (unsigned short)x1, (unsigned short)y1);
#pragma unroll
  for (int k = 0; k < 6; ++k) out.pad[k] = 0u;
  touched[e] = (uint32_t)count;
  return true;
}

// Per (view, component): project_entry, then the block's entry lines go out
// through LDS: each thread stages its 128-byte line (its eight 16-byte parts
// rotated by the thread number, against bank conflicts), and each wave
// writes its 64 threads' lines as eight contiguous 1 KB runs, whole lines
// only (a per-thread 128-byte store pattern measured 30% slower; culled
// entries' lines are not written).
template <int DEG>
__global__ __launch_bounds__(kBlock) void project_kernel(
    CamBatch cb, OptsDev op, int64_t n, const float* __restrict__ means, const float* __restrict__ scales,
    const float* __restrict__ quats, const float* __restrict__ nu, const float* __restrict__ opac,
    const float* __restrict__ sh, Entry* __restrict__ ent, uint32_t* __restrict__ keys,
    uint32_t* __restrict__ touched) {
  __shared__ uint4 stage[kBlock * 8];
  // Workgroup ids are dealt to the 8 XCDs in turn.  Ids run over chunks of
  // 8 component blocks x all views, view-major inside a chunk, so the views
  // of one component block land on one XCD close together in time and read
  // the block's parameters (the SH above all) from that XCD's L2 after the
  // first view (view-major over the whole grid, every view re-read them
  // from HBM).
  const int64_t nb = (n + kBlock - 1) / kBlock;
  const int64_t per_chunk = 8 * (int64_t)cb.n_views;
  const int64_t chunk = (int64_t)blockIdx.x / per_chunk, rem = (int64_t)blockIdx.x - chunk * per_chunk;
  const int v = (int)(rem >> 3);
  const int64_t blk = chunk * 8 + (rem & 7);
  if (blk >= nb) return;   // padding of the last chunk (whole workgroup)
  const int64_t i0 = blk * kBlock;
  const int64_t i = i0 + threadIdx.x;
  const CamDev& c = cb.v[v];
  const int64_t e = (int64_t)v * n + i;
  Entry out;
  const bool listed = i < n && project_entry<DEG>(c, op, i, e, means, scales, quats, nu, opac, sh, keys, touched, out);
  if (listed) {
    const uint4* src = reinterpret_cast<const uint4*>(&out);
#pragma unroll
    for (int k = 0; k < 8; ++k) stage[threadIdx.x * 8 + ((k + threadIdx.x) & 7)] = src[k];
  }
  const uint64_t wave_listed = __ballot(listed);
  __syncthreads();
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t wave_i0 = i0 + 64 * w;
  uint4* dst = reinterpret_cast<uint4*>(ent + (int64_t)v * n + wave_i0);
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const int j = 8 * k + (lane >> 3), part = lane & 7;   // entry within the wave, its 16-byte part
    if ((wave_listed >> j) & 1ull) dst[8 * j + part] = stage[(64 * w + j) * 8 + ((part + j) & 7)];
  }
}

// Backward of the geometry: per component, sum over views of the chain from
// d mean2d and d conic (and d o, d nu) to means, scales, quats, opacity, nu.
// FP32; the SH part is sh_bwd_kernel.  d_means is always accumulated (+=):
// sh_bwd_kernel runs first and initialises it when overwriting.
__global__ __launch_bounds__(kBlock) void project_bwd_kernel(
    CamBatch cb, OptsDev op, int64_t n, const float* means, const float* scales, const float* quats, const float* nu,
    const float* opac, const uint32_t* __restrict__ touched, const double* __restrict__ g2, float* __restrict__ d_means,
    float* __restrict__ d_scales, float* __restrict__ d_quats, float* __restrict__ d_nu, float* __restrict__ d_opac,
    int overwrite, StepArgs sa) {
  // means, scales, quats and nu are not __restrict__: with sa.on the same
  // arrays are written through sa after this thread's reads
  using F = float;
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const float* mu = means + 3 * i;
  const float* s = scales + 3 * i;
  // the update's state does not depend on the gradient: its loads are
  // issued first, so their latency hides behind the arithmetic below
  float st_r[3], st_m[9], st_v[9], st_o = 0.0f;
  if (sa.on) {
    for (int a = 0; a < 3; ++a) st_r[a] = sa.mom[3 * i + a];
    st_o = sa.opac[i];
    if (sa.adam) {
      for (int a = 0; a < 3; ++a) { st_m[a] = sa.m[0][3 * i + a]; st_v[a] = sa.v[0][3 * i + a]; }
      for (int a = 0; a < 4; ++a) { st_m[3 + a] = sa.m[1][4 * i + a]; st_v[3 + a] = sa.v[1][4 * i + a]; }
      st_m[7] = sa.m[2][i]; st_v[7] = sa.v[2][i];
      st_m[8] = sa.m[3][i]; st_v[8] = sa.v[3][i];
    }
  }
  F gmu[3] = {0, 0, 0}, gs[3] = {0, 0, 0}, gq[4] = {0, 0, 0, 0};
  F gnu = 0, gop = 0;
  bool any = false;
  // The raster's sums leave out the entry's own factors (the same float
  // values its record holds): d mean2d and d conic carry o nb (1/nu, or
  // ln 2 for the Gaussian family), d nu carries o ln(2) / 2.
  float cgeo, cnu;
  {
    const float o = opac[i];
    const bool gauss = op.family == SSS_FAMILY_GAUSSIAN;
    const double nuc = fmin(fmax((double)nu[i], (double)op.nu_min), (double)op.nu_max);
    const float nb = gauss ? (float)(-0.5 * 1.4426950408889634) : (float)(-0.5 * (nuc + 2.0));
    const float kh = gauss ? 0.6931471805599453f : (float)(1.0 / nuc);
    cgeo = o * nb * kh;
    cnu = 0.5f * o * 0.6931471805599453f;
  }
  for (int v = 0; v < cb.n_views; ++v) {
    const int64_t e = (int64_t)v * n + i;
    if (touched[e] == 0) continue;
    any = true;
    const CamDev& c = cb.v[v];
    const double2* gp = reinterpret_cast<const double2*>(g2 + e * kG2);
    const double2 g01 = gp[0], g23 = gp[1], g45 = gp[2], g89 = gp[4];
    // the raster's sums in the frame w = L^T d of the conic's Cholesky
    // factor L: mean (-2 sum dh w) and the symmetric sum dh w w^T (00, 2 x
    // 01, 11)
    const F gw0 = (F)g01.x * cgeo, gw1 = (F)g01.y * cgeo, gw00 = (F)g23.x * cgeo,
            gw01 = F(0.5) * (F)g23.y * cgeo, gw11 = (F)g45.x * cgeo;
    gop += (F)g89.x;
    gnu += (F)g89.y * cnu;

    Geo<F> g;
    geometry<F>(c, op, mu, s, quats + 4 * i, g);
    // The chain runs through P = M Rq (2x3), the projected component axes,
    // rather than through Sigma and Sigma2: with N = P diag(s), Sigma2 =
    // N N^T + lowpass I, so A and D are sums of squares and det (Cauchy-
    // Binet) is a sum of squared 2x2 minors plus positive low-pass terms,
    // and the terms of the conic's inverse that were (1/det - A D / det^2)
    // are -B^2 / det^2.  A D - B^2 in FP32 loses about 2 log2(r) bits for an
    // ellipse of axis ratio r, as does Sigma = Rq diag(s^2) Rq^T for an
    // elongated component; these forms lose none to cancellation.
    const F* M = g.M;
    const F* R = g.Rq;
    const F sv[3] = {s[0], s[1], s[2]};
    const F sq[3] = {sv[0] * sv[0], sv[1] * sv[1], sv[2] * sv[2]};
    F P[6];
    for (int r = 0; r < 2; ++r)
      for (int k = 0; k < 3; ++k) P[3 * r + k] = M[3 * r] * R[k] + M[3 * r + 1] * R[3 + k] + M[3 * r + 2] * R[6 + k];
    const F n00 = P[0] * sv[0], n01 = P[1] * sv[1], n02 = P[2] * sv[2];
    const F n10 = P[3] * sv[0], n11 = P[4] * sv[1], n12 = P[5] * sv[2];
    const F A0 = n00 * n00 + n01 * n01 + n02 * n02, D0 = n10 * n10 + n11 * n11 + n12 * n12;
    const F B = n00 * n10 + n01 * n11 + n02 * n12;
    const F m01 = n00 * n11 - n01 * n10, m02 = n00 * n12 - n02 * n10, m12 = n01 * n12 - n02 * n11;
    const F lp = op.lowpass;
    const F A = A0 + lp, D = D0 + lp;
    const F det = m01 * m01 + m02 * m02 + m12 * m12 + lp * (A0 + D0) + lp * lp;
    // the conic's Cholesky factor (Q = Sigma2^-1 = L L^T), as the
    // projection forms it: l11 = sqrt(D/det), l21 = -B/sqrt(D det), l22 =
    // 1/sqrt(D); the mean's gradient is L (gw0, gw1), and the 2D covariance's
    // G = -L (sum dh w w^T) L^T (symmetric 2x2, off-diagonal shared by B)
    const F isD = F(1) / sqrt(D), isdet = F(1) / sqrt(det);
    const F l11 = sqrt(D) * isdet, l21 = -B * isD * isdet, l22 = isD;
    const F gmx = l11 * gw0, gmy = l21 * gw0 + l22 * gw1;
    const F G00 = -(l11 * l11 * gw00);
    const F G01 = -(l11 * (l21 * gw00 + l22 * gw01));
    const F G11 = -(l21 * l21 * gw00 + F(2) * l21 * l22 * gw01 + l22 * l22 * gw11);
    F GP[6];
    for (int k = 0; k < 3; ++k) {
      GP[k] = G00 * P[k] + G01 * P[3 + k];
      GP[3 + k] = G01 * P[k] + G11 * P[3 + k];
    }
    // dM = 2 G M Sigma = 2 (G P) diag(s^2) Rq^T
    F dM[6];
    for (int r = 0; r < 2; ++r)
      for (int b = 0; b < 3; ++b)
        dM[3 * r + b] = F(2) * (GP[3 * r] * sq[0] * R[3 * b] + GP[3 * r + 1] * sq[1] * R[3 * b + 1] +
                                GP[3 * r + 2] * sq[2] * R[3 * b + 2]);
    // M = J Rview: dJ = dM Rview^T (only J00, J02, J11, J12 are non-zero)
    const F dJ00 = dM[0] * c.R[0] + dM[1] * c.R[1] + dM[2] * c.R[2];
    const F dJ02 = dM[0] * c.R[6] + dM[1] * c.R[7] + dM[2] * c.R[8];
    const F dJ11 = dM[3] * c.R[3] + dM[4] * c.R[4] + dM[5] * c.R[5];
    const F dJ12 = dM[3] * c.R[6] + dM[4] * c.R[7] + dM[5] * c.R[8];
    const F iz = F(1) / g.Z, iz2 = iz * iz;
    F dX = gmx * c.fx * iz;
    F dY = gmy * c.fy * iz;
    F dZ = -(gmx * c.fx * g.X + gmy * c.fy * g.Y) * iz2;
    dZ += -dJ00 * c.fx * iz2 - dJ11 * c.fy * iz2;
    if (g.clx) {
      dZ += dJ02 * c.fx * g.txz * iz2;
    } else {
      dX += -dJ02 * c.fx * iz2;
      dZ += F(2) * dJ02 * c.fx * g.X * iz2 * iz;
    }
    if (g.cly) {
      dZ += dJ12 * c.fy * g.tyz * iz2;
    } else {
      dY += -dJ12 * c.fy * iz2;
      dZ += F(2) * dJ12 * c.fy * g.Y * iz2 * iz;
    }
    for (int a = 0; a < 3; ++a) gmu[a] += c.R[a] * dX + c.R[3 + a] * dY + c.R[6 + a] * dZ;

    // Sigma = Rq diag(s^2) Rq^T with dSigma = M^T G M: dRq = 2 dSigma Rq
    // diag(s^2), where dSigma Rq = M^T (G P); d s_k = 2 s_k (Rq^T dSigma
    // Rq)_kk = 2 s_k P_k^T G P_k (P_k: column k of P)
    F dR[9];
    for (int r = 0; r < 3; ++r)
      for (int k = 0; k < 3; ++k) dR[3 * r + k] = F(2) * (M[r] * GP[k] + M[3 + r] * GP[3 + k]) * sq[k];
    for (int k = 0; k < 3; ++k) gs[k] += F(2) * sv[k] * (P[k] * GP[k] + P[3 + k] * GP[3 + k]);
    const F w = g.q[0], x = g.q[1], y = g.q[2], z = g.q[3];
    F gu[4];
    gu[0] = -F(2) * z * dR[1] + F(2) * y * dR[2] + F(2) * z * dR[3] - F(2) * x * dR[5] - F(2) * y * dR[6] +
            F(2) * x * dR[7];
    gu[1] = F(2) * y * dR[1] + F(2) * z * dR[2] + F(2) * y * dR[3] - F(4) * x * dR[4] - F(2) * w * dR[5] +
            F(2) * z * dR[6] + F(2) * w * dR[7] - F(4) * x * dR[8];
    gu[2] = -F(4) * y * dR[0] + F(2) * x * dR[1] + F(2) * w * dR[2] + F(2) * x * dR[3] + F(2) * z * dR[5] -
            F(2) * w * dR[6] + F(2) * z * dR[7] - F(4) * y * dR[8];
    gu[3] = -F(4) * z * dR[0] - F(2) * w * dR[1] + F(2) * x * dR[2] + F(2) * w * dR[3] - F(4) * z * dR[4] +
            F(2) * y * dR[5] + F(2) * x * dR[6] + F(2) * y * dR[7];
    const F dq = gu[0] * g.q[0] + gu[1] * g.q[1] + gu[2] * g.q[2] + gu[3] * g.q[3];
    for (int a = 0; a < 4; ++a) gq[a] += (gu[a] - g.q[a] * dq) / g.qn;
  }
  if (!any && !overwrite && !sa.on) return;
  const float nv = nu[i];
  if (!(nv >= op.nu_min && nv <= op.nu_max) || op.family == SSS_FAMILY_GAUSSIAN) gnu = 0;
  if (d_means) for (int a = 0; a < 3; ++a) d_means[3 * i + a] += gmu[a];
  if (sa.on) {
    // the component's whole gradient is here: the SH part of d_means left by
    // sh_bwd_kernel in the unused slots of the entry's screen-space record,
    // plus the geometric part; SGHMC on the mean with the old opacity (and
    // old scales and rotation for burn-in), then Adam on the other arrays
    const float* part = reinterpret_cast<const float*>(g2 + (size_t)i * kG2 + 10);
    const float G[3] = {part[0] + gmu[0], part[1] + gmu[1], part[2] + gmu[2]};
    float mu_i[3] = {mu[0], mu[1], mu[2]}, si[3] = {s[0], s[1], s[2]};
    const float4 q = *reinterpret_cast<const float4*>(quats + 4 * i);
    sghmc_one(i, mu_i, st_r, G, st_o, q, si, sa.sg);
    for (int a = 0; a < 3; ++a) {
      sa.means[3 * i + a] = mu_i[a];
      sa.mom[3 * i + a] = st_r[a];
    }
    if (sa.adam) {
      float qq[4] = {q.x, q.y, q.z, q.w};
      float op_i = st_o, nu_i = nv;
      for (int a = 0; a < 3; ++a) adam_one(si[a], gs[a], st_m[a], st_v[a], sa.lr[0], sa.lo[0], sa.hi[0], sa.ac);
      for (int a = 0; a < 4; ++a)
        adam_one(qq[a], gq[a], st_m[3 + a], st_v[3 + a], sa.lr[1], sa.lo[1], sa.hi[1], sa.ac);
      adam_one(nu_i, gnu, st_m[7], st_v[7], sa.lr[2], sa.lo[2], sa.hi[2], sa.ac);
      adam_one(op_i, gop, st_m[8], st_v[8], sa.lr[3], sa.lo[3], sa.hi[3], sa.ac);
      for (int a = 0; a < 3; ++a) {
        sa.scales[3 * i + a] = si[a];
        sa.m[0][3 * i + a] = st_m[a];
        sa.v[0][3 * i + a] = st_v[a];
      }
      *reinterpret_cast<float4*>(sa.quats + 4 * i) = make_float4(qq[0], qq[1], qq[2], qq[3]);
      for (int a = 0; a < 4; ++a) {
        sa.m[1][4 * i + a] = st_m[3 + a];
        sa.v[1][4 * i + a] = st_v[3 + a];
      }
      sa.nu[i] = nu_i;
      sa.m[2][i] = st_m[7];
      sa.v[2][i] = st_v[7];
      sa.opac[i] = op_i;
      sa.m[3][i] = st_m[8];
      sa.v[3][i] = st_v[8];
    }
  }
  if (overwrite) {
    if (d_scales) for (int a = 0; a < 3; ++a) d_scales[3 * i + a] = gs[a];
    if (d_quats) for (int a = 0; a < 4; ++a) d_quats[4 * i + a] = gq[a];
    if (d_opac) d_opac[i] = gop;
    if (d_nu) d_nu[i] = gnu;
  } else {
    if (d_scales) for (int a = 0; a < 3; ++a) d_scales[3 * i + a] += gs[a];
    if (d_quats) for (int a = 0; a < 4; ++a) d_quats[4 * i + a] += gq[a];
    if (d_opac) d_opac[i] += gop;
    if (d_nu) d_nu[i] += gnu;
  }
}

// Backward of the SH colour: d_sh[k][c] = sum over views of d colour_c Y_k
// (where the colour is not clamped), and the part of d_means that comes from
// the viewing direction.  The block's SH are staged in LDS, read for every
// view's colour and direction gradient; d_sh is summed in registers and
// passes through the same LDS slots to be written back coalesced (and, in a
// training step, to the Adam update, which takes the SH values from the
// slots first, so the coefficients are read from memory once).  d_means is
// written (overwrite) or accumulated; project_bwd_kernel adds the geometric
// part afterwards.
// Workgroup size of the SH backward (components per workgroup): 256
// measured fastest at the 1M workload (128: 4% slower, 64: 21% slower).
constexpr int kShBlock = 256;

template <int DEG>
__global__ __launch_bounds__(kShBlock) void sh_bwd_kernel(CamBatch cb, int64_t n, const float* means,
                                                        const float* sh,
                                                        const uint32_t* __restrict__ touched,
                                                        double* __restrict__ g2, float* __restrict__ d_means,
                                                        float* __restrict__ d_sh, int overwrite, StepArgs sa) {
  using F = float;
  constexpr int K = (DEG + 1) * (DEG + 1), KC = 3 * K, STR = KC + 1;
  __shared__ float shs[kShBlock * STR];
  const int64_t i0 = (int64_t)blockIdx.x * kShBlock;
  const int cnt = (int)min((int64_t)kShBlock, n - i0);
  stage_sh<DEG, kShBlock>(sh, i0, cnt, shs);
  __syncthreads();
  const int64_t i = i0 + threadIdx.x;
  float* slot = shs + threadIdx.x * STR;
  F gsh[KC];
#pragma unroll
  for (int j = 0; j < KC; ++j) gsh[j] = 0.0f;
  if (i < n) {
    const float* mu = means + 3 * i;
    F gmu[3] = {0, 0, 0};
    uint64_t clamped = 0;                      // bit 3v+c: colour c of view v clamped at 0
    for (int v = 0; v < cb.n_views; ++v) {
      const int64_t e = (int64_t)v * n + i;
      if (touched[e] == 0) continue;
      const CamDev& c = cb.v[v];
      const double* gq = g2 + e * kG2;
      const F gcol[3] = {(F)gq[5], (F)gq[6], (F)gq[7]};
      F dir[3], vn;
      view_dir<F>(c, mu, dir, &vn);
      F Yb[K];
      sh_basis<F>(DEG, dir[0], dir[1], dir[2], Yb);
      F wsum[16];
#pragma unroll
      for (int k = 0; k < K; ++k) wsum[k] = 0;
#pragma unroll
      for (int ch = 0; ch < 3; ++ch) {
        F raw = F(0.5);
#pragma unroll
        for (int k = 0; k < K; ++k) raw += Yb[k] * slot[3 * k + ch];
        if (!(raw > F(0))) {
          clamped |= 1ull << (3 * v + ch);
          continue;
        }
#pragma unroll
        for (int k = 0; k < K; ++k) wsum[k] += gcol[ch] * slot[3 * k + ch];
      }
      F gx = 0, gy = 0, gz = 0;
      if (DEG > 0) sh_basis_grad<F>(DEG, dir[0], dir[1], dir[2], wsum, &gx, &gy, &gz);
      const F dd = gx * dir[0] + gy * dir[1] + gz * dir[2];
      const F ivn = F(1) / vn;
      gmu[0] += (gx - dir[0] * dd) * ivn;
      gmu[1] += (gy - dir[1] * dd) * ivn;
      gmu[2] += (gz - dir[2] * dd) * ivn;
    }
    if (d_means) {
      if (overwrite) for (int a = 0; a < 3; ++a) d_means[3 * i + a] = gmu[a];
      else for (int a = 0; a < 3; ++a) d_means[3 * i + a] += gmu[a];
    }
    if (sa.on) {
      // for project_bwd_kernel's update: the two unused slots of entry i's
      // screen-space record (view 0) hold this part of d_means
      float* part = reinterpret_cast<float*>(g2 + (size_t)i * kG2 + 10);
      for (int a = 0; a < 3; ++a) part[a] = gmu[a];
    }
    // d_sh of this component, in registers: the slot keeps the SH values
    // for the update below
    for (int v = 0; v < cb.n_views; ++v) {
      const int64_t e = (int64_t)v * n + i;
      if (touched[e] == 0) continue;
      const CamDev& c = cb.v[v];
      const double* gq = g2 + e * kG2;
      const F gcol[3] = {(F)gq[5], (F)gq[6], (F)gq[7]};
      F dir[3], vn;
      view_dir<F>(c, mu, dir, &vn);
      F Yb[K];
      sh_basis<F>(DEG, dir[0], dir[1], dir[2], Yb);
#pragma unroll
      for (int ch = 0; ch < 3; ++ch) {
        const F gc = (clamped & (1ull << (3 * v + ch))) ? F(0) : gcol[ch];
#pragma unroll
        for (int k = 0; k < K; ++k) gsh[3 * k + ch] += gc * Yb[k];
      }
    }
  }
  if (sa.on && sa.adam) {
    // Adam on the SH coefficients, per wave over its own 64 components, in
    // the memory order of the coefficient arrays (lane l takes elements
    // l + 64 t, or 16-byte runs), so the moments stream coalesced.  The SH values come from
    // the slots (staged once), the gradient through the same slots: every
    // lane first takes its values, then the slots are overwritten with the
    // per-component gradients and read back in the same order.
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int nc = min(max(cnt - 64 * wv, 0), 64);
    const int total = nc * KC;
    const float* wsl = shs + 64 * wv * STR;
    const size_t o0 = (size_t)(i0 + 64 * wv) * KC;
    if constexpr (KC % 4 == 0) {
      // 16-byte runs: lane l takes elements 4q .. 4q + 3, q = l + 64 t (a run
      // lies in one component, KC being a multiple of 4), and each group
      // keeps 4 runs of m and v in flight: twice the bytes per lane of
      // scalar elements, where the kernel's 3 waves per SIMD (LDS and
      // registers) leave the memory pipe short of requests
      typedef float f4 __attribute__((ext_vector_type(4)));
      constexpr int Q = KC / 4;
      f4 pv[Q], gv[Q];
#pragma unroll
      for (int t = 0; t < Q; ++t) {
        const int el = 4 * (lane + 64 * t), c = el / KC, j = el - c * KC;
        const float* w = wsl + c * STR + j;
        pv[t] = el < total ? f4{w[0], w[1], w[2], w[3]} : f4{0.0f, 0.0f, 0.0f, 0.0f};
      }
      __syncthreads();
#pragma unroll
      for (int j = 0; j < KC; ++j) slot[j] = gsh[j];
      __syncthreads();
#pragma unroll
      for (int t = 0; t < Q; ++t) {
        const int el = 4 * (lane + 64 * t), c = el / KC, j = el - c * KC;
        const float* w = wsl + c * STR + j;
        gv[t] = el < total ? f4{w[0], w[1], w[2], w[3]} : f4{0.0f, 0.0f, 0.0f, 0.0f};
      }
      f4* const m4 = reinterpret_cast<f4*>(sa.m[4] + o0);
      f4* const v4 = reinterpret_cast<f4*>(sa.v[4] + o0);
      f4* const p4 = reinterpret_cast<f4*>(sa.sh + o0);
      constexpr int kGrp = 4;
#pragma unroll
      for (int t0 = 0; t0 < Q; t0 += kGrp) {
        f4 m[kGrp], v[kGrp];
#pragma unroll
        for (int u = 0; u < kGrp && t0 + u < Q; ++u) {
          const int q = lane + 64 * (t0 + u);
          if (4 * q < total) {
            m[u] = __builtin_nontemporal_load(m4 + q);
            v[u] = __builtin_nontemporal_load(v4 + q);
          }
        }
#pragma unroll
        for (int u = 0; u < kGrp && t0 + u < Q; ++u) {
          const int q = lane + 64 * (t0 + u);
          if (4 * q < total) {
            f4 pp = pv[t0 + u], mm = m[u], vv = v[u];
            const f4 gg = gv[t0 + u];
#pragma unroll
            for (int e = 0; e < 4; ++e) {
              float pe = pp[e], me = mm[e], ve = vv[e];
              adam_one(pe, gg[e], me, ve, sa.lr[4], sa.lo[4], sa.hi[4], sa.ac);
              pp[e] = pe; mm[e] = me; vv[e] = ve;
            }
            __builtin_nontemporal_store(pp, p4 + q);
            __builtin_nontemporal_store(mm, m4 + q);
            __builtin_nontemporal_store(vv, v4 + q);
          }
        }
      }
    } else {
      float pv[KC], gv[KC];
#pragma unroll
      for (int t = 0; t < KC; ++t) {
        const int el = lane + 64 * t, c = el / KC, j = el - c * KC;
        pv[t] = el < total ? wsl[c * STR + j] : 0.0f;
      }
      __syncthreads();
#pragma unroll
      for (int j = 0; j < KC; ++j) slot[j] = gsh[j];
      __syncthreads();
#pragma unroll
      for (int t = 0; t < KC; ++t) {
        const int el = lane + 64 * t, c = el / KC, j = el - c * KC;
        gv[t] = el < total ? wsl[c * STR + j] : 0.0f;
      }
      constexpr int kGrp = 8;                  // loads of a group issued before its updates
#pragma unroll
      for (int t0 = 0; t0 < KC; t0 += kGrp) {
        float m[kGrp], v[kGrp];
#pragma unroll
        for (int u = 0; u < kGrp && t0 + u < KC; ++u) {
          const int el = lane + 64 * (t0 + u);
          if (el < total) {
            m[u] = __builtin_nontemporal_load(sa.m[4] + o0 + el);
            v[u] = __builtin_nontemporal_load(sa.v[4] + o0 + el);
          }
        }
#pragma unroll
        for (int u = 0; u < kGrp && t0 + u < KC; ++u) {
          const int el = lane + 64 * (t0 + u);
          if (el < total) {
            float pp = pv[t0 + u];
            adam_one(pp, gv[t0 + u], m[u], v[u], sa.lr[4], sa.lo[4], sa.hi[4], sa.ac);
            __builtin_nontemporal_store(pp, sa.sh + o0 + el);
            __builtin_nontemporal_store(m[u], sa.m[4] + o0 + el);
            __builtin_nontemporal_store(v[u], sa.v[4] + o0 + el);
          }
        }
      }
    }
    // the slots hold the gradients (per component) for the d_sh output
  } else {
#pragma unroll
    for (int j = 0; j < KC; ++j) slot[j] = gsh[j];
  }
  __syncthreads();
  if (!d_sh) return;
  float* dst = d_sh + (size_t)i0 * KC;
  for (int g = threadIdx.x; g < cnt * KC; g += kShBlock) {
    const int c = g / KC, j = g - c * KC;
    if (overwrite) dst[g] = shs[c * STR + j];
    else dst[g] += shs[c * STR + j];
  }
}

}  // namespace

void launch_project(const CamBatch& cb, const OptsDev& op, const sss_scene_t& s, const sss_proj_t& out,
                    hipStream_t st) {
  // component blocks rounded up to the 8-block chunks of project_kernel's ids
  const int64_t nb = (s.n + kBlock - 1) / kBlock;
  dim3 grid((unsigned)(((nb + 7) / 8) * 8 * cb.n_views));
#define SSS_PROJ(D)                                                                                          \
  SSS_LAUNCH("project", project_kernel<D>, grid, dim3(kBlock), 0, st, cb, op, (int64_t)s.n, s.means, s.scales, \
             s.quats, s.nu, s.opacity, s.sh, (Entry*)out.entries, out.depth_key, out.tiles_touched)
  switch (s.sh_degree) {
    case 0: SSS_PROJ(0); break;
    case 1: SSS_PROJ(1); break;
    case 2: SSS_PROJ(2); break;
    default: SSS_PROJ(3); break;
  }
#undef SSS_PROJ
}

void launch_project_bwd(const CamBatch& cb, const OptsDev& op, const sss_scene_t& s, const uint32_t* touched,
                        double* g2, const sss_grads_t& gr, const StepArgs& sa, hipStream_t st) {
  dim3 grid((unsigned)((s.n + kBlock - 1) / kBlock));
  const dim3 grid_sh((unsigned)((s.n + kShBlock - 1) / kShBlock));
#define SSS_SHB(D)                                                                                         \
  SSS_LAUNCH("sh_bwd", sh_bwd_kernel<D>, grid_sh, dim3(kShBlock), 0, st, cb, (int64_t)s.n, s.means, s.sh, touched, \
             g2, gr.means, gr.sh, (int)gr.overwrite, sa)
  switch (s.sh_degree) {
    case 0: SSS_SHB(0); break;
    case 1: SSS_SHB(1); break;
    case 2: SSS_SHB(2); break;
    default: SSS_SHB(3); break;
  }
#undef SSS_SHB
  SSS_LAUNCH("project_bwd", project_bwd_kernel, grid, dim3(kBlock), 0, st, cb, op, (int64_t)s.n, s.means, s.scales,
             s.quats, s.nu, s.opacity, touched, (const double*)g2, gr.means, gr.scales, gr.quats, gr.nu, gr.opacity,
             (int)gr.overwrite, sa);
}

}  // namespace sss
