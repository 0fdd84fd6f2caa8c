// Tile rasterizer: signed front-to-back compositing of 2D Student's t
// components (Sec. 3.4 eq. SSS_color) and its closed-form backward pass
// (SM "Backward Pass").
//
// One workgroup of 256 threads per 16x16 tile, one pixel per thread (wave w
// covers tile rows 4w..4w+3).  The tile's depth-ordered list is consumed in
// batches of 256 records staged in LDS; every thread reads each staged record
// as a broadcast.  The 2D mean is re-based on the tile origin in FP64 while
// staging, so pixel offsets keep full FP32 relative precision.
//
// The backward pass walks the list front to back, like the forward pass: with
// out = sum_j c_j a_j T_j + T_final bg and A_i = sum_{j<=i} c_j a_j T_j,
//   d out / d a_i = c_i T_i - (out - A_i) / (1 - a_i),
// so it needs only the forward output per pixel, never a division to recover
// T.  The per-pixel gradients of each record are summed over the wave with
// DPP row shifts / broadcasts, and lane 63 adds them to the entry's
// screen-space gradient slot with hardware float atomics.
#include "common.hpp"

namespace sss {
namespace {

constexpr float kLog2e = 1.4426950408889634f;
constexpr float kLn2 = 0.6931471805599453f;

// LDS record (16 floats).
struct __align__(16) LRec {
  float mx, my, qa, qb;      // mean relative to the tile origin; conic a, b
  float qc, hs, o, inv_nu;   // conic c; truncation test level; opacity; 1/nu
  float nb, cr, cg, cb;      // -(nu+2)/2; colour
  float nu, pad0;
  uint32_t entry;
  float pad1;
};

__device__ __forceinline__ void stage(const Rec* __restrict__ srec, uint32_t rank, double ox, double oy, LRec* dst) {
  const Rec r = srec[rank];
  LRec l;
  l.mx = (float)(r.mx - ox);
  l.my = (float)(r.my - oy);
  l.qa = r.qa; l.qb = r.qb; l.qc = r.qc;
  // Conservative pre-test level; the alpha test itself decides.
  l.hs = r.hs * 1.0001f;
  l.o = r.o;
  l.inv_nu = r.inv_nu;
  l.nb = r.nb;
  l.cr = r.cr; l.cg = r.cg; l.cb = r.cb;
  l.nu = r.nu;
  l.pad0 = 0.0f;
  l.entry = r.entry;
  l.pad1 = 0.0f;
  *dst = l;
}

// Evaluation of one record at one pixel, shared bit-for-bit by the forward
// and backward kernels (explicit fma, compiled without contraction).
struct Eval {
  float dx, dy, ax, ay, h, y, u, l2, t2, alpha;
  bool hit, clamped;
};

__device__ __forceinline__ void evaluate(float px, float py, const LRec& L, float amin, float amax, Eval& E) {
  E.dx = px - L.mx;
  E.dy = py - L.my;
  E.ax = __fmaf_rn(L.qb, E.dy, L.qa * E.dx);
  E.ay = __fmaf_rn(L.qb, E.dx, L.qc * E.dy);
  E.h = __fmaf_rn(E.dx, E.ax, E.dy * E.ay);
  E.hit = false;
  E.clamped = false;
  if (!(E.h <= L.hs)) return;
  // T2D = (1 + h/nu)^(-(nu+2)/2) = 2^(nb log2(1 + y)), y = h/nu.  log2(1 + y) is
  // corrected by the rounding error of u = 1 + y while u < 2.
  E.y = E.h * L.inv_nu;
  E.u = 1.0f + E.y;
  const float z = E.u - 1.0f;
  const float corr = E.u < 2.0f ? (E.y - z) : 0.0f;
  E.l2 = __fmaf_rn(corr, kLog2e, __builtin_amdgcn_logf(E.u));
  E.t2 = __builtin_amdgcn_exp2f(L.nb * E.l2);
  float a = L.o * E.t2;
  if (fabsf(a) < amin) return;
  E.clamped = fabsf(a) > amax;
  a = fminf(fmaxf(a, -amax), amax);
  E.alpha = a;
  E.hit = true;
}

template <int kCtrl, int kRowMask>
__device__ __forceinline__ float dpp_add(float v) {
  return v + __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), kCtrl, kRowMask, 0xf, true));
}

// Sum over the 64 lanes, result in lane 63 (row shifts, then row broadcasts).
__device__ __forceinline__ float wave_sum63(float v) {
  v = dpp_add<0x111, 0xf>(v);  // row_shr:1
  v = dpp_add<0x112, 0xf>(v);  // row_shr:2
  v = dpp_add<0x114, 0xf>(v);  // row_shr:4
  v = dpp_add<0x118, 0xf>(v);  // row_shr:8
  v = dpp_add<0x142, 0xa>(v);  // row_bcast:15
  v = dpp_add<0x143, 0xc>(v);  // row_bcast:31
  return v;
}

struct TileCtx {
  int view, tx, ty, x, y;
  bool inside;
  float px, py;
  double ox, oy;
  int64_t pix;
  uint32_t start, end;
};

__device__ __forceinline__ TileCtx tile_ctx(const CamBatch& cb, const uint32_t* __restrict__ tile_start) {
  TileCtx t;
  const int g = blockIdx.x;
  int v = 0;
  for (int k = 1; k < cb.n_views; ++k)
    if (g >= cb.v[k].tile_offset) v = k;
  const CamDev& c = cb.v[v];
  const int lt = g - c.tile_offset;
  t.view = v;
  t.tx = lt % c.tiles_x;
  t.ty = lt / c.tiles_x;
  const int lx = threadIdx.x & (kTile - 1), ly = threadIdx.x / kTile;
  t.x = t.tx * kTile + lx;
  t.y = t.ty * kTile + ly;
  t.inside = t.x < c.W && t.y < c.H;
  t.px = (float)lx + 0.5f;
  t.py = (float)ly + 0.5f;
  t.ox = (double)(t.tx * kTile);
  t.oy = (double)(t.ty * kTile);
  t.pix = c.pix_offset + (int64_t)t.y * c.W + t.x;
  t.start = tile_start[g];
  t.end = tile_start[g + 1];
  return t;
}

// Forward traversal of the tile list; identical in render_fwd and in the
// recompute phase of render_bwd.
__device__ __forceinline__ void forward_walk(const TileCtx& t, const OptsDev& op, const Rec* __restrict__ srec,
                                             const uint32_t* __restrict__ pair_rank, LRec* lds, float* C,
                                             float* Tout, uint32_t* last_out) {
  bool done = !t.inside;
  float T = 1.0f, c0 = 0.0f, c1 = 0.0f, c2 = 0.0f;
  uint32_t last = 0;
  for (uint32_t base = t.start; base < t.end; base += kBlock) {
    if (__syncthreads_count(done) == kBlock) break;
    const uint32_t k = base + threadIdx.x;
    if (k < t.end) stage(srec, pair_rank[k], t.ox, t.oy, lds + threadIdx.x);
    __syncthreads();
    const int cnt = (int)min((uint32_t)kBlock, t.end - base);
    if (!done) {
      for (int j = 0; j < cnt; ++j) {
        const LRec L = lds[j];
        Eval E;
        evaluate(t.px, t.py, L, op.alpha_min, op.alpha_max, E);
        if (!E.hit) continue;
        const float Tn = T * (1.0f - E.alpha);
        if (Tn < op.t_min) {
          done = true;
          break;
        }
        const float wgt = E.alpha * T;
        c0 = __fmaf_rn(L.cr, wgt, c0);
        c1 = __fmaf_rn(L.cg, wgt, c1);
        c2 = __fmaf_rn(L.cb, wgt, c2);
        T = Tn;
        last = base - t.start + (uint32_t)j + 1u;
      }
    }
  }
  C[0] = __fmaf_rn(T, op.bg[0], c0);
  C[1] = __fmaf_rn(T, op.bg[1], c1);
  C[2] = __fmaf_rn(T, op.bg[2], c2);
  *Tout = T;
  *last_out = last;
}

__global__ __launch_bounds__(kBlock) void render_fwd_kernel(CamBatch cb, OptsDev op, const Rec* __restrict__ srec,
                                                            const uint32_t* __restrict__ tile_start,
                                                            const uint32_t* __restrict__ pair_rank,
                                                            float* __restrict__ image, float* __restrict__ t_final,
                                                            uint32_t* __restrict__ n_contrib) {
  __shared__ LRec lds[kBlock];
  const TileCtx t = tile_ctx(cb, tile_start);
  float C[3], T;
  uint32_t last;
  forward_walk(t, op, srec, pair_rank, lds, C, &T, &last);
  if (t.inside) {
    image[3 * t.pix + 0] = C[0];
    image[3 * t.pix + 1] = C[1];
    image[3 * t.pix + 2] = C[2];
    if (t_final) t_final[t.pix] = T;
    if (n_contrib) n_contrib[t.pix] = last;
  }
}

template <int kMode, int kLoss>
__global__ __launch_bounds__(kBlock) void render_bwd_kernel(CamBatch cb, OptsDev op, const Rec* __restrict__ srec,
                                                            const uint32_t* __restrict__ tile_start,
                                                            const uint32_t* __restrict__ pair_rank,
                                                            const float* __restrict__ dl_or_target,
                                                            const float* __restrict__ image,
                                                            const uint32_t* __restrict__ n_contrib,
                                                            float* __restrict__ image_out, float* __restrict__ loss_out,
                                                            float inv_count, float* __restrict__ g2) {
  __shared__ LRec lds[kBlock];
  __shared__ uint32_t s_max;
  __shared__ float s_loss[kBlock / 64];
  const TileCtx t = tile_ctx(cb, tile_start);
  const int lane = threadIdx.x & 63;

  // ---- per-pixel forward output and loss gradient ----
  float out[3] = {0.0f, 0.0f, 0.0f};
  uint32_t bound = 0;
  if (kMode == SSS_BWD_RECOMPUTE) {
    float T;
    forward_walk(t, op, srec, pair_rank, lds, out, &T, &bound);
    if (image_out && t.inside) {
      image_out[3 * t.pix + 0] = out[0];
      image_out[3 * t.pix + 1] = out[1];
      image_out[3 * t.pix + 2] = out[2];
    }
    if (!t.inside) bound = 0;
  } else if (t.inside) {
    out[0] = image[3 * t.pix + 0];
    out[1] = image[3 * t.pix + 1];
    out[2] = image[3 * t.pix + 2];
    bound = n_contrib[t.pix];
  }
  float g[3] = {0.0f, 0.0f, 0.0f};
  float l1 = 0.0f;
  if (t.inside) {
    if (kLoss == SSS_LOSS_L1) {
      for (int ch = 0; ch < 3; ++ch) {
        const float d = out[ch] - dl_or_target[3 * t.pix + ch];
        g[ch] = d > 0.0f ? inv_count : (d < 0.0f ? -inv_count : 0.0f);
        l1 += fabsf(d);
      }
    } else {
      g[0] = dl_or_target[3 * t.pix + 0];
      g[1] = dl_or_target[3 * t.pix + 1];
      g[2] = dl_or_target[3 * t.pix + 2];
    }
  }
  if (kLoss == SSS_LOSS_L1 && loss_out) {
    // |out - target| summed over the workgroup, one atomic per tile
    l1 = wave_sum63(l1);
    if (lane == 63) s_loss[threadIdx.x >> 6] = l1;
  }
  const float gout = g[0] * out[0] + g[1] * out[1] + g[2] * out[2];

  if (threadIdx.x == 0) s_max = 0;
  __syncthreads();
  atomicMax(&s_max, bound);
  __syncthreads();
  const uint32_t stop = min(t.start + s_max, t.end);
  if (kLoss == SSS_LOSS_L1 && loss_out && threadIdx.x == 0)
    atomicAdd(loss_out, (s_loss[0] + s_loss[1] + s_loss[2] + s_loss[3]) * inv_count);

  // ---- front-to-back gradient walk ----
  float T = 1.0f, gA = 0.0f;
  for (uint32_t base = t.start; base < stop; base += kBlock) {
    __syncthreads();
    const uint32_t k = base + threadIdx.x;
    if (k < stop) stage(srec, pair_rank[k], t.ox, t.oy, lds + threadIdx.x);
    __syncthreads();
    const int cnt = (int)min((uint32_t)kBlock, stop - base);
    for (int j = 0; j < cnt; ++j) {
      const uint32_t pos = base - t.start + (uint32_t)j;
      const LRec L = lds[j];
      float v0 = 0.0f, v1 = 0.0f, v2 = 0.0f, v3 = 0.0f, v4 = 0.0f;
      float v5 = 0.0f, v6 = 0.0f, v7 = 0.0f, v8 = 0.0f, v9 = 0.0f;
      bool hit = false;
      if (pos < bound) {
        Eval E;
        evaluate(t.px, t.py, L, op.alpha_min, op.alpha_max, E);
        if (E.hit) {
          hit = true;
          const float a = E.alpha;
          const float Tn = T * (1.0f - a);
          const float w = a * T;
          const float gc = __fmaf_rn(g[2], L.cb, __fmaf_rn(g[1], L.cg, g[0] * L.cr));
          gA = __fmaf_rn(w, gc, gA);
          const float gR = gout - gA;
          const float da = __fmaf_rn(-gR, __builtin_amdgcn_rcpf(1.0f - a), T * gc);
          v5 = g[0] * w;
          v6 = g[1] * w;
          v7 = g[2] * w;
          if (!E.clamped) {
            v8 = da * E.t2;
            const float dt2 = da * L.o;
            const float ru = __builtin_amdgcn_rcpf(E.u);
            const float dh = dt2 * E.t2 * L.nb * L.inv_nu * ru;
            v0 = dh * E.ax;
            v1 = dh * E.ay;
            const float tq = dh * E.dx;
            v2 = tq * E.dx;
            v3 = tq * E.dy;
            v4 = dh * E.dy * E.dy;
            // dT2D/dnu = T2D/2 [y/(1+y) - log(1+y) + 2y/(nu (1+y))]
            const float y = E.y;
            float q;
            if (y < 0.1f) {
              float s = __fmaf_rn(y, 6.0f / 7.0f, -5.0f / 6.0f);
              s = __fmaf_rn(y, s, 4.0f / 5.0f);
              s = __fmaf_rn(y, s, -3.0f / 4.0f);
              s = __fmaf_rn(y, s, 2.0f / 3.0f);
              s = __fmaf_rn(y, s, -0.5f);
              q = y * y * s;
            } else {
              q = __fmaf_rn(y, ru, -E.l2 * kLn2);
            }
            const float dtn = 0.5f * E.t2 * __fmaf_rn(2.0f * y * L.inv_nu, ru, q);
            v9 = dt2 * dtn;
          }
          T = Tn;
        }
      }
      if (__any(hit)) {
        v0 = wave_sum63(v0); v1 = wave_sum63(v1); v2 = wave_sum63(v2); v3 = wave_sum63(v3);
        v4 = wave_sum63(v4); v5 = wave_sum63(v5); v6 = wave_sum63(v6); v7 = wave_sum63(v7);
        v8 = wave_sum63(v8); v9 = wave_sum63(v9);
        if (lane == 63) {
          float* gp = g2 + (size_t)L.entry * kG2;
          atomicAdd(gp + 0, -2.0f * v0);
          atomicAdd(gp + 1, -2.0f * v1);
          atomicAdd(gp + 2, v2);
          atomicAdd(gp + 3, 2.0f * v3);
          atomicAdd(gp + 4, v4);
          atomicAdd(gp + 5, v5);
          atomicAdd(gp + 6, v6);
          atomicAdd(gp + 7, v7);
          atomicAdd(gp + 8, v8);
          atomicAdd(gp + 9, v9);
        }
      }
    }
  }
}

__global__ __launch_bounds__(kBlock) void zero_kernel(float4* __restrict__ p, int64_t n4) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < n4) p[i] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
}

}  // namespace

void launch_zero(float* p, int64_t count, hipStream_t st) {
  // count is a multiple of 4 for every caller (kG2 = 12 floats per entry)
  const int64_t n4 = count / 4;
  if (n4 <= 0) return;
  SSS_LAUNCH("zero", zero_kernel, dim3((unsigned)((n4 + kBlock - 1) / kBlock)), dim3(kBlock), 0, st,
                     (float4*)p, n4);
}

void launch_render_fwd(const CamBatch& cb, const OptsDev& op, const sss_bins_t& b, float* image, float* t_final,
                       uint32_t* n_contrib, hipStream_t st) {
  SSS_LAUNCH("render_fwd", render_fwd_kernel, dim3((unsigned)cb.total_tiles), dim3(kBlock), 0, st, cb, op,
                     (const Rec*)b.sorted_records, (const uint32_t*)b.tile_start, (const uint32_t*)b.pair_rank,
                     image, t_final, n_contrib);
}

void launch_render_bwd(const CamBatch& cb, const OptsDev& op, const sss_bins_t& b, int mode, int loss,
                       const float* dl_or_target, const float* image, const uint32_t* n_contrib, float* image_out,
                       float* loss_out, float* g2, int64_t total_pixels, hipStream_t st) {
  const float inv_count = 1.0f / (3.0f * (float)total_pixels);
  const dim3 grid((unsigned)cb.total_tiles), blk(kBlock);
  const Rec* sr = (const Rec*)b.sorted_records;
  const uint32_t* ts = b.tile_start;
  const uint32_t* pr = b.pair_rank;
#define SSS_BWD(M, L)                                                                                        \
  SSS_LAUNCH("render_bwd", (render_bwd_kernel<M, L>), grid, blk, 0, st, cb, op, sr, ts, pr, dl_or_target, image,  \
                     n_contrib, image_out, loss_out, inv_count, g2)
  if (mode == SSS_BWD_STORED && loss == SSS_LOSS_GRAD) SSS_BWD(SSS_BWD_STORED, SSS_LOSS_GRAD);
  else if (mode == SSS_BWD_STORED) SSS_BWD(SSS_BWD_STORED, SSS_LOSS_L1);
  else if (loss == SSS_LOSS_GRAD) SSS_BWD(SSS_BWD_RECOMPUTE, SSS_LOSS_GRAD);
  else SSS_BWD(SSS_BWD_RECOMPUTE, SSS_LOSS_L1);
#undef SSS_BWD
}

}  // namespace sss
