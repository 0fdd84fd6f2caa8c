// Photometric loss of Sec. 3.4: L = (1 - lambda) L1 + lambda (1 - SSIM), and
// dL/dimage.  SSIM with an 11x11 Gaussian window (sigma 1.5), C1 = 0.01^2,
// C2 = 0.03^2, zero padding, per view; L1 and SSIM are means over all 3P
// values of all views.
//
// With mx = G*x, Exx = G*(x x), Exy = G*(x y) (and my, Eyy for the target),
// S = (2 mx my + C1)(2 sxy + C2) / ((mx^2 + my^2 + C1)(sxx + syy + C2)):
//   dS/dmx  = S (2my/A1 - 2my/A2 - 2mx/B1 + 2mx/B2),
//   dS/dExx = -S / B2,   dS/dExy = 2 S / A2,
// so d(sum S)/dx = G*(dS/dmx) + 2 x G*(dS/dExx) + y G*(dS/dExy) (G symmetric).
// ssim_fwd writes the three partial maps and accumulates L; ssim_bwd filters
// them and writes dL/dimage.  Both work on 16x16 output tiles with a 5-pixel
// halo staged in LDS and separable filtering (horizontal, then vertical).
#include "common.hpp"

namespace sss {
namespace {

constexpr int kR = 5;                  // window radius
constexpr int kP = kTile + 2 * kR;     // patch edge (26)
constexpr float kC1 = 0.0001f, kC2 = 0.0009f;

struct Window {
  float g[2 * kR + 1];
};

struct TileXY {
  int view, x0, y0, W, H;
  int64_t pix0;
};

__device__ __forceinline__ TileXY loss_tile(const CamBatch& cb) {
  const int g = blockIdx.x;
  int v = 0;
  for (int k = 1; k < cb.n_views; ++k)
    if (g >= cb.v[k].tile_offset) v = k;
  const CamDev& c = cb.v[v];
  const int lt = g - c.tile_offset;
  TileXY t;
  t.view = v;
  t.x0 = (lt % c.tiles_x) * kTile;
  t.y0 = (lt / c.tiles_x) * kTile;
  t.W = c.W;
  t.H = c.H;
  t.pix0 = c.pix_offset;
  return t;
}

// Load channel-interleaved maps (nch values per pixel, channel ch) of the
// tile's patch into LDS, zero outside the image.
__device__ __forceinline__ void load_patch(const TileXY& t, const float* __restrict__ src, int nch, int ch,
                                           float* dst) {
  for (int i = threadIdx.x; i < kP * kP; i += kBlock) {
    const int py = i / kP, px = i - py * kP;
    const int x = t.x0 - kR + px, y = t.y0 - kR + py;
    float v = 0.0f;
    if (x >= 0 && y >= 0 && x < t.W && y < t.H) v = src[(t.pix0 + (int64_t)y * t.W + x) * nch + ch];
    dst[i] = v;
  }
}

__global__ __launch_bounds__(kBlock) void ssim_fwd_kernel(CamBatch cb, Window wd, const float* __restrict__ img,
                                                          const float* __restrict__ tgt, float lam, float inv_count,
                                                          float* __restrict__ partial, float* __restrict__ loss_out) {
  __shared__ float sx[kP * kP], sy[kP * kP];
  __shared__ float hs[5][kP * kTile];   // horizontal sums: x, y, xx, yy, xy
  __shared__ float red[kBlock / 64];
  const TileXY t = loss_tile(cb);
  const int lx = threadIdx.x & (kTile - 1), ly = threadIdx.x / kTile;
  const int x = t.x0 + lx, y = t.y0 + ly;
  const bool inside = x < t.W && y < t.H;
  const int64_t p = t.pix0 + (int64_t)y * t.W + x;
  float acc = 0.0f;
  for (int ch = 0; ch < 3; ++ch) {
    __syncthreads();
    load_patch(t, img, 3, ch, sx);
    load_patch(t, tgt, 3, ch, sy);
    __syncthreads();
    for (int i = threadIdx.x; i < kP * kTile; i += kBlock) {
      const int r = i / kTile, c = i - r * kTile;
      float a = 0.0f, b = 0.0f, aa = 0.0f, bb = 0.0f, ab = 0.0f;
#pragma unroll
      for (int k = 0; k < 2 * kR + 1; ++k) {
        const float u = sx[r * kP + c + k], v = sy[r * kP + c + k], w = wd.g[k];
        a = __fmaf_rn(w, u, a);
        b = __fmaf_rn(w, v, b);
        aa = __fmaf_rn(w * u, u, aa);
        bb = __fmaf_rn(w * v, v, bb);
        ab = __fmaf_rn(w * u, v, ab);
      }
      hs[0][i] = a; hs[1][i] = b; hs[2][i] = aa; hs[3][i] = bb; hs[4][i] = ab;
    }
    __syncthreads();
    float mx = 0.0f, my = 0.0f, exx = 0.0f, eyy = 0.0f, exy = 0.0f;
#pragma unroll
    for (int k = 0; k < 2 * kR + 1; ++k) {
      const int i = (ly + k) * kTile + lx;
      const float w = wd.g[k];
      mx = __fmaf_rn(w, hs[0][i], mx);
      my = __fmaf_rn(w, hs[1][i], my);
      exx = __fmaf_rn(w, hs[2][i], exx);
      eyy = __fmaf_rn(w, hs[3][i], eyy);
      exy = __fmaf_rn(w, hs[4][i], exy);
    }
    if (inside) {
      const float sxx = exx - mx * mx, syy = eyy - my * my, sxy = exy - mx * my;
      const float A1 = 2.0f * mx * my + kC1, A2 = 2.0f * sxy + kC2;
      const float B1 = mx * mx + my * my + kC1, B2 = sxx + syy + kC2;
      const float S = (A1 * A2) / (B1 * B2);
      const float dmx = S * (2.0f * my / A1 - 2.0f * my / A2 - 2.0f * mx / B1 + 2.0f * mx / B2);
      const float dxx = -S / B2;
      const float dxy = 2.0f * S / A2;
      float* q = partial + p * 9 + 3 * ch;
      q[0] = dmx;
      q[1] = dxx;
      q[2] = dxy;
      const float d = sx[(ly + kR) * kP + lx + kR] - sy[(ly + kR) * kP + lx + kR];
      acc += (1.0f - lam) * fabsf(d) + lam * (1.0f - S);
    }
  }
  if (loss_out) {
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) atomicAdd(loss_out, (red[0] + red[1] + red[2] + red[3]) * inv_count);
  }
}

__global__ __launch_bounds__(kBlock) void ssim_bwd_kernel(CamBatch cb, Window wd, const float* __restrict__ img,
                                                          const float* __restrict__ tgt, float lam, float inv_count,
                                                          const float* __restrict__ partial,
                                                          float* __restrict__ dl_dimage) {
  __shared__ float sp[3][kP * kP];
  __shared__ float hs[3][kP * kTile];
  const TileXY t = loss_tile(cb);
  const int lx = threadIdx.x & (kTile - 1), ly = threadIdx.x / kTile;
  const int x = t.x0 + lx, y = t.y0 + ly;
  const bool inside = x < t.W && y < t.H;
  const int64_t p = t.pix0 + (int64_t)y * t.W + x;
  for (int ch = 0; ch < 3; ++ch) {
    __syncthreads();
    for (int m = 0; m < 3; ++m) load_patch(t, partial, 9, 3 * ch + m, sp[m]);
    __syncthreads();
    for (int i = threadIdx.x; i < kP * kTile; i += kBlock) {
      const int r = i / kTile, c = i - r * kTile;
      float a = 0.0f, b = 0.0f, d = 0.0f;
#pragma unroll
      for (int k = 0; k < 2 * kR + 1; ++k) {
        const float w = wd.g[k];
        a = __fmaf_rn(w, sp[0][r * kP + c + k], a);
        b = __fmaf_rn(w, sp[1][r * kP + c + k], b);
        d = __fmaf_rn(w, sp[2][r * kP + c + k], d);
      }
      hs[0][i] = a; hs[1][i] = b; hs[2][i] = d;
    }
    __syncthreads();
    float ga = 0.0f, gb = 0.0f, gc = 0.0f;
#pragma unroll
    for (int k = 0; k < 2 * kR + 1; ++k) {
      const int i = (ly + k) * kTile + lx;
      const float w = wd.g[k];
      ga = __fmaf_rn(w, hs[0][i], ga);
      gb = __fmaf_rn(w, hs[1][i], gb);
      gc = __fmaf_rn(w, hs[2][i], gc);
    }
    if (inside) {
      const float xv = img[3 * p + ch], yv = tgt[3 * p + ch];
      const float dl1 = xv > yv ? inv_count : (xv < yv ? -inv_count : 0.0f);
      const float dss = ga + 2.0f * xv * gb + yv * gc;
      dl_dimage[3 * p + ch] = (1.0f - lam) * dl1 - lam * inv_count * dss;
    }
  }
}

}  // namespace

size_t loss_workspace(int64_t total_pixels) { return (size_t)total_pixels * 9 * sizeof(float); }

void launch_loss(const CamBatch& cb, const float* img, const float* tgt, float lam, float* dl, float* loss_out,
                 float* partial, int64_t total_pixels, hipStream_t st) {
  Window wd;
  double s = 0.0, g[2 * kR + 1];
  for (int k = 0; k <= 2 * kR; ++k) {
    const double u = k - kR;
    g[k] = exp(-u * u / (2.0 * 1.5 * 1.5));
    s += g[k];
  }
  for (int k = 0; k <= 2 * kR; ++k) wd.g[k] = (float)(g[k] / s);
  const float inv_count = (float)(1.0 / (3.0 * (double)total_pixels));
  SSS_LAUNCH("ssim_fwd", ssim_fwd_kernel, dim3((unsigned)cb.total_tiles), dim3(kBlock), 0, st, cb, wd, img, tgt, lam,
             inv_count, partial, loss_out);
  SSS_LAUNCH("ssim_bwd", ssim_bwd_kernel, dim3((unsigned)cb.total_tiles), dim3(kBlock), 0, st, cb, wd, img, tgt, lam,
             inv_count, (const float*)partial, dl);
}

}  // namespace sss
