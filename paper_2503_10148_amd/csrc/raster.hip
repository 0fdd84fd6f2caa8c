// Tile rasterizer: signed front-to-back compositing of 2D Student's t
// components (Sec. 3.4 eq. SSS_color) and its closed-form backward pass
// (SM "Backward Pass").
//
// Work unit: one wave of 64 threads, each thread PIX pixels, renders 4*PIX
// consecutive rows of a 16x16 tile (4/PIX units per tile), as a workgroup
// of its own, so the hardware schedules units rather than whole tiles; the
// units are launched most expensive first.  The tile's depth-ordered list is
// consumed in batches of 64 records staged in LDS, and the walk visits only
// the staged records whose strip mask meets the unit (a ballot); every lane
// reads a visited record as a broadcast.  The 2D mean is re-based on the
// tile origin in FP64 while staging and the staged record carries L^T m
// (L the conic's Cholesky factor, m that mean), so a pixel's w = L^T (p - m)
// is three FMAs on tile coordinates.
//
// The backward pass walks the list front to back, like the forward pass: with
// out = sum_j c_j a_j T_j + T_final bg and A_i = sum_{j<=i} c_j a_j T_j,
//   d out / d a_i = c_i T_i - (out - A_i) / (1 - a_i),
// so it needs only the forward output per pixel, never a division to recover
// T.  The ten per-pixel gradient sums of a record are reduced over the wave
// in transposed form (wave_sum10_transposed), and ten lanes add them to the
// entry's screen-space gradient slot with one FP64 atomic instruction.
//
// Deterministic variant: instead of the atomics, those lanes store the sums
// of each (tile, component) pair in the pair's own slot, addressed by the
// pair's position in emission order (the component's rank offset plus the
// tile's row-major index in its rectangle).  A second kernel then adds, for
// every component, its slots in emission order with a fixed reduction tree,
// so the result does not depend on scheduling.
#include <stdlib.h>

#include "common.hpp"
#include "tiles.hpp"

namespace sss {
namespace {

constexpr float kLog2e = 1.4426950408889634f;

// LDS record (16 floats).
struct __align__(16) LRec {
  float q0, q1, l11, l21;    // L^T m (m: mean relative to the tile origin); conic's Cholesky factor
  float l22, pad, o, inv_nu; // (L = [[l11, 0], [l21, l22]], h = |L^T p - L^T m|^2); (unused); opacity; 1/nu
  float nb, cr, cg, cb;      // -(nu+2)/2; colour
  uint32_t smask;            // bit s: the ellipse reaches strip s (rows 4s..4s+3), of the unit's strips
  float c2;                  // 2 log2(e) / nu (the backward's nu term; 0 for the Gaussian family)
  uint32_t entry;
  uint32_t slot;             // deterministic backward: the pair's emission position
};

// Forward-only LDS record (64 bytes): the colour is converted to FP64 once
// when staged rather than per pixel in the compositing loop.
struct __align__(16) FRec {
  float q0, q1, l11, l21;
  float l22, pad, o, inv_nu;
  float nb;
  uint32_t smask;
  double cr, cg, cb;
};

// Strips of 4 pixel rows (bit st: pixel centres x in [1/2, 31/2], y in
// [4 st + 1/2, 4 st + 7/2], tile coordinates) that the ellipse h <= h* of a
// record reaches, for the N strips first .. first + N - 1 (the caller's
// unit; first is wave-uniform).  Exact rather than by the ellipse's row
// extent, which visits 9% more strips on the 1M-component workload (tilted
// ellipses that cross a tile's corner).
//
// The minimum of h over a box is 0 with the mean inside it, else it lies on
// an edge.  On a row y = Y it is qa (x - x*)^2 + (Y - my)^2 / Sigma_yy, with
// x* = mx - (qb/qa)(Y - my) the row's minimiser clamped to the box
// (completing the square: two non-negative terms, so FP32 loses nothing to
// cancellation, however elongated the ellipse); on a column x = X likewise
// qc (y - y*)^2 + (X - mx)^2 / Sigma_xx.  The record gives 1/Sigma_yy =
// h*/ey^2 and Sigma_xx / Sigma_yy = qc / qa.  A strip is kept when the
// minimum is within 1% above h* (the level set of the cut-off, |o| T2D(h*)
// = alpha_min): the rounding of these few operations is far below that,
// and so is the band of h in which a rounded alpha can still pass the
// cut-off, except for an opacity within about 1e-4 of alpha_min, whose
// alpha is at the cut-off to rounding everywhere.  Without a finite
// positive h* (alpha_min = 0) the row extent decides, as it does for a
// zero-size ellipse.
template <int N>
__device__ __forceinline__ uint32_t strip_mask(const Rec& r, float mx, float my, int first) {
  uint32_t m = 0;
  const float ey = r.ey;
  if (!(r.hs > 0.0f && r.hs < __builtin_inff() && ey > 0.0f)) {
    const float e = ey * 1.0001f + 1e-3f;
#pragma unroll
    for (int k = 0; k < N; ++k) {
      const float y0 = (float)(4 * (first + k)) + 0.5f;
      if (my + e >= y0 && my - e <= y0 + 3.0f) m |= 1u << (first + k);
    }
    return m;
  }
  // the conic's entries from its factor (qa = l11^2, qb = l11 l21, qc =
  // l21^2 + l22^2: sums of products, no cancellation in qa and qc)
  const float qa = r.l11 * r.l11, qb = r.l11 * r.l21, qc = __fmaf_rn(r.l21, r.l21, r.l22 * r.l22);
  const float iyy = r.hs * __builtin_amdgcn_rcpf(ey * ey);
  const float ixx = iyy * qa * __builtin_amdgcn_rcpf(qc);
  const float kx = r.l21 * __builtin_amdgcn_rcpf(r.l11), ky = qb * __builtin_amdgcn_rcpf(qc);
  const float lvl = (r.hs * 1.0001f) * 1.01f;
  constexpr float x0 = 0.5f, x1 = (float)kTile - 0.5f;
  const bool in_x = mx >= x0 && mx <= x1;
#pragma unroll
  for (int k = 0; k < N; ++k) {
    const float y0 = (float)(4 * (first + k)) + 0.5f, y1 = y0 + 3.0f;
    bool keep = in_x && my >= y0 && my <= y1;
    // rows y0, y1, then columns x0, x1
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      const float dy = (e ? y1 : y0) - my;
      const float xs = __fmaf_rn(-kx, dy, mx);
      const float d = __builtin_amdgcn_fmed3f(xs, x0, x1) - xs;
      keep |= __fmaf_rn(qa * d, d, dy * dy * iyy) <= lvl;
    }
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      const float dx = (e ? x1 : x0) - mx;
      const float ys = __fmaf_rn(-ky, dx, my);
      const float d = __builtin_amdgcn_fmed3f(ys, y0, y1) - ys;
      keep |= __fmaf_rn(qc * d, d, dx * dx * ixx) <= lvl;
    }
    if (keep) m |= 1u << (first + k);
  }
  return m;
}

// The tile origin as FP64, converted where a batch is staged: the empty asm
// makes the integer look redefined there, so the conversion is not hoisted
// out of the walk and the origin stays in scalar registers (two FP64 values
// held in vector registers across the walk cost the backward a wave per
// SIMD).
__device__ __forceinline__ double origin_f64(int o) {
  asm volatile("" : "+s"(o));
  return (double)o;
}

// The record's mean relative to the tile origin (m, for the strip test) and
// L^T m, both from the FP64 mean and rounded once: a pixel p of the tile then
// has w = L^T (p - m) = L^T p - L^T m, two FMAs for w0 and one for w1.
__device__ __forceinline__ void tile_frame(const Rec& r, int ox, int oy, float* q0, float* q1, float* mx,
                                           float* my) {
  const double dx = r.mx - origin_f64(ox), dy = r.my - origin_f64(oy);
  *q0 = (float)__fma_rn((double)r.l21, dy, (double)r.l11 * dx);
  *q1 = (float)((double)r.l22 * dy);
  *mx = (float)dx;
  *my = (float)dy;
}

// Stages one forward-only record in LDS; returns its mask over the strips
// first .. first + N - 1 (the same fields and strip test as the general
// record below).
template <int N>
__device__ __forceinline__ uint32_t stage(const Rec* __restrict__ srec, uint32_t rank, int ox, int oy,
                                          int first, FRec* dst, uint32_t* entry) {
  const Rec r = srec[rank];
  FRec l;
  float mx, my;
  tile_frame(r, ox, oy, &l.q0, &l.q1, &mx, &my);
  l.l11 = r.l11; l.l21 = r.l21; l.l22 = r.l22;
  l.pad = 0.0f;
  l.o = r.o;
  l.inv_nu = r.inv_nu;
  l.nb = r.nb;
  l.cr = (double)r.cr; l.cg = (double)r.cg; l.cb = (double)r.cb;
  const uint32_t m = strip_mask<N>(r, mx, my, first);
  l.smask = m;
  *dst = l;
  *entry = r.entry;
  return m;
}

// Stages one record in LDS; returns its mask over the strips first ..
// first + N - 1, and the entry.
template <int N>
__device__ __forceinline__ uint32_t stage(const Rec* __restrict__ srec, uint32_t rank, int ox, int oy,
                                          int first, LRec* dst, uint32_t* entry) {
  const Rec r = srec[rank];
  LRec l;
  float mx, my;
  tile_frame(r, ox, oy, &l.q0, &l.q1, &mx, &my);
  l.l11 = r.l11; l.l21 = r.l21; l.l22 = r.l22;
  // Conservative pre-test level; the alpha test itself decides.
  l.pad = 0.0f;
  l.o = r.o;
  l.inv_nu = r.inv_nu;
  l.nb = r.nb;
  l.cr = r.cr; l.cg = r.cg; l.cb = r.cb;
  l.c2 = 2.0f * r.inv_nu * kLog2e;
  l.smask = 0u;
  l.entry = r.entry;
  l.slot = 0u;
  *entry = r.entry;
  // the record goes to LDS before the mask is computed, so that its
  // registers are free by then (the backward's accumulators are live here)
  *dst = l;
  const uint32_t m = strip_mask<N>(r, mx, my, first);
  dst->smask = m;
  return m;
}

// Evaluation of one record at one pixel, shared bit-for-bit by the forward
// and backward kernels (explicit fma, compiled without contraction).
struct Eval {
  float w0, w1, h, y, u, l2, t2, a, alpha;   // (w0, w1) = L^T (p - m); a = o T2D, alpha = a clamped
  bool hit, clamped;   // hit: |a| >= alpha_min (false for NaN)
};

// kGauss: the Gaussian family (every record has inv_nu = 0 and
// nb = -log2(e)/2); the kernels are instantiated per family, which the
// caller's options select for the whole call.
template <bool kGauss, typename R>
__device__ __forceinline__ void evaluate(float px, float py, const R& L, float amin, float amax, Eval& E) {
  // h = |w|^2 with w = L^T (p - m) (the conic's Cholesky factor L): a sum
  // of two squares, so near an elongated ellipse's major axis FP32 keeps h
  // to about (axis ratio) x 6e-8 relative, where the conic entries' form
  // lost (axis ratio)^2 x 6e-8.  The backward's sums are taken in w as well.
  // L^T m comes with the record, rounded once from FP64 (its error is that
  // of rounding m itself, times L's entries).
  E.w0 = __fmaf_rn(L.l11, px, __fmaf_rn(L.l21, py, -L.q0));
  E.w1 = __fmaf_rn(L.l22, py, -L.q1);
  E.h = __fmaf_rn(E.w0, E.w0, E.w1 * E.w1);
  // Branch-free: once a record passes the strip test nearly every wave has
  // a lane inside the ellipse, so the whole chain runs anyway; selects keep
  // the exec mask untouched.
  if constexpr (kGauss) {
    // T2D = exp(-h/2) = 2^(nb h)
    E.y = 0.0f;
    E.u = 1.0f;
    E.l2 = E.h;
  } else {
    // T2D = (1 + h/nu)^(-(nu+2)/2) = 2^(nb log2(1 + y)), y = h/nu.  log2(1 + y)
    // is corrected by the rounding error of u = 1 + y, which y - (u - 1) gives
    // exactly for every u (both subtractions are exact), taken with the slope
    // log2(e) of log2 at u = 1: where the slope 1/u differs the correction is
    // below 1e-7 relative, and with |nb| large there T2D is far below alpha_min.
    E.y = E.h * L.inv_nu;
    E.u = 1.0f + E.y;
    const float corr = E.y - (E.u - 1.0f);
    E.l2 = __fmaf_rn(corr, kLog2e, __builtin_amdgcn_logf(E.u));
  }
  E.t2 = __builtin_amdgcn_exp2f(L.nb * E.l2);
  const float a = L.o * E.t2;
  E.a = a;
  // the cut-off alone decides a hit: h* is the level set |o| T2D(h*) =
  // alpha_min, so a test of h against it could only differ from this one
  // within rounding of the level
  E.hit = fabsf(a) >= amin;
  E.clamped = fabsf(a) > amax;
  E.alpha = __builtin_amdgcn_fmed3f(a, -amax, amax);
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

template <int kCtrl>
__device__ __forceinline__ float dpp_mov(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), kCtrl, 0xf, 0xf, false));
}

// One halving step of the transposed reduction: the n values are split into
// a low half [0, h) and a high half [h, n) (zero-padded to h); a lane whose
// selector bit is 0 keeps the low half and sends the high one to its partner
// (which keeps the high half), and adds what the partner sends.
template <int kCtrl, int N>
__device__ __forceinline__ void halve(const float (&a)[N], float (&out)[(N + 1) / 2], bool bit) {
  constexpr int H = (N + 1) / 2;
#pragma unroll
  for (int i = 0; i < H; ++i) {
    const float hi = (H + i < N) ? a[H + i] : 0.0f;
    const float keep = bit ? hi : a[i];
    const float send = bit ? a[i] : hi;
    out[i] = keep + dpp_mov<kCtrl>(send);
  }
}

// Wave sums of ten per-lane values, transposed: afterwards lane l holds the
// wave sum of value tr_index(l) (lanes where tr_index is -1 hold 0).  Four
// halving steps inside each row of 16 lanes, with partners l^8 (row_ror:8),
// l^7 (row_half_mirror), l^3 and l^1 (quad permutations), whose xor masks
// span all 16 lanes, then two exchanges across rows.  About 30 instructions
// instead of ten 6-step reductions, and the ten sums end in ten lanes of one
// row, so one memory instruction can store or add them all.
//
// The first two steps pair lanes in different 4-lane banks (l^8: banks 0,1
// with 2,3; l^7: banks 0,2 with 1,3), so the DPP bank mask can pick which
// lanes an add writes: each pair costs two adds, one per half of the lanes,
// instead of two selects and an add.  The compiler's DPP builtins cannot
// express an add that leaves the other lanes' destination untouched, hence
// the asm.  Its wait states: 5 before the first DPP read (a VALU or EXEC
// write just before it), 2 between the steps and after the last write (a
// DPP read of a VGPR written by the VALU), since the compiler's hazard
// checks do not look inside it.  Same sums, same order as the halving
// steps (keep + received, a commutative add).
__device__ __forceinline__ float wave_sum10_transposed(const float (&v)[10]) {
  const int lane = threadIdx.x & 63;
  float a0, a1, a2, a3, a4, b[3], c[2], d[1];
  asm("s_nop 4\n\t"
      // l^8 (row_ror:8): lanes 0-7 of a row keep values 0-4, lanes 8-15 values 5-9
      "v_add_f32_dpp %0, %13, %13 row_ror:8 row_mask:0xf bank_mask:0xc\n\t"
      "v_add_f32_dpp %1, %14, %14 row_ror:8 row_mask:0xf bank_mask:0xc\n\t"
      "v_add_f32_dpp %2, %15, %15 row_ror:8 row_mask:0xf bank_mask:0xc\n\t"
      "v_add_f32_dpp %3, %16, %16 row_ror:8 row_mask:0xf bank_mask:0xc\n\t"
      "v_add_f32_dpp %4, %17, %17 row_ror:8 row_mask:0xf bank_mask:0xc\n\t"
      "v_add_f32_dpp %0, %8, %8 row_ror:8 row_mask:0xf bank_mask:0x3\n\t"
      "v_add_f32_dpp %1, %9, %9 row_ror:8 row_mask:0xf bank_mask:0x3\n\t"
      "v_add_f32_dpp %2, %10, %10 row_ror:8 row_mask:0xf bank_mask:0x3\n\t"
      "v_add_f32_dpp %3, %11, %11 row_ror:8 row_mask:0xf bank_mask:0x3\n\t"
      "v_add_f32_dpp %4, %12, %12 row_ror:8 row_mask:0xf bank_mask:0x3\n\t"
      "s_nop 1\n\t"
      // l^7 (row_half_mirror): banks 0,2 keep (a0, a1, a2), banks 1,3 (a3, a4);
      // b[2] of banks 1,3 (the zero padding) is left unwritten: the later
      // steps carry it only into lanes tr_index marks empty
      "v_add_f32_dpp %5, %3, %3 row_half_mirror row_mask:0xf bank_mask:0xa\n\t"
      "v_add_f32_dpp %6, %4, %4 row_half_mirror row_mask:0xf bank_mask:0xa\n\t"
      "v_add_f32_dpp %5, %0, %0 row_half_mirror row_mask:0xf bank_mask:0x5\n\t"
      "v_add_f32_dpp %6, %1, %1 row_half_mirror row_mask:0xf bank_mask:0x5\n\t"
      "v_add_f32_dpp %7, %2, %2 row_half_mirror row_mask:0xf bank_mask:0x5\n\t"
      "s_nop 1"
      : "=&v"(a0), "=&v"(a1), "=&v"(a2), "=&v"(a3), "=&v"(a4), "=&v"(b[0]), "=&v"(b[1]), "=&v"(b[2])
      : "v"(v[0]), "v"(v[1]), "v"(v[2]), "v"(v[3]), "v"(v[4]), "v"(v[5]), "v"(v[6]), "v"(v[7]), "v"(v[8]),
        "v"(v[9]));
  halve<0x1B, 3>(b, c, lane & 2);     // quad_perm [3,2,1,0]
  halve<0xB1, 2>(c, d, lane & 1);     // quad_perm [1,0,3,2]
  float x = d[0];
  x += __shfl_xor(x, 16, 64);
  x += __shfl_xor(x, 32, 64);
  return x;
}

// Which of the ten values lane l holds after wave_sum10_transposed (-1: none).
__device__ __forceinline__ int tr_index(int lane) {
  const int b3 = (lane >> 3) & 1, b2 = (lane >> 2) & 1, b1 = (lane >> 1) & 1, b0 = lane & 1;
  if ((b1 & b0) | (b2 & b1)) return -1;
  return 5 * b3 + 3 * b2 + 2 * b1 + b0;
}

// Scale of each screen-space gradient component as stored: the two mean
// sums carry the -2 of dh/d mean = -2 L w, and the off-diagonal sum of
// dh w w^T is stored doubled (it appears twice in the symmetric matrix).
__device__ __forceinline__ float g2_scale(int idx) { return idx < 2 ? -2.0f : (idx == 3 ? 2.0f : 1.0f); }

// Pixels of a unit owned by a thread: unit `sub` of a tile covers rows
// r0 = 4*PIX*sub .. r0 + 4*PIX - 1; thread t (of 64) owns column t % 16 and
// rows r0 + t/16 + 4k, k < PIX, so its k-th pixel lies in the tile's 16x4
// strip PIX*sub + k.
constexpr int kUnitThreads = 64;
template <int PIX>
constexpr int kUnits = 4 / PIX;   // units per tile

template <int PIX>
struct TileCtx {
  int g;       // global tile id
  int sub;     // unit within the tile
  bool skip;   // g is outside the grid (an order entry that is not a tile)
  int view, tx, ty;
  uint32_t start, end;
  int ox, oy;   // tile origin (pixels)
  float px;
  float py[PIX];
  bool inside[PIX];
  int64_t pix[PIX];
};

template <int PIX>
__device__ __forceinline__ TileCtx<PIX> tile_ctx(const CamBatch& cb, const uint32_t* __restrict__ tile_start,
                                                 const uint32_t* __restrict__ order, bool unit_order, uint32_t blk) {
  TileCtx<PIX> t;
  // The units with the most work are launched first, so that they do not
  // run alone at the end of the grid: with a unit order, launch slot blk
  // renders unit order[blk]; with a tile order, the units of tile
  // order[blk / units] follow each other.  blk is the workgroup number, or
  // in the persistent backward the number a wave took from the work queue.
  uint32_t gu, sub;
  if (unit_order) {
    const uint32_t u = order[blk];
    gu = u / kUnits<PIX>;
    sub = u % kUnits<PIX>;
  } else {
    const uint32_t b = blk / kUnits<PIX>;
    sub = blk % kUnits<PIX>;
    gu = order ? order[b] : b;
  }
  t.g = (int)gu;
  t.sub = (int)sub;
  t.skip = gu >= (uint32_t)cb.total_tiles;
  if (t.skip) return t;
  const int g = t.g;
  int v = 0;
  for (int k = 1; k < cb.n_views; ++k)
    if (g >= cb.v[k].tile_offset) v = k;
  const CamDev& c = cb.v[v];
  const int lt = g - c.tile_offset;
  const int tx = lt % c.tiles_x, ty = lt / c.tiles_x;
  t.view = v;
  t.tx = tx;
  t.ty = ty;
  const int lx = threadIdx.x & (kTile - 1), ly0 = (int)threadIdx.x / kTile + 4 * PIX * t.sub;
  const int x = tx * kTile + lx;
  t.px = (float)lx + 0.5f;
#pragma unroll
  for (int k = 0; k < PIX; ++k) {
    const int ly = ly0 + 4 * k;
    const int y = ty * kTile + ly;
    t.py[k] = (float)ly + 0.5f;
    t.inside[k] = x < c.W && y < c.H;
    t.pix[k] = c.pix_offset + (int64_t)y * c.W + x;
  }
  t.ox = tx * kTile;
  t.oy = ty * kTile;
  t.start = tile_start[g];
  t.end = tile_start[g + 1];
  return t;
}

// The 16x4 pixel strips a unit covers: its k-th pixel group is strip
// PIX*sub + k.  Returns the strip bits of all groups (wave-uniform) and each
// group's bit.
template <int PIX>
struct WaveStrips {
  uint32_t all;
  uint32_t bit[PIX];
};

template <int PIX>
__device__ __forceinline__ WaveStrips<PIX> wave_strips(int sub) {
  WaveStrips<PIX> ws;
  ws.all = 0;
#pragma unroll
  for (int k = 0; k < PIX; ++k) {
    ws.bit[k] = 1u << (PIX * sub + k);
    ws.all |= ws.bit[k];
  }
  return ws;
}

__device__ __forceinline__ uint32_t wave_max_u32(uint32_t v) {
#pragma unroll
  for (int d = 32; d > 0; d >>= 1) v = max(v, (uint32_t)__shfl_xor((int)v, d, 64));
  return v;
}

// A batch is one staged record per thread.  Returns the wave's set of
// staged records whose strip mask meets `strips` (bit j: record j), so the
// walk visits those records only.
template <int PIX, typename R>
__device__ __forceinline__ uint64_t stage_batch(const TileCtx<PIX>& t, const Rec* __restrict__ srec,
                                                const uint32_t* __restrict__ pair_rank, uint32_t base, uint32_t stop,
                                                R* lds, uint32_t strips) {
  const uint32_t k = base + threadIdx.x;
  uint32_t m = 0, e;
  if (k < stop) m = stage<PIX>(srec, pair_rank[k], t.ox, t.oy, PIX * t.sub, lds + threadIdx.x, &e);
  return __ballot((m & strips) != 0u);
}

// The same, also recording each pair's emission position: the rank's offset
// plus the number of the entry's listed tiles before this one (rows above,
// then columns to the left in this row), from the same row_run as the
// emission.
// Every visited pair's slot is written: a record that meets none of the
// strips gets zeros here, from the thread that staged it.
template <int PIX>
__device__ __forceinline__ uint64_t stage_batch_slot(const TileCtx<PIX>& t, const Rec* __restrict__ srec,
                                                     const uint32_t* __restrict__ pair_rank, const DetArgs& det,
                                                     uint32_t base, uint32_t stop, LRec* lds, uint32_t strips) {
  const uint32_t k = base + threadIdx.x;
  uint32_t m = 0;
  if (k < stop) {
    const uint32_t rank = pair_rank[k];
    uint32_t e;
    m = stage<PIX>(srec, rank, t.ox, t.oy, PIX * t.sub, lds + threadIdx.x, &e);
    const ushort4 rc = det.ent[e].rect;
    const RowGeo g = make_row_geo(srec[rank].mx, srec[rank].my, det.ent[e].ell);
    uint32_t pos = det.rank_off[rank];
    int t0;
    for (int ty = rc.y; ty < t.ty; ++ty) pos += (uint32_t)row_run(g, ty, rc.x, rc.z, &t0);
    row_run(g, t.ty, rc.x, rc.z, &t0);
    const uint32_t slot = pos + (uint32_t)(t.tx - t0);
    lds[threadIdx.x].slot = slot;
    if (!(m & strips) && slot < det.n_pairs) {
#pragma unroll
      for (int f = 0; f < 10; ++f) det.part[(size_t)slot * kG2 + f] = 0.0f;
    }
  }
  return __ballot((m & strips) != 0u);
}

// Forward traversal of the tile list; the same arithmetic in render_fwd and
// in the recompute phase of render_bwd.  kSelect picks how a record is
// composited: straight-line code with selects (the forward kernel: 3% faster)
// or branches on hit and termination (the recompute phase, where the selects
// measured 1-2% slower next to the backward body's registers).
template <int PIX, bool kGauss, bool kSelect, typename R>
__device__ __forceinline__ void forward_walk(const TileCtx<PIX>& t, const OptsDev& op, const Rec* __restrict__ srec,
                                             const uint32_t* __restrict__ pair_rank, R* lds, float (*C)[3],
                                             float* Tout, uint32_t* last_out) {
  // The colour sums are kept in FP64: the backward pass subtracts the colour
  // accumulated up to a component from the output, and for components deep
  // in a list (small T) an FP32 running sum's accumulated rounding would be
  // a large part of that difference.  FP64 FMA issues at the FP32 rate here.
  // A pixel is finished when its T is negative: T stays at or above t_min
  // (> 0) while it composites (1 - alpha lies in [1 - alpha_max, 1 +
  // alpha_max], alpha_max < 1), and termination negates it, so the final
  // transmittance is |T|.
  float T[PIX];
  double c0[PIX], c1[PIX], c2[PIX];
  uint32_t last[PIX];
  // kSelect: the last compositing record of the current batch as its LDS
  // byte offset (the address the record is read from), kNoRec if none;
  // turned into a list position once per batch
  constexpr uint32_t kNoRec = 0xFFFFFFFFu;
  uint32_t lastj[PIX];
#pragma unroll
  for (int k = 0; k < PIX; ++k) {
    T[k] = t.inside[k] ? 1.0f : -1.0f;
    c0[k] = 0.0; c1[k] = 0.0; c2[k] = 0.0;
    last[k] = 0;
  }
  constexpr uint32_t kBatch = kUnitThreads;
  const WaveStrips<PIX> ws = wave_strips<PIX>(t.sub);
  for (uint32_t base = t.start; base < t.end; base += kBatch) {
    bool alive = false;
#pragma unroll
    for (int k = 0; k < PIX; ++k) alive |= T[k] > 0.0f;
    if (__syncthreads_count(alive) == 0) break;
    // records that miss every strip of this unit are never visited
    uint64_t hits = stage_batch<PIX, R>(t, srec, pair_rank, base, t.end, lds, ws.all);
    __syncthreads();
    // Finished pixels are masked off; whether the whole wave is finished is
    // asked every 8 visited records only (a per-record test cost more than
    // the few records a finished wave may still walk), at the top of the
    // loop, so that T is not read between its update and the next record
    // (a test after the update cost a register copy of T per record).
    int since = 0;
#pragma unroll
    for (int k = 0; k < PIX; ++k) lastj[k] = kNoRec;
    while (hits) {
      if (++since == 9) {
        since = 1;
        bool left = false;
#pragma unroll
        for (int k = 0; k < PIX; ++k) left |= T[k] > 0.0f;
        if (!__any(left)) break;
      }
      const int j = (int)__builtin_ctzll(hits);
      hits &= hits - 1;
      const R L = lds[j];
      const uint32_t sm = PIX > 1 ? __builtin_amdgcn_readfirstlane(L.smask) : ws.all;
#pragma unroll
      for (int k = 0; k < PIX; ++k) {
        if constexpr (kSelect) {
          if (!(sm & ws.bit[k])) continue;  // wave-uniform
          // A lane that misses the ellipse or terminates here adds a zero
          // weight (x + 0 is x exactly) and keeps its T.  A finished lane
          // needs no test of its own: its T (1 - alpha) is negative, below
          // t_min, so it takes the termination branch and keeps -|T| = T.
          Eval E;
          evaluate<kGauss>(t.px, t.py[k], L, op.alpha_min, op.alpha_max, E);
          const float Tn = __fmaf_rn(-T[k], E.alpha, T[k]);   // T (1 - alpha), one rounding
          const bool term = Tn < op.t_min;
          const bool comp = __builtin_unpredictable(E.hit && !term);
          // the select on alpha, not on the product: one FP32 select
          const double wgt = (double)((comp ? E.alpha : 0.0f) * T[k]);
          c0[k] = __fma_rn((double)L.cr, wgt, c0[k]);
          c1[k] = __fma_rn((double)L.cg, wgt, c1[k]);
          c2[k] = __fma_rn((double)L.cb, wgt, c2[k]);
          T[k] = __builtin_unpredictable(E.hit) ? (term ? -fabsf(T[k]) : Tn) : T[k];
          lastj[k] = comp ? (uint32_t)j * (uint32_t)sizeof(R) : lastj[k];
        } else {
          if (!(T[k] > 0.0f) || !(sm & ws.bit[k])) continue;
          Eval E;
          evaluate<kGauss>(t.px, t.py[k], L, op.alpha_min, op.alpha_max, E);
          if (E.hit) {
            const float Tn = __fmaf_rn(-T[k], E.alpha, T[k]);
            if (Tn < op.t_min) {
              T[k] = -T[k];
            } else {
              const float wgt = E.alpha * T[k];
              c0[k] = __fma_rn((double)L.cr, (double)wgt, c0[k]);
              c1[k] = __fma_rn((double)L.cg, (double)wgt, c1[k]);
              c2[k] = __fma_rn((double)L.cb, (double)wgt, c2[k]);
              T[k] = Tn;
              last[k] = base - t.start + (uint32_t)j + 1u;
            }
          }
        }
      }
    }
    if constexpr (kSelect) {
#pragma unroll
      for (int k = 0; k < PIX; ++k)
        if (lastj[k] != kNoRec) last[k] = base - t.start + lastj[k] / (uint32_t)sizeof(R) + 1u;
    }
  }
#pragma unroll
  for (int k = 0; k < PIX; ++k) {
    const float Tf = fabsf(T[k]);
    C[k][0] = (float)__fma_rn((double)Tf, (double)op.bg[0], c0[k]);
    C[k][1] = (float)__fma_rn((double)Tf, (double)op.bg[1], c1[k]);
    C[k][2] = (float)__fma_rn((double)Tf, (double)op.bg[2], c2[k]);
    Tout[k] = Tf;
    last_out[k] = last[k];
  }
}

template <int PIX, bool kGauss>
__global__ __launch_bounds__(kUnitThreads) void render_fwd_kernel(CamBatch cb, OptsDev op,
                                                                  const Rec* __restrict__ srec,
                                                                  const uint32_t* __restrict__ tile_start,
                                                                  const uint32_t* __restrict__ pair_rank,
                                                                  float* __restrict__ image,
                                                                  float* __restrict__ t_final,
                                                                  uint32_t* __restrict__ n_contrib,
                                                                  const uint32_t* __restrict__ tile_order,
                                                                  uint32_t* __restrict__ tile_work) {
  __shared__ FRec lds[kUnitThreads];
  const TileCtx<PIX> t = tile_ctx<PIX>(cb, tile_start, tile_order, false, blockIdx.x);
  if (t.skip) return;
  float C[PIX][3], T[PIX];
  uint32_t last[PIX];
  forward_walk<PIX, kGauss, true>(t, op, srec, pair_rank, lds, C, T, last);
#pragma unroll
  for (int k = 0; k < PIX; ++k) {
    if (!t.inside[k]) continue;
    const int64_t p = t.pix[k];
    image[3 * p + 0] = C[k][0];
    image[3 * p + 1] = C[k][1];
    image[3 * p + 2] = C[k][2];
    if (t_final) t_final[p] = T[k];
    if (n_contrib) n_contrib[p] = last[k];
  }
  if (tile_work) {
    // per 16x4 strip, the longest prefix any of its pixels used (outside
    // pixels have last = 0)
#pragma unroll
    for (int k = 0; k < PIX; ++k) {
      const uint32_t w = wave_max_u32(last[k]);
      if (threadIdx.x == 0) tile_work[4 * (int64_t)t.g + PIX * t.sub + k] = w;
    }
  }
}

// One unit of the backward pass (launch slot blk).
template <int PIX, int kMode, int kLoss, bool kDet, bool kGauss>
__device__ __forceinline__ void render_bwd_unit(
    uint32_t blk, LRec* lds, const CamBatch& cb, const OptsDev& op, const Rec* __restrict__ srec,
    const uint32_t* __restrict__ tile_start, const uint32_t* __restrict__ pair_rank,
    const float* __restrict__ dl_or_target, const float* __restrict__ image, const uint32_t* __restrict__ n_contrib,
    float* __restrict__ image_out, float* __restrict__ loss_out, float inv_count, double* __restrict__ g2,
    const DetArgs& det) {
  static_assert(!kDet || PIX == 4, "the deterministic variant runs one unit per tile");
  constexpr uint32_t kBatch = kUnitThreads;
  const TileCtx<PIX> t = tile_ctx<PIX>(cb, tile_start, det.tile_order, det.unit_order != 0, blk);
  if (t.skip) return;
  const int lane = threadIdx.x & 63;

  // ---- per-pixel forward output and loss gradient ----
  float out[PIX][3];
  uint32_t bound[PIX];
  if (kMode == SSS_BWD_RECOMPUTE) {
    float T[PIX];
    forward_walk<PIX, kGauss, false>(t, op, srec, pair_rank, lds, out, T, bound);
#pragma unroll
    for (int k = 0; k < PIX; ++k) {
      if (!t.inside[k]) {
        bound[k] = 0;
        continue;
      }
      if (image_out) {
        image_out[3 * t.pix[k] + 0] = out[k][0];
        image_out[3 * t.pix[k] + 1] = out[k][1];
        image_out[3 * t.pix[k] + 2] = out[k][2];
      }
    }
  } else {
#pragma unroll
    for (int k = 0; k < PIX; ++k) {
      out[k][0] = out[k][1] = out[k][2] = 0.0f;
      bound[k] = 0;
      if (!t.inside[k]) continue;
      out[k][0] = image[3 * t.pix[k] + 0];
      out[k][1] = image[3 * t.pix[k] + 1];
      out[k][2] = image[3 * t.pix[k] + 2];
      bound[k] = n_contrib[t.pix[k]];
    }
  }
  float g[PIX][3];
  double gout[PIX];
  float l1 = 0.0f;
#pragma unroll
  for (int k = 0; k < PIX; ++k) {
    g[k][0] = g[k][1] = g[k][2] = 0.0f;
    if (t.inside[k]) {
      if (kLoss == SSS_LOSS_L1) {
        for (int ch = 0; ch < 3; ++ch) {
          const float d = out[k][ch] - dl_or_target[3 * t.pix[k] + ch];
          g[k][ch] = d > 0.0f ? inv_count : (d < 0.0f ? -inv_count : 0.0f);
          l1 += fabsf(d);
        }
      } else {
        g[k][0] = dl_or_target[3 * t.pix[k] + 0];
        g[k][1] = dl_or_target[3 * t.pix[k] + 1];
        g[k][2] = dl_or_target[3 * t.pix[k] + 2];
      }
    }
    gout[k] = __fma_rn((double)g[k][2], (double)out[k][2],
                       __fma_rn((double)g[k][1], (double)out[k][1], (double)g[k][0] * (double)out[k][0]));
  }
  if (kLoss == SSS_LOSS_L1 && loss_out) {
    // |out - target| summed over the unit; the units' values are added in a
    // fixed order afterwards
    l1 = wave_sum63(l1);
    if (lane == 63) det.loss_part[(int64_t)t.g * kUnits<PIX> + t.sub] = l1 * inv_count;
  }

  // per pixel group, the walk bound of its longest pixel (wave-uniform): a
  // group is skipped on a scalar branch once the walk passes it
  uint32_t gmax[PIX], mb = 0;
#pragma unroll
  for (int k = 0; k < PIX; ++k) {
    gmax[k] = __builtin_amdgcn_readfirstlane(wave_max_u32(bound[k]));
    mb = max(mb, gmax[k]);
  }
  const uint32_t stop = min(t.start + mb, t.end);
  // pairs of this tile up to rank lastp1 - 1 are visited (lists ascend in rank)
  if (kDet && threadIdx.x == 0) det.lastp1[t.g] = stop > t.start ? pair_rank[stop - 1] + 1u : 0u;

  // ---- front-to-back gradient walk ----
  const WaveStrips<PIX> ws = wave_strips<PIX>(t.sub);
  // gB: g . (the part of the output behind the current component), the
  // output minus the colour accumulated so far, kept in FP64 like the
  // forward's sums so that it keeps its precision deep in a list
  float T[PIX];
  double gB[PIX];
#pragma unroll
  for (int k = 0; k < PIX; ++k) {
    T[k] = 1.0f;
    gB[k] = gout[k];
  }
  for (uint32_t base = t.start; base < stop; base += kBatch) {
    __syncthreads();
    uint64_t hits = kDet ? stage_batch_slot<PIX>(t, srec, pair_rank, det, base, stop, lds, ws.all)
                         : stage_batch<PIX, LRec>(t, srec, pair_rank, base, stop, lds, ws.all);
    __syncthreads();
    while (hits) {
      const int j = (int)__builtin_ctzll(hits);
      hits &= hits - 1;
      const uint32_t pos = base - t.start + (uint32_t)j;
      const LRec L = lds[j];
      const uint32_t sm = PIX > 1 ? __builtin_amdgcn_readfirstlane(L.smask) : ws.all;
      // v: the record's ten gradient sums over this lane's pixels.  Pixel
      // group 0 assigns them (zeros when it does not run) and later groups
      // accumulate, a choice made at compile time: zeroing ten registers on
      // every record, or choosing at run time, cost more.
      float v[10];
      bool hit = false;
#pragma unroll
      for (int k = 0; k < PIX; ++k) {
        bool run = (sm & ws.bit[k]) && pos < gmax[k];
        // Predicated rather than branched (see evaluate): lanes past their
        // walk bound or outside the ellipse add zeros and keep T.
        Eval E;
        bool hk = false;
        if (run) {
          evaluate<kGauss>(t.px, t.py[k], L, op.alpha_min, op.alpha_max, E);
          hk = pos < bound[k] && E.hit;
          // ballot(hk) as the AND of the ballots of its two compares: the
          // lane masks combine on the scalar unit.  The second ballot takes
          // its own compare, the complement of |a| < alpha_min (the same
          // lanes as E.hit, NaN aside, where it only adds a lane that
          // contributes zeros): a ballot of E.hit itself, or of the combined
          // bool, went through two more vector instructions.
          run = (__builtin_amdgcn_ballot_w64(pos < bound[k]) &
                 __builtin_amdgcn_ballot_w64(!(fabsf(E.a) < op.alpha_min))) != 0;
        }
        if (!run) {
          if (k == 0) {
#pragma unroll
            for (int f = 0; f < 10; ++f) v[f] = 0.0f;
          }
          continue;
        }
        const float a = E.alpha;
        const float Tk = T[k];
        const float w = hk ? a * Tk : 0.0f;
        const float gc = __fmaf_rn(g[k][2], L.cb, __fmaf_rn(g[k][1], L.cg, g[k][0] * L.cr));
        gB[k] = __fma_rn(-(double)w, (double)gc, gB[k]);
        const float gR = (float)gB[k];
        // a clamped alpha passes no gradient to T2D
        const float da0 = __fmaf_rn(-gR, __builtin_amdgcn_rcpf(1.0f - a), Tk * gc);
        const float da = hk && !E.clamped ? da0 : 0.0f;
        T[k] = hk ? __fmaf_rn(-Tk, a, Tk) : Tk;   // as the forward walk
        const float ru = kGauss ? 1.0f : __builtin_amdgcn_rcpf(E.u);
        // d T2D / dh = T2D nb kh with d log2 T / dh = nb / (nu (1 + y)), or nb
        // ln 2 for the Gaussian family: kh = (1/nu or ln 2) ru.  The factors
        // that are the entry's own (o from dt2 = da o, nb, 1/nu or ln 2, and
        // ln(2)/2 of the nu term) are left out of the per-pixel terms and
        // applied once per entry where the sums are read (the projection
        // backward): dh here is dh / (o nb (1/nu or ln 2)).
        const float dt = da * E.t2;
        const float dh = kGauss ? dt : dt * ru;
        // the ten terms as products A[f] * B[f]: dh w (2), dh w w^T (3: 00,
        // 01, 11), d colour (3), d opacity, d nu / (o ln(2) / 2).  With Q =
        // L L^T and d = pixel - mean, dh/d mean = -2 Q d = -2 L w and the
        // gradient of the 2D covariance is -Q (sum dh d d^T) Q = -L (sum dh w
        // w^T) L^T: the projection backward applies L once per entry.  In w
        // the quadratic is isotropic, so its three sums stay of one size; in
        // pixel coordinates the thin axis's share of sum dh d d^T was
        // (axis ratio)^2 below the rest and lost to FP32.
        const float tq = dh * E.w0;
        float A[10] = {dh, dh, tq, tq, dh * E.w1, g[k][0], g[k][1], g[k][2], dt, dt};
        float B[10] = {E.w0, E.w1, E.w0, E.w1, E.w1, w, w, w, 1.0f, 0.0f};
        if constexpr (!kGauss) {
          // dT2D/dnu = T2D/2 [y/(1+y) - ln(1+y) + 2y/(nu (1+y))], here the
          // bracket / ln 2.  The first two terms cancel for small y: below
          // y = 0.1 they come from their series (coefficients times log2 e),
          // evaluated only when a lane of the wave needs it.  The Gaussian
          // family has no nu.
          const float y = E.y, yr = y * ru;
          float q = __fmaf_rn(yr, kLog2e, -E.l2);
          if (__builtin_amdgcn_ballot_w64(y < 0.1f)) {   // wave-uniform
            float s = __fmaf_rn(y, (float)(6.0 / 7.0 * 1.4426950408889634), (float)(-5.0 / 6.0 * 1.4426950408889634));
            s = __fmaf_rn(y, s, (float)(4.0 / 5.0 * 1.4426950408889634));
            s = __fmaf_rn(y, s, (float)(-3.0 / 4.0 * 1.4426950408889634));
            s = __fmaf_rn(y, s, (float)(2.0 / 3.0 * 1.4426950408889634));
            s = __fmaf_rn(y, s, (float)(-0.5 * 1.4426950408889634));
            q = y < 0.1f ? y * y * s : q;
          }
          B[9] = __fmaf_rn(yr, L.c2, q);
        }
        if (k == 0) {
#pragma unroll
          for (int f = 0; f < 10; ++f) v[f] = A[f] * B[f];
        } else {
#pragma unroll
          for (int f = 0; f < 10; ++f) v[f] = __fmaf_rn(A[f], B[f], v[f]);
        }
        hit = true;
      }
      // sums over the wave, transposed: lane tr_index(l) of the first row
      // holds component tr_index(l) of the entry's screen-space gradient
      const int idx = tr_index(lane);
      if (kDet) {
        // every visited pair's slot is written, zeros when no pixel was hit
        const float x = hit ? wave_sum10_transposed(v) : 0.0f;
        if (lane < 16 && idx >= 0 && L.slot < det.n_pairs) det.part[(size_t)L.slot * kG2 + idx] = g2_scale(idx) * x;
      } else if (hit) {   // wave-uniform
        const float x = wave_sum10_transposed(v);
        if (lane < 16 && idx >= 0) atomicAdd(g2 + (size_t)L.entry * kG2 + idx, (double)(g2_scale(idx) * x));
      }
    }
  }
}

// kQueue: a persistent grid (as many waves as are resident); each wave takes
// launch slots from the work counter det.queue, in launch order, until the
// counter passes det.n_units (every wave reaches that exit).  Otherwise one
// workgroup per unit.
template <int PIX, int kMode, int kLoss, bool kDet, bool kGauss, bool kQueue>
__global__ __launch_bounds__(kUnitThreads) void render_bwd_kernel(
    CamBatch cb, OptsDev op, const Rec* __restrict__ srec, const uint32_t* __restrict__ tile_start,
    const uint32_t* __restrict__ pair_rank, const float* __restrict__ dl_or_target, const float* __restrict__ image,
    const uint32_t* __restrict__ n_contrib, float* __restrict__ image_out, float* __restrict__ loss_out,
    float inv_count, double* __restrict__ g2, DetArgs det) {
  __shared__ LRec lds[kUnitThreads];
  if constexpr (kQueue) {
    for (;;) {
      uint32_t b = 0;
      if (threadIdx.x == 0) b = atomicAdd(det.queue, 1u);
      b = (uint32_t)__builtin_amdgcn_readfirstlane(__shfl((int)b, 0, 64));
      if (b >= det.n_units) break;
      render_bwd_unit<PIX, kMode, kLoss, kDet, kGauss>(b, lds, cb, op, srec, tile_start, pair_rank, dl_or_target,
                                                        image, n_contrib, image_out, loss_out, inv_count, g2, det);
      __syncthreads();   // the next unit restages the LDS batch
    }
  } else {
    render_bwd_unit<PIX, kMode, kLoss, kDet, kGauss>(blockIdx.x, lds, cb, op, srec, tile_start, pair_rank,
                                                      dl_or_target, image, n_contrib, image_out, loss_out, inv_count,
                                                      g2, det);
  }
}

// One step of a segmented inclusive scan over the wave: the value of the
// lane the DPP control selects is added where that lane has the same key
// (keys are non-decreasing over lanes and >= 1; lanes outside the row or
// masked rows read key 0).
template <int kCtrl, int kRowMask>
__device__ __forceinline__ void seg_step(int key, float (&v)[10]) {
  const int kk = __builtin_amdgcn_update_dpp(0, key, kCtrl, kRowMask, 0xf, true);
  const bool same = kk == key;
#pragma unroll
  for (int f = 0; f < 10; ++f) {
    const float t = __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v[f]), kCtrl, kRowMask, 0xf, true));
    v[f] += same ? t : 0.0f;
  }
}

// Deterministic sum of the pair slots.  A wave takes 64 consecutive visible
// ranks, whose slots are one contiguous range in emission order.  Each lane
// first evaluates its rank's rows into the wave's row table; the wave then
// streams through the slot range 64 slots at a time (coalesced loads), each
// lane finding its slot's rank and tile by binary search and zeroing slots
// whose tile walk stopped before the rank; a segmented scan by rank sums each
// rank's slots within the chunk and the segment's last lane adds the sum to
// the rank's accumulator in LDS, chunk after chunk.  Ranks whose rows do not
// fit the table are summed afterwards with for_each_listed_tile.  The result
// depends only on the data, never on scheduling.
__global__ __launch_bounds__(kBlock) void det_reduce_kernel(CamBatch cb, int64_t n, int64_t n_vis, uint32_t m,
                                                            const Rec* __restrict__ srec, DetArgs det,
                                                            double* __restrict__ g2) {
  struct WaveMeta {
    uint32_t off[65];
    int base[64], h[64], total[64], y0[64], toff[64], tiles_x[64], fits[64];
    double acc[64][10];
    int mark[64];
  };
  __shared__ RowTable s_rows[kBlock / 64];
  __shared__ WaveMeta s_meta[kBlock / 64];
  const int64_t r = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const int lane = threadIdx.x & 63;
  RowTable* table = &s_rows[threadIdx.x >> 6];
  WaveMeta& M = s_meta[threadIdx.x >> 6];
  const bool valid = r < n_vis;
  int my_e = 0, my_toff = 0, my_tx = 1;
  uint32_t my_off = m;
  ushort4 rc = make_ushort4(0, 0, 0, 0);
  double mx = 0.0, my = 0.0;
  Ellipse el{1.0, 0.0, 1.0, 0.0};
  if (valid) {
    const uint32_t e = det.order[r];
    my_e = (int)e;
    my_off = det.rank_off[r];
    rc = det.ent[e].rect;
    el = det.ent[e].ell;
    mx = srec[r].mx;
    my = srec[r].my;
    const int v = (int)(e / (uint64_t)n);
    for (int k = 0; k < cb.n_views; ++k)
      if (k == v) { my_toff = cb.v[k].tile_offset; my_tx = cb.v[k].tiles_x; }
  }
  const WaveRows wr = wave_row_table(valid, mx, my, el, rc.x, rc.y, rc.z, rc.w, table);
  const int64_t r0 = r - lane;
  M.off[lane] = my_off;
  if (lane == 63) M.off[64] = r0 + 64 < n_vis ? det.rank_off[r0 + 64] : m;
  M.base[lane] = wr.base;
  M.h[lane] = wr.h;
  M.total[lane] = wr.total;
  M.y0[lane] = rc.y;
  M.toff[lane] = my_toff;
  M.tiles_x[lane] = my_tx;
  M.fits[lane] = valid && wr.fits;
#pragma unroll
  for (int f = 0; f < 10; ++f) M.acc[lane][f] = 0.0;
  __syncthreads();
  if (r0 >= n_vis) return;   // uniform per wave; no barrier follows
  const uint32_t s0 = M.off[0], s1 = M.off[64];
  const int my_cnt = valid ? (int)(M.off[lane + 1] - my_off) : 0;
  int carry = 0;
  for (uint32_t c0 = s0; c0 < s1; c0 += 64) {
    const uint32_t s = c0 + (uint32_t)lane;
    const bool in = s < s1;
    // rank of the slot: a rank starting inside the window marks its start;
    // the inclusive max-scan of the marks (or the rank running into the
    // window) is the last rank with off <= s
    M.mark[lane] = 0;
    __builtin_amdgcn_wave_barrier();
    if (my_cnt > 0 && my_off >= c0 && my_off < c0 + 64u) M.mark[my_off - c0] = lane + 1;
    __builtin_amdgcn_wave_barrier();
    const int mk = wave_incl_max(M.mark[lane]);
    const int rho = mk > 0 ? mk - 1 : carry;
    carry = __builtin_amdgcn_readlane(rho, 63);
    float v[10];
#pragma unroll
    for (int f = 0; f < 10; ++f) v[f] = 0.0f;
    if (in && M.fits[rho]) {
      const int k = (int)(s - M.off[rho]);
      if (k < M.total[rho]) {
        const int b = M.base[rho];
        const int qlo = find_row(table, b, M.h[rho], k);
        const int x = (int)table->t0[b + qlo] + (k - (int)table->cum[b + qlo]);
        const int y = M.y0[rho] + qlo;
        if ((uint32_t)(r0 + rho) < det.lastp1[M.toff[rho] + y * M.tiles_x[rho] + x]) {
          const float4* p = reinterpret_cast<const float4*>(det.part + (size_t)s * kG2);
          const float4 u = p[0], w = p[1], z = p[2];
          v[0] = u.x; v[1] = u.y; v[2] = u.z; v[3] = u.w;
          v[4] = w.x; v[5] = w.y; v[6] = w.z; v[7] = w.w;
          v[8] = z.x; v[9] = z.y;
        }
      }
    }
    const int key = in ? rho + 1 : 65;
    seg_step<0x111, 0xf>(key, v);   // row_shr:1
    seg_step<0x112, 0xf>(key, v);   // row_shr:2
    seg_step<0x114, 0xf>(key, v);   // row_shr:4
    seg_step<0x118, 0xf>(key, v);   // row_shr:8
    seg_step<0x142, 0xa>(key, v);   // row_bcast:15
    seg_step<0x143, 0xc>(key, v);   // row_bcast:31
    const int next = __shfl_down(key, 1, 64);
    if (in && (lane == 63 || next != key)) {
#pragma unroll
      for (int f = 0; f < 10; ++f) M.acc[rho][f] += (double)v[f];
    }
  }
  // ranks whose rows did not fit the table
  for (int j = 0; j < 64; ++j) {
    if (r0 + j >= n_vis) break;   // uniform
    if (M.fits[j]) continue;
    const uint32_t rank = (uint32_t)(r0 + j);
    const uint32_t off = M.off[j];
    const int cnt = (int)(M.off[j + 1] - off);
    const int toff = M.toff[j], tiles_x = M.tiles_x[j];
    float a[10];
#pragma unroll
    for (int f = 0; f < 10; ++f) a[f] = 0.0f;
    const Ellipse ej{bcast_d(el.A, j), bcast_d(el.B, j), bcast_d(el.D, j), bcast_d(el.hr, j)};
    for_each_listed_tile(bcast_d(mx, j), bcast_d(my, j), ej, bcast_i(rc.x, j), bcast_i(rc.y, j), bcast_i(rc.z, j),
                         bcast_i(rc.w, j), [&](int k, int x, int y) {
                           if (k < cnt && rank < det.lastp1[toff + y * tiles_x + x]) {
                             const float4* p =
                                 reinterpret_cast<const float4*>(det.part + (size_t)(off + (uint32_t)k) * kG2);
                             const float4 u = p[0], w = p[1], z = p[2];
                             a[0] += u.x; a[1] += u.y; a[2] += u.z; a[3] += u.w;
                             a[4] += w.x; a[5] += w.y; a[6] += w.z; a[7] += w.w;
                             a[8] += z.x; a[9] += z.y;
                           }
                         });
#pragma unroll
    for (int f = 0; f < 10; ++f) a[f] = wave_sum63(a[f]);
    if (lane == 63) {
#pragma unroll
      for (int f = 0; f < 10; ++f) M.acc[j][f] = (double)a[f];
    }
  }
  if (valid) {
    double2* g = reinterpret_cast<double2*>(g2 + (size_t)my_e * kG2);
#pragma unroll
    for (int f = 0; f < 5; ++f) g[f] = make_double2(M.acc[lane][2 * f], M.acc[lane][2 * f + 1]);
    g[5] = make_double2(0.0, 0.0);
  }
}

// Fixed-order sum of the per-tile loss values (one workgroup): one add to
// loss_out instead of one atomic per tile on a single address, and the same
// value on every run.
// Sum of the per-unit loss values in a fixed order (each thread a fixed
// strided subset, then a fixed tree), added to *loss_out.
constexpr int kLossThreads = 1024;
__global__ __launch_bounds__(kLossThreads) void loss_reduce_kernel(const float* __restrict__ part, int64_t n,
                                                                 float* __restrict__ loss_out) {
  __shared__ float red[kLossThreads];
  float s = 0.0f;
  const int64_t n4 = n / 4;
  const float4* __restrict__ p4 = (const float4*)part;
  for (int64_t i = threadIdx.x; i < n4; i += kLossThreads) {
    const float4 v = p4[i];
    s += (v.x + v.y) + (v.z + v.w);
  }
  for (int64_t i = 4 * n4 + threadIdx.x; i < n; i += kLossThreads) s += part[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int h = kLossThreads / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) atomicAdd(loss_out, red[0]);
}

// Launch order of the tiles: a counting sort by a logarithmic bucket of the
// cost (12 buckets per doubling), most expensive bucket first.  One
// workgroup; the order inside a bucket follows the LDS atomics.
constexpr int kOrderThreads = 1024;
constexpr int kOrderBuckets = 256;
constexpr int kOrderBatch = 8;

__device__ __forceinline__ int order_bucket(uint32_t c) {
  const int b = (int)(12.0f * __log2f(1.0f + (float)c));
  return kOrderBuckets - 1 - min(b, kOrderBuckets - 1);
}

// Cost of item t: the largest of strip_cost[spi*t .. spi*t + spi) when
// strip_cost is given (kSpi > 0: spi = kSpi; kSpi < 0: spi at run time),
// else (kSpi = 0) the list length of tile t.  Straight-line loads, so the
// costs of a round of items are all in flight together.
template <int kSpi>
__device__ __forceinline__ uint32_t item_cost(const uint32_t* __restrict__ strip_cost, int spi,
                                              const uint32_t* __restrict__ tile_start, int64_t t) {
  if constexpr (kSpi == 0) {
    return tile_start[t + 1] - tile_start[t];
  } else if constexpr (kSpi > 0) {
    uint32_t c = 0;
#pragma unroll
    for (int j = 0; j < kSpi; ++j) c = max(c, strip_cost[kSpi * t + j]);
    return c;
  } else {
    uint32_t c = 0;
    for (int j = 0; j < spi; ++j) c = max(c, strip_cost[spi * t + j]);
    return c;
  }
}

template <int kSpi>
__global__ __launch_bounds__(kOrderThreads) void tile_order_kernel(const uint32_t* __restrict__ strip_cost, int spi,
                                                                   const uint32_t* __restrict__ tile_start,
                                                                   int64_t n_items, uint32_t* __restrict__ order) {
  __shared__ uint32_t hist[kOrderBuckets];
  for (int i = threadIdx.x; i < kOrderBuckets; i += kOrderThreads) hist[i] = 0;
  __syncthreads();
  // kOrderBatch items per thread and round, their costs loaded before any is
  // used (indices clamped into range, so the loads need no branch): a round
  // waits for one memory latency rather than one per item
  constexpr int64_t kStride = (int64_t)kOrderBatch * kOrderThreads;
  for (int64_t t0 = threadIdx.x; t0 < n_items; t0 += kStride) {
    uint32_t c[kOrderBatch];
#pragma unroll
    for (int j = 0; j < kOrderBatch; ++j)
      c[j] = item_cost<kSpi>(strip_cost, spi, tile_start, min(t0 + (int64_t)j * kOrderThreads, n_items - 1));
#pragma unroll
    for (int j = 0; j < kOrderBatch; ++j)
      if (t0 + (int64_t)j * kOrderThreads < n_items) atomicAdd(&hist[order_bucket(c[j])], 1u);
  }
  __syncthreads();
  if (threadIdx.x < 64) {
    // exclusive scan of the 256 counts by one wave, 4 per lane
    uint32_t c[4], s = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      c[k] = hist[4 * threadIdx.x + k];
      s += c[k];
    }
    const uint32_t incl = (uint32_t)wave_incl_scan((int)s);
    uint32_t run = incl - s;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      hist[4 * threadIdx.x + k] = run;
      run += c[k];
    }
  }
  __syncthreads();
  for (int64_t t0 = threadIdx.x; t0 < n_items; t0 += kStride) {
    uint32_t c[kOrderBatch];
#pragma unroll
    for (int j = 0; j < kOrderBatch; ++j)
      c[j] = item_cost<kSpi>(strip_cost, spi, tile_start, min(t0 + (int64_t)j * kOrderThreads, n_items - 1));
#pragma unroll
    for (int j = 0; j < kOrderBatch; ++j) {
      const int64_t t = t0 + (int64_t)j * kOrderThreads;
      if (t < n_items) order[atomicAdd(&hist[order_bucket(c[j])], 1u)] = (uint32_t)t;
    }
  }
}

__global__ __launch_bounds__(kBlock) void zero_kernel(float4* __restrict__ p, int64_t n4) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < n4) p[i] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
}

}  // namespace

void launch_tile_order(const uint32_t* strip_cost, int strips_per_item, const uint32_t* tile_start, int64_t n_items,
                       uint32_t* order, hipStream_t st) {
  if (n_items <= 0) return;
#define SSS_ORDER(K)                                                                                          \
  SSS_LAUNCH("tile_order", tile_order_kernel<K>, dim3(1), dim3(kOrderThreads), 0, st, strip_cost, strips_per_item, \
             tile_start, n_items, order)
  if (!strip_cost) SSS_ORDER(0);
  else if (strips_per_item == 1) SSS_ORDER(1);
  else if (strips_per_item == 2) SSS_ORDER(2);
  else if (strips_per_item == 4) SSS_ORDER(4);
  else SSS_ORDER(-1);
#undef SSS_ORDER
}

void launch_zero(float* p, int64_t count, hipStream_t st) {
  // count is a multiple of 4 for every caller (kG2 = 12 floats per entry)
  const int64_t n4 = count / 4;
  if (n4 <= 0) return;
  SSS_LAUNCH("zero", zero_kernel, dim3((unsigned)((n4 + kBlock - 1) / kBlock)), dim3(kBlock), 0, st,
                     (float4*)p, n4);
}

static size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

// Deterministic-mode workspace: screen-space gradients [E][kG2], per-pair
// sums [M][kG2], per-tile visit bounds [T], loss values [4T] and unit order
// [4T] (up to 4 units per tile), each 256-byte aligned.
static size_t det_parts(int64_t n_entries, int64_t n_pairs, int64_t n_tiles, size_t part[5]) {
  part[0] = sizeof(double) * kG2 * (size_t)n_entries;
  part[1] = sizeof(float) * kG2 * (size_t)(n_pairs > 0 ? n_pairs : 1);
  part[2] = sizeof(uint32_t) * (size_t)n_tiles;
  part[3] = sizeof(float) * 4 * (size_t)n_tiles;
  part[4] = sizeof(uint32_t) * 4 * (size_t)n_tiles;
  size_t total = 0;
  for (int k = 0; k < 5; ++k) total += align256(part[k]);
  return total;
}

size_t render_bwd_det_workspace(int64_t n_entries, int64_t n_pairs, int64_t n_tiles) {
  size_t part[5];
  return det_parts(n_entries, n_pairs, n_tiles, part);
}

// Workspace of the atomic mode: screen-space gradients [E][kG2] FP64, the
// per-unit loss values [4T] and the unit order [4T].
size_t render_bwd_workspace(int64_t n_entries, int64_t n_tiles) {
  // screen-space sums, per-unit loss, unit order, work counter (16 B)
  return align256(sizeof(double) * kG2 * (size_t)n_entries) + align256(sizeof(float) * 4 * (size_t)n_tiles) +
         align256(sizeof(uint32_t) * 4 * (size_t)n_tiles) + 16;
}

DetArgs carve_bwd(void* ws, int64_t n_entries, int64_t n_tiles, double** g2) {
  DetArgs d{};
  char* p = (char*)ws;
  *g2 = (double*)p;
  p += align256(sizeof(double) * kG2 * (size_t)n_entries);
  d.loss_part = (float*)p;
  p += align256(sizeof(float) * 4 * (size_t)n_tiles);
  d.order_ws = (uint32_t*)p;
  p += align256(sizeof(uint32_t) * 4 * (size_t)n_tiles);
  d.queue = (uint32_t*)p;
  return d;
}

DetArgs carve_det(void* ws, int64_t n_entries, int64_t n_pairs, int64_t n_tiles, double** g2) {
  size_t part[5];
  det_parts(n_entries, n_pairs, n_tiles, part);
  char* q[5];
  char* p = (char*)ws;
  for (int k = 0; k < 5; ++k) {
    q[k] = p;
    p += align256(part[k]);
  }
  DetArgs d{};
  *g2 = (double*)q[0];
  d.part = (float*)q[1];
  d.lastp1 = (uint32_t*)q[2];
  d.loss_part = (float*)q[3];
  d.order_ws = (uint32_t*)q[4];
  return d;
}

int env_pix(const char* name, int dflt) {
  const char* e = getenv(name);
  const int v = e ? atoi(e) : dflt;
  return (v == 1 || v == 2 || v == 4) ? v : dflt;
}

void launch_render_fwd(const CamBatch& cb, const OptsDev& op, const sss_bins_t& b, float* image, float* t_final,
                       uint32_t* n_contrib, hipStream_t st) {
  static const int pix = env_pix("SSS_PIX_FWD", 1);
  const dim3 grid((unsigned)(cb.total_tiles * (4 / pix)));
  const Rec* sr = (const Rec*)b.sorted_records;
  const bool gauss = op.family == SSS_FAMILY_GAUSSIAN;
#define SSS_FWD(P, G)                                                                                       \
  SSS_LAUNCH("render_fwd", (render_fwd_kernel<P, G>), grid, dim3(kUnitThreads), 0, st, cb, op, sr,         \
             (const uint32_t*)b.tile_start, (const uint32_t*)b.pair_rank, image, t_final, n_contrib,           \
             (const uint32_t*)b.tile_order, b.tile_work)
#define SSS_FWD_G(P)                \
  if (gauss) SSS_FWD(P, true);      \
  else SSS_FWD(P, false)
  if (pix == 1) { SSS_FWD_G(1); }
  else if (pix == 2) { SSS_FWD_G(2); }
  else { SSS_FWD_G(4); }
#undef SSS_FWD_G
#undef SSS_FWD
}

// The recompute-mode backward as one persistent launch over a work queue
// (see render_bwd_kernel) when SSS_BWD_PERSISTENT=1; off by default: on the
// 3M- and 5M-component workloads it measured 12-18% slower than one
// workgroup per unit in launch order.
static bool persistent_recompute() {
  static const int on = env_pix("SSS_BWD_PERSISTENT", 0);
  return on != 0;
}

// Waves of a persistent grid: what the occupancy lets every CU hold, and no
// more than there are units.
static unsigned resident_waves(const void* kernel, int64_t units) {
  int dev = 0, cus = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) !=
                                               hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, kUnitThreads, 0) != hipSuccess || per_cu < 1 ||
      cus < 1) {
    cus = 256;
    per_cu = 8;
  }
  const int64_t w = (int64_t)cus * per_cu;
  return (unsigned)(w < units ? w : (units > 0 ? units : 1));
}

void launch_render_bwd(const CamBatch& cb, const OptsDev& op, const sss_bins_t& b, int mode, int loss,
                       const float* dl_or_target, const float* image, const uint32_t* n_contrib, float* image_out,
                       float* loss_out, double* g2, int64_t total_pixels, bool det_mode, const DetArgs& dargs,
                       int64_t n, hipStream_t st) {
  // Pixels per lane: the deterministic variant runs one unit (one wave of 4
  // pixels per thread) per tile, so each pair's sums come from one wave;
  // otherwise 2 when the walk bounds are stored; when the unit first
  // recomputes the forward walk, 1 for calls of up to kRecomputePix2Tiles
  // tiles and 2 beyond (measured: one 1920x1080 view of 3M components,
  // 8160 tiles, 2.00 ms at 1 against 2.43 at 2; eight 1600x1064 views of
  // 5M, 53600 tiles, 11.7 ms at 1 against 10.1 at 2), unless SSS_PIX_BWD
  // says otherwise.
  constexpr int64_t kRecomputePix2Tiles = 16384;
  static const int env_bwd = env_pix("SSS_PIX_BWD", 0);
  const int pix = det_mode ? 4
                  : env_bwd ? env_bwd
                  : mode == SSS_BWD_RECOMPUTE ? (cb.total_tiles > kRecomputePix2Tiles ? 2 : 1)
                                               : 2;
  const int64_t units = cb.total_tiles * (4 / pix);
  // schedule: units ordered by the forward's per-strip walk lengths when
  // the backward walks the stored prefixes, else the binning's tile order
  DetArgs da = dargs;
  da.tile_order = b.tile_order;
  da.unit_order = 0;
  if (mode == SSS_BWD_STORED && b.tile_work && da.order_ws) {
    launch_tile_order(b.tile_work, pix, nullptr, units, da.order_ws, st);
    da.tile_order = da.order_ws;
    da.unit_order = 1;
  }
  const float inv_count = 1.0f / (3.0f * (float)total_pixels);
  const dim3 grid((unsigned)units);
  da.n_units = (uint32_t)units;
  const Rec* sr = (const Rec*)b.sorted_records;
  const uint32_t* ts = b.tile_start;
  const uint32_t* pr = b.pair_rank;
  const bool gauss = op.family == SSS_FAMILY_GAUSSIAN;
  if (det_mode) {
#define SSS_BWD_DET1(M, L, G)                                                                                       \
  SSS_LAUNCH("render_bwd", (render_bwd_kernel<4, M, L, true, G, false>), grid, dim3(kUnitThreads), 0, st, cb, op, sr, \
             ts, pr, dl_or_target, image, n_contrib, image_out, loss_out, inv_count, g2, da)
#define SSS_BWD_DET(M, L)            \
  if (gauss) SSS_BWD_DET1(M, L, true); \
  else SSS_BWD_DET1(M, L, false)
    if (mode == SSS_BWD_STORED && loss == SSS_LOSS_GRAD) { SSS_BWD_DET(SSS_BWD_STORED, SSS_LOSS_GRAD); }
    else if (mode == SSS_BWD_STORED) { SSS_BWD_DET(SSS_BWD_STORED, SSS_LOSS_L1); }
    else if (loss == SSS_LOSS_GRAD) { SSS_BWD_DET(SSS_BWD_RECOMPUTE, SSS_LOSS_GRAD); }
    else { SSS_BWD_DET(SSS_BWD_RECOMPUTE, SSS_LOSS_L1); }
#undef SSS_BWD_DET
#undef SSS_BWD_DET1
    // then the fixed-order sums
    if (b.n_visible > 0) {
      const unsigned gr = (unsigned)((b.n_visible + kBlock - 1) / kBlock);
      SSS_LAUNCH("det_reduce", det_reduce_kernel, dim3(gr), dim3(kBlock), 0, st, cb, n, b.n_visible,
                 (uint32_t)b.n_pairs, sr, da, g2);
    }
  } else {
#define SSS_BWD1(P, M, L, G)                                                                                  \
  do {                                                                                                        \
    if (M == SSS_BWD_RECOMPUTE && persistent_recompute()) {                                                  \
      auto kern = render_bwd_kernel<P, SSS_BWD_RECOMPUTE, L, false, G, true>;                                  \
      launch_zero((float*)da.queue, 4, st);                                                                   \
      SSS_LAUNCH("render_bwd", kern, dim3(resident_waves((const void*)kern, units)), dim3(kUnitThreads), 0, st,  \
                 cb, op, sr, ts, pr, dl_or_target, image, n_contrib, image_out, loss_out, inv_count, g2, da);    \
    } else {                                                                                                  \
      SSS_LAUNCH("render_bwd", (render_bwd_kernel<P, M, L, false, G, false>), grid, dim3(kUnitThreads), 0, st,  \
                 cb, op, sr, ts, pr, dl_or_target, image, n_contrib, image_out, loss_out, inv_count, g2, da);    \
    }                                                                                                         \
  } while (0)
#define SSS_BWD(P, M, L)                 \
  do {                                   \
    if (gauss) SSS_BWD1(P, M, L, true);  \
    else SSS_BWD1(P, M, L, false);       \
  } while (0)
#define SSS_BWD_P(M, L)                \
  if (pix == 1) SSS_BWD(1, M, L);      \
  else if (pix == 2) SSS_BWD(2, M, L); \
  else SSS_BWD(4, M, L)
    if (mode == SSS_BWD_STORED && loss == SSS_LOSS_GRAD) { SSS_BWD_P(SSS_BWD_STORED, SSS_LOSS_GRAD); }
    else if (mode == SSS_BWD_STORED) { SSS_BWD_P(SSS_BWD_STORED, SSS_LOSS_L1); }
    else if (loss == SSS_LOSS_GRAD) { SSS_BWD_P(SSS_BWD_RECOMPUTE, SSS_LOSS_GRAD); }
    else { SSS_BWD_P(SSS_BWD_RECOMPUTE, SSS_LOSS_L1); }
#undef SSS_BWD_P
#undef SSS_BWD
#undef SSS_BWD1
  }
  if (loss == SSS_LOSS_L1 && loss_out)
    SSS_LAUNCH("loss_reduce", loss_reduce_kernel, dim3(1), dim3(kLossThreads), 0, st, (const float*)da.loss_part, units,
               loss_out);
}

}  // namespace sss
