// Exact tile rows of a projected ellipse, shared by the projection (count),
// the pair emission (enumeration) and the deterministic backward pass (pair
// positions): the three must agree bit for bit, so they call these functions
// on the same FP64 values (the projection stores them per entry).
#pragma once

#include "common.hpp"

namespace sss {

// Per-entry constants of the row test, formed once per entry.
struct RowGeo {
  double mx, my, k, S, ds, ey, iD, hr;
  bool inf;
};

__device__ __forceinline__ RowGeo make_row_geo(double mx, double my, const Ellipse& e) {
  RowGeo g;
  g.mx = mx;
  g.my = my;
  g.hr = e.hr;
  g.inf = __builtin_isinf(e.hr);
  g.iD = 1.0 / e.D;
  g.k = e.B * g.iD;
  g.S = e.A - e.B * g.k;
  g.ds = e.B * sqrt(e.hr / e.A);
  g.ey = sqrt(e.hr * e.D);
  return g;
}

// Tiles of tile row ty (clipped to the rectangle's columns [x0, x1]) whose
// pixel-centre box meets the ellipse.  The ellipse is convex, so over the
// band of pixel-centre rows [16 ty + 1/2, 16 ty + 15.5] its x-extent is one
// interval: the chord at height dy runs over
// (B/D) dy +- sqrt((A - B^2/D)(hr - dy^2/D)), the right end peaking at the
// ellipse's rightmost point dy = B sqrt(hr/A) and the left end at the
// opposite point, each clamped into the band.  A tile is kept when the
// interval reaches its pixel-centre columns [16 tx + 1/2, 16 tx + 15.5].
// Returns the number of tiles and their first column in *t0.
__device__ __forceinline__ int row_run(const RowGeo& g, int ty, int x0, int x1, int* t0) {
  *t0 = x0;
  if (g.inf) return x1 - x0 + 1;
  const double y0 = 16.0 * ty + 0.5 - g.my, y1 = 16.0 * ty + 15.5 - g.my;
  const double lo = fmax(y0, -g.ey), hi = fmin(y1, g.ey);
  if (lo > hi) return 0;
  const double dr = fmin(fmax(g.ds, lo), hi), dl = fmin(fmax(-g.ds, lo), hi);
  const double wr = g.S * (g.hr - dr * dr * g.iD), wl = g.S * (g.hr - dl * dl * g.iD);
  const double xr = g.mx + (g.k * dr + (wr > 0.0 ? sqrt(wr) : 0.0));
  const double xl = g.mx + (g.k * dl - (wl > 0.0 ? sqrt(wl) : 0.0));
  const int a = (int)fmin(fmax(ceil((xl - 15.5) * 0.0625), (double)x0), (double)x1 + 1.0);
  const int b = (int)fmax(fmin(floor((xr - 0.5) * 0.0625), (double)x1), (double)x0 - 1.0);
  *t0 = a;
  return b >= a ? b - a + 1 : 0;
}

// Lane j's value of v, as a wave-uniform value.
__device__ __forceinline__ int bcast_i(int v, int j) { return __builtin_amdgcn_readlane(v, j); }


// Inclusive prefix sum over the 64 lanes of a wave (all lanes active): DPP
// row shifts by 1, 2, 4, 8 (a lane outside the row reads 0), then row 0's
// last lane into row 1 and row 2's into row 3, then lane 31 into rows 2 and
// 3.  Six VALU adds where shuffles took six LDS round trips.
template <int kCtrl, int kRowMask>
__device__ __forceinline__ int dpp_add_i(int v) {
  return v + __builtin_amdgcn_update_dpp(0, v, kCtrl, kRowMask, 0xf, true);
}

__device__ __forceinline__ int wave_incl_scan(int v) {
  v = dpp_add_i<0x111, 0xf>(v);  // row_shr:1
  v = dpp_add_i<0x112, 0xf>(v);  // row_shr:2
  v = dpp_add_i<0x114, 0xf>(v);  // row_shr:4
  v = dpp_add_i<0x118, 0xf>(v);  // row_shr:8
  v = dpp_add_i<0x142, 0xa>(v);  // row_bcast:15
  v = dpp_add_i<0x143, 0xc>(v);  // row_bcast:31
  return v;
}

// Row runs of the 64 entries of a wave, one entry per lane, in a per-wave
// LDS table: entry j's rows occupy slots [base_j, base_j + h_j) holding the
// row's first column (t0) and the number of the entry's tiles in the rows
// above it (cum).  The FP64 row tests run once per row, spread over the
// lanes.  Entries whose rows would overflow the table are marked
// (fits = false) and walked by the caller with for_each_listed_tile.
constexpr int kRowSlots = 640;

struct RowTable {
  uint32_t t0[kRowSlots];
  uint32_t cum[kRowSlots];
};

struct WaveRows {
  int base, h, total;
  bool fits;
};

__device__ __forceinline__ WaveRows wave_row_table(bool valid, double mx, double my, const Ellipse& el, int x0, int y0,
                                                   int x1, int y1, RowTable* table) {
  WaveRows w;
  w.h = valid ? y1 - y0 + 1 : 0;
  const int incl = wave_incl_scan(w.h);
  w.base = incl - w.h;
  w.fits = incl <= kRowSlots;
  w.total = 0;
  if (valid && w.fits) {
    const RowGeo g = make_row_geo(mx, my, el);
    for (int q = 0; q < w.h; ++q) {
      int t0;
      const int len = row_run(g, y0 + q, x0, x1, &t0);
      table->t0[w.base + q] = (uint32_t)t0;
      table->cum[w.base + q] = (uint32_t)w.total;
      w.total += len;
    }
  }
  return w;
}

// Inclusive max-scan over the wave of non-negative values (DPP row shifts,
// then row broadcasts; lanes outside a row or in masked rows read 0).
template <int kCtrl, int kRowMask>
__device__ __forceinline__ int dpp_max(int v) {
  return max(v, __builtin_amdgcn_update_dpp(0, v, kCtrl, kRowMask, 0xf, true));
}

__device__ __forceinline__ int wave_incl_max(int v) {
  v = dpp_max<0x111, 0xf>(v);  // row_shr:1
  v = dpp_max<0x112, 0xf>(v);  // row_shr:2
  v = dpp_max<0x114, 0xf>(v);  // row_shr:4
  v = dpp_max<0x118, 0xf>(v);  // row_shr:8
  v = dpp_max<0x142, 0xa>(v);  // row_bcast:15
  v = dpp_max<0x143, 0xc>(v);  // row_bcast:31
  return v;
}

// Row of the k-th listed tile of an entry whose h rows start at table
// slot `base`: cum is the exclusive prefix of the row lengths, so the row is
// the last one with cum <= k (binary search; entries span a few rows, and a
// counted scan of 16 predicated reads measured slower).
__device__ __forceinline__ int find_row(const RowTable* table, int base, int h, int k) {
  int lo = 0, hi = h - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if ((int)table->cum[base + mid] <= k) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// Wave-cooperative walk over the `total` listed tiles of one entry of the
// table, in emission order: the lanes take positions k = lane, lane + 64,
// ... and find their row as the last one whose cum is <= k (binary search),
// then call f(k, tile_x, tile_y).
template <typename F>
__device__ __forceinline__ void for_each_tile_in_table(const RowTable* table, int base, int h, int total, int y0,
                                                       F&& f) {
  const int lane = threadIdx.x & 63;
  for (int k = lane; k < total; k += 64) {
    const int lo = find_row(table, base, h, k);
    f(k, (int)table->t0[base + lo] + (k - (int)table->cum[base + lo]), y0 + lo);
  }
}

// The same walk for an entry that did not fit the table (wave-uniform
// arguments): rows are evaluated 64 at a time, one per lane.
template <typename F>
__device__ __forceinline__ int for_each_listed_tile(double mx, double my, const Ellipse& el, int x0, int y0, int x1,
                                                    int y1, F&& f) {
  const int lane = threadIdx.x & 63;
  const int h = y1 - y0 + 1;
  const RowGeo g = make_row_geo(mx, my, el);
  int base = 0;
  for (int q0 = 0; q0 < h; q0 += 64) {
    int t0 = x0, len = 0;
    if (q0 + lane < h) len = row_run(g, y0 + q0 + lane, x0, x1, &t0);
    const int incl = wave_incl_scan(len);
    const int rows = min(64, h - q0);
    for (int qq = 0; qq < rows; ++qq) {
      const int L = bcast_i(len, qq);
      if (L == 0) continue;
      const int T0 = bcast_i(t0, qq);
      const int B = base + bcast_i(incl, qq) - L;
      for (int c = lane; c < L; c += 64) f(B + c, T0 + c, y0 + q0 + qq);
    }
    base += bcast_i(incl, 63);
  }
  return base;
}

__device__ __forceinline__ double bcast_d(double v, int j) {
  return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), j),
                          __builtin_amdgcn_readlane(__double2loint(v), j));
}

}  // namespace sss
