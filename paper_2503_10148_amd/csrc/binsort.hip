// Tile binning and depth ordering.
//
//  1. every entry gets its depth key (culled ones 2^32 - 1) and per-block
//     counts of visible entries, pairs and the visible key range are reduced
//     into a device record (SortDyn) that every later kernel reads its sizes
//     from, so nothing after this waits for the host; on request the counts
//     are also read back (the call then waits once) or copied to the
//     caller's device buffer;
//  2. a stable LSD radix sort by the depth key, relative to the smallest
//     visible key and over only the bits that vary, gives each visible entry
//     its rank (ties keep entry order, i.e. component index); culled entries
//     sort last;
//  3. every (tile, rank) pair of a visible entry's listed tiles is written in
//     rank order (exclusive scan of tiles_touched over ranks; each wave
//     streams its ranks' contiguous slot range), the projected records are
//     gathered into rank order alongside;
//  4. a stable radix sort of the pairs by global tile id leaves each tile's
//     ranks ascending, i.e. in (depth key, component index) order;
//  5. tile_start[] marks where each tile's run begins;
//  6. if the caller asks for it, the tiles' launch order for the raster
//     kernels, longest list first.
//
// All passes stream through HBM with coalesced accesses where the data
// allows; the radix scatter ranks keys inside a wave with ballots (64-wide
// match) so the sort is stable without per-thread digit counters.
#include "common.hpp"
#include "tiles.hpp"
#include "scan.hpp"

namespace sss {
namespace {


// ---------------------------------------------------------------------------
// 1. sort input and counts
// ---------------------------------------------------------------------------
// Every entry goes into the depth sort; a culled one gets the key 2^32 - 1,
// which the depth passes map above every visible key, so the n_visible
// visible entries come first in depth order.  Each block writes its count of
// visible entries, its pair total and the range of its visible keys to its
// own slot (no atomics), and one workgroup reduces the slots.
struct BlockStat {
  unsigned long long pairs;
  uint32_t visible, kmin, kmax, pad;
};

constexpr int kPrepItems = 4;

__global__ __launch_bounds__(kBlock) void prepare_kernel(const uint32_t* __restrict__ touched,
                                                         const uint32_t* __restrict__ keys, int64_t n,
                                                         uint32_t* __restrict__ out_keys,
                                                         uint32_t* __restrict__ out_vals,
                                                         BlockStat* __restrict__ stats) {
  __shared__ BlockStat red[kBlock / 64];
  // kPrepItems entries per thread, kBlock apart, loaded before use; one
  // statistics record per block of kPrepItems * kBlock entries
  const int64_t j0 = (int64_t)blockIdx.x * (kBlock * kPrepItems) + threadIdx.x;
  uint32_t t[kPrepItems], k[kPrepItems];
#pragma unroll
  for (int q = 0; q < kPrepItems; ++q) {
    const int64_t j = j0 + (int64_t)q * kBlock;
    t[q] = j < n ? touched[j] : 0u;
    k[q] = j < n ? keys[j] : 0u;
  }
  unsigned long long pairs = 0;
  uint32_t vis = 0, lo = 0xFFFFFFFFu, hi = 0u;
#pragma unroll
  for (int q = 0; q < kPrepItems; ++q) {
    const int64_t j = j0 + (int64_t)q * kBlock;
    if (j < n) {
      out_keys[j] = t[q] > 0 ? k[q] : 0xFFFFFFFFu;
      out_vals[j] = (uint32_t)j;
    }
    pairs += t[q];
    if (t[q] > 0) {
      vis += 1u;
      lo = min(lo, k[q]);
      hi = max(hi, k[q]);
    }
  }
  for (int d = 32; d > 0; d >>= 1) {
    pairs += __shfl_xor(pairs, d, 64);
    vis += __shfl_xor(vis, d, 64);
    lo = min(lo, (uint32_t)__shfl_xor((int)lo, d, 64));
    hi = max(hi, (uint32_t)__shfl_xor((int)hi, d, 64));
  }
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = BlockStat{pairs, vis, lo, hi, 0u};
  __syncthreads();
  if (threadIdx.x == 0) {
    BlockStat b = red[0];
    for (int w = 1; w < kBlock / 64; ++w) {
      b.pairs += red[w].pairs;
      b.visible += red[w].visible;
      b.kmin = min(b.kmin, red[w].kmin);
      b.kmax = max(b.kmax, red[w].kmax);
    }
    stats[blockIdx.x] = b;
  }
}

// Sizes of one bin sort on the device, written by stat_reduce_kernel and
// read by every later kernel of the call (the host sizes the grids from
// upper bounds: all entries, the pair capacity).
struct SortDyn {
  uint32_t n_vis;        // visible entries
  uint32_t depth_base;   // smallest visible depth key
  uint32_t depth_cap;    // relative key of culled entries (range + 1)
  uint32_t depth_bits;   // bits the depth passes sort (>= 1)
  uint32_t m;            // pairs emitted and sorted: min(required, capacity)
  uint32_t nb[2];        // radix blocks of the depth sort and of the pair sort
  uint32_t scan_n[2][4]; // histogram entries each pass scans (0: the pass is idle)
  uint32_t pad;
};

// The radix passes' digit layout, fixed on the host: items per block, and
// per pass the number of digits (histogram rows).
struct SortLayout {
  int64_t n_entries;
  int per_block[2];
  int rows[2][4];
  int passes[2];
};

// smallest b >= 1 with 2^b >= v (v <= 2^32)
__device__ __forceinline__ uint32_t bits_for_dev(unsigned long long v) {
  return v <= 2ull ? 1u : (uint32_t)(64 - __clzll((long long)(v - 1ull)));
}

// counters: visible entries, pairs (required), smallest and largest visible
// key; dyn: the sizes the later kernels use; counts_out (nullable, device):
// the caller's copy of (visible, required pairs).
__global__ __launch_bounds__(kBlock) void stat_reduce_kernel(const BlockStat* __restrict__ stats, int64_t nb,
                                                             SortLayout lay, unsigned long long pair_capacity,
                                                             unsigned long long* __restrict__ counters,
                                                             SortDyn* __restrict__ dyn,
                                                             unsigned long long* __restrict__ counts_out,
                                                             ScanSync* __restrict__ sync) {
  __shared__ BlockStat red[kBlock];
  scan_sync_clear(sync);   // for the sort's single-pass scans
  BlockStat b{0ull, 0u, 0xFFFFFFFFu, 0u, 0u};
  // rounds of 8 statistics per thread, loaded before any is combined, so a
  // round waits for one memory latency (every later kernel waits on this one)
  constexpr int kRound = 8;
  for (int64_t i0 = threadIdx.x; i0 < nb; i0 += (int64_t)kRound * kBlock) {
    BlockStat s[kRound];
#pragma unroll
    for (int j = 0; j < kRound; ++j) {
      const int64_t i = i0 + (int64_t)j * kBlock;
      s[j] = i < nb ? stats[i] : BlockStat{0ull, 0u, 0xFFFFFFFFu, 0u, 0u};
    }
#pragma unroll
    for (int j = 0; j < kRound; ++j) {
      b.pairs += s[j].pairs;
      b.visible += s[j].visible;
      b.kmin = min(b.kmin, s[j].kmin);
      b.kmax = max(b.kmax, s[j].kmax);
    }
  }
  red[threadIdx.x] = b;
  __syncthreads();
  for (int h = kBlock / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) {
      BlockStat& a = red[threadIdx.x];
      const BlockStat& c = red[threadIdx.x + h];
      a.pairs += c.pairs;
      a.visible += c.visible;
      a.kmin = min(a.kmin, c.kmin);
      a.kmax = max(a.kmax, c.kmax);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const BlockStat& t = red[0];
    counters[0] = t.visible;
    counters[1] = t.pairs;
    counters[2] = t.kmin;
    counters[3] = t.kmax;
    // depth keys relative to the smallest visible key; culled entries at
    // range + 1, after every visible one; only the bits that vary are sorted
    SortDyn d{};
    d.n_vis = t.visible;
    if (t.visible > 0) {
      const uint32_t range = t.kmax - t.kmin;
      d.depth_base = t.kmin;
      d.depth_cap = range == 0xFFFFFFFFu ? range : range + 1u;
    } else {
      d.depth_base = 0u;
      d.depth_cap = 0u;
    }
    d.depth_bits = bits_for_dev((unsigned long long)d.depth_cap + 1ull);
    d.m = (uint32_t)min(t.pairs, pair_capacity);
    // radix blocks and the histogram length of each pass: a depth pass runs
    // only while its digit lies inside the bits that vary (pass 0 always)
    d.nb[0] = (uint32_t)((lay.n_entries + lay.per_block[0] - 1) / lay.per_block[0]);
    d.nb[1] = (uint32_t)(((int64_t)d.m + lay.per_block[1] - 1) / lay.per_block[1]);
    for (int p = 0; p < 4; ++p) {
      const bool on = p < lay.passes[0] && (p == 0 || 8 * p < (int)d.depth_bits);
      d.scan_n[0][p] = on ? (uint32_t)lay.rows[0][p] * d.nb[0] : 0u;
      d.scan_n[1][p] = p < lay.passes[1] ? (uint32_t)lay.rows[1][p] * d.nb[1] : 0u;
    }
    *dyn = d;
    if (counts_out) {
      counts_out[0] = t.visible;
      counts_out[1] = t.pairs;
    }
  }
}

// ---------------------------------------------------------------------------
// 2./4. stable LSD radix sort, digits of up to 8 bits
// ---------------------------------------------------------------------------
// Items per thread of a radix pass: 16 for 8-bit digits, 8 (blocks of 2048,
// half the LDS, so twice the workgroups per CU) for digits of up to 7 bits,
// where a block's runs per digit stay as long (A/B on the 1M workload: the
// pair scatter 0.217 -> 0.197 ms; 8-bit passes measured slower with 8).
constexpr int kRItemsWide = 16;
constexpr int kRItemsNarrow = 8;
constexpr int radix_items(int width) { return width <= 7 ? kRItemsNarrow : kRItemsWide; }
// Keys enter the passes as min(key - base, cap) (unsigned): the depth sort
// subtracts the smallest visible key and maps culled entries to cap, so only
// the bits that vary are sorted; the pair sort uses base 0, cap 2^32 - 1.
__device__ __forceinline__ uint32_t radix_digit(uint32_t key, uint32_t base, uint32_t cap, int shift, uint32_t mask) {
  return (min(key - base, cap) >> shift) & mask;
}

// A pass's sizes.  The host gives upper bounds (n_max items, a grid of at
// most kRadixGrid workgroups) and the digit layout; the device record gives
// the rest.  The depth sort (kDepthSort) sorts all n_max entries by keys
// relative to dyn->depth_base: the host launches four 8-bit passes and a
// pass whose digit lies beyond dyn->depth_bits does nothing; the last pass
// that runs writes the values to their final buffer.  The pair sort
// (kPairSort) sorts the first dyn->m items over the host's bit count, and
// every pass runs.  Each pass covers dyn->nb[kind] radix blocks.
enum { kDepthSort = 0, kPairSort = 1 };
struct PassArgs {
  const SortDyn* dyn;
  int64_t n_max;
  int kind;
  int pass;
  int shift;   // first bit of this pass's digit
  int width;   // digit width of every pass (the last may use fewer bits)
  int nbits;   // bits of the whole sort (kPairSort)
};
struct PassDev {
  int64_t n, nb;
  uint32_t base, cap;
  bool active, last;
};
__device__ __forceinline__ PassDev pass_dev(const PassArgs& a) {
  PassDev p;
  int nbits;
  if (a.kind == kDepthSort) {
    p.n = a.n_max;
    p.base = a.dyn->depth_base;
    p.cap = a.dyn->depth_cap;
    nbits = (int)a.dyn->depth_bits;
  } else {
    p.n = min(a.n_max, (int64_t)a.dyn->m);
    p.base = 0u;
    p.cap = 0xFFFFFFFFu;
    nbits = a.nbits;
  }
  p.nb = a.dyn->nb[a.kind];
  p.active = a.shift == 0 || a.shift < nbits;
  p.last = a.shift + a.width >= nbits;
  return p;
}

// Workgroups are dispatched to the chip's 8 XCDs in turn, each XCD with an
// L2 of its own.  Radix block numbers that give every XCD one contiguous
// range put neighbouring blocks on the same L2, so the cache lines they
// share (adjacent words of a histogram row; the ends of digit runs that
// meet in the scatter's output) are completed there before write-back.
// The grid is a multiple of 8 workgroups and may be smaller than the block
// count, which the device decides: workgroup g of XCD x walks x's range
// [x * per, (x + 1) * per) from its own position in steps of grid / 8.
// One workgroup per radix block measured fastest (multiview pair scatter
// 6.1 ms, against 7.7-8.5 ms with 8192-2048 workgroups looping over the
// blocks); the loop only matters for grids beyond this bound.
constexpr int64_t kRadixGrid = int64_t(1) << 20;
struct XcdRange {
  int64_t first, end, step;
};
__device__ __forceinline__ XcdRange xcd_range(int64_t nblocks) {
  const int64_t per = (nblocks + 7) / 8;
  const int64_t x = blockIdx.x % 8;
  XcdRange r;
  r.first = x * per + blockIdx.x / 8;
  r.end = min((x + 1) * per, nblocks);
  r.step = gridDim.x / 8;
  return r;
}

template <int kRItems>
__global__ __launch_bounds__(kBlock) void radix_hist_kernel(const uint32_t* __restrict__ keys, PassArgs pa,
                                                            uint32_t mask, uint32_t* __restrict__ hist) {
  const PassDev pd = pass_dev(pa);
  if (!pd.active) return;       // uniform over the grid
  const int64_t n = pd.n, nblocks = pd.nb;
  __shared__ uint32_t h[256];
  constexpr int kRPerBlock = kBlock * kRItems;
  const XcdRange xr = xcd_range(nblocks);
  for (int64_t blk = xr.first; blk < xr.end; blk += xr.step) {
    __syncthreads();            // the previous block's rows are written
    h[threadIdx.x] = 0;
    __syncthreads();
    const int64_t base = blk * kRPerBlock;
    // all loads first, so their latencies overlap (LDS atomics in between
    // would keep the compiler from hoisting them)
    uint32_t kk[kRItems];
#pragma unroll
    for (int k = 0; k < kRItems; ++k) {
      const int64_t j = base + (int64_t)k * kBlock + threadIdx.x;
      kk[k] = j < n ? keys[j] : 0u;
    }
#pragma unroll
    for (int k = 0; k < kRItems; ++k) {
      const int64_t j = base + (int64_t)k * kBlock + threadIdx.x;
      if (j < n) atomicAdd(&h[radix_digit(kk[k], pd.base, pd.cap, pa.shift, mask)], 1u);
    }
    __syncthreads();
    // digit-major rows; only the mask + 1 digits of this pass (the scan
    // covers just those rows)
    if (threadIdx.x <= mask) hist[(int64_t)threadIdx.x * nblocks + blk] = h[threadIdx.x];
  }
}

// Block b owns items [b*B, (b+1)*B), B = 256 * kRItems; wave w owns the w-th
// quarter and walks it in kRItems rounds of 64 consecutive items, so (wave,
// round, lane) is item order and ranks computed in that order are stable.
// The block is then reordered by digit in LDS and written out digit run by
// digit run, so consecutive threads store to consecutive addresses.
template <int kRItems>
__global__ __launch_bounds__(kBlock) void radix_scatter_kernel(
    const uint32_t* __restrict__ keys, const uint32_t* __restrict__ vals, PassArgs pa, int bits,
    const uint32_t* __restrict__ offsets, uint32_t* __restrict__ okeys, uint32_t* __restrict__ ovals_mid,
    uint32_t* __restrict__ ovals_last, const uint32_t* __restrict__ gsrc, int64_t gn, uint32_t* __restrict__ gout) {
  __shared__ uint32_t cnt[4][256];
  __shared__ uint32_t gbase[256];
  __shared__ uint32_t dofs[256];
  constexpr int kRPerBlock = kBlock * kRItems;
  __shared__ uint32_t sk[kRPerBlock];
  __shared__ uint32_t sv[kRPerBlock];
  const PassDev pd = pass_dev(pa);
  if (!pd.active) return;       // uniform over the grid: an idle pass
  const int64_t n = pd.n, nblocks = pd.nb;
  const uint32_t base_key = pd.base, cap = pd.cap;
  const int shift = pa.shift;
  uint32_t* __restrict__ ovals = pd.last ? ovals_last : ovals_mid;
  if (!pd.last) gsrc = nullptr;
  const int tid = threadIdx.x;
  const int w = tid >> 6, lane = tid & 63;
  const uint32_t mask = (1u << bits) - 1u;
  const XcdRange xr = xcd_range(nblocks);
  for (int64_t blk = xr.first; blk < xr.end; blk += xr.step) {
    __syncthreads();              // the previous block's LDS reads are done
    for (int k = 0; k < 4; ++k) cnt[k][tid] = 0;
    gbase[tid] = (uint32_t)tid <= mask ? offsets[(int64_t)tid * nblocks + blk] : 0u;
    __syncthreads();
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    const int64_t block0 = blk * kRPerBlock;
    const int64_t base = block0 + (int64_t)w * (kRPerBlock / 4);
    uint32_t key[kRItems], val[kRItems], loc[kRItems];
    // all loads first: the ranking below writes LDS between rounds, which
    // would otherwise serialise one memory latency per round.  Each item is
    // read once per pass: streaming (non-temporal) loads, measured 4% faster.
#pragma unroll
    for (int r = 0; r < kRItems; ++r) {
      const int64_t j = base + (int64_t)r * 64 + lane;
      key[r] = j < n ? __builtin_nontemporal_load(keys + j) : 0u;
      val[r] = j < n ? __builtin_nontemporal_load(vals + j) : 0u;
    }
#pragma unroll
    for (int r = 0; r < kRItems; ++r) {
      const int64_t j = base + (int64_t)r * 64 + lane;
      const bool ok = j < n;
      const uint32_t d = radix_digit(key[r], base_key, cap, shift, mask);
      uint64_t peers = __ballot(ok);
      for (int b = 0; b < bits; ++b) {
        const bool bit = (d >> b) & 1u;
        const uint64_t on = __ballot(bit);
        peers &= bit ? on : ~on;
      }
      const uint32_t before = (uint32_t)__popcll(peers & lt);
      const uint32_t cur = cnt[w][d];
      loc[r] = cur + before;
      const int leader = __ffsll((unsigned long long)peers) - 1;
      __builtin_amdgcn_wave_barrier();
      if (ok && lane == leader) cnt[w][d] = cur + (uint32_t)__popcll(peers);
      __builtin_amdgcn_wave_barrier();
    }
    __syncthreads();
    // per digit: exclusive prefix over waves, and the block-level digit offset
    const uint32_t c0 = cnt[0][tid], c1 = cnt[1][tid], c2 = cnt[2][tid], c3 = cnt[3][tid];
    const uint32_t dstart = block_excl_scan<uint32_t>(c0 + c1 + c2 + c3, dofs, (uint32_t*)nullptr);
    cnt[0][tid] = dstart;
    cnt[1][tid] = dstart + c0;
    cnt[2][tid] = dstart + c0 + c1;
    cnt[3][tid] = dstart + c0 + c1 + c2;
    dofs[tid] = dstart;
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kRItems; ++r) {
      const int64_t j = base + (int64_t)r * 64 + lane;
      if (j < n) {
        const uint32_t d = radix_digit(key[r], base_key, cap, shift, mask);
        const uint32_t bp = cnt[w][d] + loc[r];
        sk[bp] = key[r];
        sv[bp] = val[r];
      }
    }
    __syncthreads();
    const int in_block = (int)min((int64_t)kRPerBlock, n - block0);
    for (int i = tid; i < in_block; i += kBlock) {
      const uint32_t k = sk[i];
      const uint32_t d = radix_digit(k, base_key, cap, shift, mask);
      const uint32_t p = gbase[d] + ((uint32_t)i - dofs[d]);
      okeys[p] = k;
      ovals[p] = sv[i];
      // optional gather by the output value for the first gn positions (the
      // depth sort's last pass: the visible entries' tile counts in rank
      // order; issuing these loads in batches measured no faster and, by the
      // registers it took, slowed every other pass of this kernel)
      if (gsrc && (int64_t)p < gn) gout[p] = gsrc[sv[i]];
    }
  }  // radix blocks
}

// ---------------------------------------------------------------------------
// 3. emission
// ---------------------------------------------------------------------------


// Per-wave metadata of the emission: the 64 ranks' first slots and row
// table coordinates, read by the lanes that write those ranks' pairs.
struct EmitMeta {
  uint32_t off[64];
  int base[64], h[64], total[64], y0[64], toff[64], tx[64], fits[64];
  int mark[64];
};

// One lane per rank reads that rank's entry line (record, ellipse,
// rectangle: one 128-byte read) and copies the record to rank order.  The
// rows of the wave's 64 rectangles are evaluated spread over the lanes into
// the wave's row table (start slot, first tile key, rank lane).  The 64
// ranks' pairs are one contiguous slot range, which the wave then writes 64
// slots at a time: the non-empty rows that start inside the window mark
// their start, an inclusive max-scan of the marks gives every slot its row,
// and the slot's key is the row's first key plus the slot's distance from
// the row start.  Stores are coalesced and each step does the same work
// whatever the ranks' sizes.  Exactly tiles_touched pairs are written per
// rank (the scan reserved that many, and the projection counted them with
// the same row_run on the same values).  If the two ever disagreed, the wave
// instead rebuilds the table per rank (wave_row_table) and writes by rank:
// each slot's rank from marks at the ranks' first slots, its row by binary
// search (find_row); slots a rank reserved beyond its rows get the sentinel
// key n_tiles, which sorts after every real tile, and no store leaves the
// rank's range.  Ranks whose rows do not fit the table are written
// afterwards with for_each_listed_tile.  No slot at or beyond the pair
// capacity is written (the caller learns from the required count that the
// lists are incomplete).  The grid covers every entry; the number of
// visible ranks comes from the device record.
__global__ __launch_bounds__(kBlock) void emit_kernel(CamBatch cb, int64_t n, const uint32_t* __restrict__ order,
                                                      const Entry* __restrict__ ent,
                                                      const uint32_t* __restrict__ off,
                                                      const uint32_t* __restrict__ cnt, const SortDyn* __restrict__ dyn,
                                                      uint32_t capacity, uint4* __restrict__ rec_out,
                                                      uint32_t* __restrict__ tkeys, uint32_t* __restrict__ tvals) {
  __shared__ RowTable s_rows[kBlock / 64];
  __shared__ EmitMeta s_meta[kBlock / 64];
  const int64_t r = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const int lane = threadIdx.x & 63;
  RowTable* table = &s_rows[threadIdx.x >> 6];
  EmitMeta& M = s_meta[threadIdx.x >> 6];
  int my_off = 0, my_cnt = 0, my_x0 = 0, my_y0 = 0, my_x1 = 0, my_y1 = 0, my_toff = 0, my_tx = 1;
  double my_mx = 0.0, my_my = 0.0;
  Ellipse my_el{1.0, 0.0, 1.0, 0.0};
  const int64_t n_vis = dyn->n_vis;
  const bool valid = r < n_vis;
  if (valid) {
    // the entry's line: record (4 x 16 B), ellipse (2 x 16 B), rectangle;
    // all loads issued before any is used
    const uint32_t e = order[r];
    const uint4* src = reinterpret_cast<const uint4*>(ent + e);
    uint4 q[7];
#pragma unroll
    for (int k = 0; k < 7; ++k) q[k] = src[k];
    uint4* dst = rec_out + (size_t)r * 4;
    dst[0] = q[0]; dst[1] = q[1]; dst[2] = q[2]; dst[3] = q[3];
    my_mx = __hiloint2double((int)q[0].y, (int)q[0].x);   // Rec: 2D mean in FP64 first
    my_my = __hiloint2double((int)q[0].w, (int)q[0].z);
    my_el.A = __hiloint2double((int)q[4].y, (int)q[4].x);
    my_el.B = __hiloint2double((int)q[4].w, (int)q[4].z);
    my_el.D = __hiloint2double((int)q[5].y, (int)q[5].x);
    my_el.hr = __hiloint2double((int)q[5].w, (int)q[5].z);
    my_x0 = (int)(q[6].x & 0xFFFFu); my_y0 = (int)(q[6].x >> 16);
    my_x1 = (int)(q[6].y & 0xFFFFu); my_y1 = (int)(q[6].y >> 16);
    const int v = (int)(e / (uint64_t)n);
    for (int k = 0; k < cb.n_views; ++k)
      if (k == v) { my_toff = cb.v[k].tile_offset; my_tx = cb.v[k].tiles_x; }
    my_off = (int)off[r];
    my_cnt = (int)cnt[r];
  }
  // The rows of the wave's entries, spread over the lanes: the entries'
  // rows are numbered in rank order (entry j's h_j rows from base_j, an
  // exclusive scan of the heights), and lane l evaluates rows l, l + 64, ...
  // of those that fit the table (the entries that fit are a prefix).  A
  // row's entry comes from a max-scan of marks at the entries' first rows,
  // its constants from that entry's lane.  Each row is stored as (its start
  // slot relative to the wave's first slot, first tile key | entry lane << 25
  // | empty << 31); the start slots are a running sum of the row lengths,
  // which equals the offsets scan whenever every entry's rows add up to its
  // reserved count.
  const int h = valid ? my_y1 - my_y0 + 1 : 0;
  const int incl = wave_incl_scan(h);
  const int base = incl - h;
  const bool listed = valid && incl <= kRowSlots;
  const uint64_t fitm = __ballot(listed);
  const int nrows = fitm ? __builtin_amdgcn_readlane(incl, 63 - __builtin_clzll(fitm)) : 0;
  const bool keys25 = cb.total_tiles < (1 << 25);
  RowGeo geo{};
  if (valid) geo = make_row_geo(my_mx, my_my, my_el);
  uint32_t gsum = 0;                 // slots of the rows of earlier rounds
  int own_carry = 0;
  for (int q0 = 0; q0 < nrows; q0 += 64) {
    M.mark[lane] = 0;
    __builtin_amdgcn_wave_barrier();
    if (listed && h > 0 && base >= q0 && base < q0 + 64) M.mark[base - q0] = lane + 1;
    __builtin_amdgcn_wave_barrier();
    const int mk = wave_incl_max(M.mark[lane]);
    const int own = mk > 0 ? mk - 1 : own_carry;
    own_carry = __builtin_amdgcn_readlane(own, 63);
    RowGeo og;
    og.mx = __shfl(geo.mx, own, 64);
    og.my = __shfl(geo.my, own, 64);
    og.k = __shfl(geo.k, own, 64);
    og.S = __shfl(geo.S, own, 64);
    og.ds = __shfl(geo.ds, own, 64);
    og.ey = __shfl(geo.ey, own, 64);
    og.iD = __shfl(geo.iD, own, 64);
    og.hr = __shfl(geo.hr, own, 64);
    og.inf = __shfl((int)geo.inf, own, 64) != 0;
    const int ob = __shfl(base, own, 64), oy0 = __shfl(my_y0, own, 64);
    const int ox0 = __shfl(my_x0, own, 64), ox1 = __shfl(my_x1, own, 64);
    const int otoff = __shfl(my_toff, own, 64), otx = __shfl(my_tx, own, 64);
    const int rw = q0 + lane;
    const int y = oy0 + (rw - ob);
    int len = 0, t0 = ox0;
    if (rw < nrows) len = row_run(og, y, ox0, ox1, &t0);
    const int li = wave_incl_scan(len);
    if (rw < nrows) {
      const uint32_t key = (uint32_t)(otoff + y * otx + t0) & 0x1FFFFFFu;
      table->t0[rw] = key | ((uint32_t)own << 25) | (len == 0 ? 0x80000000u : 0u);
      table->cum[rw] = gsum + (uint32_t)(li - len);
    }
    gsum += (uint32_t)__builtin_amdgcn_readlane(li, 63);
  }
  __builtin_amdgcn_wave_barrier();
  int total = 0;
  if (listed && h > 0) total = (int)((base + h < nrows ? table->cum[base + h] : gsum) - table->cum[base]);
  M.off[lane] = (uint32_t)my_off;
  M.y0[lane] = my_y0;
  M.toff[lane] = my_toff;
  M.tx[lane] = my_tx;
  __syncthreads();
  const int64_t r0 = r - lane;
  if (r0 >= n_vis) return;   // uniform per wave; no barrier follows
  const int last = (int)min((int64_t)63, n_vis - 1 - r0);
  const uint32_t s0 = (uint32_t)__builtin_amdgcn_readfirstlane(my_off);
  const uint32_t s1 = min((uint32_t)__builtin_amdgcn_readlane(my_off + my_cnt, last), capacity);
  int carry = 0;
  // Row path, when every listed entry's rows add up to its reserved count
  // and a tile key fits 25 bits: in each 64-slot window the non-empty rows
  // that start there mark their start, and the max-scan hands every slot its
  // row directly (key = the row's first key plus the slot's distance from the
  // row start).
  const bool row_path = !__any(listed && total != my_cnt) && keys25;
  if (row_path) {
    uint32_t s1m = s0;
    if (fitm) {
      const int lf = 63 - __builtin_clzll(fitm);                 // listed ranks are a prefix
      s1m = lf == last ? s1 : min(s1, (uint32_t)__builtin_amdgcn_readlane(my_off, lf + 1));
    }
    uint32_t rptr = 0;
    for (uint32_t c0 = s0; c0 < s1m; c0 += 64) {
      M.mark[lane] = 0;
      __builtin_amdgcn_wave_barrier();
      // rows are consumed in order: every row before rptr starts before c0
      uint32_t taken;
      do {
        const uint32_t rw = rptr + (uint32_t)lane;
        const uint32_t st = rw < (uint32_t)nrows ? s0 + table->cum[rw] : 0xFFFFFFFFu;
        const bool in = st < c0 + 64u;
        if (in && !(table->t0[rw] >> 31)) M.mark[st - c0] = (int)rw + 1;
        taken = (uint32_t)__popcll(__ballot(in));
        rptr += taken;
      } while (taken == 64u);
      __builtin_amdgcn_wave_barrier();
      const int m = wave_incl_max(M.mark[lane]);
      const int rw = m > 0 ? m - 1 : carry;
      carry = __builtin_amdgcn_readlane(rw, 63);
      const uint32_t sl = c0 + (uint32_t)lane;
      if (sl < s1m) {
        const uint32_t pk = table->t0[rw];
        tkeys[sl] = (pk & 0x1FFFFFFu) + (sl - s0 - table->cum[rw]);
        tvals[sl] = (uint32_t)r0 + ((pk >> 25) & 63u);
      }
    }
  } else {
    // the per-rank path: the table again in its plain form (first column and
    // the tiles of the rows above, per entry), each slot's rank by the marks
    // of the ranks' first slots and its row by binary search
    const WaveRows wr = wave_row_table(valid, my_mx, my_my, my_el, my_x0, my_y0, my_x1, my_y1, table);
    M.base[lane] = wr.base;
    M.h[lane] = wr.h;
    M.total[lane] = wr.total;
    M.fits[lane] = valid && wr.fits;
    __builtin_amdgcn_wave_barrier();
    for (uint32_t c0 = s0; c0 < s1; c0 += 64) {
      M.mark[lane] = 0;
      __builtin_amdgcn_wave_barrier();
      if (valid && my_cnt > 0 && (uint32_t)my_off >= c0 && (uint32_t)my_off < c0 + 64u) M.mark[my_off - c0] = lane + 1;
      __builtin_amdgcn_wave_barrier();
      const int m = wave_incl_max(M.mark[lane]);
      const int rk = m > 0 ? m - 1 : carry;
      carry = __builtin_amdgcn_readlane(rk, 63);
      const uint32_t sl = c0 + (uint32_t)lane;
      if (sl < s1 && M.fits[rk]) {
        const int k = (int)(sl - M.off[rk]);
        uint32_t key = (uint32_t)cb.total_tiles;
        if (k < M.total[rk]) {
          const int b = M.base[rk];
          const int row = find_row(table, b, M.h[rk], k);
          const int x = (int)table->t0[b + row] + (k - (int)table->cum[b + row]);
          key = (uint32_t)(M.toff[rk] + (M.y0[rk] + row) * M.tx[rk] + x);
        }
        tkeys[sl] = key;
        tvals[sl] = (uint32_t)(r0 + rk);
      }
    }
  }
  // ranks whose rows did not fit the table, one at a time
  uint64_t rest = __ballot(valid && my_cnt > 0 && !listed);
  while (rest) {
    const int j = (int)__builtin_ctzll(rest);
    rest &= rest - 1;
    const int cntj = bcast_i(my_cnt, j);
    const uint32_t offj = (uint32_t)bcast_i(my_off, j);
    const uint32_t rank = (uint32_t)(r0 + j);
    const int toff = bcast_i(my_toff, j), tx = bcast_i(my_tx, j);
    auto put = [&](int k, int x, int y) {
      if (k < cntj && offj + (uint32_t)k < capacity) {
        tkeys[offj + k] = (uint32_t)(toff + y * tx + x);
        tvals[offj + k] = rank;
      }
    };
    const Ellipse el{bcast_d(my_el.A, j), bcast_d(my_el.B, j), bcast_d(my_el.D, j), bcast_d(my_el.hr, j)};
    const int written = for_each_listed_tile(bcast_d(my_mx, j), bcast_d(my_my, j), el, bcast_i(my_x0, j),
                                             bcast_i(my_y0, j), bcast_i(my_x1, j), bcast_i(my_y1, j), put);
    for (int k = written + lane; k < cntj && offj + (uint32_t)k < capacity; k += 64) {
      tkeys[offj + k] = (uint32_t)cb.total_tiles;
      tvals[offj + k] = rank;
    }
  }
}

// ---------------------------------------------------------------------------
// 5. tile ranges
// ---------------------------------------------------------------------------
// Tile ranges from the sorted tile keys: position i starts every tile in
// (key[i-1], key[i]] (key[-1] = -1, key[m] = n_tiles).  Each thread takes four
// consecutive positions with one 16-byte load (keys is 16-byte aligned).
__device__ __forceinline__ void mark_starts(int64_t prev, int64_t cur, int64_t n_tiles, uint32_t i,
                                            uint32_t* __restrict__ start) {
  if (prev > n_tiles) prev = n_tiles;
  if (cur > n_tiles) cur = n_tiles;
  for (int64_t t = prev + 1; t <= cur; ++t) start[t] = i;
}

// Tile starts from the four positions i0 .. i0 + 3 (and the end, m).
__device__ __forceinline__ void tile_start_at(const uint32_t* __restrict__ tkeys, int64_t m, int64_t n_tiles,
                                              int64_t i0, uint32_t* __restrict__ start) {
  int64_t prev = i0 == 0 ? -1 : (int64_t)tkeys[i0 - 1];
  if (i0 + 4 <= m) {
    const uint4 k = *(const uint4*)(tkeys + i0);
    const uint32_t kk[4] = {k.x, k.y, k.z, k.w};
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      if ((int64_t)kk[j] != prev) mark_starts(prev, kk[j], n_tiles, (uint32_t)(i0 + j), start);
      prev = kk[j];
    }
  } else {
    // the last positions, up to and including m
    for (int64_t i = i0; i <= m; ++i) {
      const int64_t cur = i == m ? n_tiles : (int64_t)tkeys[i];
      if (cur != prev) mark_starts(prev, cur, n_tiles, (uint32_t)i, start);
      prev = cur;
    }
  }
}

constexpr int64_t kTileStartGrid = 4096;

__global__ __launch_bounds__(kBlock) void tile_start_kernel(const uint32_t* __restrict__ tkeys,
                                                            const SortDyn* __restrict__ dyn, int64_t n_tiles,
                                                            uint32_t* __restrict__ start) {
  const int64_t m = dyn->m;   // positions 0..m; the grid strides over them
  for (int64_t i0 = 4 * ((int64_t)blockIdx.x * kBlock + threadIdx.x); i0 <= m;
       i0 += 4 * (int64_t)gridDim.x * kBlock)
    tile_start_at(tkeys, m, n_tiles, i0, start);
}

// ---------------------------------------------------------------------------
// workspace
// ---------------------------------------------------------------------------
struct Ws {
  uint32_t *flags, *pos, *ka, *va, *kb, *vb, *hist, *scan;
  ScanSync* sync;
  unsigned long long* counters;
  SortDyn* dyn;
  BlockStat* stats;
  size_t bytes;
};

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

Ws carve(void* base, int64_t n_entries, int64_t pair_cap) {
  const int64_t big = n_entries > pair_cap ? n_entries : pair_cap;
  // blocks of the narrowest pass (the most blocks, so the largest histogram)
  const int64_t nb = (big + kBlock * kRItemsNarrow - 1) / (kBlock * kRItemsNarrow);
  Ws w;
  char* p = (char*)base;
  size_t off = 0;
  auto take = [&](size_t bytes) { char* q = p ? p + off : nullptr; off += align256(bytes); return q; };
  w.counters = (unsigned long long*)take(4 * sizeof(unsigned long long));
  w.dyn = (SortDyn*)take(sizeof(SortDyn));
  w.sync = (ScanSync*)take(sizeof(ScanSync));
  w.stats = (BlockStat*)take(sizeof(BlockStat) * (size_t)((n_entries + kBlock - 1) / kBlock + 1));
  w.flags = (uint32_t*)take(sizeof(uint32_t) * (size_t)n_entries);
  w.pos = (uint32_t*)take(sizeof(uint32_t) * (size_t)n_entries);
  w.ka = (uint32_t*)take(sizeof(uint32_t) * (size_t)big);
  w.va = (uint32_t*)take(sizeof(uint32_t) * (size_t)big);
  w.kb = (uint32_t*)take(sizeof(uint32_t) * (size_t)big);
  w.vb = (uint32_t*)take(sizeof(uint32_t) * (size_t)big);
  w.hist = (uint32_t*)take(sizeof(uint32_t) * 256 * (size_t)nb);
  w.scan = (uint32_t*)take(sizeof(uint32_t) * (size_t)scan_ws_words(256 * nb > big ? 256 * nb : big));
  w.bytes = off;
  return w;
}

// Digit layout of a sort: kDepthSort four 8-bit passes; kPairSort nbits in
// as few passes of at most 8 bits as possible, the bits spread evenly (e.g.
// 13 as 7 + 6: wider runs per digit and block make the scatter's stores
// longer).
struct Digits {
  int passes, width, items, bits[4];
};
Digits digits(int kind, int nbits) {
  if (kind == kDepthSort) nbits = 32;
  Digits d;
  d.passes = (nbits + 7) / 8;
  d.width = (nbits + d.passes - 1) / d.passes;
  d.items = radix_items(d.width);
  for (int p = 0; p < 4; ++p) {
    const int shift = d.width * p;
    d.bits[p] = p < d.passes ? ((nbits - shift) < d.width ? (nbits - shift) : d.width) : 0;
  }
  return d;
}

// Stable sort of (keys, vals) with at most n_max items (see PassArgs for
// the sizes the device supplies).  The data starts in (ka, va); keys
// ping-pong between ka and kb, values between va and vb, and the last pass
// that runs writes the values to out_v.  Returns the buffer holding the
// sorted keys for kPairSort, nullptr for kDepthSort (its keys are not used).
// With gsrc, the last pass also writes gout[p] = gsrc[out_v[p]] for p < gn.
uint32_t* radix_sort(uint32_t* ka, uint32_t* va, uint32_t* kb, uint32_t* vb, int64_t n_max, int kind, int nbits,
                     uint32_t* out_v, Ws& w, hipStream_t st, const uint32_t* gsrc = nullptr, int64_t gn = 0,
                     uint32_t* gout = nullptr) {
  const Digits dg = digits(kind, nbits);
  uint32_t* final_keys = kind == kDepthSort ? nullptr : (((dg.passes - 1) % 2 == 0) ? kb : ka);
  if (n_max <= 0) return final_keys;
  const int64_t nb = (n_max + kBlock * dg.items - 1) / (kBlock * dg.items);
  const int64_t g = nb < kRadixGrid ? nb : kRadixGrid;
  const dim3 grid((unsigned)(8 * ((g + 7) / 8)));
  for (int p = 0; p < dg.passes; ++p) {
    const int bits = dg.bits[p];
    uint32_t* ik = (p % 2 == 0) ? ka : kb;
    uint32_t* iv = (p % 2 == 0) ? va : vb;
    uint32_t* okk = (p % 2 == 0) ? kb : ka;
    uint32_t* ovv = (p % 2 == 0) ? vb : va;
    const uint32_t mask = (1u << bits) - 1u;
    const PassArgs pa{w.dyn, n_max, kind, p, dg.width * p, dg.width, nbits};
    if (dg.items == kRItemsNarrow)
      SSS_LAUNCH("radix_hist", radix_hist_kernel<kRItemsNarrow>, grid, dim3(kBlock), 0, st, ik, pa, mask, w.hist);
    else
      SSS_LAUNCH("radix_hist", radix_hist_kernel<kRItemsWide>, grid, dim3(kBlock), 0, st, ik, pa, mask, w.hist);
    // the histogram of the blocks the device counted (0 for an idle pass)
    scan_excl_sync(w.hist, w.hist, ((int64_t)1 << bits) * nb, w.scan, w.sync, st,
                   (const uint32_t*)&w.dyn->scan_n[kind][p]);
    if (dg.items == kRItemsNarrow)
      SSS_LAUNCH("radix_scatter", radix_scatter_kernel<kRItemsNarrow>, grid, dim3(kBlock), 0, st, ik, iv, pa, bits,
                 (const uint32_t*)w.hist, okk, ovv, out_v, gsrc, gn, gout);
    else
      SSS_LAUNCH("radix_scatter", radix_scatter_kernel<kRItemsWide>, grid, dim3(kBlock), 0, st, ik, iv, pa, bits,
                 (const uint32_t*)w.hist, okk, ovv, out_v, gsrc, gn, gout);
  }
  return final_keys;
}

int bits_for(int64_t v) {
  int b = 1;
  while (b < 32 && (int64_t(1) << b) < v) ++b;
  return b;
}

}  // namespace

size_t bin_sort_workspace(int64_t n_entries, int64_t pair_capacity) {
  return carve(nullptr, n_entries, pair_capacity).bytes;
}

int run_bin_sort(const CamBatch& cb, const sss_proj_t& proj, int64_t n, sss_bins_t* bins, void* ws,
                 size_t ws_bytes, hipStream_t st) {
  const int64_t n_entries = n * cb.n_views;
  const bool wait = !bins->no_wait;
  Ws w = carve(ws, n_entries, bins->pair_capacity);
  if (ws_bytes < w.bytes) {
    set_error("sss_bin_sort: workspace of %zu bytes, %zu needed", ws_bytes, w.bytes);
    return SSS_ERR_INVALID;
  }
  if (bins->pair_capacity > (int64_t)0xFFFFFFFFll) {
    set_error("sss_bin_sort: pair capacity %lld exceeds 2^32 - 1", (long long)bins->pair_capacity);
    return SSS_ERR_UNSUPPORTED;
  }
  bins->n_visible = -1;
  bins->n_pairs = -1;
  // 1. sort input and counts
  const unsigned g1 = (unsigned)((n_entries + kBlock * kPrepItems - 1) / (kBlock * kPrepItems));
  SSS_LAUNCH("prepare", prepare_kernel, dim3(g1), dim3(kBlock), 0, st, proj.tiles_touched, proj.depth_key, n_entries,
             w.ka, w.va, w.stats);
  const int pair_bits = bits_for((int64_t)cb.total_tiles + 1);
  SortLayout lay{};
  lay.n_entries = n_entries;
  for (int k = 0; k < 2; ++k) {
    const Digits dg = digits(k == 0 ? kDepthSort : kPairSort, pair_bits);
    lay.per_block[k] = kBlock * dg.items;
    lay.passes[k] = dg.passes;
    for (int p = 0; p < 4; ++p) lay.rows[k][p] = p < dg.passes ? 1 << dg.bits[p] : 0;
  }
  SSS_LAUNCH("stat_reduce", stat_reduce_kernel, dim3(1), dim3(kBlock), 0, st, (const BlockStat*)w.stats, (int64_t)g1,
             lay, (unsigned long long)bins->pair_capacity, w.counters, w.dyn, (unsigned long long*)bins->counts,
             w.sync);
  // the grids of the pair passes cover the pair capacity, or, when the call
  // waits for the counts, just the pairs
  int64_t pair_grid = bins->pair_capacity;
  if (wait) {
    unsigned long long counts[4];
    if (!hip_ok(hipMemcpyAsync(counts, w.counters, sizeof(counts), hipMemcpyDeviceToHost, st), "count readback"))
      return SSS_ERR_HIP;
    if (!hip_ok(hipStreamSynchronize(st), "count sync")) return SSS_ERR_HIP;
    bins->n_visible = (int64_t)counts[0];
    bins->n_pairs = (int64_t)counts[1];
    if (bins->n_pairs > bins->pair_capacity) {
      set_error("sss_bin_sort: %lld pairs exceed the capacity %lld", (long long)bins->n_pairs,
                (long long)bins->pair_capacity);
      return SSS_ERR_CAPACITY;
    }
    pair_grid = bins->n_pairs;
  }
  // 2. depth order over all entries (culled ones last); the last pass also
  //    gathers each rank's tile count (0 for culled entries)
  radix_sort(w.ka, w.va, w.kb, w.vb, n_entries, kDepthSort, 32, bins->order, w, st, proj.tiles_touched, n_entries,
             w.flags);
  // 3. pair offsets in rank order, emission, record gather; the caller may
  //    keep the offsets (deterministic backward pass)
  uint32_t* offs = bins->rank_offset ? bins->rank_offset : w.pos;
  scan_excl_sync(w.flags, offs, n_entries, w.scan, w.sync, st);
  const unsigned ge = (unsigned)((n_entries + kBlock - 1) / kBlock);
  SSS_LAUNCH("emit", emit_kernel, dim3(ge), dim3(kBlock), 0, st, cb, n, bins->order, (const Entry*)proj.entries,
             (const uint32_t*)offs, (const uint32_t*)w.flags, (const SortDyn*)w.dyn, (uint32_t)bins->pair_capacity,
             (uint4*)bins->sorted_records, w.ka, w.va);
  // 4. stable sort of the pairs by tile
  const uint32_t* tkeys = radix_sort(w.ka, w.va, w.kb, w.vb, pair_grid, kPairSort, pair_bits, bins->pair_rank, w, st);
  // 5. tile ranges
  const int64_t gt_need = ((pair_grid + 4) / 4 + kBlock - 1) / kBlock;
  const unsigned gt = (unsigned)(gt_need < kTileStartGrid ? gt_need : kTileStartGrid);
  SSS_LAUNCH("tile_start", tile_start_kernel, dim3(gt), dim3(kBlock), 0, st, tkeys, (const SortDyn*)w.dyn,
             (int64_t)cb.total_tiles, bins->tile_start);
  // 6. launch order of the tiles for the raster kernels, longest list first
  if (bins->tile_order) launch_tile_order(nullptr, 0, bins->tile_start, cb.total_tiles, bins->tile_order, st);
  if (!hip_ok(hipGetLastError(), "bin_sort launch")) return SSS_ERR_HIP;
  return SSS_OK;
}

}  // namespace sss
