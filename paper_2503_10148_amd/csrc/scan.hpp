// Exclusive prefix sums over device arrays (uint32 or uint64), any length:
// blocks of 256 threads x 16 items reduce, their sums are scanned
// recursively, then each block scans its items and adds its prefix.
#pragma once

#include "common.hpp"

namespace sss {
namespace {

constexpr int kItems = 16;                 // items per thread in scans / radix passes
constexpr int kPerBlock = kBlock * kItems; // 4096

constexpr int kScanWaves = kBlock / 64;

// Inclusive prefix sum over the 64 lanes of a wave.
template <typename T>
__device__ __forceinline__ T wave_incl_sum(T v) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const T u = __shfl_up(v, d, 64);
    if (lane >= d) v += u;
  }
  return v;
}

// Exclusive prefix of v over the 256 threads of the block (in thread order):
// a scan inside each wave, then the totals of the waves before.  lds holds
// at least kScanWaves values; it may be reused once this returns.
template <typename T>
__device__ __forceinline__ T block_excl_scan(T v, T* lds, T* total) {
  const int w = threadIdx.x >> 6;
  const T incl = wave_incl_sum(v);
  if ((threadIdx.x & 63) == 63) lds[w] = incl;
  __syncthreads();
  T before = 0, all = 0;
#pragma unroll
  for (int k = 0; k < kScanWaves; ++k) {
    const T c = lds[k];
    before += k < w ? c : T(0);
    all += c;
  }
  if (total) *total = all;
  __syncthreads();
  return before + incl - v;
}

// Item count of a scan: n, or the smaller count *n_dev when the device
// supplies it (the grid is sized for n).
__device__ __forceinline__ int64_t scan_count(int64_t n, const uint32_t* n_dev) {
  return n_dev ? min(n, (int64_t)*n_dev) : n;
}

template <typename T>
__global__ __launch_bounds__(kBlock) void scan_reduce_kernel(const T* __restrict__ in, int64_t n_max,
                                                             const uint32_t* __restrict__ n_dev,
                                                             T* __restrict__ sums) {
  __shared__ T red[kScanWaves];
  const int64_t n = scan_count(n_max, n_dev);
  const int64_t base = (int64_t)blockIdx.x * kPerBlock;
  if (base >= n) {              // uniform per block; past the device's count
    if (threadIdx.x == 0) sums[blockIdx.x] = T(0);
    return;
  }
  // all loads before the sum, so one memory latency is waited for, not 16
  T v[kItems];
#pragma unroll
  for (int k = 0; k < kItems; ++k) {
    const int64_t j = base + (int64_t)k * kBlock + threadIdx.x;
    v[k] = j < n ? in[j] : T(0);
  }
  T s = 0;
#pragma unroll
  for (int k = 0; k < kItems; ++k) s += v[k];
  s = wave_incl_sum(s);   // lane 63 holds the wave's sum
  if ((threadIdx.x & 63) == 63) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    T t = 0;
#pragma unroll
    for (int k = 0; k < kScanWaves; ++k) t += red[k];
    sums[blockIdx.x] = t;
  }
}

// Exclusive scan of one 4096-item block plus the block's prefix (in may alias
// out).  The prefix is prefix[block] when prefix is given, else the sum of
// block_sums[0 .. block) when that is given (each block adds the raw sums of
// the blocks before it, which for up to kFusedBlocks blocks is cheaper than
// a launch that scans them), else 0.  Loads and stores are coalesced (item k*256 + t by thread t) and
// staged in LDS with one pad word per 16, so that thread t can scan its 16
// consecutive items without bank conflicts.
template <typename T>
__global__ __launch_bounds__(kBlock) void scan_apply_kernel(const T* in, int64_t n_max, const uint32_t* __restrict__ n_dev,
                                                            const T* __restrict__ prefix,
                                                            const T* __restrict__ block_sums, T* out) {
  constexpr int kPad = kItems + 1;
  __shared__ T lds[kBlock];
  __shared__ T tile[kBlock * kPad];
  const int64_t n = scan_count(n_max, n_dev);
  const int64_t base = (int64_t)blockIdx.x * kPerBlock;
  if (base >= n) return;        // uniform per block, before any barrier
  const int t = threadIdx.x;
  T ld[kItems];
#pragma unroll
  for (int k = 0; k < kItems; ++k) {
    const int64_t j = base + (int64_t)k * kBlock + t;
    ld[k] = j < n ? in[j] : T(0);
  }
#pragma unroll
  for (int k = 0; k < kItems; ++k) {
    const int i = k * kBlock + t;                // item index inside the block
    tile[(i / kItems) * kPad + i % kItems] = ld[k];
  }
  __syncthreads();
  T v[kItems];
  T s = 0;
#pragma unroll
  for (int k = 0; k < kItems; ++k) {
    v[k] = tile[t * kPad + k];
    s += v[k];
  }
  T pre = prefix ? prefix[blockIdx.x] : T(0);
  if (!prefix && block_sums) {
    T ps = 0;
    for (int64_t i = t; i < (int64_t)blockIdx.x; i += kBlock) ps += block_sums[i];
    block_excl_scan<T>(ps, lds, &pre);
  }
  T run = block_excl_scan<T>(s, lds, nullptr) + pre;
#pragma unroll
  for (int k = 0; k < kItems; ++k) {
    tile[t * kPad + k] = run;
    run += v[k];
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < kItems; ++k) {
    const int i = k * kBlock + t;
    const int64_t j = base + i;
    if (j < n) out[j] = tile[(i / kItems) * kPad + i % kItems];
  }
}

// Single-pass exclusive scan of uint32 counts over at most kFusedBlocks
// blocks, one launch instead of the reduce + apply pair (whose cost here is
// mostly the second launch).  A block takes its number from a ticket counter
// when it starts, so every block with a smaller number is already running;
// it publishes its sum as soon as it has it (one 64-bit word: a ready bit
// above the 32-bit sum), adds the published sums of all blocks before it,
// then scans its items.  The wait for a predecessor's word is bounded (the
// predecessors never wait themselves, so it ends long before the bound).
// The last block to finish clears the counters and the words it used, so
// the next scan starts from zeros; the first scan of a sort needs them zeroed
// by an earlier kernel (scan_sync_clear).
struct ScanSync {
  uint32_t ticket, done;
  uint32_t pad[62];
  unsigned long long word[1024];
};

constexpr int kScanSpin = 1 << 22;

// Zeroes a ScanSync with the calling block's threads.
__device__ __forceinline__ void scan_sync_clear(ScanSync* sync) {
  for (int i = threadIdx.x; i < 1024; i += blockDim.x) sync->word[i] = 0ull;
  if (threadIdx.x == 0) {
    sync->ticket = 0u;
    sync->done = 0u;
  }
}

__global__ __launch_bounds__(kBlock) void scan_1pass_kernel(const uint32_t* in, int64_t n_max,
                                                            const uint32_t* __restrict__ n_dev, ScanSync* sync,
                                                            uint32_t* out) {
  constexpr int kPad = kItems + 1;
  __shared__ uint32_t lds[kBlock];
  __shared__ uint32_t tile[kBlock * kPad];
  __shared__ uint32_t s_ticket, s_last;
  const int t = threadIdx.x;
  if (t == 0) s_ticket = atomicAdd(&sync->ticket, 1u);
  __syncthreads();
  const uint32_t b = s_ticket;
  const int64_t n = scan_count(n_max, n_dev);
  const int64_t base = (int64_t)b * kPerBlock;
  if (base < n) {                                    // uniform per block
    uint32_t ld[kItems];
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
      const int64_t j = base + (int64_t)k * kBlock + t;
      ld[k] = j < n ? in[j] : 0u;
    }
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
      const int i = k * kBlock + t;
      tile[(i / kItems) * kPad + i % kItems] = ld[k];
    }
    __syncthreads();
    uint32_t v[kItems];
    uint32_t s = 0;
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
      v[k] = tile[t * kPad + k];
      s += v[k];
    }
    uint32_t total;
    const uint32_t run0 = block_excl_scan<uint32_t>(s, lds, &total);
    if (t == 0)
      __hip_atomic_store(&sync->word[b], (1ull << 32) | (unsigned long long)total, __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_AGENT);
    // the sums of the blocks before this one
    uint32_t ps = 0;
    for (uint32_t i = (uint32_t)t; i < b; i += kBlock) {
      unsigned long long wv = 0ull;
      for (int spin = 0; spin < kScanSpin; ++spin) {
        wv = __hip_atomic_load(&sync->word[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (wv >> 32) break;
        __builtin_amdgcn_s_sleep(1);
      }
      ps += (uint32_t)wv;
    }
    uint32_t pre;
    block_excl_scan<uint32_t>(ps, lds, &pre);
    uint32_t run = run0 + pre;
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
      tile[t * kPad + k] = run;
      run += v[k];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
      const int i = k * kBlock + t;
      const int64_t j = base + i;
      if (j < n) out[j] = tile[(i / kItems) * kPad + i % kItems];
    }
  }
  // the last block to finish leaves the counters and words at zero
  __syncthreads();
  if (t == 0) s_last = atomicAdd(&sync->done, 1u) == gridDim.x - 1u;
  __syncthreads();
  if (s_last) {
    for (uint32_t i = (uint32_t)t; i < gridDim.x; i += kBlock) sync->word[i] = 0ull;
    if (t == 0) {
      sync->ticket = 0u;
      sync->done = 0u;
    }
  }
}

// Scratch elements (of T) that scan_excl needs for n items.
inline int64_t scan_ws_words(int64_t n) {
  int64_t w = 0;
  while (n > kPerBlock) {
    n = (n + kPerBlock - 1) / kPerBlock;
    w += 2 * n;
  }
  return w + 16;
}

constexpr int64_t kFusedBlocks = 1024;

// scan_excl for uint32 counts with a ScanSync (zeroed before the first use,
// left zeroed by every single-pass scan): one launch for up to kFusedBlocks
// blocks of items, the two-launch scan beyond.
inline void scan_excl_sync(const uint32_t* in, uint32_t* out, int64_t n, uint32_t* ws, ScanSync* sync,
                           hipStream_t st, const uint32_t* n_dev = nullptr);

// Exclusive scan of in[0, n) into out.  With n_dev, the device supplies the
// count (at most n; n sizes the grids): blocks past it do nothing, so a
// scan sized for a bound costs little more than one sized for the count.
template <typename T>
void scan_excl(const T* in, T* out, int64_t n, T* ws, hipStream_t st, const uint32_t* n_dev = nullptr) {
  if (n <= 0) return;
  const int64_t nb = (n + kPerBlock - 1) / kPerBlock;
  if (nb == 1) {
    SSS_LAUNCH("scan_apply", scan_apply_kernel<T>, dim3(1), dim3(kBlock), 0, st, in, n, n_dev, (const T*)nullptr,
               (const T*)nullptr, out);
    return;
  }
  T* sums = ws;
  T* sums_scan = ws + nb;
  SSS_LAUNCH("scan_reduce", scan_reduce_kernel<T>, dim3((unsigned)nb), dim3(kBlock), 0, st, in, n, n_dev, sums);
  if (nb <= kFusedBlocks) {
    SSS_LAUNCH("scan_apply", scan_apply_kernel<T>, dim3((unsigned)nb), dim3(kBlock), 0, st, in, n, n_dev,
               (const T*)nullptr, (const T*)sums, out);
    return;
  }
  // the block sums of blocks past the device's count are zero
  scan_excl<T>(sums, sums_scan, nb, ws + 2 * nb, st);
  SSS_LAUNCH("scan_apply", scan_apply_kernel<T>, dim3((unsigned)nb), dim3(kBlock), 0, st, in, n, n_dev,
             (const T*)sums_scan, (const T*)nullptr, out);
}

inline void scan_excl_sync(const uint32_t* in, uint32_t* out, int64_t n, uint32_t* ws, ScanSync* sync,
                           hipStream_t st, const uint32_t* n_dev) {
  if (n <= 0) return;
  const int64_t nb = (n + kPerBlock - 1) / kPerBlock;
  if (nb == 1 || nb > kFusedBlocks) {
    scan_excl<uint32_t>(in, out, n, ws, st, n_dev);
    return;
  }
  SSS_LAUNCH("scan_1pass", scan_1pass_kernel, dim3((unsigned)nb), dim3(kBlock), 0, st, in, n, n_dev, sync, out);
}

}  // namespace
}  // namespace sss
