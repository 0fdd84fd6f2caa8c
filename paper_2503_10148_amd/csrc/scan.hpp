// Exclusive prefix sums over device arrays (uint32 or uint64), any length:
// blocks of 256 threads x 16 items reduce, their sums are scanned
// recursively, then each block scans its items and adds its prefix.
#pragma once

#include "common.hpp"

namespace sss {
namespace {

constexpr int kItems = 16;                 // items per thread in scans / radix passes
constexpr int kPerBlock = kBlock * kItems; // 4096

template <typename T>
__device__ __forceinline__ T block_excl_scan(T v, T* lds, T* total) {
  // Hillis-Steele over 256 values in LDS; returns the exclusive prefix.
  const int t = threadIdx.x;
  lds[t] = v;
  __syncthreads();
  for (int off = 1; off < kBlock; off <<= 1) {
    const T add = t >= off ? lds[t - off] : T(0);
    __syncthreads();
    lds[t] += add;
    __syncthreads();
  }
  const T incl = lds[t];
  if (total) *total = lds[kBlock - 1];
  __syncthreads();
  return incl - v;
}

template <typename T>
__global__ __launch_bounds__(kBlock) void scan_reduce_kernel(const T* __restrict__ in, int64_t n, T* __restrict__ sums) {
  __shared__ T red[kBlock];
  const int64_t base = (int64_t)blockIdx.x * kPerBlock;
  T s = 0;
  for (int k = 0; k < kItems; ++k) {
    const int64_t j = base + (int64_t)k * kBlock + threadIdx.x;
    if (j < n) s += in[j];
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int off = kBlock / 2; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) sums[blockIdx.x] = red[0];
}

// Exclusive scan of one 4096-item block plus the block's prefix (in may alias
// out).  Loads and stores are coalesced (item k*256 + t by thread t) and
// staged in LDS with one pad word per 16, so that thread t can scan its 16
// consecutive items without bank conflicts.
template <typename T>
__global__ __launch_bounds__(kBlock) void scan_apply_kernel(const T* in, int64_t n, const T* __restrict__ prefix,
                                                            T* out) {
  constexpr int kPad = kItems + 1;
  __shared__ T lds[kBlock];
  __shared__ T tile[kBlock * kPad];
  const int64_t base = (int64_t)blockIdx.x * kPerBlock;
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
  T run = block_excl_scan<T>(s, lds, nullptr) + (prefix ? prefix[blockIdx.x] : T(0));
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

// Scratch elements (of T) that scan_excl needs for n items.
inline int64_t scan_ws_words(int64_t n) {
  int64_t w = 0;
  while (n > kPerBlock) {
    n = (n + kPerBlock - 1) / kPerBlock;
    w += 2 * n;
  }
  return w + 16;
}

template <typename T>
void scan_excl(const T* in, T* out, int64_t n, T* ws, hipStream_t st) {
  if (n <= 0) return;
  const int64_t nb = (n + kPerBlock - 1) / kPerBlock;
  if (nb == 1) {
    SSS_LAUNCH("scan_apply", scan_apply_kernel<T>, dim3(1), dim3(kBlock), 0, st, in, n, (const T*)nullptr, out);
    return;
  }
  T* sums = ws;
  T* sums_scan = ws + nb;
  SSS_LAUNCH("scan_reduce", scan_reduce_kernel<T>, dim3((unsigned)nb), dim3(kBlock), 0, st, in, n, sums);
  scan_excl<T>(sums, sums_scan, nb, ws + 2 * nb, st);
  SSS_LAUNCH("scan_apply", scan_apply_kernel<T>, dim3((unsigned)nb), dim3(kBlock), 0, st, in, n, (const T*)sums_scan,
             out);
}

}  // namespace
}  // namespace sss
