// Workgroup- and wave-level building blocks for gfx950 (wave64).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace bilu {

__device__ __forceinline__ int lane_id() { return __lane_id(); }

// Wave-wide sum of an int (all 64 lanes participate).
__device__ __forceinline__ int wave_sum(int v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}

// Exclusive scan of one int per thread over a workgroup of nthreads (multiple
// of 64, <= 1024).  tmp: LDS scratch of >= nthreads/64 + 1 ints.  Returns the
// exclusive prefix; *total receives the sum (all threads).
__device__ __forceinline__ int wg_exclusive_scan(int v, int* tmp, int* total) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
  int incl = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    int t = __shfl_up(incl, o, 64);
    if (lane >= o) incl += t;
  }
  if (lane == 63) tmp[wid] = incl;
  __syncthreads();
  if (threadIdx.x == 0) {
    int acc = 0;
    for (int w = 0; w < nw; ++w) {
      int t = tmp[w];
      tmp[w] = acc;
      acc += t;
    }
    tmp[nw] = acc;
  }
  __syncthreads();
  int res = tmp[wid] + incl - v;
  *total = tmp[nw];
  __syncthreads();
  return res;
}

// Bitonic sort of keys[0..m) in LDS (ascending), padded with INT32_MAX up to
// the next power of two (the array must hold that many slots).
__device__ inline void wg_bitonic_sort(int* keys, int m) {
  int p2 = 1;
  while (p2 < m) p2 <<= 1;
  for (int i = m + threadIdx.x; i < p2; i += blockDim.x) keys[i] = INT32_MAX;
  __syncthreads();
  for (int k = 2; k <= p2; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int i = threadIdx.x; i < p2; i += blockDim.x) {
        int ixj = i ^ j;
        if (ixj > i) {
          int a = keys[i], b = keys[ixj];
          bool up = (i & k) == 0;
          if ((a > b) == up) {
            keys[i] = b;
            keys[ixj] = a;
          }
        }
      }
      __syncthreads();
    }
  }
}

// First index in sorted a[0..m) with a[idx] >= key.
__device__ __forceinline__ int lower_bound(const int* a, int m, int key) {
  int lo = 0, hi = m;
  while (lo < hi) {
    int mid = (lo + hi) >> 1;
    if (a[mid] < key)
      lo = mid + 1;
    else
      hi = mid;
  }
  return lo;
}

}  // namespace bilu
