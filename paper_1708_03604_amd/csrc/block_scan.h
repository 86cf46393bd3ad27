// Exclusive prefix sum over one workgroup, shared by the symbolic pass, the
// class lists of the small-block path and the device-wide scans.
#pragma once

#include <hip/hip_runtime.h>

namespace bsmm {

// Exclusive scan of v over a workgroup of kThreads threads (whole waves):
// an inclusive scan within each wave by shuffles, then the wave sums through
// LDS.  *total receives the workgroup sum.  Every thread of the workgroup
// must call it (it holds two barriers).
template <int kThreads, class T>
__device__ __forceinline__ T block_exclusive_scan(T v, T* total) {
  static_assert(kThreads % 64 == 0 && kThreads <= 1024, "whole waves");
  __shared__ T wsum[kThreads / 64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  T x = v;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const T y = __shfl_up(x, d, 64);
    if (lane >= d) x += y;
  }
  if (lane == 63) wsum[wave] = x;
  __syncthreads();
  T off = 0, tot = 0;
#pragma unroll
  for (int w = 0; w < kThreads / 64; ++w) {
    if (w < wave) off += wsum[w];
    tot += wsum[w];
  }
  __syncthreads();
  *total = tot;
  return off + x - v;
}

}  // namespace bsmm
