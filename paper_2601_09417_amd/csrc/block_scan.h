// Wave64 and 256-thread block scans shared by the scan, sort and selection kernels.
#pragma once

#include <hip/hip_runtime.h>

#include "common.h"

namespace vbm {

constexpr int kScanThreads = 256;
constexpr int kScanWaves = kScanThreads / 64;

// Inclusive scan across the 64 lanes of a wave.
template <class T>
__device__ __forceinline__ T wave_incl_scan(T v) {
  const uint32_t lane = lane_id();
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    T o = __shfl_up(v, d, 64);
    if (lane >= static_cast<uint32_t>(d)) v += o;
  }
  return v;
}

// Exclusive scan of one value per thread across a 256-thread block; block total in *total.
// Every thread of the block must call it (it synchronises).
template <class T>
__device__ __forceinline__ T block_excl_scan(T v, T* total) {
  __shared__ T s_wave[kScanWaves];
  const int w = threadIdx.x >> 6;
  T incl = wave_incl_scan(v);
  if (lane_id() == 63) s_wave[w] = incl;
  __syncthreads();
  T base = 0, tot = 0;
#pragma unroll
  for (int i = 0; i < kScanWaves; ++i) {
    T x = s_wave[i];
    if (i < w) base += x;
    tot += x;
  }
  __syncthreads();
  *total = tot;
  return base + incl - v;
}

}  // namespace vbm
