// Device-wide exclusive prefix sums (three launches: per-block reduce, scan
// of the block sums in one workgroup, per-block scan with the block's
// offset).  out[n] receives the total.
#pragma once

#include "common.h"

namespace tgs {

constexpr int kScanThreads = 256;
constexpr int kScanItems = 8;
constexpr int kScanTile = kScanThreads * kScanItems;

inline int64_t scan_partials(int64_t n) { return ceil_div(n, kScanTile); }

template <typename T>
__device__ __forceinline__ T wave_inclusive_scan_t(T v) {
  const int lane = lane_id();
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    T t = __shfl_up(v, o, kWave);
    if (lane >= o) v += t;
  }
  return v;
}

// Workgroup-wide exclusive scan of one value per thread; returns the
// exclusive prefix and writes the workgroup total to *total.
template <int kThreads, typename T>
__device__ __forceinline__ T block_exclusive_scan(T v, T* lds_waves, T* total) {
  constexpr int kWaves = kThreads / kWave;
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  const T incl = wave_inclusive_scan_t<T>(v);
  if (lane == kWave - 1) lds_waves[wave] = incl;
  __syncthreads();
  T wave_off = 0, sum = 0;
  for (int w = 0; w < kWaves; ++w) {
    const T c = lds_waves[w];
    if (w < wave) wave_off += c;
    sum += c;
  }
  __syncthreads();
  *total = sum;
  return wave_off + incl - v;
}

void exclusive_scan_u32(const uint32_t* in, uint32_t* out, int64_t n, uint32_t* partials,
                        hipStream_t s);

}  // namespace tgs
