// Device-wide exclusive prefix sum of uint32 values (three launches:
// per-block reduce, scan of the block sums in one workgroup, per-block scan
// with the block's offset).  out[n] receives the total.
#pragma once

#include "common.h"

namespace tgs {

constexpr int kScanThreads = 256;
constexpr int kScanItems = 8;
constexpr int kScanTile = kScanThreads * kScanItems;

inline int64_t scan_partials(int64_t n) { return ceil_div(n, kScanTile); }

// Workgroup-wide exclusive scan of one value per thread; returns the
// exclusive prefix and writes the workgroup total to *total.
template <int kThreads>
__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t v, uint32_t* lds_waves,
                                                         uint32_t* total) {
  constexpr int kWaves = kThreads / kWave;
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  const uint32_t incl = wave_inclusive_scan_u32(v);
  if (lane == kWave - 1) lds_waves[wave] = incl;
  __syncthreads();
  uint32_t wave_off = 0, sum = 0;
  for (int w = 0; w < kWaves; ++w) {
    const uint32_t c = lds_waves[w];
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
