// Tile x depth binning, LSD radix sort of (key, Gaussian id) pairs, and the
// per-tile [start, end) ranges.
//
//   count   one thread per Gaussian: number of valid tiles in its rectangle
//   scan    exclusive prefix of the counts -> write offsets, pair total
//   emit    one thread per Gaussian: key = (tile << 32) | bits(depth), value =
//           Gaussian id, tiles row-major inside the rectangle; Gaussians in
//           id order, so equal keys already sit in id order
//   sort    8-bit LSD passes over the significant key bits (32 depth bits
//           plus ceil(log2(n_tiles)) tile bits); each pass is a stable
//           counting sort: per-block digit histograms, one scan of the
//           digit-major histogram table, then a per-block stable scatter whose
//           in-block ranks come from wave ballots (a 64-lane match on the
//           8 digit bits) and a per-round digit prefix across the 4 waves
//   ranges  one thread per sorted pair marks tile boundaries
#include <algorithm>
#include <utility>

#include "scan.h"

namespace tgs {

__global__ void __launch_bounds__(256) fill_u32_kernel(uint32_t* __restrict__ p, int64_t n, uint32_t v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// ------------------------------------------------------------------ scan
__global__ void __launch_bounds__(kScanThreads) scan_reduce_kernel(const uint32_t* __restrict__ in,
                                                                  int64_t n,
                                                                  uint32_t* __restrict__ part) {
  const int64_t base = (int64_t)blockIdx.x * kScanTile;
  uint32_t s = 0;
  for (int k = 0; k < kScanItems; ++k) {
    const int64_t i = base + (int64_t)k * kScanThreads + threadIdx.x;
    if (i < n) s += in[i];
  }
  __shared__ uint32_t lds[kScanThreads / kWave];
  uint32_t total;
  block_exclusive_scan<kScanThreads>(s, lds, &total);
  if (threadIdx.x == 0) part[blockIdx.x] = total;
}

// In-place exclusive scan of the block sums by one workgroup.
__global__ void __launch_bounds__(1024) scan_partials_kernel(uint32_t* __restrict__ part,
                                                             int64_t np) {
  __shared__ uint32_t lds[1024 / kWave];
  uint32_t carry = 0;
  for (int64_t b = 0; b < np; b += 1024) {
    const int64_t i = b + threadIdx.x;
    const uint32_t v = i < np ? part[i] : 0;
    uint32_t total;
    const uint32_t ex = block_exclusive_scan<1024>(v, lds, &total);
    if (i < np) part[i] = carry + ex;
    carry += total;
  }
}

__global__ void __launch_bounds__(kScanThreads) scan_down_kernel(const uint32_t* __restrict__ in,
                                                                int64_t n,
                                                                const uint32_t* __restrict__ part,
                                                                uint32_t* __restrict__ out) {
  // each thread owns kScanItems consecutive elements
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
  uint32_t v[kScanItems];
  uint32_t s = 0;
  for (int k = 0; k < kScanItems; ++k) {
    const int64_t i = base + k;
    v[k] = i < n ? in[i] : 0;
    s += v[k];
  }
  __shared__ uint32_t lds[kScanThreads / kWave];
  uint32_t total;
  uint32_t run = part[blockIdx.x] + block_exclusive_scan<kScanThreads>(s, lds, &total);
  for (int k = 0; k < kScanItems; ++k) {
    const int64_t i = base + k;
    if (i < n) out[i] = run;
    run += v[k];
  }
  if (blockIdx.x == gridDim.x - 1 && threadIdx.x == kScanThreads - 1) out[n] = run;
}

void exclusive_scan_u32(const uint32_t* in, uint32_t* out, int64_t n, uint32_t* partials,
                        hipStream_t s) {
  const int64_t nb = scan_partials(n);
  if (nb == 0) {
    hipLaunchKernelGGL(fill_u32_kernel, dim3(1), dim3(256), 0, s, out, (int64_t)1, 0u);
    return;
  }
  hipLaunchKernelGGL(scan_reduce_kernel, dim3((unsigned)nb), dim3(kScanThreads), 0, s, in, n, partials);
  hipLaunchKernelGGL(scan_partials_kernel, dim3(1), dim3(1024), 0, s, partials, nb);
  hipLaunchKernelGGL(scan_down_kernel, dim3((unsigned)nb), dim3(kScanThreads), 0, s, in, n, partials, out);
}

// ------------------------------------------------------------------ binning
__global__ void __launch_bounds__(256) count_kernel(const int4* __restrict__ rect, int64_t n,
                                                    const int32_t* __restrict__ tile_slot,
                                                    int tiles_x, uint32_t* __restrict__ counts,
                                                    uint8_t* __restrict__ touched) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int4 r = rect[i];
  uint32_t c = 0;
  if (tile_slot == nullptr) {
    c = (uint32_t)((r.z - r.x) * (r.w - r.y));
  } else {
    for (int ty = r.y; ty < r.w; ++ty)
      for (int tx = r.x; tx < r.z; ++tx) c += tile_slot[ty * tiles_x + tx] >= 0 ? 1u : 0u;
  }
  counts[i] = c;
  if (touched != nullptr && c > 0) touched[i] = 1;
}

__global__ void __launch_bounds__(256) emit_kernel(const int4* __restrict__ rect,
                                                   const float* __restrict__ depth, int64_t n,
                                                   const int32_t* __restrict__ tile_slot,
                                                   int tiles_x, const uint32_t* __restrict__ offsets,
                                                   uint64_t* __restrict__ keys,
                                                   uint32_t* __restrict__ vals) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int4 r = rect[i];
  uint32_t o = offsets[i];
  const uint64_t dbits = (uint64_t)__float_as_uint(depth[i]);
  for (int ty = r.y; ty < r.w; ++ty)
    for (int tx = r.x; tx < r.z; ++tx) {
      const int t = ty * tiles_x + tx;
      if (tile_slot != nullptr && tile_slot[t] < 0) continue;
      keys[o] = ((uint64_t)t << 32) | dbits;
      vals[o] = (uint32_t)i;
      ++o;
    }
}

// ------------------------------------------------------------------ radix sort
constexpr int kSortThreads = 256;
constexpr int kSortRounds = 8;
constexpr int kSortTile = kSortThreads * kSortRounds;  // keys per block
constexpr int kSortWaves = kSortThreads / kWave;

__global__ void __launch_bounds__(kSortThreads) radix_hist_kernel(const uint64_t* __restrict__ keys,
                                                                 const uint32_t* __restrict__ n_dev,
                                                                 int shift, int nblocks,
                                                                 uint32_t* __restrict__ hist) {
  __shared__ uint32_t h[256];
  h[threadIdx.x] = 0;
  __syncthreads();
  const uint32_t n = *n_dev;
  const int64_t base = (int64_t)blockIdx.x * kSortTile;
  for (int k = 0; k < kSortRounds; ++k) {
    const int64_t i = base + (int64_t)k * kSortThreads + threadIdx.x;
    if (i < n) atomicAdd(&h[(keys[i] >> shift) & 255u], 1u);
  }
  __syncthreads();
  hist[(int64_t)threadIdx.x * nblocks + blockIdx.x] = h[threadIdx.x];
}

__global__ void __launch_bounds__(kSortThreads) radix_scatter_kernel(
    const uint64_t* __restrict__ keys_in, const uint32_t* __restrict__ vals_in,
    const uint32_t* __restrict__ n_dev, int shift, int nblocks, const uint32_t* __restrict__ offs,
    uint64_t* __restrict__ keys_out, uint32_t* __restrict__ vals_out) {
  __shared__ uint32_t base[256];               // running count of each digit in this block
  __shared__ uint32_t wcount[kSortWaves][256];  // per-wave digit counts of the current round
  const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
  base[tid] = offs[(int64_t)tid * nblocks + blockIdx.x];
  for (int w = 0; w < kSortWaves; ++w) wcount[w][tid] = 0;
  __syncthreads();
  const uint32_t n = *n_dev;
  const int64_t blk = (int64_t)blockIdx.x * kSortTile;
  const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  for (int k = 0; k < kSortRounds; ++k) {
    const int64_t i = blk + (int64_t)k * kSortThreads + tid;
    const bool valid = i < n;
    uint64_t key = 0;
    uint32_t val = 0;
    if (valid) {
      key = keys_in[i];
      val = vals_in[i];
    }
    const uint32_t d = (uint32_t)(key >> shift) & 255u;
    uint64_t peers = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const bool bit = (d >> b) & 1u;
      const uint64_t bal = __ballot(bit);
      peers &= bit ? bal : ~bal;
    }
    const int rank = __popcll(peers & lt_mask);
    if (valid && rank == 0) wcount[wave][d] = (uint32_t)__popcll(peers);
    __syncthreads();
    // digit tid: exclusive prefix over the waves, then advance the running base
    {
      uint32_t run = base[tid];
      for (int w = 0; w < kSortWaves; ++w) {
        const uint32_t c = wcount[w][tid];
        wcount[w][tid] = run;
        run += c;
      }
      base[tid] = run;
    }
    __syncthreads();
    if (valid) {
      const uint32_t dst = wcount[wave][d] + (uint32_t)rank;
      keys_out[dst] = key;
      vals_out[dst] = val;
    }
    __syncthreads();
    for (int w = 0; w < kSortWaves; ++w) wcount[w][tid] = 0;
    __syncthreads();
  }
}

// ------------------------------------------------------------------ ranges
__global__ void __launch_bounds__(256) ranges_kernel(const uint64_t* __restrict__ keys,
                                                     const uint32_t* __restrict__ n_dev,
                                                     uint2* __restrict__ ranges) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint32_t n = *n_dev;
  if (i >= n) return;
  const uint32_t t = (uint32_t)(keys[i] >> 32);
  if (i == 0 || (uint32_t)(keys[i - 1] >> 32) != t) ranges[t].x = (uint32_t)i;
  if (i == n - 1 || (uint32_t)(keys[i + 1] >> 32) != t) ranges[t].y = (uint32_t)(i + 1);
}

struct SortWs {
  uint32_t* counts;    // [n + 1] counts, then offsets
  uint32_t* offsets;   // [n + 1]
  uint32_t* partials;  // scan block sums
  uint32_t* hist;      // [256 * max_blocks]
  uint32_t* hoffs;     // [256 * max_blocks + 1]
  uint64_t* keys_alt;  // [capacity]
  uint32_t* vals_alt;  // [capacity]
  size_t bytes;
};

static SortWs layout(void* ws, int64_t n, int64_t capacity) {
  const int64_t max_blocks = std::max<int64_t>(1, ceil_div(capacity, kSortTile));
  const int64_t hist_n = 256 * max_blocks;
  const int64_t part_n = std::max(scan_partials(n), scan_partials(hist_n)) + 1;
  size_t off = 0;
  char* b = (char*)ws;
  SortWs w;
  auto take = [&](size_t bytes) {
    char* p = b ? b + off : nullptr;
    off += align_up(bytes, 256);
    return p;
  };
  w.counts = (uint32_t*)take(sizeof(uint32_t) * (n + 1));
  w.offsets = (uint32_t*)take(sizeof(uint32_t) * (n + 1));
  w.partials = (uint32_t*)take(sizeof(uint32_t) * part_n);
  w.hist = (uint32_t*)take(sizeof(uint32_t) * hist_n);
  w.hoffs = (uint32_t*)take(sizeof(uint32_t) * (hist_n + 1));
  w.keys_alt = (uint64_t*)take(sizeof(uint64_t) * std::max<int64_t>(capacity, 1));
  w.vals_alt = (uint32_t*)take(sizeof(uint32_t) * std::max<int64_t>(capacity, 1));
  w.bytes = off;
  return w;
}

static int key_tile_bits(int n_tiles) {
  int b = 0;
  while ((1ll << b) < (long long)n_tiles) ++b;
  return b;
}

}  // namespace tgs

using namespace tgs;

extern "C" size_t tgs_bin_sort_workspace_size(int64_t n, int64_t capacity, int32_t n_tiles) {
  (void)n_tiles;
  if (n < 0 || capacity < 0) return 0;
  return layout(nullptr, n, capacity).bytes;
}

extern "C" int32_t tgs_bin_sort(const int32_t* rect, const float* depth, int64_t n,
                                const int32_t* tile_slot, int32_t tiles_x, int32_t tiles_y,
                                uint64_t* keys, uint32_t* vals, int64_t capacity, uint32_t* ranges,
                                uint8_t* touched, int64_t* n_pairs, void* ws, size_t ws_bytes,
                                void* stream) {
  TGS_REQUIRE(n >= 0 && n < (1ll << 32), "tgs_bin_sort: n out of range");
  TGS_REQUIRE(tiles_x > 0 && tiles_y > 0 && (int64_t)tiles_x * tiles_y < (1ll << 31),
              "tgs_bin_sort: bad tile grid");
  TGS_REQUIRE(capacity >= 0 && capacity < (1ll << 32), "tgs_bin_sort: capacity out of range");
  TGS_REQUIRE(keys && vals && ranges && n_pairs && ws, "tgs_bin_sort: null pointer");
  TGS_REQUIRE(n == 0 || (rect && depth), "tgs_bin_sort: null rect/depth");
  TGS_REQUIRE(((uintptr_t)rect & 15) == 0, "tgs_bin_sort: rect must be 16-byte aligned");
  const SortWs w = layout(ws, n, capacity);
  TGS_REQUIRE(ws_bytes >= w.bytes, "tgs_bin_sort: workspace %zu bytes < %zu", ws_bytes, w.bytes);
  hipStream_t s = as_stream(stream);
  const int64_t n_t = (int64_t)tiles_x * tiles_y;

  hipLaunchKernelGGL(fill_u32_kernel, dim3((unsigned)ceil_div(2 * n_t, 256)), dim3(256), 0, s,
                     ranges, 2 * n_t, 0u);
  if (n > 0)
    hipLaunchKernelGGL(count_kernel, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, s,
                       (const int4*)rect, n, tile_slot, tiles_x, w.counts, touched);
  exclusive_scan_u32(w.counts, w.offsets, n, w.partials, s);
  uint32_t total = 0;
  if (hipMemcpyAsync(&total, w.offsets + n, sizeof(uint32_t), hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return hip_status("tgs_bin_sort: pair count readback");
  *n_pairs = total;
  if ((int64_t)total > capacity) {
    set_error("tgs_bin_sort: %u pairs exceed capacity %lld", total, (long long)capacity);
    return TGS_ERR_CAPACITY;
  }
  if (total == 0) return hip_status("tgs_bin_sort");

  const int bits = 32 + key_tile_bits((int)n_t);
  const int passes = (bits + 7) / 8;
  // emit so that the last pass lands in the caller's buffers
  uint64_t* kA = keys;
  uint32_t* vA = vals;
  uint64_t* kB = w.keys_alt;
  uint32_t* vB = w.vals_alt;
  uint64_t* k_src = (passes % 2 == 0) ? kA : kB;
  uint32_t* v_src = (passes % 2 == 0) ? vA : vB;
  uint64_t* k_dst = (passes % 2 == 0) ? kB : kA;
  uint32_t* v_dst = (passes % 2 == 0) ? vB : vA;
  hipLaunchKernelGGL(emit_kernel, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, s,
                     (const int4*)rect, depth, n, tile_slot, tiles_x, w.offsets, k_src, v_src);
  const uint32_t* n_dev = w.offsets + n;
  const int nblocks = (int)ceil_div(total, kSortTile);
  for (int p = 0; p < passes; ++p) {
    const int shift = 8 * p;
    hipLaunchKernelGGL(radix_hist_kernel, dim3(nblocks), dim3(kSortThreads), 0, s, k_src, n_dev,
                       shift, nblocks, w.hist);
    exclusive_scan_u32(w.hist, w.hoffs, (int64_t)256 * nblocks, w.partials, s);
    hipLaunchKernelGGL(radix_scatter_kernel, dim3(nblocks), dim3(kSortThreads), 0, s, k_src, v_src,
                       n_dev, shift, nblocks, w.hoffs, k_dst, v_dst);
    std::swap(k_src, k_dst);
    std::swap(v_src, v_dst);
  }
  hipLaunchKernelGGL(ranges_kernel, dim3((unsigned)ceil_div(total, 256)), dim3(256), 0, s, keys, n_dev,
                     (uint2*)ranges);
  return hip_status("tgs_bin_sort");
}
