// Tile x depth binning, sort and per-tile ranges.
//
// The per-tile Gaussian lists must follow (tile, FP32 depth bits, Gaussian
// id).  Rather than radix-sorting a 64-bit (tile, depth) key with an id for
// every (Gaussian, tile) pair, the Gaussians are put in (depth, id) order once
// (a 32-bit sort of n keys) and the pairs are emitted in that order; a
// stable sort on the tile bits alone then yields the full order.  The pair
// key is (tile << id_bits) | Gaussian id, usually 32 bits: the id bits only
// ride along, since a stable sort never compares them.
//
//   count     per Gaussian: rectangle area, visibility, touched flag and the
//             depth key (culled Gaussians get a key above every depth); the
//             rectangle's four corners go into a 2-D difference grid, whose
//             prefix sums are the per-tile pair counts
//   sort      LSD radix sort of (depth key, id) over n: stable, so ties keep
//             id order; visible Gaussians come first
//   gather    rectangles and pair counts in depth order, exclusive scan ->
//             pair offsets and the total (read back once)
//   ranges    2-D prefix of the difference grid, then a scan over the valid
//             tiles in tile order: each tile's [start, end)
//   emit      4096 pairs per workgroup: the Gaussians that start inside the
//             block mark their first slot in LDS and a max-scan hands every
//             slot its Gaussian (a load-balanced search); keys are written
//             coalesced, tiles outside the valid set get the sentinel tile
//             id n_tiles (after every real tile), and the block's histogram
//             of the first radix digit is taken on the way
//   sort      LSD radix sort of the pair keys on the tile bits only; the
//             last pass writes the ids (and, if asked, the 64-bit keys)
//
// A radix pass is a stable counting sort over blocks of 256 x kItems keys:
// per-block digit histograms (peer lanes found by a ballot match add their
// count once), one scan of the digit-major histogram table, and a scatter
// that ranks the block's keys (each wave owns a contiguous quarter of the
// block), reorders them by digit in LDS and writes runs of equal digits to
// consecutive addresses.
#include <algorithm>
#include <utility>

#include "scan.h"

namespace tgs {

__global__ void __launch_bounds__(256) fill_u32_kernel(uint32_t* __restrict__ p, int64_t n, uint32_t v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// ------------------------------------------------------------------ scans
template <typename T>
__global__ void __launch_bounds__(kScanThreads) scan_reduce_kernel(const T* __restrict__ in, int64_t n,
                                                                  T* __restrict__ part) {
  const int64_t base = (int64_t)blockIdx.x * kScanTile;
  T s = 0;
  for (int k = 0; k < kScanItems; ++k) {
    const int64_t i = base + (int64_t)k * kScanThreads + threadIdx.x;
    if (i < n) s += in[i];
  }
  __shared__ T lds[kScanThreads / kWave];
  T total;
  block_exclusive_scan<kScanThreads, T>(s, lds, &total);
  if (threadIdx.x == 0) part[blockIdx.x] = total;
}

template <typename T>
__global__ void __launch_bounds__(1024) scan_partials_kernel(T* __restrict__ part, int64_t np) {
  __shared__ T lds[1024 / kWave];
  T carry = 0;
  for (int64_t b = 0; b < np; b += 1024) {
    const int64_t i = b + threadIdx.x;
    const T v = i < np ? part[i] : 0;
    T total;
    const T ex = block_exclusive_scan<1024, T>(v, lds, &total);
    if (i < np) part[i] = carry + ex;
    carry += total;
  }
}

template <typename T>
__global__ void __launch_bounds__(kScanThreads) scan_down_kernel(const T* __restrict__ in, int64_t n,
                                                                const T* __restrict__ part,
                                                                T* __restrict__ out) {
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
  T v[kScanItems];
  T s = 0;
  for (int k = 0; k < kScanItems; ++k) {
    const int64_t i = base + k;
    v[k] = i < n ? in[i] : 0;
    s += v[k];
  }
  __shared__ T lds[kScanThreads / kWave];
  T total;
  T run = part[blockIdx.x] + block_exclusive_scan<kScanThreads, T>(s, lds, &total);
  for (int k = 0; k < kScanItems; ++k) {
    const int64_t i = base + k;
    if (i < n) out[i] = run;
    run += v[k];
  }
  if (blockIdx.x == gridDim.x - 1 && threadIdx.x == kScanThreads - 1) out[n] = run;
}

template <typename T>
__global__ void __launch_bounds__(64) set_kernel(T* __restrict__ p, T v) {
  if (threadIdx.x == 0) *p = v;
}

template <typename T>
static void exclusive_scan(const T* in, T* out, int64_t n, T* partials, hipStream_t s) {
  const int64_t nb = scan_partials(n);
  if (nb == 0) {
    hipLaunchKernelGGL(set_kernel<T>, dim3(1), dim3(64), 0, s, out, (T)0);
    return;
  }
  hipLaunchKernelGGL(scan_reduce_kernel<T>, dim3((unsigned)nb), dim3(kScanThreads), 0, s, in, n, partials);
  hipLaunchKernelGGL(scan_partials_kernel<T>, dim3(1), dim3(1024), 0, s, partials, nb);
  hipLaunchKernelGGL(scan_down_kernel<T>, dim3((unsigned)nb), dim3(kScanThreads), 0, s, in, n, partials, out);
}



// ------------------------------------------------------------------ count
// Depth key of a culled Gaussian: above every finite positive depth bit pattern.
constexpr uint32_t kCulledKey = 0xffffffffu;

// Rectangles are clamped to the tile grid (projection already does so; the
// clamp keeps every index of the binning in bounds for any input).
__device__ __forceinline__ int4 clamp_rect(int4 r, int tiles_x, int tiles_y) {
  r.x = min(max(r.x, 0), tiles_x);
  r.z = min(max(r.z, r.x), tiles_x);
  r.y = min(max(r.y, 0), tiles_y);
  r.w = min(max(r.w, r.y), tiles_y);
  return r;
}

// Difference grid of the pair counts: (tiles_y + 1) x (tiles_x + 1) cells; a
// Gaussian with a pair adds +1 at (y0, x0) and (y1, x1), -1 at (y0, x1) and
// (y1, x0), so the 2-D inclusive prefix sum at (ty, tx) counts the rectangles
// that cover tile (tx, ty).  Each count workgroup accumulates its own grid in
// LDS and writes it out whole (contended device-wide atomics are slow), and
// the grids are summed per cell afterwards.  Grids above kLdsCells cells use
// device atomics on a single grid instead.
constexpr int kCountThreads = 1024;
constexpr int kCountBlocks = 64;   // at most; partial grids to sum
constexpr int kLdsCells = 12288;   // 48 KiB of LDS

__global__ void __launch_bounds__(kCountThreads) count_kernel(const int4* __restrict__ rect,
                                                              const float* __restrict__ depth, int64_t n,
                                                              const int32_t* __restrict__ tile_slot, int tiles_x,
                                                              int tiles_y, uint32_t* __restrict__ dkeys,
                                                              uint32_t* __restrict__ dvals,
                                                              uint8_t* __restrict__ touched,
                                                              int32_t* __restrict__ partial, bool lds_grid,
                                                              unsigned long long* __restrict__ valid_total) {
  __shared__ int32_t s_diff[kLdsCells];
  __shared__ uint32_t lds[kCountThreads / kWave];
  const int gw = tiles_x + 1;
  const int cells = gw * (tiles_y + 1);
  if (lds_grid) {
    for (int c = threadIdx.x; c < cells; c += kCountThreads) s_diff[c] = 0;
    __syncthreads();
  }
  int32_t* gdiff = lds_grid ? s_diff : partial;
  uint32_t valid_sum = 0;
  for (int64_t i = (int64_t)blockIdx.x * kCountThreads + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kCountThreads) {
    const int4 r = clamp_rect(rect[i], tiles_x, tiles_y);
    const uint32_t area = (uint32_t)((r.z - r.x) * (r.w - r.y));
    uint32_t valid = 0;
    if (tile_slot == nullptr) {
      valid = area;
    } else {
      for (int ty = r.y; ty < r.w; ++ty)
        for (int tx = r.x; tx < r.z; ++tx) valid += tile_slot[ty * tiles_x + tx] >= 0 ? 1u : 0u;
    }
    dkeys[i] = valid > 0 ? __float_as_uint(depth[i]) : kCulledKey;
    dvals[i] = (uint32_t)i;
    if (valid > 0) {
      atomicAdd(&gdiff[r.y * gw + r.x], 1);
      atomicAdd(&gdiff[r.y * gw + r.z], -1);
      atomicAdd(&gdiff[r.w * gw + r.x], -1);
      atomicAdd(&gdiff[r.w * gw + r.z], 1);
      if (touched != nullptr) touched[i] = 1;
    }
    valid_sum += valid;
  }
  if (tile_slot != nullptr) {  // pairs in valid tiles, spread over the slots
    uint32_t tot;
    block_exclusive_scan<kCountThreads, uint32_t>(valid_sum, lds, &tot);
    if (threadIdx.x == 0 && tot > 0)
      atomicAdd(&valid_total[blockIdx.x & (TGS_COUNTER_SLOTS - 1)], (unsigned long long)tot);
  }
  if (lds_grid) {
    __syncthreads();
    int32_t* out = partial + (int64_t)blockIdx.x * cells;
    for (int c = threadIdx.x; c < cells; c += kCountThreads) out[c] = s_diff[c];
  }
}

// diff[c] = sum over the partial grids of cell c: 64 cells per workgroup
// (a lane each), its 8 waves take every 8th grid, then LDS combines them.
constexpr int kSumWaves = 8;

__global__ void __launch_bounds__(kSumWaves * kWave) diff_sum_kernel(const int32_t* __restrict__ partial,
                                                                     int n_grids, int cells,
                                                                     int32_t* __restrict__ diff) {
  __shared__ int32_t s_part[kSumWaves][kWave];
  const int lane = lane_id(), wave = threadIdx.x / kWave;
  const int c = blockIdx.x * kWave + lane;
  int32_t acc = 0;
  if (c < cells)
    for (int b = wave; b < n_grids; b += kSumWaves) acc += partial[(int64_t)b * cells + c];
  s_part[wave][lane] = acc;
  __syncthreads();
  if (wave == 0 && c < cells) {
    int32_t t = 0;
#pragma unroll
    for (int w = 0; w < kSumWaves; ++w) t += s_part[w][lane];
    diff[c] = t;
  }
}

// Rectangles and pair counts in depth order (a Gaussian without a valid tile
// has the culled key and sits after the visible ones; its count is 0).
__global__ void __launch_bounds__(256) gather_kernel(const uint32_t* __restrict__ perm,
                                                     const uint32_t* __restrict__ dkeys_sorted,
                                                     const int4* __restrict__ rect, int64_t n,
                                                     int tiles_x, int tiles_y,
                                                     int4* __restrict__ rect_sorted,
                                                     uint32_t* __restrict__ area_sorted) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  const int4 r = clamp_rect(rect[perm[j]], tiles_x, tiles_y);
  rect_sorted[j] = r;
  area_sorted[j] = dkeys_sorted[j] == kCulledKey ? 0u : (uint32_t)((r.z - r.x) * (r.w - r.y));
}

// ------------------------------------------------------------------ ranges
// One workgroup: 2-D inclusive prefix of the difference grid (rows, then
// columns; in LDS when it fits), then an exclusive scan of the valid tiles'
// counts in tile order.  Empty and invalid tiles get [0, 0).
constexpr int kRangeThreads = 1024;

__global__ void __launch_bounds__(kRangeThreads) ranges_kernel(int32_t* __restrict__ diff, int tiles_x,
                                                               int tiles_y, const int32_t* __restrict__ tile_slot,
                                                               uint2* __restrict__ ranges) {
  __shared__ int32_t s_grid[kLdsCells];
  __shared__ uint32_t lds[kRangeThreads / kWave];
  const int gw = tiles_x + 1;
  const int cells = gw * (tiles_y + 1);
  const bool in_lds = cells <= kLdsCells;
  int32_t* g = in_lds ? s_grid : diff;
  if (in_lds) {
    for (int c = threadIdx.x; c < cells; c += kRangeThreads) s_grid[c] = diff[c];
    __syncthreads();
  }
  // rows: one wave per row, 64 columns per step with a wave scan
  const int lane = lane_id(), wave = threadIdx.x / kWave;
  for (int y = wave; y < tiles_y; y += kRangeThreads / kWave) {
    int32_t* row = g + (int64_t)y * gw;
    int32_t carry = 0;
    for (int x0 = 0; x0 < tiles_x; x0 += kWave) {
      const int x = x0 + lane;
      const int32_t v = x < tiles_x ? row[x] : 0;
      const int32_t incl = wave_inclusive_scan_i(v) + carry;
      if (x < tiles_x) row[x] = incl;
      carry = __shfl(incl, kWave - 1, kWave);
    }
  }
  __syncthreads();
  // columns: a thread per column
  for (int x = threadIdx.x; x < tiles_x; x += kRangeThreads) {
    int32_t acc = 0;
#pragma unroll 8
    for (int y = 0; y < tiles_y; ++y) {
      acc += g[(int64_t)y * gw + x];
      g[(int64_t)y * gw + x] = acc;
    }
  }
  __syncthreads();
  const int n_t = tiles_x * tiles_y;
  uint32_t carry = 0;
  for (int t0 = 0; t0 < n_t; t0 += kRangeThreads) {
    const int t = t0 + (int)threadIdx.x;
    uint32_t c = 0;
    if (t < n_t && (tile_slot == nullptr || tile_slot[t] >= 0))
      c = (uint32_t)g[(int64_t)(t / tiles_x) * gw + (t % tiles_x)];
    uint32_t tot;
    const uint32_t start = carry + block_exclusive_scan<kRangeThreads, uint32_t>(c, lds, &tot);
    if (t < n_t) ranges[t] = c > 0 ? make_uint2(start, start + c) : make_uint2(0u, 0u);
    carry += tot;
  }
}

// ------------------------------------------------------------------ radix sort
constexpr int kSortThreads = 256;
constexpr int kSortWaves = kSortThreads / kWave;
constexpr int kPairItems = 16;  // keys per thread of the pair sort (and of emit)

// Keys per thread: 16 for large sorts, 4 for small ones (more workgroups).
static int sort_items(int64_t n) { return n >= (1ll << 20) ? 16 : 4; }

static int64_t sort_blocks(int64_t n, int items) { return ceil_div(n, (int64_t)kSortThreads * items); }

__device__ __forceinline__ uint64_t lanes_below() {
  const int lane = lane_id();
  return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

// Lanes of the wave holding the same kBits-bit digit (inactive lanes excluded).
template <int kBits>
__device__ __forceinline__ uint64_t digit_peers(uint32_t d, bool valid) {
  uint64_t peers = __ballot(valid);
#pragma unroll
  for (int b = 0; b < kBits; ++b) {
    const bool bit = (d >> b) & 1u;
    const uint64_t bal = __ballot(bit);
    peers &= bit ? bal : ~bal;
  }
  return peers;
}

// Per-block histogram: block b covers keys [b * 256 * kItems, ...), wave w
// the contiguous quarter w of it, 64 keys per round.
template <typename K, int kBits, int kItems>
__global__ void __launch_bounds__(kSortThreads) radix_hist_kernel(const K* __restrict__ keys, uint32_t n,
                                                                 int shift, int nblocks,
                                                                 uint32_t* __restrict__ hist) {
  constexpr int kDigits = 1 << kBits;
  __shared__ uint32_t h[kDigits];
  for (int i = threadIdx.x; i < kDigits; i += kSortThreads) h[i] = 0;
  const int lane = lane_id(), wave = threadIdx.x / kWave;
  const int64_t wbase = (int64_t)blockIdx.x * kSortThreads * kItems + (int64_t)wave * kWave * kItems;
  K key[kItems];
#pragma unroll
  for (int k = 0; k < kItems; ++k) {
    const int64_t i = wbase + k * kWave + lane;
    key[k] = i < n ? keys[i] : (K)0;
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < kItems; ++k)
    if (wbase + k * kWave + lane < n) atomicAdd(&h[(uint32_t)(key[k] >> shift) & (kDigits - 1u)], 1u);
  __syncthreads();
  for (int dg = threadIdx.x; dg < kDigits; dg += kSortThreads)
    hist[(int64_t)dg * nblocks + blockIdx.x] = h[dg];
}

// One workgroup per digit: exclusive prefix of the digit's per-block counts
// (a contiguous row of the digit-major table) and the digit's total.
__global__ void __launch_bounds__(1024) digit_scan_kernel(const uint32_t* __restrict__ hist, int nblocks,
                                                          uint32_t* __restrict__ hoffs,
                                                          uint32_t* __restrict__ dtot) {
  __shared__ uint32_t lds[1024 / kWave];
  const int64_t row = (int64_t)blockIdx.x * nblocks;
  uint32_t carry = 0;
  for (int b0 = 0; b0 < nblocks; b0 += 1024) {
    const int b = b0 + (int)threadIdx.x;
    const uint32_t v = b < nblocks ? hist[row + b] : 0u;
    uint32_t tot;
    const uint32_t ex = block_exclusive_scan<1024, uint32_t>(v, lds, &tot);
    if (b < nblocks) hoffs[row + b] = carry + ex;
    carry += tot;
  }
  if (threadIdx.x == 0) dtot[blockIdx.x] = carry;
}

// Output of a scatter pass: keys (and values) for the next pass, or, in the
// last pass of the pair sort, the Gaussian ids carried in the low key bits
// and optionally the 64-bit (tile << 32) | depth-bits keys.
struct ScatterOut {
  void* keys;
  uint32_t* vals;
  int id_bits;           // final pass: key = (tile << id_bits) | id
  const float* depth;    // final pass, for keys64
  uint64_t* keys64;      // final pass, nullable
};

template <typename K, bool kVals, bool kFinal, int kBits, int kItems>
__global__ void __launch_bounds__(kSortThreads) radix_scatter_kernel(
    const K* __restrict__ keys_in, const uint32_t* __restrict__ vals_in, uint32_t n, int shift, int nblocks,
    const uint32_t* __restrict__ offs, const uint32_t* __restrict__ dtot, ScatterOut o) {
  constexpr int kDigits = 1 << kBits;
  constexpr int kBlockKeys = kSortThreads * kItems;
  __shared__ uint32_t s_cnt[kSortWaves][kDigits];  // per-wave digit counts, then block-local offsets
  __shared__ uint32_t s_gbase[kDigits];            // global position of block-local position 0 of the digit
  __shared__ K s_keys[kBlockKeys];
  __shared__ uint32_t s_vals[kVals ? kBlockKeys : 1];
  __shared__ uint32_t s_red[kSortWaves];
  const int tid = threadIdx.x, lane = lane_id(), wave = tid / kWave;
  for (int i = tid; i < kSortWaves * kDigits; i += kSortThreads) (&s_cnt[0][0])[i] = 0;
  const int64_t blk0 = (int64_t)blockIdx.x * kBlockKeys;
  const int64_t wbase = blk0 + (int64_t)wave * kWave * kItems;
  K key[kItems];
  uint32_t val[kItems];
#pragma unroll
  for (int k = 0; k < kItems; ++k) {
    const int64_t i = wbase + k * kWave + lane;
    key[k] = i < n ? keys_in[i] : (K)0;
    if (kVals) val[k] = i < n ? vals_in[i] : 0u;
  }
  __syncthreads();
  // rank of each key among the wave's keys of the same digit (stable: by
  // round, then lane); the wave's running counts live in s_cnt[wave]
  const uint64_t below = lanes_below();
  uint32_t rank[kItems];
#pragma unroll
  for (int k = 0; k < kItems; ++k) {
    const bool valid = wbase + k * kWave + lane < n;
    const uint32_t d = (uint32_t)(key[k] >> shift) & (kDigits - 1u);
    const uint64_t peers = digit_peers<kBits>(d, valid);
    const uint32_t r = (uint32_t)__popcll(peers & below);
    const uint32_t before = valid ? s_cnt[wave][d] : 0u;
    rank[k] = before + r;
    if (valid && r == 0) s_cnt[wave][d] = before + (uint32_t)__popcll(peers);
  }
  __syncthreads();
  // block-local start of each (digit, wave) and the digit's global base
  uint32_t pre[kSortWaves];
  uint32_t tot = 0;
  if (tid < kDigits)
    for (int w = 0; w < kSortWaves; ++w) {
      pre[w] = tot;
      tot += s_cnt[w][tid];
    }
  uint32_t all;
  const uint32_t lstart = block_exclusive_scan<kSortThreads, uint32_t>(tid < kDigits ? tot : 0u, s_red, &all);
  const uint32_t gstart =
      block_exclusive_scan<kSortThreads, uint32_t>(tid < kDigits ? dtot[tid] : 0u, s_red, &all);
  if (tid < kDigits) {
    for (int w = 0; w < kSortWaves; ++w) s_cnt[w][tid] = lstart + pre[w];
    s_gbase[tid] = gstart + offs[(int64_t)tid * nblocks + blockIdx.x] - lstart;
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < kItems; ++k) {
    if (wbase + k * kWave + lane < n) {
      const uint32_t d = (uint32_t)(key[k] >> shift) & (kDigits - 1u);
      const uint32_t lp = s_cnt[wave][d] + rank[k];
      s_keys[lp] = key[k];
      if (kVals) s_vals[lp] = val[k];
    }
  }
  __syncthreads();
  // runs of equal digits go to consecutive addresses
  const int count = (int)min((int64_t)kBlockKeys, (int64_t)n - blk0);
#pragma unroll
  for (int k = 0; k < kItems; ++k) {
    const int lp = k * kSortThreads + tid;
    if (lp < count) {
      const K kk = s_keys[lp];
      const uint32_t dst = s_gbase[(uint32_t)(kk >> shift) & (kDigits - 1u)] + (uint32_t)lp;
      if (kFinal) {
        const uint32_t g = (uint32_t)(kk & (((K)1 << o.id_bits) - 1));
        o.vals[dst] = g;
        if (o.keys64 != nullptr)
          o.keys64[dst] = ((uint64_t)(kk >> o.id_bits) << 32) | (uint64_t)__float_as_uint(o.depth[g]);
      } else {
        ((K*)o.keys)[dst] = kk;
        if (kVals) o.vals[dst] = s_vals[lp];
      }
    }
  }
}

// One radix pass over n keys on bits [shift, shift + kBits); the histogram
// table is taken here unless the caller already wrote it (hist_ready).
template <typename K, bool kVals, bool kFinal, int kBits, int kItems>
static void radix_pass(const K* keys, const uint32_t* vals, uint32_t n, int shift, bool hist_ready,
                       uint32_t* hist, uint32_t* hoffs, uint32_t* dtot, const ScatterOut& o, hipStream_t s) {
  const int nblocks = (int)sort_blocks(n, kItems);
  if (!hist_ready)
    hipLaunchKernelGGL((radix_hist_kernel<K, kBits, kItems>), dim3(nblocks), dim3(kSortThreads), 0, s, keys, n,
                       shift, nblocks, hist);
  hipLaunchKernelGGL(digit_scan_kernel, dim3(1 << kBits), dim3(1024), 0, s, hist, nblocks, hoffs, dtot);
  hipLaunchKernelGGL((radix_scatter_kernel<K, kVals, kFinal, kBits, kItems>), dim3(nblocks), dim3(kSortThreads),
                     0, s, keys, vals, n, shift, nblocks, hoffs, dtot, o);
}

template <typename K, bool kVals, bool kFinal, int kItems>
static void radix_pass_bits(int bits, const K* keys, const uint32_t* vals, uint32_t n, int shift,
                            bool hist_ready, uint32_t* hist, uint32_t* hoffs, uint32_t* dtot,
                            const ScatterOut& o, hipStream_t s) {
  switch (bits) {
#define TGS_PASS(B) \
  case B: radix_pass<K, kVals, kFinal, B, kItems>(keys, vals, n, shift, hist_ready, hist, hoffs, dtot, o, s); break;
    TGS_PASS(1) TGS_PASS(2) TGS_PASS(3) TGS_PASS(4) TGS_PASS(5) TGS_PASS(6) TGS_PASS(7)
    default: radix_pass<K, kVals, kFinal, 8, kItems>(keys, vals, n, shift, hist_ready, hist, hoffs, dtot, o, s);
#undef TGS_PASS
  }
}

// Passes of at most 8 bits over [lo, lo + bits), split evenly.
static int pass_count(int bits) { return (bits + 7) / 8; }
static int pass_bits(int bits, int p) {
  const int per = (bits + pass_count(bits) - 1) / pass_count(bits);
  return std::min(per, bits - p * per);
}

// ------------------------------------------------------------------ emit
constexpr int kEmitThreads = kSortThreads;
constexpr int kEmitTile = kSortThreads * kPairItems;  // = a pair-sort block
constexpr int kEmitWin = 512;                          // Gaussians staged in LDS per block

// block_j0[b]: the Gaussian (depth position) holding pair b * kEmitTile.
__global__ void __launch_bounds__(256) block_start_kernel(const uint32_t* __restrict__ off, int64_t n,
                                                          int32_t* __restrict__ block_j0) {
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (j >= n) return;
  const uint32_t a = off[j], e = off[j + 1];
  for (uint32_t b = (uint32_t)ceil_div(a, kEmitTile); (uint64_t)b * kEmitTile < e; ++b) block_j0[b] = (int32_t)j;
}

// q = a / b and r = a % b for b > 0: below 2^22 a float estimate of the
// quotient is off by at most one and is corrected; larger a divide exactly.
__device__ __forceinline__ void divmod_small(uint32_t a, uint32_t b, uint32_t& q, uint32_t& r) {
  if (a >= (1u << 22)) {
    q = a / b;
    r = a - q * b;
    return;
  }
  int qi = (int)((float)a * __builtin_amdgcn_rcpf((float)b));
  int ri = (int)a - qi * (int)b;
  if (ri < 0) { --qi; ri += (int)b; }
  if (ri >= (int)b) { ++qi; ri -= (int)b; }
  q = (uint32_t)qi;
  r = (uint32_t)ri;
}

// Pairs [p0, p0 + kEmitTile) of the depth-ordered pair list.  The Gaussians
// that start inside the block (and j0, which holds p0) mark their first slot
// with their index relative to j0 and stage rectangle, offset and id in LDS;
// an inclusive max-scan then gives every slot its Gaussian.  Every
// Gaussian before the culled tail has at least one pair, so the marked
// slots are distinct.
template <typename K, int kBits0>
__global__ void __launch_bounds__(kEmitThreads) emit_kernel(
    const int4* __restrict__ rect_sorted, const uint32_t* __restrict__ ids_sorted,
    const uint32_t* __restrict__ off, const int32_t* __restrict__ block_j0, int64_t n, uint32_t total,
    const int32_t* __restrict__ tile_slot, int tiles_x, uint32_t n_t, int id_bits, K* __restrict__ keys,
    int nblocks, uint32_t* __restrict__ hist) {
  constexpr int kDigits = 1 << kBits0;
  __shared__ int32_t s_j[kEmitTile];
  __shared__ int4 s_rect[kEmitWin];
  __shared__ uint32_t s_off[kEmitWin];
  __shared__ uint32_t s_id[kEmitWin];
  __shared__ uint32_t s_h[kDigits];
  __shared__ int32_t s_red[kEmitThreads / kWave];
  const int tid = threadIdx.x;
  const uint32_t p0 = blockIdx.x * (uint32_t)kEmitTile;
  const uint32_t p_end = min(total, p0 + (uint32_t)kEmitTile);
  for (int i = tid; i < kEmitTile; i += kEmitThreads) s_j[i] = -1;
  for (int i = tid; i < kDigits; i += kEmitThreads) s_h[i] = 0;
  const int64_t j0 = block_j0[blockIdx.x];
  __syncthreads();
  for (int jb = 0;; jb += kEmitThreads) {
    const int jl = jb + tid;
    const int64_t j = j0 + jl;
    bool in = false;
    if (j < n) {
      const uint32_t o = off[j];
      in = jl == 0 || o < p_end;
      if (in) {
        s_j[jl == 0 ? 0 : (int)(o - p0)] = jl;
        if (jl < kEmitWin) {
          s_rect[jl] = rect_sorted[j];
          s_off[jl] = o;
          s_id[jl] = ids_sorted[j];
        }
      }
    }
    if (__syncthreads_count(in) == 0) break;
  }
  // inclusive max-scan: thread t owns slots [t * kPairItems, (t + 1) * kPairItems)
  int32_t run = -1;
#pragma unroll
  for (int k = 0; k < kPairItems; ++k) run = max(run, s_j[tid * kPairItems + k]);
  {
    const int lane = lane_id(), wave = tid / kWave;
    int32_t incl = run;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
      const int32_t t = __shfl_up(incl, o, kWave);
      if (lane >= o) incl = max(incl, t);
    }
    if (lane == kWave - 1) s_red[wave] = incl;
    __syncthreads();
    int32_t prev = __shfl_up(incl, 1, kWave);
    if (lane == 0) prev = -1;
    for (int w = 0; w < wave; ++w) prev = max(prev, s_red[w]);
    run = prev;
  }
#pragma unroll
  for (int k = 0; k < kPairItems; ++k) {
    run = max(run, s_j[tid * kPairItems + k]);
    s_j[tid * kPairItems + k] = run;
  }
  __syncthreads();
#pragma unroll 4
  for (int k = 0; k < kPairItems; ++k) {
    const int lp = k * kEmitThreads + tid;
    const uint32_t p = p0 + (uint32_t)lp;
    if (p < p_end) {
      const int32_t jl = s_j[lp];
      int4 r;
      uint32_t o, g;
      if (jl < kEmitWin) {
        r = s_rect[jl];
        o = s_off[jl];
        g = s_id[jl];
      } else {
        const int64_t j = j0 + jl;
        r = rect_sorted[j];
        o = off[j];
        g = ids_sorted[j];
      }
      uint32_t dy, dx;
      divmod_small(p - o, (uint32_t)(r.z - r.x), dy, dx);
      uint32_t tile = ((uint32_t)r.y + dy) * (uint32_t)tiles_x + (uint32_t)r.x + dx;
      if (tile_slot != nullptr && tile_slot[tile] < 0) tile = n_t;
      keys[p] = ((K)tile << id_bits) | (K)g;
      atomicAdd(&s_h[tile & (kDigits - 1u)], 1u);
    }
  }
  __syncthreads();
  for (int dg = tid; dg < kDigits; dg += kEmitThreads) hist[(int64_t)dg * nblocks + blockIdx.x] = s_h[dg];
}

// ------------------------------------------------------------------ workspace
struct SortWs {
  unsigned long long* scalars;  // [TGS_COUNTER_SLOTS] partial valid-pair totals
  int32_t* diff;                // [cells] difference grid, cells = (tiles_y + 1) * (tiles_x + 1)
  int32_t* partial;             // [kCountBlocks][cells] per-workgroup grids
  int32_t* block_j0;            // [max_blocks] first Gaussian of each emit block
  int4* rect_sorted;            // [n] rectangles in depth order
  uint32_t* area_sorted;        // [n] pair counts in depth order
  uint32_t* off;                // [n + 1] pair offsets in depth order
  uint32_t* dkeys[2];           // [n] depth keys (ping-pong)
  uint32_t* dvals[2];           // [n] ids
  uint32_t* partials;           // scan block sums, digit totals
  uint32_t* hist;               // [256 * max_blocks]
  uint32_t* hoffs;              // [256 * max_blocks]
  void* pkeys[2];               // [capacity] pair keys (u32 or u64), ping-pong
  size_t bytes;
};

static SortWs layout(void* ws, int64_t n, int64_t capacity, int64_t n_tiles) {
  const int64_t cap = std::max<int64_t>(capacity, 1), nn = std::max<int64_t>(n, 1);
  const int64_t m = std::max(cap, nn);
  // blocks of any sort of up to m keys: 1024-key blocks below 2^20 keys, 4096-key blocks above
  const int64_t max_blocks = std::max<int64_t>(1024, sort_blocks(m, kPairItems)) + 1;
  const int64_t hist_n = 256 * max_blocks;
  const int64_t part_n = std::max<int64_t>(256, scan_partials(nn + 1)) + 1;
  // (tiles_x + 1)(tiles_y + 1) <= 2 n_tiles + 2 for any grid of n_tiles tiles
  const int64_t diff_n = 2 * std::max<int64_t>(n_tiles, 1) + 2;
  size_t o = 0;
  char* b = (char*)ws;
  auto take = [&](size_t bytes) {
    char* p = b ? b + o : nullptr;
    o += align_up(bytes, 256);
    return (void*)p;
  };
  SortWs w;
  w.scalars = (unsigned long long*)take(sizeof(unsigned long long) * TGS_COUNTER_SLOTS);
  w.diff = (int32_t*)take(sizeof(int32_t) * diff_n);
  w.partial = (int32_t*)take(sizeof(int32_t) * diff_n * kCountBlocks);
  w.block_j0 = (int32_t*)take(sizeof(int32_t) * max_blocks);
  w.rect_sorted = (int4*)take(sizeof(int4) * nn);
  w.area_sorted = (uint32_t*)take(sizeof(uint32_t) * nn);
  w.off = (uint32_t*)take(sizeof(uint32_t) * (nn + 1));
  for (int k = 0; k < 2; ++k) {
    w.dkeys[k] = (uint32_t*)take(sizeof(uint32_t) * nn);
    w.dvals[k] = (uint32_t*)take(sizeof(uint32_t) * nn);
  }
  w.partials = (uint32_t*)take(sizeof(uint32_t) * part_n);
  w.hist = (uint32_t*)take(sizeof(uint32_t) * hist_n);
  w.hoffs = (uint32_t*)take(sizeof(uint32_t) * hist_n);
  for (int k = 0; k < 2; ++k) w.pkeys[k] = take(sizeof(uint64_t) * cap);
  w.bytes = o;
  return w;
}

static int bits_for(uint64_t max_value) {  // bits needed to represent 0..max_value
  int b = 0;
  while (b < 64 && (max_value >> b) != 0) ++b;
  return b;
}

// Stable LSD sort of the n depth keys with their ids; returns the buffers
// holding the sorted keys and ids.
template <int kItems>
static void sort_depth(const SortWs& w, uint32_t n, uint32_t** keys_out, uint32_t** ids_out, hipStream_t s) {
  uint32_t* k[2] = {w.dkeys[0], w.dkeys[1]};
  uint32_t* v[2] = {w.dvals[0], w.dvals[1]};
  int cur = 0;
  for (int p = 0; p < 4; ++p) {
    const ScatterOut o = {k[cur ^ 1], v[cur ^ 1], 0, nullptr, nullptr};
    radix_pass<uint32_t, true, false, 8, kItems>(k[cur], v[cur], n, 8 * p, false, w.hist, w.hoffs, w.partials, o, s);
    cur ^= 1;
  }
  *keys_out = k[cur];
  *ids_out = v[cur];
}

template <typename K>
static void sort_pairs(const SortWs& w, const uint32_t* ids, int64_t n, uint32_t total, const int32_t* tile_slot,
                       int tiles_x, uint32_t n_t, int id_bits, int tbits, const float* depth, uint32_t* vals,
                       uint64_t* keys64, hipStream_t s) {
  K* kb[2] = {(K*)w.pkeys[0], (K*)w.pkeys[1]};
  const int nblocks = (int)sort_blocks(total, kPairItems);
  hipLaunchKernelGGL(block_start_kernel, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, s, w.off, n, w.block_j0);
  const int passes = pass_count(tbits);
  const int b0 = pass_bits(tbits, 0);
  switch (b0) {
#define TGS_EMIT(B)                                                                                          \
  case B:                                                                                                    \
    hipLaunchKernelGGL((emit_kernel<K, B>), dim3(nblocks), dim3(kEmitThreads), 0, s, w.rect_sorted, ids,     \
                       w.off, w.block_j0, n, total, tile_slot, tiles_x, n_t, id_bits, kb[0], nblocks, w.hist); \
    break;
    TGS_EMIT(1) TGS_EMIT(2) TGS_EMIT(3) TGS_EMIT(4) TGS_EMIT(5) TGS_EMIT(6) TGS_EMIT(7)
    default:
      hipLaunchKernelGGL((emit_kernel<K, 8>), dim3(nblocks), dim3(kEmitThreads), 0, s, w.rect_sorted, ids, w.off,
                         w.block_j0, n, total, tile_slot, tiles_x, n_t, id_bits, kb[0], nblocks, w.hist);
#undef TGS_EMIT
  }
  int cur = 0, shift = id_bits;
  for (int p = 0; p < passes; ++p) {
    const int b = pass_bits(tbits, p);
    const bool last = p == passes - 1;
    const ScatterOut o = {kb[cur ^ 1], vals, id_bits, depth, keys64};
    if (last)
      radix_pass_bits<K, false, true, kPairItems>(b, kb[cur], nullptr, total, shift, p == 0, w.hist, w.hoffs,
                                                  w.partials, o, s);
    else
      radix_pass_bits<K, false, false, kPairItems>(b, kb[cur], nullptr, total, shift, p == 0, w.hist, w.hoffs,
                                                   w.partials, o, s);
    cur ^= 1;
    shift += b;
  }
}

}  // namespace tgs

using namespace tgs;

extern "C" size_t tgs_bin_sort_workspace_size(int64_t n, int64_t capacity, int32_t n_tiles) {
  if (n < 0 || capacity < 0 || n_tiles < 0) return 0;
  return layout(nullptr, n, capacity, n_tiles).bytes;
}

extern "C" int32_t tgs_bin_sort(const int32_t* rect, const float* depth, int64_t n,
                                const int32_t* tile_slot, int32_t tiles_x, int32_t tiles_y,
                                uint64_t* keys, uint32_t* vals, int64_t capacity, uint32_t* ranges,
                                uint8_t* touched, int64_t* n_pairs, void* ws, size_t ws_bytes,
                                void* stream) {
  TGS_REQUIRE(n >= 0 && n < (1ll << 31), "tgs_bin_sort: n out of range");
  TGS_REQUIRE(tiles_x > 0 && tiles_y > 0 && (int64_t)tiles_x * tiles_y < (1ll << 30),
              "tgs_bin_sort: bad tile grid");
  TGS_REQUIRE(capacity >= 0 && capacity < (1ll << 32), "tgs_bin_sort: capacity out of range");
  TGS_REQUIRE(vals && ranges && n_pairs && ws, "tgs_bin_sort: null pointer");  // keys may be null
  TGS_REQUIRE(n == 0 || (rect && depth), "tgs_bin_sort: null rect/depth");
  TGS_REQUIRE(((uintptr_t)rect & 15) == 0, "tgs_bin_sort: rect must be 16-byte aligned");
  const uint32_t n_t = (uint32_t)tiles_x * (uint32_t)tiles_y;
  const SortWs w = layout(ws, n, capacity, n_t);
  TGS_REQUIRE(ws_bytes >= w.bytes, "tgs_bin_sort: workspace %zu bytes < %zu (is n_tiles right?)", ws_bytes,
              w.bytes);
  hipStream_t s = as_stream(stream);
  const int cells = (tiles_x + 1) * (tiles_y + 1);
  const bool lds_grid = cells <= kLdsCells;
  const int count_blocks = lds_grid ? (int)std::min<int64_t>(kCountBlocks, std::max<int64_t>(1, ceil_div(n, kCountThreads)))
                                    : (int)std::max<int64_t>(1, std::min<int64_t>(ceil_div(n, kCountThreads), 1024));
  if (!lds_grid)  // one grid accumulated with device atomics
    hipLaunchKernelGGL(fill_u32_kernel, dim3((unsigned)ceil_div(cells, 256)), dim3(256), 0, s,
                       (uint32_t*)w.partial, (int64_t)cells, 0u);
  hipLaunchKernelGGL(fill_u32_kernel, dim3(1), dim3(256), 0, s, (uint32_t*)w.scalars,
                     (int64_t)(2 * TGS_COUNTER_SLOTS), 0u);
  const int n_grids = n == 0 ? 0 : (lds_grid ? count_blocks : 1);
  if (n > 0)
    hipLaunchKernelGGL(count_kernel, dim3((unsigned)count_blocks), dim3(kCountThreads), 0, s, (const int4*)rect,
                       depth, n, tile_slot, tiles_x, tiles_y, w.dkeys[0], w.dvals[0], touched, w.partial, lds_grid,
                       w.scalars);
  hipLaunchKernelGGL(diff_sum_kernel, dim3((unsigned)ceil_div(cells, kWave)), dim3(kSumWaves * kWave), 0, s,
                     w.partial, n_grids, cells, w.diff);
  hipLaunchKernelGGL(ranges_kernel, dim3(1), dim3(kRangeThreads), 0, s, w.diff, tiles_x, tiles_y, tile_slot,
                     (uint2*)ranges);
  if (n == 0) {
    *n_pairs = 0;
    return hip_status("tgs_bin_sort");
  }
  // (depth, id) order; culled Gaussians last
  uint32_t* dk = nullptr;
  uint32_t* perm = nullptr;
  if (sort_items(n) == 16) sort_depth<16>(w, (uint32_t)n, &dk, &perm, s);
  else sort_depth<4>(w, (uint32_t)n, &dk, &perm, s);
  hipLaunchKernelGGL(gather_kernel, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, s, perm, dk,
                     (const int4*)rect, n, tiles_x, tiles_y, w.rect_sorted, w.area_sorted);
  exclusive_scan<uint32_t>(w.area_sorted, w.off, n, w.partials, s);
  uint32_t total = 0;
  unsigned long long slots[TGS_COUNTER_SLOTS] = {};
  if (hipMemcpyAsync(&total, w.off + n, sizeof(uint32_t), hipMemcpyDeviceToHost, s) != hipSuccess ||
      (tile_slot != nullptr &&
       hipMemcpyAsync(slots, w.scalars, sizeof(slots), hipMemcpyDeviceToHost, s) != hipSuccess) ||
      hipStreamSynchronize(s) != hipSuccess)
    return hip_status("tgs_bin_sort: count readback");
  unsigned long long valid_total = 0;
  for (int k = 0; k < TGS_COUNTER_SLOTS; ++k) valid_total += slots[k];
  if (tile_slot == nullptr) valid_total = total;
  if ((int64_t)total > capacity) {
    *n_pairs = (int64_t)total;
    set_error("tgs_bin_sort: %u pairs exceed capacity %lld", total, (long long)capacity);
    return TGS_ERR_CAPACITY;
  }
  *n_pairs = (int64_t)valid_total;
  if (total == 0) return hip_status("tgs_bin_sort");

  const int id_bits = std::max(1, bits_for((uint64_t)n - 1));
  const int tbits = bits_for(n_t);  // the sentinel tile id n_t must fit
  if (id_bits + tbits <= 32)
    sort_pairs<uint32_t>(w, perm, n, total, tile_slot, tiles_x, n_t, id_bits, tbits, depth, vals, keys, s);
  else
    sort_pairs<uint64_t>(w, perm, n, total, tile_slot, tiles_x, n_t, id_bits, tbits, depth, vals, keys, s);
  return hip_status("tgs_bin_sort");
}
