// Tile x depth binning, sort and per-tile ranges.
//
// The per-tile Gaussian lists must follow (tile, FP32 depth bits, Gaussian
// id).  Rather than radix-sorting a 64-bit (tile, depth) key with an id for
// every (Gaussian, tile) pair, the Gaussians are put in (depth, id) order once
// (a 32-bit sort of n keys) and the pairs are emitted in that order; a
// stable sort on the tile bits alone then yields the full order.  The pair
// key is (tile << pos_bits) | position-in-depth-order, usually 32 bits, and
// the id is read back from the depth order after the sort:
//
//   count     per Gaussian: rectangle area, visibility, touched flag and the
//             depth key (culled Gaussians get a key above every depth)
//   sort      LSD radix sort of (depth key, id) over n: stable, so ties keep
//             id order; visible Gaussians come first
//   gather    areas in depth order, exclusive scan -> pair offsets, total
//   emit      one thread per pair (load-balanced: each block finds its first
//             Gaussian with a 256-way search of the offsets), coalesced key
//             writes; tiles outside the valid set get the sentinel tile id
//             n_tiles, which sorts after every real tile
//   sort      LSD radix sort of the pair keys on the tile bits only
//   finalize  ids from depth positions, tile boundaries -> ranges and
//             (optionally) the 64-bit (tile << 32) | depth-bits keys
//
// Each radix pass is a stable counting sort: per-block digit histograms
// (peer groups found by a 64-lane ballot match add their counts once), one
// scan of the digit-major histogram table, and a per-block scatter whose
// in-block ranks come from the same ballot match and a digit prefix across
// the workgroup's waves.
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

void exclusive_scan_u32(const uint32_t* in, uint32_t* out, int64_t n, uint32_t* partials, hipStream_t s) {
  exclusive_scan<uint32_t>(in, out, n, partials, s);
}


// ------------------------------------------------------------------ count
// Depth key of a culled Gaussian: above every finite positive depth bit pattern.
constexpr uint32_t kCulledKey = 0xffffffffu;

__global__ void __launch_bounds__(256) count_kernel(const int4* __restrict__ rect,
                                                    const float* __restrict__ depth, int64_t n,
                                                    const int32_t* __restrict__ tile_slot, int tiles_x,
                                                    uint32_t* __restrict__ dkeys, uint32_t* __restrict__ dvals,
                                                    uint8_t* __restrict__ touched,
                                                    unsigned long long* __restrict__ valid_total) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  uint32_t valid = 0;
  if (i < n) {
    const int4 r = rect[i];
    const uint32_t area = (uint32_t)((r.z - r.x) * (r.w - r.y));
    if (tile_slot == nullptr) {
      valid = area;
    } else {
      for (int ty = r.y; ty < r.w; ++ty)
        for (int tx = r.x; tx < r.z; ++tx) valid += tile_slot[ty * tiles_x + tx] >= 0 ? 1u : 0u;
    }
    dkeys[i] = valid > 0 ? __float_as_uint(depth[i]) : kCulledKey;
    dvals[i] = (uint32_t)i;
    if (touched != nullptr && valid > 0) touched[i] = 1;
  }
  if (tile_slot != nullptr) {  // pairs in valid tiles: one atomic per workgroup
    __shared__ uint32_t lds[256 / kWave];
    uint32_t tot;
    block_exclusive_scan<256, uint32_t>(valid, lds, &tot);
    if (threadIdx.x == 0 && tot > 0) atomicAdd(valid_total, (unsigned long long)tot);
  }
}

// Rectangles and pair counts in depth order (a Gaussian without a valid tile
// has the culled key and sits after the visible ones; its count is 0).
__global__ void __launch_bounds__(256) gather_kernel(const uint32_t* __restrict__ perm,
                                                     const uint32_t* __restrict__ dkeys_sorted,
                                                     const int4* __restrict__ rect, int64_t n,
                                                     int4* __restrict__ rect_sorted,
                                                     uint32_t* __restrict__ area_sorted) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  const int4 r = rect[perm[j]];
  rect_sorted[j] = r;
  area_sorted[j] = dkeys_sorted[j] == kCulledKey ? 0u : (uint32_t)((r.z - r.x) * (r.w - r.y));
}

// ------------------------------------------------------------------ radix sort
constexpr int kSortThreads = 256;
constexpr int kSortWaves = kSortThreads / kWave;

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

template <typename K, int kBits>
__global__ void __launch_bounds__(kSortThreads) radix_hist_kernel(const K* __restrict__ keys, uint32_t n,
                                                                 int shift, int rounds, int nblocks,
                                                                 uint32_t* __restrict__ hist) {
  constexpr int kDigits = 1 << kBits;
  __shared__ uint32_t h[kDigits];
  if (threadIdx.x < kDigits) h[threadIdx.x] = 0;
  __syncthreads();
  const int lane = threadIdx.x & (kWave - 1);
  const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  const int64_t base = (int64_t)blockIdx.x * kSortThreads * rounds;
  for (int k = 0; k < rounds; ++k) {
    const int64_t i = base + (int64_t)k * kSortThreads + threadIdx.x;
    const bool valid = i < n;
    const uint32_t d = valid ? (uint32_t)(keys[i] >> shift) & (kDigits - 1u) : 0u;
    const uint64_t peers = digit_peers<kBits>(d, valid);
    if (valid && (peers & lt_mask) == 0) atomicAdd(&h[d], (uint32_t)__popcll(peers));
  }
  __syncthreads();
  if (threadIdx.x < kDigits) hist[(int64_t)threadIdx.x * nblocks + blockIdx.x] = h[threadIdx.x];
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

template <typename K, bool kVals, int kBits>
__global__ void __launch_bounds__(kSortThreads) radix_scatter_kernel(
    const K* __restrict__ keys_in, const uint32_t* __restrict__ vals_in, uint32_t n, int shift, int rounds,
    int nblocks, const uint32_t* __restrict__ offs, const uint32_t* __restrict__ dtot,
    K* __restrict__ keys_out, uint32_t* __restrict__ vals_out) {
  constexpr int kDigits = 1 << kBits;
  __shared__ uint32_t base[kDigits];                // running position of each digit
  __shared__ uint32_t wcount[kSortWaves][kDigits];  // per-wave counts, then offsets, of this round
  __shared__ uint32_t lds[kSortThreads / kWave];
  const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
  // start of each digit = totals of the smaller digits + this block's prefix within the digit
  uint32_t dall;
  const uint32_t dstart = block_exclusive_scan<kSortThreads, uint32_t>(tid < kDigits ? dtot[tid] : 0u, lds, &dall);
  if (tid < kDigits) {
    base[tid] = dstart + offs[(int64_t)tid * nblocks + blockIdx.x];
    for (int w = 0; w < kSortWaves; ++w) wcount[w][tid] = 0;
  }
  __syncthreads();
  const int64_t blk = (int64_t)blockIdx.x * kSortThreads * rounds;
  const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  for (int k = 0; k < rounds; ++k) {
    if (blk + (int64_t)k * kSortThreads >= n) break;  // uniform across the workgroup
    const int64_t i = blk + (int64_t)k * kSortThreads + tid;
    const bool valid = i < n;
    K key = 0;
    uint32_t val = 0;
    if (valid) {
      key = keys_in[i];
      if (kVals) val = vals_in[i];
    }
    const uint32_t d = (uint32_t)(key >> shift) & (kDigits - 1u);
    const uint64_t peers = digit_peers<kBits>(d, valid);
    const int rank = __popcll(peers & lt_mask);
    if (valid && rank == 0) wcount[wave][d] = (uint32_t)__popcll(peers);
    __syncthreads();
    if (tid < kDigits) {
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
      if (kVals) vals_out[dst] = val;
    }
    __syncthreads();
    if (tid < kDigits)
      for (int w = 0; w < kSortWaves; ++w) wcount[w][tid] = 0;
    __syncthreads();
  }
}

// Keys per thread for n keys: enough workgroups to fill the GPU, at most 16.
static int sort_rounds(uint32_t n) {
  int r = (int)ceil_div(n, (int64_t)kSortThreads * 2048);
  return std::min(16, std::max(1, r));
}

template <typename K, bool kVals, int kBits>
static void radix_pass(K*& keys, uint32_t*& vals, K*& keys_alt, uint32_t*& vals_alt, uint32_t n, int shift,
                       uint32_t* hist, uint32_t* hoffs, uint32_t* partials, hipStream_t s) {
  const int rounds = sort_rounds(n);
  const int nblocks = (int)ceil_div(n, (int64_t)kSortThreads * rounds);
  hipLaunchKernelGGL((radix_hist_kernel<K, kBits>), dim3(nblocks), dim3(kSortThreads), 0, s, keys, n, shift,
                     rounds, nblocks, hist);
  uint32_t* dtot = partials;  // one total per digit
  hipLaunchKernelGGL(digit_scan_kernel, dim3(1 << kBits), dim3(1024), 0, s, hist, nblocks, hoffs, dtot);
  hipLaunchKernelGGL((radix_scatter_kernel<K, kVals, kBits>), dim3(nblocks), dim3(kSortThreads), 0, s, keys,
                     vals, n, shift, rounds, nblocks, hoffs, dtot, keys_alt, vals_alt);
  std::swap(keys, keys_alt);
  std::swap(vals, vals_alt);
}

// Sorts n keys (and values) on bits [lo, lo + bits); passes of at most 8
// bits, split evenly.  The result lands in keys/vals (pointers are swapped).
template <typename K, bool kVals>
static void radix_sort(K*& keys, uint32_t*& vals, K*& keys_alt, uint32_t*& vals_alt, uint32_t n, int lo,
                       int bits, uint32_t* hist, uint32_t* hoffs, uint32_t* partials, hipStream_t s) {
  if (n <= 1 || bits <= 0) return;
  const int passes = (bits + 7) / 8;
  const int per = (bits + passes - 1) / passes;
  int shift = lo;
  for (int p = 0; p < passes; ++p) {
    const int b = std::min(per, lo + bits - shift);
    switch (b) {
      case 1: radix_pass<K, kVals, 1>(keys, vals, keys_alt, vals_alt, n, shift, hist, hoffs, partials, s); break;
      case 2: radix_pass<K, kVals, 2>(keys, vals, keys_alt, vals_alt, n, shift, hist, hoffs, partials, s); break;
      case 3: radix_pass<K, kVals, 3>(keys, vals, keys_alt, vals_alt, n, shift, hist, hoffs, partials, s); break;
      case 4: radix_pass<K, kVals, 4>(keys, vals, keys_alt, vals_alt, n, shift, hist, hoffs, partials, s); break;
      case 5: radix_pass<K, kVals, 5>(keys, vals, keys_alt, vals_alt, n, shift, hist, hoffs, partials, s); break;
      case 6: radix_pass<K, kVals, 6>(keys, vals, keys_alt, vals_alt, n, shift, hist, hoffs, partials, s); break;
      case 7: radix_pass<K, kVals, 7>(keys, vals, keys_alt, vals_alt, n, shift, hist, hoffs, partials, s); break;
      default: radix_pass<K, kVals, 8>(keys, vals, keys_alt, vals_alt, n, shift, hist, hoffs, partials, s); break;
    }
    shift += b;
  }
}

// ------------------------------------------------------------------ emit
constexpr int kEmitThreads = 256;
constexpr int kEmitItems = 8;
constexpr int kEmitTile = kEmitThreads * kEmitItems;
constexpr int kEmitWindow = 2048;

// Largest j in [0, n) with off[j] <= target, by a 256-way search per round
// (off[0] = 0 <= target; offsets are non-decreasing).
__device__ __forceinline__ int64_t block_last_le(const uint32_t* __restrict__ off, int64_t n, uint32_t target) {
  int64_t lo = 0, hi = n;
  while (hi - lo > 1) {
    const int64_t step = ceil_div(hi - lo, kEmitThreads);
    const int64_t j = lo + (int64_t)threadIdx.x * step;
    const bool pred = j < hi && off[j] <= target;
    const int cnt = __syncthreads_count(pred);
    lo = lo + (int64_t)(cnt - 1) * step;
    hi = min(hi, lo + step);
  }
  return lo;
}

template <typename K>
__global__ void __launch_bounds__(kEmitThreads) emit_kernel(
    const int4* __restrict__ rect_sorted, const uint32_t* __restrict__ off, int64_t n, uint32_t total,
    const int32_t* __restrict__ tile_slot, int tiles_x, uint32_t n_t, int pbits, K* __restrict__ keys) {
  __shared__ uint32_t s_off[kEmitWindow];
  const uint32_t p0 = blockIdx.x * (uint32_t)kEmitTile;
  const uint32_t p_last = min(total, p0 + (uint32_t)kEmitTile) - 1u;
  const int64_t j0 = block_last_le(off, n, p0);
  const int64_t j1 = block_last_le(off, n, p_last);
  const int64_t cnt = j1 - j0 + 1;
  const bool windowed = cnt <= kEmitWindow;
  if (windowed)
    for (int64_t k = threadIdx.x; k < cnt; k += kEmitThreads) s_off[k] = off[j0 + k];
  __syncthreads();
  for (int it = 0; it < kEmitItems; ++it) {
    const uint32_t p = p0 + (uint32_t)(it * kEmitThreads) + threadIdx.x;
    if (p >= total) break;
    int64_t lo = 0, hi = cnt;  // last entry of the window with offset <= p
    while (hi - lo > 1) {
      const int64_t mid = (lo + hi) >> 1;
      const uint32_t o = windowed ? s_off[mid] : off[j0 + mid];
      if (o <= p) lo = mid; else hi = mid;
    }
    const int64_t j = j0 + lo;
    const uint32_t l = p - (windowed ? s_off[lo] : off[j]);
    const int4 r = rect_sorted[j];
    const uint32_t w = (uint32_t)(r.z - r.x);
    const uint32_t ty = (uint32_t)r.y + l / w, tx = (uint32_t)r.x + l % w;
    uint32_t tile = ty * (uint32_t)tiles_x + tx;
    if (tile_slot != nullptr && tile_slot[tile] < 0) tile = n_t;
    keys[p] = ((K)tile << pbits) | (K)j;
  }
}

// ------------------------------------------------------------------ finalize
template <typename K>
__global__ void __launch_bounds__(256) finalize_kernel(const K* __restrict__ keys, uint32_t total, int pbits,
                                                       uint32_t n_t, const uint32_t* __restrict__ perm,
                                                       const float* __restrict__ depth,
                                                       uint32_t* __restrict__ vals, uint64_t* __restrict__ keys64,
                                                       uint2* __restrict__ ranges) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= total) return;
  const K key = keys[i];
  const uint32_t t = (uint32_t)(key >> pbits);
  if (t >= n_t) return;  // sentinel pairs (tiles outside the valid set) sit at the end
  const uint32_t g = perm[(uint32_t)(key & (((K)1 << pbits) - 1))];
  vals[i] = g;
  if (keys64 != nullptr) keys64[i] = ((uint64_t)t << 32) | (uint64_t)__float_as_uint(depth[g]);
  if (i == 0 || (uint32_t)(keys[i - 1] >> pbits) != t) ranges[t].x = i;
  if (i == total - 1 || (uint32_t)(keys[i + 1] >> pbits) != t) ranges[t].y = i + 1;
}

// ------------------------------------------------------------------ workspace
struct SortWs {
  unsigned long long* scalars;  // [0] valid pair total
  int4* rect_sorted;            // [n] rectangles in depth order
  uint32_t* area_sorted;        // [n] pair counts in depth order
  uint32_t* off;                // [n + 1] pair offsets in depth order
  uint32_t* dkeys[2];           // [n] depth keys (ping-pong)
  uint32_t* dvals[2];           // [n] ids
  uint32_t* partials;           // scan block sums
  uint32_t* hist;               // [256 * max_blocks]
  uint32_t* hoffs;              // [256 * max_blocks + 1]
  void* pkeys[2];               // [capacity] pair keys (u32 or u64), ping-pong
  size_t bytes;
};

static SortWs layout(void* ws, int64_t n, int64_t capacity) {
  const int64_t cap = std::max<int64_t>(capacity, 1), nn = std::max<int64_t>(n, 1);
  const int64_t m = std::max(cap, nn);
  // sort_rounds keeps the grid at <= 2048 workgroups up to 16 x 2048 x 256 keys
  const int64_t max_blocks = std::max<int64_t>(2048, ceil_div(m, (int64_t)kSortThreads * 16)) + 1;
  const int64_t hist_n = 256 * (max_blocks + 1);
  const int64_t part_n = std::max<int64_t>(256, scan_partials(nn + 1)) + 1;
  size_t o = 0;
  char* b = (char*)ws;
  auto take = [&](size_t bytes) {
    char* p = b ? b + o : nullptr;
    o += align_up(bytes, 256);
    return (void*)p;
  };
  SortWs w;
  w.scalars = (unsigned long long*)take(64);
  w.rect_sorted = (int4*)take(sizeof(int4) * nn);
  w.area_sorted = (uint32_t*)take(sizeof(uint32_t) * nn);
  w.off = (uint32_t*)take(sizeof(uint32_t) * (nn + 1));
  for (int k = 0; k < 2; ++k) {
    w.dkeys[k] = (uint32_t*)take(sizeof(uint32_t) * nn);
    w.dvals[k] = (uint32_t*)take(sizeof(uint32_t) * nn);
  }
  w.partials = (uint32_t*)take(sizeof(uint32_t) * part_n);
  w.hist = (uint32_t*)take(sizeof(uint32_t) * hist_n);
  w.hoffs = (uint32_t*)take(sizeof(uint32_t) * (hist_n + 1));
  for (int k = 0; k < 2; ++k) w.pkeys[k] = take(sizeof(uint64_t) * cap);
  w.bytes = o;
  return w;
}

static int bits_for(uint64_t max_value) {  // bits needed to represent 0..max_value
  int b = 0;
  while (b < 64 && (max_value >> b) != 0) ++b;
  return b;
}

template <typename K>
static void sort_pairs(const SortWs& w, const uint32_t* perm, int64_t n, uint32_t total,
                       const int32_t* tile_slot, int tiles_x, uint32_t n_t, int pbits, int tbits,
                       const float* depth, uint32_t* vals, uint64_t* keys64, uint32_t* ranges, hipStream_t s) {
  K* ka = (K*)w.pkeys[0];
  K* kb = (K*)w.pkeys[1];
  uint32_t* va = nullptr;
  uint32_t* vb = nullptr;
  hipLaunchKernelGGL((emit_kernel<K>), dim3((unsigned)ceil_div(total, kEmitTile)), dim3(kEmitThreads), 0, s,
                     w.rect_sorted, w.off, n, total, tile_slot, tiles_x, n_t, pbits, ka);
  radix_sort<K, false>(ka, va, kb, vb, total, pbits, tbits, w.hist, w.hoffs, w.partials, s);
  hipLaunchKernelGGL((finalize_kernel<K>), dim3((unsigned)ceil_div(total, 256)), dim3(256), 0, s, ka, total,
                     pbits, n_t, perm, depth, vals, keys64, (uint2*)ranges);
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
  TGS_REQUIRE(n >= 0 && n < (1ll << 31), "tgs_bin_sort: n out of range");
  TGS_REQUIRE(tiles_x > 0 && tiles_y > 0 && (int64_t)tiles_x * tiles_y < (1ll << 30),
              "tgs_bin_sort: bad tile grid");
  TGS_REQUIRE(capacity >= 0 && capacity < (1ll << 32), "tgs_bin_sort: capacity out of range");
  TGS_REQUIRE(vals && ranges && n_pairs && ws, "tgs_bin_sort: null pointer");  // keys may be null
  TGS_REQUIRE(n == 0 || (rect && depth), "tgs_bin_sort: null rect/depth");
  TGS_REQUIRE(((uintptr_t)rect & 15) == 0, "tgs_bin_sort: rect must be 16-byte aligned");
  const SortWs w = layout(ws, n, capacity);
  TGS_REQUIRE(ws_bytes >= w.bytes, "tgs_bin_sort: workspace %zu bytes < %zu", ws_bytes, w.bytes);
  hipStream_t s = as_stream(stream);
  const uint32_t n_t = (uint32_t)tiles_x * (uint32_t)tiles_y;

  hipLaunchKernelGGL(fill_u32_kernel, dim3((unsigned)ceil_div(2 * (int64_t)n_t, 256)), dim3(256), 0, s,
                     ranges, 2 * (int64_t)n_t, 0u);
  hipLaunchKernelGGL(set_kernel<unsigned long long>, dim3(1), dim3(64), 0, s, w.scalars, 0ull);
  if (n == 0) {
    *n_pairs = 0;
    return hip_status("tgs_bin_sort");
  }
  hipLaunchKernelGGL(count_kernel, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, s, (const int4*)rect, depth,
                     n, tile_slot, tiles_x, w.dkeys[0], w.dvals[0], touched, w.scalars);
  // (depth, id) order; culled Gaussians last
  uint32_t* dk = w.dkeys[0];
  uint32_t* dv = w.dvals[0];
  uint32_t* dk2 = w.dkeys[1];
  uint32_t* dv2 = w.dvals[1];
  radix_sort<uint32_t, true>(dk, dv, dk2, dv2, (uint32_t)n, 0, 32, w.hist, w.hoffs, w.partials, s);
  const uint32_t* perm = dv;
  hipLaunchKernelGGL(gather_kernel, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, s, perm, dk,
                     (const int4*)rect, n, w.rect_sorted, w.area_sorted);
  exclusive_scan<uint32_t>(w.area_sorted, w.off, n, w.partials, s);
  uint32_t total = 0;
  unsigned long long valid_total = 0;
  if (hipMemcpyAsync(&total, w.off + n, sizeof(uint32_t), hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipMemcpyAsync(&valid_total, w.scalars, sizeof(valid_total), hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return hip_status("tgs_bin_sort: count readback");
  if (tile_slot == nullptr) valid_total = total;
  if ((int64_t)total > capacity) {
    *n_pairs = (int64_t)total;
    set_error("tgs_bin_sort: %u pairs exceed capacity %lld", total, (long long)capacity);
    return TGS_ERR_CAPACITY;
  }
  *n_pairs = (int64_t)valid_total;
  if (total == 0) return hip_status("tgs_bin_sort");

  const int pbits = std::max(1, bits_for((uint64_t)n - 1));
  const int tbits = bits_for(n_t);  // the sentinel tile id n_t must fit
  if (pbits + tbits <= 32)
    sort_pairs<uint32_t>(w, perm, n, total, tile_slot, tiles_x, n_t, pbits, tbits, depth, vals,
                         keys, ranges, s);
  else
    sort_pairs<uint64_t>(w, perm, n, total, tile_slot, tiles_x, n_t, pbits, tbits, depth, vals,
                         keys, ranges, s);
  return hip_status("tgs_bin_sort");
}
