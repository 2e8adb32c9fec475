// Shared device helpers of the turbogs HIP library (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "turbogs.h"

namespace tgs {

constexpr int kTile = 16;
constexpr int kTilePixels = kTile * kTile;
constexpr int kWave = 64;

// ---------------------------------------------------------------- errors
void set_error(const char* fmt, ...);
int32_t hip_status(const char* where);  // TGS_OK or TGS_ERR_HIP (+ message)

#define TGS_REQUIRE(cond, ...)          \
  do {                                  \
    if (!(cond)) {                      \
      ::tgs::set_error(__VA_ARGS__);    \
      return TGS_ERR_INVALID;           \
    }                                   \
  } while (0)

inline hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

__host__ __device__ inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

__host__ __device__ inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// ---------------------------------------------------------------- wave-level
// DPP control words of the GFX9 family (CDNA).
constexpr int kDppQuadPerm1032 = 0xB1;  // quad_perm [1, 0, 3, 2]
constexpr int kDppQuadPerm2301 = 0x4E;  // quad_perm [2, 3, 0, 1]
constexpr int kDppRowHalfMirror = 0x141;
constexpr int kDppRowMirror = 0x140;
constexpr int kDppRowBcast15 = 0x142;
constexpr int kDppRowBcast31 = 0x143;
constexpr int kDppRowShr1 = 0x111;
constexpr int kDppWaveShr1 = 0x138;

template <int Ctrl, int RowMask = 0xf, int BankMask = 0xf, bool BoundCtrl = false>
__device__ __forceinline__ float dpp_f(float old, float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(old), __float_as_int(v), Ctrl,
                                                    RowMask, BankMask, BoundCtrl));
}

template <int Ctrl, int RowMask = 0xf, int BankMask = 0xf, bool BoundCtrl = false>
__device__ __forceinline__ int dpp_i(int old, int v) {
  return __builtin_amdgcn_update_dpp(old, v, Ctrl, RowMask, BankMask, BoundCtrl);
}

// Sum over the 64 lanes of a wave; the result is returned in every lane.
// Rows of 16 are reduced with quad permutations and mirrors, then the row
// sums are chained with the row broadcasts into lane 63 and read back.
__device__ __forceinline__ float wave_sum(float v) {
  v += dpp_f<kDppQuadPerm1032>(0.f, v);
  v += dpp_f<kDppQuadPerm2301>(0.f, v);
  v += dpp_f<kDppRowHalfMirror>(0.f, v);
  v += dpp_f<kDppRowMirror>(0.f, v);
  v += dpp_f<kDppRowBcast15, 0xa>(0.f, v);
  v += dpp_f<kDppRowBcast31, 0xc>(0.f, v);
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
}

__device__ __forceinline__ int wave_sum_i(int v) {
  v += dpp_i<kDppQuadPerm1032>(0, v);
  v += dpp_i<kDppQuadPerm2301>(0, v);
  v += dpp_i<kDppRowHalfMirror>(0, v);
  v += dpp_i<kDppRowMirror>(0, v);
  v += dpp_i<kDppRowBcast15, 0xa>(0, v);
  v += dpp_i<kDppRowBcast31, 0xc>(0, v);
  return __builtin_amdgcn_readlane(v, 63);
}

__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }

__device__ __forceinline__ int lane_id() { return __lane_id(); }

// Number of set bits of `mask` below this lane.
__device__ __forceinline__ int mask_rank(uint64_t mask) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                   __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

// Inclusive prefix sum over the wave (Hillis-Steele with shuffles).
__device__ __forceinline__ uint64_t wave_inclusive_scan_u64(uint64_t v) {
  const int lane = lane_id();
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    uint64_t t = __shfl_up(v, o, kWave);
    if (lane >= o) v += t;
  }
  return v;
}

// The same scan on DPP alone: rows of 16 by shifts of 1, 2, 4 and 8 lanes,
// then the row totals chained by the row broadcasts of lanes 15 and 31.  A
// lane whose DPP source lies before its row (or in a masked row) reads 0.
template <int Ctrl, int RowMask = 0xf>
__device__ __forceinline__ uint64_t dpp_u64(uint64_t v) {
  const uint32_t lo = (uint32_t)dpp_i<Ctrl, RowMask>(0, (int)(uint32_t)v);
  const uint32_t hi = (uint32_t)dpp_i<Ctrl, RowMask>(0, (int)(uint32_t)(v >> 32));
  return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ uint64_t wave_inclusive_scan_u64_dpp(uint64_t v) {
  v += dpp_u64<kDppRowShr1>(v);
  v += dpp_u64<kDppRowShr1 + 1>(v);  // row_shr:2
  v += dpp_u64<kDppRowShr1 + 3>(v);  // row_shr:4
  v += dpp_u64<kDppRowShr1 + 7>(v);  // row_shr:8
  v += dpp_u64<kDppRowBcast15, 0xa>(v);
  v += dpp_u64<kDppRowBcast31, 0xc>(v);
  return v;
}

__device__ __forceinline__ int wave_inclusive_scan_i_dpp(int v) {
  v += dpp_i<kDppRowShr1>(0, v);
  v += dpp_i<kDppRowShr1 + 1>(0, v);
  v += dpp_i<kDppRowShr1 + 3>(0, v);
  v += dpp_i<kDppRowShr1 + 7>(0, v);
  v += dpp_i<kDppRowBcast15, 0xa>(0, v);
  v += dpp_i<kDppRowBcast31, 0xc>(0, v);
  return v;
}

// Maximum over the 64 lanes (every lane receives it).
__device__ __forceinline__ uint32_t wave_max_u32(uint32_t v) {
  for (int o = kWave / 2; o > 0; o >>= 1) v = max(v, (uint32_t)__shfl_xor((int)v, o, kWave));
  return v;
}

__device__ __forceinline__ uint32_t wave_inclusive_scan_u32(uint32_t v) {
  const int lane = lane_id();
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    uint32_t t = __shfl_up(v, o, kWave);
    if (lane >= o) v += t;
  }
  return v;
}

__device__ __forceinline__ int wave_inclusive_scan_i(int v) {
  const int lane = lane_id();
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    int t = __shfl_up(v, o, kWave);
    if (lane >= o) v += t;
  }
  return v;
}

}  // namespace tgs
