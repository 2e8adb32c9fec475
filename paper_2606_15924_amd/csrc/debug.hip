// Debug helper: counts the non-finite entries of a float array on the
// device (NaN and +-inf: exponent bits all set).  A grid-stride loop with
// 16-byte loads, one wave reduction and one 64-bit atomic per wave.
#include <algorithm>

#include "common.h"

namespace tgs {

__global__ void __launch_bounds__(64) clear_count_kernel(unsigned long long* __restrict__ c) {
  if (threadIdx.x == 0) *c = 0ull;
}

__device__ __forceinline__ int nonfinite(float f) {
  return (__float_as_uint(f) & 0x7f800000u) == 0x7f800000u ? 1 : 0;
}

__global__ void __launch_bounds__(256) count_nonfinite_kernel(const float* __restrict__ x, int64_t n,
                                                              unsigned long long* __restrict__ count) {
  const int64_t n4 = n / 4;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  int c = 0;
  const float4* x4 = reinterpret_cast<const float4*>(x);
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n4; i += stride) {
    const float4 v = x4[i];
    c += nonfinite(v.x) + nonfinite(v.y) + nonfinite(v.z) + nonfinite(v.w);
  }
  for (int64_t i = 4 * n4 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
    c += nonfinite(x[i]);
  c = wave_sum_i(c);
  if (lane_id() == 0 && c != 0) atomicAdd(count, (unsigned long long)c);
}

}  // namespace tgs

using namespace tgs;

extern "C" int32_t tgs_check_finite(const float* x, int64_t n, int64_t* count, void* stream) {
  TGS_REQUIRE(n >= 0, "tgs_check_finite: n < 0");
  TGS_REQUIRE(count != nullptr, "tgs_check_finite: null count");
  TGS_REQUIRE(n == 0 || x != nullptr, "tgs_check_finite: null array");
  TGS_REQUIRE(((uintptr_t)x & 15) == 0, "tgs_check_finite: array must be 16-byte aligned");
  TGS_REQUIRE(((uintptr_t)count & 7) == 0, "tgs_check_finite: count must be 8-byte aligned");
  hipStream_t s = as_stream(stream);
  hipLaunchKernelGGL(clear_count_kernel, dim3(1), dim3(64), 0, s, (unsigned long long*)count);
  if (n > 0) {
    const unsigned grid = (unsigned)std::min<int64_t>(ceil_div(ceil_div(n, 4), 256), 2048);
    hipLaunchKernelGGL(count_nonfinite_kernel, dim3(grid), dim3(256), 0, s, x, n, (unsigned long long*)count);
  }
  return hip_status("tgs_check_finite");
}
