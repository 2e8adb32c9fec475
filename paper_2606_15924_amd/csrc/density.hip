// Difficulty score of the error-driven density control (Sec. 3.8,
// Eq. gauss_score) from the back-projected sums of tgs_density_accumulate:
// e_i = E_i / (W_i + eps), d_i = D_i / (W_i + eps), s_i = e_i + lambda_eff d_i
// with lambda_eff = lambda_base (1 - rho).  Elementwise and HBM-bound:
// 16 bytes read (one [E, W, D, -] slot) and up to 12 written per Gaussian,
// one Gaussian per thread.
#include <algorithm>

#include "common.h"

namespace tgs {

__device__ __forceinline__ void score_one(float E, float W, float D, float eps, float lam, float& e, float& d,
                                          float& sc) {
#pragma clang fp contract(off)
  const float den = W + eps;
  e = E / den;
  d = D / den;
  sc = e + lam * d;
}

__global__ void __launch_bounds__(256) density_score_kernel(const float* __restrict__ stats, int64_t n, float eps,
                                                            float lam, float* __restrict__ e_out,
                                                            float* __restrict__ d_out, float* __restrict__ s_out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float4 st = reinterpret_cast<const float4*>(stats)[i];
  float e, d, sc;
  score_one(st.x, st.y, st.z, eps, lam, e, d, sc);
  if (e_out != nullptr) e_out[i] = e;
  if (d_out != nullptr) d_out[i] = d;
  s_out[i] = sc;
}

// ------------------------------------------------------------------ percentile
// Exact k-th largest of n floats by an MSB-first radix select over the
// order-preserving 32-bit keys (sign flipped for non-negative values, all
// bits flipped for negative ones): four rounds of an 8-bit digit histogram
// of the keys that still match the chosen prefix, each followed by a
// one-workgroup pick of the digit that holds the k-th largest.  The state
// (prefix, remaining rank, histogram) stays on the device, so the rounds
// queue without a host round trip.
struct SelectState {
  uint32_t hist[256];
  uint32_t prefix;
  uint32_t k_rem;  // rank of the target among the keys that match the prefix
  uint32_t pad[2];
};

__device__ __forceinline__ uint32_t order_key(float f) {
  const uint32_t b = __float_as_uint(f);
  return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}

__device__ __forceinline__ float key_value(uint32_t k) {
  return __uint_as_float((k & 0x80000000u) ? (k & 0x7fffffffu) : ~k);
}

__global__ void __launch_bounds__(256) select_init_kernel(SelectState* __restrict__ st, uint32_t k) {
  st->hist[threadIdx.x] = 0u;
  if (threadIdx.x == 0) {
    st->prefix = 0u;
    st->k_rem = k;
  }
}

__global__ void __launch_bounds__(256) select_hist_kernel(const float* __restrict__ v, int64_t n, int shift,
                                                          SelectState* __restrict__ st) {
  __shared__ uint32_t h[256];
  h[threadIdx.x] = 0u;
  __syncthreads();
  const uint32_t prefix = st->prefix;
  const uint32_t hi_mask = shift == 24 ? 0u : ~((1u << (shift + 8)) - 1u);
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    const uint32_t key = order_key(v[i]);
    if ((key & hi_mask) == prefix) atomicAdd(&h[(key >> shift) & 255u], 1u);
  }
  __syncthreads();
  if (h[threadIdx.x] != 0u) atomicAdd(&st->hist[threadIdx.x], h[threadIdx.x]);
}

// One workgroup of 256: digit d's count of keys with a larger digit is a
// suffix sum (an inclusive Hillis-Steele scan from the top, eight rounds);
// the digit with above < k_rem <= above + hist[d] holds the target.
__global__ void __launch_bounds__(256) select_pick_kernel(int shift, SelectState* __restrict__ st,
                                                          float* __restrict__ out) {
  __shared__ uint32_t sfx[256];
  const int d = threadIdx.x;
  const uint32_t hd = st->hist[d];
  sfx[d] = hd;
  __syncthreads();
  for (int off = 1; off < 256; off <<= 1) {
    const uint32_t add = d + off < 256 ? sfx[d + off] : 0u;
    __syncthreads();
    sfx[d] += add;
    __syncthreads();
  }
  const uint32_t above = sfx[d] - hd;
  const uint32_t k = st->k_rem;
  __syncthreads();
  const bool mine = above < k && k <= above + hd;
  st->hist[d] = 0u;  // cleared for the next round
  __syncthreads();
  if (mine) {
    const uint32_t prefix = st->prefix | ((uint32_t)d << shift);
    st->prefix = prefix;
    st->k_rem = k - above;
    if (shift == 0) *out = key_value(prefix);
  }
}

__global__ void __launch_bounds__(256) threshold_mask_kernel(const float* __restrict__ v, int64_t n,
                                                             const float* __restrict__ thr,
                                                             uint8_t* __restrict__ mask) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  mask[i] = order_key(v[i]) >= order_key(*thr) ? 1u : 0u;
}

}  // namespace tgs

using namespace tgs;

extern "C" size_t tgs_select_workspace_size(void) { return sizeof(SelectState); }

extern "C" int32_t tgs_select_kth_largest(const float* values, int64_t n, int64_t k, float* out, void* ws,
                                          size_t ws_bytes, void* stream) {
  TGS_REQUIRE(n > 0 && n < (1ll << 31), "tgs_select_kth_largest: n %lld out of range", (long long)n);
  TGS_REQUIRE(k >= 1 && k <= n, "tgs_select_kth_largest: k %lld not in [1, %lld]", (long long)k, (long long)n);
  TGS_REQUIRE(values && out && ws, "tgs_select_kth_largest: null pointer");
  TGS_REQUIRE(ws_bytes >= sizeof(SelectState), "tgs_select_kth_largest: workspace %zu bytes < %zu", ws_bytes,
              sizeof(SelectState));
  TGS_REQUIRE(((uintptr_t)ws & 15) == 0, "tgs_select_kth_largest: workspace must be 16-byte aligned");
  hipStream_t s = as_stream(stream);
  SelectState* st = (SelectState*)ws;
  const unsigned grid = (unsigned)std::min<int64_t>(ceil_div(n, (int64_t)256 * 8), 2048);
  hipLaunchKernelGGL(select_init_kernel, dim3(1), dim3(256), 0, s, st, (uint32_t)k);
  for (int shift = 24; shift >= 0; shift -= 8) {
    hipLaunchKernelGGL(select_hist_kernel, dim3(grid), dim3(256), 0, s, values, n, shift, st);
    hipLaunchKernelGGL(select_pick_kernel, dim3(1), dim3(256), 0, s, shift, st, out);
  }
  return hip_status("tgs_select_kth_largest");
}

extern "C" int32_t tgs_threshold_mask(const float* values, int64_t n, const float* thr, uint8_t* mask,
                                      void* stream) {
  TGS_REQUIRE(n >= 0 && n < (1ll << 31), "tgs_threshold_mask: n out of range");
  if (n == 0) return TGS_OK;
  TGS_REQUIRE(values && thr && mask, "tgs_threshold_mask: null pointer");
  hipStream_t s = as_stream(stream);
  hipLaunchKernelGGL(threshold_mask_kernel, dim3((unsigned)ceil_div(n, (int64_t)256)), dim3(256), 0, s, values, n,
                     thr, mask);
  return hip_status("tgs_threshold_mask");
}

extern "C" int32_t tgs_density_score(const float* stats, int64_t n, float lambda_base, float rho, float eps,
                                     float* e_out, float* d_out, float* s_out, void* stream) {
  TGS_REQUIRE(n >= 0 && n < (1ll << 31), "tgs_density_score: n out of range");
  TGS_REQUIRE(eps > 0.f, "tgs_density_score: eps %g must be positive", (double)eps);
  TGS_REQUIRE(rho >= 0.f && rho <= 1.f, "tgs_density_score: rho %g not in [0, 1]", (double)rho);
  if (n == 0) return TGS_OK;
  TGS_REQUIRE(stats && s_out, "tgs_density_score: null pointer");
  TGS_REQUIRE(((uintptr_t)stats & 15) == 0, "tgs_density_score: stats must be 16-byte aligned");
  hipStream_t s = as_stream(stream);
  const float lam = lambda_base * (1.0f - rho);
  hipLaunchKernelGGL(density_score_kernel, dim3((unsigned)ceil_div(n, (int64_t)256)), dim3(256), 0, s, stats, n,
                     eps, lam, e_out, d_out, s_out);
  return hip_status("tgs_density_score");
}
