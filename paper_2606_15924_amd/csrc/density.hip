// Difficulty score of the error-driven density control (Sec. 3.8,
// Eq. gauss_score) from the back-projected sums of tgs_density_accumulate:
// e_i = E_i / (W_i + eps), d_i = D_i / (W_i + eps), s_i = e_i + lambda_eff d_i
// with lambda_eff = lambda_base (1 - rho).  Elementwise and HBM-bound:
// 12 bytes read and up to 12 written per Gaussian, one Gaussian per thread.
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
  float e, d, sc;
  score_one(stats[i], stats[n + i], stats[2 * n + i], eps, lam, e, d, sc);
  if (e_out != nullptr) e_out[i] = e;
  if (d_out != nullptr) d_out[i] = d;
  s_out[i] = sc;
}

}  // namespace tgs

using namespace tgs;

extern "C" int32_t tgs_density_score(const float* stats, int64_t n, float lambda_base, float rho, float eps,
                                     float* e_out, float* d_out, float* s_out, void* stream) {
  TGS_REQUIRE(n >= 0 && n < (1ll << 31), "tgs_density_score: n out of range");
  TGS_REQUIRE(eps > 0.f, "tgs_density_score: eps %g must be positive", (double)eps);
  TGS_REQUIRE(rho >= 0.f && rho <= 1.f, "tgs_density_score: rho %g not in [0, 1]", (double)rho);
  if (n == 0) return TGS_OK;
  TGS_REQUIRE(stats && s_out, "tgs_density_score: null pointer");
  hipStream_t s = as_stream(stream);
  const float lam = lambda_base * (1.0f - rho);
  hipLaunchKernelGGL(density_score_kernel, dim3((unsigned)ceil_div(n, (int64_t)256)), dim3(256), 0, s, stats, n,
                     eps, lam, e_out, d_out, s_out);
  return hip_status("tgs_density_score");
}
