// Hybrid moment-damped LM / Adam update.
//
// HBM-bound: per touched Gaussian it reads params, grad, m, v (4 x 59 floats)
// and writes params, m, v.  Two launches split the rows by their kind of
// work:
//   lm_kernel     one thread per Gaussian, the two LM blocks (rows 0-13):
//                 10x10 and 4x4 damped systems solved exactly in FP64
//   adam_kernel   one thread per Gaussian, the plain Adam rows (14-58, or
//                 all rows in Adam mode)
#include "optimizer.h"

namespace tgs {

__global__ void __launch_bounds__(256) lm_kernel(float* __restrict__ p, const float* __restrict__ grad,
                                                 float* __restrict__ m, float* __restrict__ v, int64_t n,
                                                 const uint8_t* __restrict__ touched, OptArgs o) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (touched != nullptr && touched[i] == 0) return;
  float gg[10], ga[4];
#pragma unroll
  for (int k = 0; k < 10; ++k) gg[k] = grad[(int64_t)kGeomRows[k] * n + i];
#pragma unroll
  for (int k = 0; k < 4; ++k) ga[k] = grad[(int64_t)kAppRows[k] * n + i];
  lm_update<10>(p, m, v, n, i, kGeomRows, gg, o);
  lm_update<4>(p, m, v, n, i, kAppRows, ga, o);
}

// Rows [row0, TGS_PARAM_ROWS) of one Gaussian per thread: params and grad
// rows coalesced across the wave, the Gaussian's moments contiguous.
__global__ void __launch_bounds__(256) adam_kernel(float* __restrict__ p, const float* __restrict__ grad,
                                                   float* __restrict__ m, float* __restrict__ v, int64_t n,
                                                   const uint8_t* __restrict__ touched, int row0, OptArgs o) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (touched != nullptr && touched[i] == 0) return;
  for (int row = row0; row < TGS_PARAM_ROWS; ++row) {
    const int64_t idx = (int64_t)row * n + i;
    float pp = p[idx], mm = m[mom(i, row)], vv = v[mom(i, row)];
    adam_elem(pp, grad[idx], mm, vv, row_lr_bc1(o, row), o);
    p[idx] = pp;
    m[mom(i, row)] = mm;
    v[mom(i, row)] = vv;
  }
}

}  // namespace tgs

using namespace tgs;

extern "C" int32_t tgs_optimizer_step(float* params, const float* grad, float* m, float* v,
                                      int64_t n, const uint8_t* touched,
                                      const tgs_optim_params* op, int64_t step, void* stream) {
  TGS_REQUIRE(n >= 0, "tgs_optimizer_step: n < 0");
  OptArgs o;
  if (int32_t e = make_opt_args(op, step, "tgs_optimizer_step", o)) return e;
  if (n == 0) return TGS_OK;
  TGS_REQUIRE(params && grad && m && v, "tgs_optimizer_step: null pointer");
  hipStream_t s = as_stream(stream);
  if (o.lm_mode != 2)
    hipLaunchKernelGGL(lm_kernel, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, s, params, grad, m, v, n,
                       touched, o);
  const int row0 = o.lm_mode == 2 ? 0 : 14;
  hipLaunchKernelGGL(adam_kernel, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, s, params, grad, m, v, n, touched,
                     row0, o);
  return hip_status("tgs_optimizer_step");
}
