// Hybrid moment-damped LM / Adam update.
//
// HBM-bound: per touched Gaussian it reads params, grad, m, v (4 x 59 floats)
// and writes params, m, v.  Two launches split the rows by their kind of
// work so each runs at its own occupancy:
//   lm_kernel     one thread per Gaussian, the two LM blocks (rows 0-13):
//                 10x10 and 4x4 damped systems solved exactly in FP64
//   adam_kernel   the plain Adam rows (14-58, or all rows in Adam mode): a
//                 row per grid line, four consecutive Gaussians per thread
//                 with 16-byte loads when the row length allows
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

// Rows row0 + blockIdx.y; thread handles Gaussians [i0, i0 + 4).  kVec: the
// row length is a multiple of 4, so the four values are one aligned float4.
template <bool kVec>
__global__ void __launch_bounds__(256) adam_kernel(float* __restrict__ p, const float* __restrict__ grad,
                                                   float* __restrict__ m, float* __restrict__ v, int64_t n,
                                                   const uint8_t* __restrict__ touched, int row0, OptArgs o) {
  const int row = row0 + (int)blockIdx.y;
  const int64_t i0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * 4;
  if (i0 >= n) return;
  const double lr = row_lr_bc1(o, row);
  const int64_t base = (int64_t)row * n + i0;
  if (kVec) {
    bool t[4] = {true, true, true, true};
    if (touched != nullptr) {
      const uchar4 tt = *reinterpret_cast<const uchar4*>(touched + i0);
      t[0] = tt.x != 0; t[1] = tt.y != 0; t[2] = tt.z != 0; t[3] = tt.w != 0;
      if (!(t[0] || t[1] || t[2] || t[3])) return;
    }
    float4 pp = *reinterpret_cast<const float4*>(p + base);
    const float4 gg = *reinterpret_cast<const float4*>(grad + base);
    float4 mm = *reinterpret_cast<const float4*>(m + base);
    float4 vv = *reinterpret_cast<const float4*>(v + base);
    if (t[0]) adam_elem(pp.x, gg.x, mm.x, vv.x, lr, o);
    if (t[1]) adam_elem(pp.y, gg.y, mm.y, vv.y, lr, o);
    if (t[2]) adam_elem(pp.z, gg.z, mm.z, vv.z, lr, o);
    if (t[3]) adam_elem(pp.w, gg.w, mm.w, vv.w, lr, o);
    // untouched lanes store back the values they read
    *reinterpret_cast<float4*>(p + base) = pp;
    *reinterpret_cast<float4*>(m + base) = mm;
    *reinterpret_cast<float4*>(v + base) = vv;
  } else {
    for (int k = 0; k < 4 && i0 + k < n; ++k) {
      if (touched != nullptr && touched[i0 + k] == 0) continue;
      const int64_t idx = base + k;
      float pp = p[idx], mm = m[idx], vv = v[idx];
      adam_elem(pp, grad[idx], mm, vv, lr, o);
      p[idx] = pp;
      m[idx] = mm;
      v[idx] = vv;
    }
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
  const dim3 grid((unsigned)ceil_div(n, 1024), (unsigned)(TGS_PARAM_ROWS - row0));
  const bool vec = n % 4 == 0 && ((uintptr_t)params & 15) == 0 && ((uintptr_t)grad & 15) == 0 &&
                   ((uintptr_t)m & 15) == 0 && ((uintptr_t)v & 15) == 0 && ((uintptr_t)touched & 3) == 0;
  if (vec)
    hipLaunchKernelGGL(adam_kernel<true>, grid, dim3(256), 0, s, params, grad, m, v, n, touched, row0, o);
  else
    hipLaunchKernelGGL(adam_kernel<false>, grid, dim3(256), 0, s, params, grad, m, v, n, touched, row0, o);
  return hip_status("tgs_optimizer_step");
}
