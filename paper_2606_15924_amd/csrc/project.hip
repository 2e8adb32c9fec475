// EWA projection with SH colour (forward) and its chain rule (backward).
//
// One thread per Gaussian, FP64 arithmetic.  Both kernels are HBM-bound
// (59 floats in, 12-17 out per Gaussian), so FP64 costs nothing measurable
// on gfx950 (78.6 TFLOP/s FP64) and keeps the integer decisions (depth key
// bits, tile rectangle, radius) identical to an FP64 reference written in
// the same operation order.  Parameters are read row by row from the
// [59][n] store, so every load is coalesced across the wave.
#include "projection.h"

// The depth, centre and rectangle must follow a fixed sequence of rounded
// operations; no multiply-add contraction in this file.
#pragma clang fp contract(off)

namespace tgs {

// PT = float: the training path.  PT = double: the FP64 instantiation for
// gradient checks, which also writes the splat record in doubles (rec64:
// centre x, y; conic a, b, c; opacity; r, g, b; depth; two zeros).
// The splat records (48 bytes per Gaussian) and the cleared gradient
// records (36 bytes) of a wave's 64 Gaussians are contiguous, so they are
// written as whole runs: the splat floats staged in LDS, then every lane
// storing consecutive 16-byte pieces (and 4-byte zeros for the gradient),
// instead of each lane writing its own records at a 48- or 36-byte stride.
template <typename PT, int kDeg>
__global__ void __launch_bounds__(256) project_fwd_kernel(
    const PT* __restrict__ params, int64_t n, CamArgs cam, double z_near,
    double dil, float4* __restrict__ splat, float* __restrict__ depth, int* __restrict__ radius,
    int4* __restrict__ rect, uint8_t* __restrict__ clampm, float* __restrict__ g2d_clear,
    double* __restrict__ rec64) {
  __shared__ float4 s_rec[256 / kWave][3 * kWave];
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t b0 = (int64_t)blockIdx.x * blockDim.x;
  if (b0 >= n) return;  // workgroup-uniform
  const bool valid = i < n;
  const int64_t ic = valid ? i : n - 1;  // lanes past the end compute on a valid Gaussian and store nothing
  const int lane = lane_id(), wave = (int)threadIdx.x / kWave;
  const int64_t w0 = i - lane;  // the wave's first Gaussian
  // the SH coefficients are loaded with the geometry rows, before anything
  // depends on them (one round trip to memory; culled Gaussians read them
  // for nothing, a small share of the traffic)
  constexpr int nk = (kDeg + 1) * (kDeg + 1);
  PT cf[3 * nk];
#pragma unroll
  for (int q = 0; q < 3 * nk; ++q) cf[q] = params[(int64_t)(11 + q) * n + ic];
  if (g2d_clear != nullptr && w0 < n) {
    const int64_t end = n * TGS_G2D_FLOATS;
#pragma unroll
    for (int q = 0; q < TGS_G2D_FLOATS; ++q) {
      const int64_t e = w0 * TGS_G2D_FLOATS + q * kWave + lane;
      if (e < end) g2d_clear[e] = 0.f;
    }
  }
  Geom g;
  geometry(params, n, ic, cam, z_near, dil, g);
  float4 r0 = make_float4(0.f, 0.f, 0.f, 0.f), r1 = r0, r2 = make_float4(0.f, 0.f, 0.f, (float)g.t[2]);
  int rad = 0;
  int4 rc = make_int4(0, 0, 0, 0);
  uint8_t cm = 0;
  if (g.visible) {
    // view-dependent colour
    const double dx = g.mu[0] - cam.center[0], dy = g.mu[1] - cam.center[1],
                 dz = g.mu[2] - cam.center[2];
    const double dn = sqrt(dx * dx + dy * dy + dz * dz);
    const double ux = dx / dn, uy = dy / dn, uz = dz / dn;
    double rgb[3] = {0.5, 0.5, 0.5};
#pragma unroll
    for (int k = 0; k < nk; ++k) {
      double Yk, g0, g1, g2;
      sh_term(k, ux, uy, uz, Yk, g0, g1, g2);
      for (int ch = 0; ch < 3; ++ch) rgb[ch] += Yk * (double)cf[3 * k + ch];
    }
    for (int ch = 0; ch < 3; ++ch)
      if (rgb[ch] < 0.0) {
        rgb[ch] = 0.0;
        cm |= (uint8_t)(1u << ch);
      }
    const double opac = 1.0 / (1.0 + exp(-(double)params[10 * n + ic]));
    const double fxp = floor(g.px), fyp = floor(g.py);
    r0 = make_float4((float)fxp, (float)fyp, (float)(g.px - fxp), (float)(g.py - fyp));
    // the conic Q = Sigma'^-1 = [[c, -b], [-b, a]] / det in its LDL^T form:
    // Q_00 = c / det, beta = Q_01 / Q_00 = -b / c, delta = det Q / Q_00 = 1 / c
    r1 = make_float4((float)(g.c / g.det), (float)(-g.b / g.c), (float)(1.0 / g.c), (float)opac);
    r2 = make_float4((float)rgb[0], (float)rgb[1], (float)rgb[2], (float)g.t[2]);
    rad = (int)g.radius;
    rc = make_int4(g.rect[0], g.rect[1], g.rect[2], g.rect[3]);
    if (rec64 != nullptr && valid) {
      const double r64[12] = {g.px, g.py, g.c / g.det, -g.b / g.det, g.a / g.det, opac,
                              rgb[0], rgb[1], rgb[2], g.t[2], 0.0, 0.0};
      for (int k = 0; k < 12; ++k) rec64[12 * i + k] = r64[k];
    }
  } else if (rec64 != nullptr && valid) {
    for (int k = 0; k < 12; ++k) rec64[12 * i + k] = k == 9 ? g.t[2] : 0.0;
  }
  if (valid) {
    depth[i] = (float)g.t[2];
    radius[i] = rad;
    rect[i] = rc;
    clampm[i] = cm;
  }
  float4* sr = s_rec[wave];
  sr[3 * lane] = r0;
  sr[3 * lane + 1] = r1;
  sr[3 * lane + 2] = r2;
  __syncthreads();
  if (w0 < n) {
    const int64_t end = n * 3;
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      const int64_t e = w0 * 3 + q * kWave + lane;
      if (e < end) splat[e] = sr[q * kWave + lane];
    }
  }
}

// accumulate: grad += gradient; otherwise grad = gradient, with zeros for
// culled Gaussians (every row of every Gaussian is written once).
template <typename PT>
__global__ void __launch_bounds__(256) project_bwd_kernel(
    const PT* __restrict__ params, int64_t n, CamArgs cam, int sh_degree, double z_near,
    double dil, const int* __restrict__ radius, const uint8_t* __restrict__ clampm,
    const PT* __restrict__ g2d, PT* __restrict__ grad, bool accumulate) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double gg[9];
  bool any = false;
  for (int k = 0; k < 9; ++k) {
    gg[k] = (double)g2d[i * 9 + k];
    any = any || gg[k] != 0.0;
  }
  // culled, or no screen-space gradient in this view (at sparse rates most
  // Gaussians): the gradient is zero, so nothing is added, or zeros are
  // written, without reading the parameters
  if (radius[i] == 0 || !any) {
    if (!accumulate)
      for (int r = 0; r < TGS_PARAM_ROWS; ++r) grad[(int64_t)r * n + i] = (PT)0;
    return;
  }
  Geom g;
  geometry(params, n, i, cam, z_near, dil, g);
  chain_rule(params, n, i, cam, sh_degree, g, gg, clampm[i], [&](int row, double v) {
    const int64_t idx = (int64_t)row * n + i;
    grad[idx] = accumulate ? grad[idx] + (PT)v : (PT)v;
  });
}

}  // namespace tgs

using namespace tgs;


extern "C" int32_t tgs_project(const float* params, int64_t n, const tgs_camera* cam,
                               const tgs_raster_params* rp, float* splat, float* depth,
                               int32_t* radius, int32_t* rect, uint8_t* clamp, float* g2d_clear,
                               void* stream) {
  TGS_REQUIRE(n >= 0, "tgs_project: n < 0");
  TGS_REQUIRE(cam != nullptr && cam->width > 0 && cam->height > 0, "tgs_project: bad camera");
  if (int32_t e = check_raster_params(rp)) return e;
  if (n == 0) return TGS_OK;
  TGS_REQUIRE(params && splat && depth && radius && rect && clamp, "tgs_project: null pointer");
  TGS_REQUIRE(((uintptr_t)splat & 15) == 0 && ((uintptr_t)rect & 15) == 0,
              "tgs_project: splat and rect must be 16-byte aligned");
  const CamArgs ca = make_cam(cam);
  const int block = 256;
  const dim3 grid((unsigned)ceil_div(n, block));
  hipStream_t s = as_stream(stream);
#define TGS_PROJECT(D)                                                                                           \
  hipLaunchKernelGGL((project_fwd_kernel<float, D>), grid, dim3(block), 0, s, params, n, ca, (double)rp->z_near, \
                     (double)rp->dilation, (float4*)splat, depth, radius, (int4*)rect, clamp, g2d_clear,      \
                     (double*)nullptr)
  switch (rp->sh_degree) {
    case 0: TGS_PROJECT(0); break;
    case 1: TGS_PROJECT(1); break;
    case 2: TGS_PROJECT(2); break;
    default: TGS_PROJECT(3); break;
  }
#undef TGS_PROJECT
  return hip_status("tgs_project");
}

extern "C" int32_t tgs_project_bwd(const float* params, int64_t n, const tgs_camera* cam,
                                   const tgs_raster_params* rp, const int32_t* radius,
                                   const uint8_t* clamp, const float* g2d, float* grad,
                                   int32_t accumulate, void* stream) {
  TGS_REQUIRE(n >= 0, "tgs_project_bwd: n < 0");
  TGS_REQUIRE(cam != nullptr && cam->width > 0 && cam->height > 0, "tgs_project_bwd: bad camera");
  if (int32_t e = check_raster_params(rp)) return e;
  if (n == 0) return TGS_OK;
  TGS_REQUIRE(params && radius && clamp && g2d && grad, "tgs_project_bwd: null pointer");
  const CamArgs ca = make_cam(cam);
  const int block = 256;
  hipLaunchKernelGGL(project_bwd_kernel<float>, dim3((unsigned)ceil_div(n, block)), dim3(block), 0,
                     as_stream(stream), params, n, ca, rp->sh_degree, (double)rp->z_near,
                     (double)rp->dilation, radius, clamp, g2d, grad, accumulate != 0);
  return hip_status("tgs_project_bwd");
}

// ---- FP64 instantiation (gradient checks): the same kernels over double
// parameters; the float outputs feed tgs_bin_sort as usual.
extern "C" int32_t tgs_project_f64(const double* params, int64_t n, const tgs_camera* cam,
                                   const tgs_raster_params* rp, double* rec64, float* splat, float* depth,
                                   int32_t* radius, int32_t* rect, uint8_t* clamp, void* stream) {
  TGS_REQUIRE(n >= 0, "tgs_project_f64: n < 0");
  TGS_REQUIRE(cam != nullptr && cam->width > 0 && cam->height > 0, "tgs_project_f64: bad camera");
  if (int32_t e = check_raster_params(rp)) return e;
  if (n == 0) return TGS_OK;
  TGS_REQUIRE(params && rec64 && splat && depth && radius && rect && clamp, "tgs_project_f64: null pointer");
  TGS_REQUIRE(((uintptr_t)splat & 15) == 0 && ((uintptr_t)rect & 15) == 0,
              "tgs_project_f64: splat and rect must be 16-byte aligned");
  const CamArgs ca = make_cam(cam);
  const int block = 256;
  const dim3 grid((unsigned)ceil_div(n, block));
  hipStream_t s = as_stream(stream);
#define TGS_PROJECT64(D)                                                                                         \
  hipLaunchKernelGGL((project_fwd_kernel<double, D>), grid, dim3(block), 0, s, params, n, ca,                    \
                     (double)rp->z_near, (double)rp->dilation, (float4*)splat, depth, radius, (int4*)rect, clamp, \
                     (float*)nullptr, rec64)
  switch (rp->sh_degree) {
    case 0: TGS_PROJECT64(0); break;
    case 1: TGS_PROJECT64(1); break;
    case 2: TGS_PROJECT64(2); break;
    default: TGS_PROJECT64(3); break;
  }
#undef TGS_PROJECT64
  return hip_status("tgs_project_f64");
}

extern "C" int32_t tgs_project_bwd_f64(const double* params, int64_t n, const tgs_camera* cam,
                                       const tgs_raster_params* rp, const int32_t* radius, const uint8_t* clamp,
                                       const double* g2d, double* grad, int32_t accumulate, void* stream) {
  TGS_REQUIRE(n >= 0, "tgs_project_bwd_f64: n < 0");
  TGS_REQUIRE(cam != nullptr && cam->width > 0 && cam->height > 0, "tgs_project_bwd_f64: bad camera");
  if (int32_t e = check_raster_params(rp)) return e;
  if (n == 0) return TGS_OK;
  TGS_REQUIRE(params && radius && clamp && g2d && grad, "tgs_project_bwd_f64: null pointer");
  const CamArgs ca = make_cam(cam);
  const int block = 256;
  hipLaunchKernelGGL(project_bwd_kernel<double>, dim3((unsigned)ceil_div(n, block)), dim3(block), 0,
                     as_stream(stream), params, n, ca, rp->sh_degree, (double)rp->z_near, (double)rp->dilation,
                     radius, clamp, g2d, grad, accumulate != 0);
  return hip_status("tgs_project_bwd_f64");
}
