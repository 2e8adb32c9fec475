// Projection backward fused with the optimizer step, for the last view of
// a training step: the chain rule produces each parameter row's gradient in
// registers and the row is updated in the same pass, so the gradient never
// goes through HBM.  Two launches split the rows by their work:
//   sh_rest_kernel   the SH rows of degree >= 1 (rows 14-58, always Adam
//                    rows): their gradient Y_k(u) * dL/drgb,
//                    the Adam update, and the partial dL/du of these rows
//                    (three doubles per Gaussian in the workspace); each
//                    SH term's rows are loaded while the previous term is
//                    updated, so the kernel streams at close to HBM rate
//   geom_lm_kernel   the geometry chain rule and rows 0-13 (SH DC, opacity,
//                    mean, scale, quaternion) with the LM (or Adam) update;
//                    its rows reach LDS while the chain rule runs
// The SH-rest kernel reads the coefficients before updating them, and the
// geometry kernel only touches rows 0-13, so running them in this order
// gives each the values the unfused path sees.  Results equal
// tgs_project_bwd followed by tgs_optimizer_step bit for bit: gradients are
// rounded to float as the unfused path stores them, the dL/du sum keeps
// its order (the DC term contributes an exact zero), and both paths share
// the update functions.
#include <algorithm>

#include "optimizer.h"
#include "projection.h"

namespace tgs {

template <int kDeg>
__global__ void __launch_bounds__(256) sh_rest_kernel(
    float* params, int64_t n, CamArgs cam, const int* __restrict__ radius, const uint8_t* __restrict__ clampm,
    const float* __restrict__ g2d, const float* __restrict__ grad_prev, float* __restrict__ m,
    float* __restrict__ v, const uint8_t* __restrict__ touched, OptArgs o, double* __restrict__ dL_du_out) {
#pragma clang fp contract(off)
  constexpr int nk = (kDeg + 1) * (kDeg + 1);
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (touched != nullptr && touched[i] == 0) return;  // untouched: parameters and moments stay
  const bool vis = radius[i] != 0;
  double drgb[3] = {0.0, 0.0, 0.0}, dL_du[3] = {0.0, 0.0, 0.0};
  ViewDir u{};
  if (vis) {
    double mu[3], gg[9];
    for (int k = 0; k < 3; ++k) mu[k] = (double)params[(int64_t)k * n + i];
    for (int k = 0; k < 9; ++k) gg[k] = (double)g2d[i * 9 + k];
    u = view_dir(mu, cam);
    color_grad(gg, clampm[i], drgb);
  }
  // SH terms k = 1..15 (rows 11 + 3k + ch), software-pipelined: the rows of
  // term k + 1 are loaded before term k is updated and stored.  The
  // arithmetic is that of the projection backward (SH part) followed by Adam.
  struct Rows { float p[3], m[3], v[3], g[3]; };
  auto load = [&](int k, Rows& r) {
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) {
      const int64_t idx = (int64_t)(11 + 3 * k + ch) * n + i;
      r.p[ch] = params[idx];
      r.m[ch] = m[idx];
      r.v[ch] = v[idx];
      r.g[ch] = grad_prev != nullptr ? grad_prev[idx] : 0.f;
    }
  };
  Rows cur, nxt;
  load(1, cur);
#pragma unroll
  for (int k = 1; k < 16; ++k) {
    if (k + 1 < 16) load(k + 1, nxt);
    __builtin_amdgcn_sched_barrier(0);
    double grad[3] = {0.0, 0.0, 0.0};
    if (vis && k < nk) {
      double Yk, d0, d1, d2;
      sh_term(k, u.ux, u.uy, u.uz, Yk, d0, d1, d2);
      double gk = 0.0;
#pragma unroll
      for (int ch = 0; ch < 3; ++ch) {
        gk += (double)cur.p[ch] * drgb[ch];
        grad[ch] = Yk * drgb[ch];
      }
      dL_du[0] += d0 * gk;
      dL_du[1] += d1 * gk;
      dL_du[2] += d2 * gk;
    }
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) {
      const int row = 11 + 3 * k + ch;
      const int64_t idx = (int64_t)row * n + i;
      float pp = cur.p[ch], mm = cur.m[ch], vv = cur.v[ch];
      const float gf = grad_prev != nullptr ? cur.g[ch] + (float)grad[ch] : (float)grad[ch];
      adam_elem(pp, gf, mm, vv, row_lr_bc1(o, row), o);
      params[idx] = pp;
      m[idx] = mm;
      v[idx] = vv;
    }
    if (k + 1 < 16) cur = nxt;
  }
  if (vis)
    for (int k = 0; k < 3; ++k) dL_du_out[i * 3 + k] = dL_du[k];
}

// Rows 0-13 of every Gaussian the wave updates: parameters, moments and (when
// there is one) the earlier views' gradient are copied into LDS by the
// memory system while the chain rule runs, so the update does not wait for
// them at the end.  One wave per workgroup; LDS holds kPre (or kPre + 14)
// rows of 64 floats.
constexpr int kGeoRows = 14;
constexpr int kPre = 3 * kGeoRows;  // params, m, v

__global__ void __launch_bounds__(kWave) geom_lm_kernel(
    float* params, int64_t n, CamArgs cam, int sh_degree, double z_near, double dil,
    const int* __restrict__ radius, const uint8_t* __restrict__ clampm, const float* __restrict__ g2d,
    const float* __restrict__ grad_prev, float* __restrict__ m, float* __restrict__ v,
    const uint8_t* __restrict__ touched, OptArgs o, const double* __restrict__ dL_du_in) {
  extern __shared__ float s_rows[];  // [kPre (+ 14)][64]
  const int lane = threadIdx.x;
  const int64_t i = (int64_t)blockIdx.x * kWave + lane;
  const int64_t ic = i < n ? i : n - 1;  // lanes past the end load a valid element
  // asynchronous row copies global -> LDS: lane l's value lands at [row][l]
  const float* srcs[4] = {params, m, v, grad_prev};
  const int n_src = grad_prev != nullptr ? 4 : 3;
  for (int q = 0; q < n_src; ++q)
#pragma unroll
    for (int r = 0; r < kGeoRows; ++r)
      __builtin_amdgcn_global_load_lds(srcs[q] + (int64_t)r * n + ic, s_rows + (q * kGeoRows + r) * kWave, 4, 0, 0);

  const bool live = i < n && (touched == nullptr || touched[i] != 0);  // untouched: nothing changes
  float gl[kGeoRows];  // this view's gradient of rows 0-13, rounded to float
  if (live) {
    auto sink = [&](int row, double val) { gl[row] = (float)val; };
    if (radius[i] != 0) {
      Geom g;
      geometry(params, n, i, cam, z_near, dil, g);
      double gg[9];
      for (int k = 0; k < 9; ++k) gg[k] = (double)g2d[i * 9 + k];
      const ViewDir u = view_dir(g.mu, cam);
      double drgb[3];
      color_grad(gg, clampm[i], drgb);
      double dc_du[3] = {0.0, 0.0, 0.0};  // the DC basis is constant: no dL/du
      sh_backward(params, n, i, u, drgb, n_sh(sh_degree), 0, 1, dc_du, sink);
      const double dL_du[3] = {dL_du_in[i * 3], dL_du_in[i * 3 + 1], dL_du_in[i * 3 + 2]};
      geom_backward(params, n, i, cam, g, gg, u, dL_du, sink);
    } else {
#pragma unroll
      for (int r = 0; r < kGeoRows; ++r) gl[r] = 0.f;
    }
  }
  __builtin_amdgcn_s_waitcnt(0);  // the row copies have landed
  __syncthreads();
  if (!live) return;
  auto at = [&](int q, int row) -> float& { return s_rows[(q * kGeoRows + row) * kWave + lane]; };
  // the step's gradient as the unfused path stores it
  if (grad_prev != nullptr)
#pragma unroll
    for (int r = 0; r < kGeoRows; ++r) gl[r] = at(3, r) + gl[r];
  auto store = [&](int row, float pp, float mm, float vv) {
    const int64_t idx = (int64_t)row * n + i;
    m[idx] = mm;
    v[idx] = vv;
    params[idx] = pp;
  };
  if (o.lm_mode == 2) {
#pragma unroll
    for (int r = 0; r < kGeoRows; ++r) {
      float pp = at(0, r), mm = at(1, r), vv = at(2, r);
      adam_elem(pp, gl[r], mm, vv, row_lr_bc1(o, r), o);
      store(r, pp, mm, vv);
    }
    return;
  }
  float pg[10], mg[10], vg[10], gg[10];
#pragma unroll
  for (int k = 0; k < 10; ++k) {
    pg[k] = at(0, kGeomRows[k]);
    mg[k] = at(1, kGeomRows[k]);
    vg[k] = at(2, kGeomRows[k]);
    gg[k] = gl[kGeomRows[k]];
  }
  lm_block<10>(pg, mg, vg, kGeomRows, gg, o);
#pragma unroll
  for (int k = 0; k < 10; ++k) store(kGeomRows[k], pg[k], mg[k], vg[k]);
  float pa[4], ma[4], va[4], ga[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    pa[k] = at(0, kAppRows[k]);
    ma[k] = at(1, kAppRows[k]);
    va[k] = at(2, kAppRows[k]);
    ga[k] = gl[kAppRows[k]];
  }
  lm_block<4>(pa, ma, va, kAppRows, ga, o);
#pragma unroll
  for (int k = 0; k < 4; ++k) store(kAppRows[k], pa[k], ma[k], va[k]);
}

// ---- every view of a step in one pass: the chain rule of each view is
// evaluated in registers and summed (in FP64) before the update, so neither
// the earlier views' projection backward nor their gradient array is
// needed.  Same split as above; the SH kernel leaves each view's partial
// dL/du in the workspace ([view][n][3] doubles) for the geometry kernel.
constexpr int kMaxViews = 16;

struct ViewSet {
  CamArgs cam[kMaxViews];
  const int* radius[kMaxViews];
  const uint8_t* clampm[kMaxViews];
  const float* g2d[kMaxViews];
  int nv;
};

// SH rows in three groups of five terms (15 rows): per group the view loop
// sums each row's gradient and adds the group's share of each view's
// dL/du to the workspace (the first group stores it), which keeps the
// registers of one group live rather than all 45 rows'.
template <int kDeg>
__global__ void __launch_bounds__(256) sh_rest_views_kernel(float* params, int64_t n, ViewSet vs, float* __restrict__ m,
                                                            float* __restrict__ v, const uint8_t* __restrict__ touched,
                                                            OptArgs o, double* __restrict__ dL_du_out) {
#pragma clang fp contract(off)
  constexpr int nk = (kDeg + 1) * (kDeg + 1);
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (touched != nullptr && touched[i] == 0) return;  // untouched: parameters and moments stay
  double mu[3];
  for (int k = 0; k < 3; ++k) mu[k] = (double)params[(int64_t)k * n + i];
#pragma unroll
  for (int grp = 0; grp < 3; ++grp) {
    float cf[15];
#pragma unroll
    for (int r = 0; r < 15; ++r) cf[r] = params[(int64_t)(14 + 15 * grp + r) * n + i];
    double gs[15];
#pragma unroll
    for (int r = 0; r < 15; ++r) gs[r] = 0.0;
    for (int j = 0; j < vs.nv; ++j) {
      double* du_out = dL_du_out + ((int64_t)j * n + i) * 3;
      const bool vis = vs.radius[j][i] != 0;
      double du[3] = {0.0, 0.0, 0.0};
      if (vis && 1 + 5 * grp < nk) {
        double gg[9];
        for (int k = 0; k < 9; ++k) gg[k] = (double)vs.g2d[j][i * 9 + k];
        const ViewDir u = view_dir(mu, vs.cam[j]);
        double drgb[3];
        color_grad(gg, vs.clampm[j][i], drgb);
#pragma unroll
        for (int t = 0; t < 5; ++t) {
          const int k = 1 + 5 * grp + t;
          if (k >= nk) break;
          double Yk, d0, d1, d2;
          sh_term(k, u.ux, u.uy, u.uz, Yk, d0, d1, d2);
          double gk = 0.0;
#pragma unroll
          for (int ch = 0; ch < 3; ++ch) {
            gk += (double)cf[3 * t + ch] * drgb[ch];
            gs[3 * t + ch] += Yk * drgb[ch];
          }
          du[0] += d0 * gk;
          du[1] += d1 * gk;
          du[2] += d2 * gk;
        }
      }
      if (grp == 0) {
        for (int k = 0; k < 3; ++k) du_out[k] = du[k];
      } else if (vis && 1 + 5 * grp < nk) {
        for (int k = 0; k < 3; ++k) du_out[k] = du_out[k] + du[k];
      }
    }
#pragma unroll
    for (int r = 0; r < 15; ++r) {
      const int row = 14 + 15 * grp + r;
      const int64_t idx = (int64_t)row * n + i;
      float pp = cf[r], mm = m[idx], vv = v[idx];
      adam_elem(pp, (float)gs[r], mm, vv, row_lr_bc1(o, row), o);
      params[idx] = pp;
      m[idx] = mm;
      v[idx] = vv;
    }
  }
}

__global__ void __launch_bounds__(64) geom_lm_views_kernel(float* params, int64_t n, ViewSet vs, int sh_degree,
                                                           double z_near, double dil, float* __restrict__ m,
                                                           float* __restrict__ v, const uint8_t* __restrict__ touched,
                                                           OptArgs o, const double* __restrict__ dL_du_in) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (touched != nullptr && touched[i] == 0) return;
  double gsum[kGeoRows];
#pragma unroll
  for (int r = 0; r < kGeoRows; ++r) gsum[r] = 0.0;
  auto sink = [&](int row, double val) { gsum[row] += val; };
  for (int j = 0; j < vs.nv; ++j) {
    if (vs.radius[j][i] == 0) continue;
    Geom g;
    geometry(params, n, i, vs.cam[j], z_near, dil, g);
    double gg[9];
    for (int k = 0; k < 9; ++k) gg[k] = (double)vs.g2d[j][i * 9 + k];
    const ViewDir u = view_dir(g.mu, vs.cam[j]);
    double drgb[3];
    color_grad(gg, vs.clampm[j][i], drgb);
    double dc_du[3] = {0.0, 0.0, 0.0};  // the DC basis is constant: no dL/du
    sh_backward(params, n, i, u, drgb, n_sh(sh_degree), 0, 1, dc_du, sink);
    const int64_t w = ((int64_t)j * n + i) * 3;
    const double dL_du[3] = {dL_du_in[w], dL_du_in[w + 1], dL_du_in[w + 2]};
    geom_backward(params, n, i, vs.cam[j], g, gg, u, dL_du, sink);
  }
  auto store = [&](int row, float pp, float mm, float vv) {
    const int64_t idx = (int64_t)row * n + i;
    m[idx] = mm;
    v[idx] = vv;
    params[idx] = pp;
  };
  auto load = [&](int row, float& pp, float& mm, float& vv) {
    const int64_t idx = (int64_t)row * n + i;
    pp = params[idx];
    mm = m[idx];
    vv = v[idx];
  };
  if (o.lm_mode == 2) {
#pragma unroll
    for (int r = 0; r < kGeoRows; ++r) {
      float pp, mm, vv;
      load(r, pp, mm, vv);
      adam_elem(pp, (float)gsum[r], mm, vv, row_lr_bc1(o, r), o);
      store(r, pp, mm, vv);
    }
    return;
  }
  float pg[10], mg[10], vg[10], gq[10];
#pragma unroll
  for (int k = 0; k < 10; ++k) {
    load(kGeomRows[k], pg[k], mg[k], vg[k]);
    gq[k] = (float)gsum[kGeomRows[k]];
  }
  lm_block<10>(pg, mg, vg, kGeomRows, gq, o);
#pragma unroll
  for (int k = 0; k < 10; ++k) store(kGeomRows[k], pg[k], mg[k], vg[k]);
  float pa[4], ma[4], va[4], ga[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    load(kAppRows[k], pa[k], ma[k], va[k]);
    ga[k] = (float)gsum[kAppRows[k]];
  }
  lm_block<4>(pa, ma, va, kAppRows, ga, o);
#pragma unroll
  for (int k = 0; k < 4; ++k) store(kAppRows[k], pa[k], ma[k], va[k]);
}

}  // namespace tgs

using namespace tgs;

extern "C" size_t tgs_project_bwd_optimizer_views_workspace_size(int64_t n, int32_t n_views) {
  if (n < 0 || n_views < 0) return 0;
  return align_up((size_t)(3 * std::max<int64_t>(n, 1)) * (size_t)std::max(n_views, 1) * sizeof(double), 256);
}

extern "C" int32_t tgs_project_bwd_optimizer_step_views(float* params, int64_t n, int32_t n_views,
                                                        const tgs_camera* cams, const tgs_raster_params* rp,
                                                        const int32_t* const* radius, const uint8_t* const* clamp,
                                                        const float* const* g2d, float* m, float* v,
                                                        const uint8_t* touched, const tgs_optim_params* op,
                                                        int64_t step, void* ws, size_t ws_bytes, void* stream) {
  const char* who = "tgs_project_bwd_optimizer_step_views";
  TGS_REQUIRE(n >= 0, "%s: n < 0", who);
  TGS_REQUIRE(n_views >= 1 && n_views <= kMaxViews, "%s: %d views not in 1..%d", who, n_views, kMaxViews);
  TGS_REQUIRE(cams && radius && clamp && g2d, "%s: null view arrays", who);
  if (int32_t e = check_raster_params(rp)) return e;
  OptArgs o;
  if (int32_t e = make_opt_args(op, step, who, o)) return e;
  if (n == 0) return TGS_OK;
  TGS_REQUIRE(params && m && v && ws, "%s: null pointer", who);
  ViewSet vs;
  vs.nv = n_views;
  for (int j = 0; j < n_views; ++j) {
    TGS_REQUIRE(cams[j].width > 0 && cams[j].height > 0, "%s: bad camera %d", who, j);
    TGS_REQUIRE(radius[j] && clamp[j] && g2d[j], "%s: null pointer of view %d", who, j);
    vs.cam[j] = make_cam(&cams[j]);
    vs.radius[j] = radius[j];
    vs.clampm[j] = clamp[j];
    vs.g2d[j] = g2d[j];
  }
  for (int j = n_views; j < kMaxViews; ++j) {
    vs.cam[j] = vs.cam[0];
    vs.radius[j] = nullptr;
    vs.clampm[j] = nullptr;
    vs.g2d[j] = nullptr;
  }
  const size_t need = tgs_project_bwd_optimizer_views_workspace_size(n, n_views);
  TGS_REQUIRE(ws_bytes >= need, "%s: workspace %zu bytes < %zu", who, ws_bytes, need);
  TGS_REQUIRE(((uintptr_t)ws & 7) == 0, "%s: workspace must be 8-byte aligned", who);
  hipStream_t s = as_stream(stream);
  const dim3 grid((unsigned)ceil_div(n, 256));
#define TGS_SH_VIEWS(D)                                                                                       \
  hipLaunchKernelGGL(sh_rest_views_kernel<D>, grid, dim3(256), 0, s, params, n, vs, m, v, touched, o, (double*)ws)
  switch (rp->sh_degree) {
    case 0: TGS_SH_VIEWS(0); break;
    case 1: TGS_SH_VIEWS(1); break;
    case 2: TGS_SH_VIEWS(2); break;
    default: TGS_SH_VIEWS(3); break;
  }
#undef TGS_SH_VIEWS
  hipLaunchKernelGGL(geom_lm_views_kernel, dim3((unsigned)ceil_div(n, 64)), dim3(64), 0, s, params, n, vs,
                     rp->sh_degree, (double)rp->z_near, (double)rp->dilation, m, v, touched, o, (const double*)ws);
  return hip_status(who);
}

extern "C" size_t tgs_project_bwd_optimizer_workspace_size(int64_t n) {
  return n < 0 ? 0 : align_up((size_t)(3 * std::max<int64_t>(n, 1)) * sizeof(double), 256);
}

extern "C" int32_t tgs_project_bwd_optimizer_step(float* params, int64_t n, const tgs_camera* cam,
                                                  const tgs_raster_params* rp, const int32_t* radius,
                                                  const uint8_t* clamp, const float* g2d,
                                                  const float* grad_prev, float* m, float* v,
                                                  const uint8_t* touched, const tgs_optim_params* op,
                                                  int64_t step, void* ws, size_t ws_bytes, void* stream) {
  const char* who = "tgs_project_bwd_optimizer_step";
  TGS_REQUIRE(n >= 0, "%s: n < 0", who);
  TGS_REQUIRE(cam != nullptr && cam->width > 0 && cam->height > 0, "%s: bad camera", who);
  if (int32_t e = check_raster_params(rp)) return e;
  OptArgs o;
  if (int32_t e = make_opt_args(op, step, who, o)) return e;
  if (n == 0) return TGS_OK;
  TGS_REQUIRE(params && radius && clamp && g2d && m && v && ws, "%s: null pointer", who);
  TGS_REQUIRE(ws_bytes >= tgs_project_bwd_optimizer_workspace_size(n), "%s: workspace %zu bytes < %zu", who,
              ws_bytes, tgs_project_bwd_optimizer_workspace_size(n));
  TGS_REQUIRE(((uintptr_t)ws & 7) == 0, "%s: workspace must be 8-byte aligned", who);
  const CamArgs ca = make_cam(cam);
  hipStream_t s = as_stream(stream);
  const dim3 grid((unsigned)ceil_div(n, 256));
#define TGS_SH_REST(D)                                                                                \
  hipLaunchKernelGGL(sh_rest_kernel<D>, grid, dim3(256), 0, s, params, n, ca, radius, clamp, g2d, grad_prev, m, v, \
                     touched, o, (double*)ws)
  switch (rp->sh_degree) {
    case 0: TGS_SH_REST(0); break;
    case 1: TGS_SH_REST(1); break;
    case 2: TGS_SH_REST(2); break;
    default: TGS_SH_REST(3); break;
  }
#undef TGS_SH_REST
  const size_t lds = (size_t)(grad_prev != nullptr ? kPre + kGeoRows : kPre) * kWave * sizeof(float);
  hipLaunchKernelGGL(geom_lm_kernel, dim3((unsigned)ceil_div(n, kWave)), dim3(kWave), lds, s, params, n, ca,
                     rp->sh_degree, (double)rp->z_near, (double)rp->dilation, radius, clamp, g2d, grad_prev, m, v,
                     touched, o, (const double*)ws);
  return hip_status(who);
}
