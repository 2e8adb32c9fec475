// Difficulty score of the error-driven density control (Sec. 3.8,
// Eq. gauss_score) from the back-projected sums of tgs_density_accumulate:
// e_i = E_i / (W_i + eps), d_i = D_i / (W_i + eps), s_i = e_i + lambda_eff d_i
// with lambda_eff = lambda_base (1 - rho).  Elementwise and HBM-bound:
// 16 bytes read (one [E, W, D, -] slot) and up to 12 written per Gaussian,
// one Gaussian per thread.
#include <algorithm>

#include "common.h"
#include "scan.h"

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

// ------------------------------------------------------------------ densify and prune
// The step that acts on the selections (Alg. 1 step 11): Gaussians with
// keep = 0 are dropped, the kept ones stay in order, then one new Gaussian
// per kept Gaussian with densify = 1, in order.  A densified Gaussian whose
// largest log-scale exceeds log_split is split: with o = R(q/|q|) diag(exp(s)) z
// the kept slot moves to mean + o and the new one to mean - o, both with the
// log-scales lowered by ln 1.6; otherwise the new one is a clone.  Split
// and new Gaussians restart their moments at zero.  Output positions come
// from exclusive scans of the two flag arrays (the count call), so a thread
// per Gaussian writes its rows with no atomics.
constexpr float kLnSplit = 0.47000362924573558f;  // ln 1.6

struct TopoWs {
  uint32_t* kflag;
  uint32_t* dflag;
  uint32_t* koff;  // [n + 1]
  uint32_t* doff;  // [n + 1]
  uint32_t* part;
  size_t bytes;
};

static TopoWs topo_layout(void* base, int64_t n) {
  TopoWs w{};
  size_t o = 0;
  auto take = [&](size_t b) {
    void* p = base ? (void*)((char*)base + o) : nullptr;
    o += (b + 255) / 256 * 256;
    return (uint32_t*)p;
  };
  w.kflag = take(sizeof(uint32_t) * n);
  w.dflag = take(sizeof(uint32_t) * n);
  w.koff = take(sizeof(uint32_t) * (n + 1));
  w.doff = take(sizeof(uint32_t) * (n + 1));
  w.part = take(sizeof(uint32_t) * scan_partials(n));
  w.bytes = o;
  return w;
}

__global__ void __launch_bounds__(256) topo_flags_kernel(const uint8_t* __restrict__ keep,
                                                         const uint8_t* __restrict__ dens, int64_t n,
                                                         uint32_t* __restrict__ kflag,
                                                         uint32_t* __restrict__ dflag) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const uint32_t k = keep[i] != 0 ? 1u : 0u;
  kflag[i] = k;
  dflag[i] = k & (dens[i] != 0 ? 1u : 0u);
}

__global__ void __launch_bounds__(256) topo_apply_kernel(const float* __restrict__ p, const float* __restrict__ m,
                                                         const float* __restrict__ v, int64_t n,
                                                         const uint32_t* __restrict__ kflag,
                                                         const uint32_t* __restrict__ dflag,
                                                         const uint32_t* __restrict__ koff,
                                                         const uint32_t* __restrict__ doff,
                                                         const float* __restrict__ z, float log_split,
                                                         float* __restrict__ po, float* __restrict__ mo,
                                                         float* __restrict__ vo, int64_t n_out) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n || kflag[i] == 0u) return;
  const bool dn = dflag[i] != 0u;
  const int64_t dst = koff[i];
  const int64_t dst2 = (int64_t)koff[n] + doff[i];
  if (dst >= n_out || (dn && dst2 >= n_out)) return;  // an n_out not from the count call: stay in bounds
  const float s0 = p[3 * n + i], s1 = p[4 * n + i], s2 = p[5 * n + i];
  const bool split = dn && fmaxf(s0, fmaxf(s1, s2)) > log_split;
  float o[3] = {0.f, 0.f, 0.f};
  if (split) {
    float qw = p[6 * n + i], qx = p[7 * n + i], qy = p[8 * n + i], qz = p[9 * n + i];
    const float inv = 1.0f / sqrtf(qw * qw + qx * qx + qy * qy + qz * qz);
    qw *= inv; qx *= inv; qy *= inv; qz *= inv;
    const float e0 = expf(s0) * z[3 * i], e1 = expf(s1) * z[3 * i + 1], e2 = expf(s2) * z[3 * i + 2];
    const float R00 = 1.f - 2.f * (qy * qy + qz * qz), R01 = 2.f * (qx * qy - qw * qz), R02 = 2.f * (qx * qz + qw * qy);
    const float R10 = 2.f * (qx * qy + qw * qz), R11 = 1.f - 2.f * (qx * qx + qz * qz), R12 = 2.f * (qy * qz - qw * qx);
    const float R20 = 2.f * (qx * qz - qw * qy), R21 = 2.f * (qy * qz + qw * qx), R22 = 1.f - 2.f * (qx * qx + qy * qy);
    o[0] = R00 * e0 + R01 * e1 + R02 * e2;
    o[1] = R10 * e0 + R11 * e1 + R12 * e2;
    o[2] = R20 * e0 + R21 * e1 + R22 * e2;
  }
  for (int r = 0; r < TGS_PARAM_ROWS; ++r) {
    const float val = p[(int64_t)r * n + i];
    float kv = val, nv = val;
    if (split && r < 3) {
      kv = val + o[r];
      nv = val - o[r];
    } else if (split && r < 6) {
      kv = nv = val - kLnSplit;
    }
    po[(int64_t)r * n_out + dst] = kv;
    if (dn) po[(int64_t)r * n_out + dst2] = nv;
  }
  // the moments are Gaussian-major: each record (TGS_MOMENT_STRIDE floats)
  // moves whole, 16 bytes per access, all loads before the stores (a row at
  // a time would touch every record's lines once per row)
  constexpr int kQ = TGS_MOMENT_STRIDE / 4;
  const float4* ms = reinterpret_cast<const float4*>(m) + i * kQ;
  const float4* vs = reinterpret_cast<const float4*>(v) + i * kQ;
  float4* md = reinterpret_cast<float4*>(mo) + dst * kQ;
  float4* vd = reinterpret_cast<float4*>(vo) + dst * kQ;
  const float4 z4 = make_float4(0.f, 0.f, 0.f, 0.f);
  for (int h = 0; h < 2; ++h) {  // two halves, eight 16-byte pieces each
    float4 a[kQ / 2], b[kQ / 2];
#pragma unroll
    for (int q = 0; q < kQ / 2; ++q) {
      a[q] = split ? z4 : ms[h * (kQ / 2) + q];
      b[q] = split ? z4 : vs[h * (kQ / 2) + q];
    }
#pragma unroll
    for (int q = 0; q < kQ / 2; ++q) {
      md[h * (kQ / 2) + q] = a[q];
      vd[h * (kQ / 2) + q] = b[q];
    }
  }
  if (dn) {
    float4* md2 = reinterpret_cast<float4*>(mo) + dst2 * kQ;
    float4* vd2 = reinterpret_cast<float4*>(vo) + dst2 * kQ;
#pragma unroll
    for (int q = 0; q < kQ; ++q) {
      md2[q] = z4;
      vd2[q] = z4;
    }
  }
}

// ------------------------------------------------------------------ screen-space statistics
// Per view, after its backward: the norm of each projected Gaussian's 2D
// centre gradient (g2d fields 0-1) in NDC units (the pixel gradient times
// W/2 and H/2) is added to acc[i][0], the view count to acc[i][1], and
// acc[i][2] keeps the largest radius (the statistics the gradient threshold
// of densification reads).  16 bytes read-modify-written and 8 + 4 read per
// Gaussian.
__global__ void __launch_bounds__(256) grad_screen_kernel(const float* __restrict__ g2d,
                                                          const int32_t* __restrict__ radius, int64_t n,
                                                          float sx, float sy, float4* __restrict__ acc) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const int32_t r = radius[i];
  if (r <= 0) return;
  const float gx = sx * g2d[9 * i], gy = sy * g2d[9 * i + 1];
  float4 a = acc[i];
  a.x += sqrtf(gx * gx + gy * gy);
  a.y += 1.f;
  a.z = fmaxf(a.z, (float)r);
  acc[i] = a;
}

// Both selections of one density step in one pass (Sec. 3.8 percentile
// thresholds, gated by the gradient thresholds tau_grad and tau_grad^abs of
// the hyper-parameter table): keep = s >= thr[1] on a final-pruning step,
// else 1; densify = keep and s >= thr[0] and (gmean >= tau_grad or
// amean >= tau_abs), with gmean = gstats[i][0] / gstats[i][1] and
// amean = dstats[i][3] / gstats[i][1] (means over the views in which the
// Gaussian was projected; never projected: not densified).  The score
// comparisons use the total order of tgs_threshold_mask.
__global__ void __launch_bounds__(256) density_masks_kernel(const float* __restrict__ sc,
                                                            const float4* __restrict__ gstats,
                                                            const float4* __restrict__ dstats, int64_t n,
                                                            const float* __restrict__ thr, float tau_grad,
                                                            float tau_abs, int prune, uint8_t* __restrict__ dens,
                                                            uint8_t* __restrict__ keep) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const uint32_t k = order_key(sc[i]);
  const bool kp = prune == 0 || k >= order_key(thr[1]);
  const float4 g = gstats[i];
  bool gate = false;
  if (g.y > 0.f) {
    const float gm = g.x / g.y;
    const float am = dstats != nullptr ? dstats[i].w / g.y : 0.f;
    gate = gm >= tau_grad || (dstats != nullptr && am >= tau_abs);
  }
  keep[i] = kp ? 1u : 0u;
  dens[i] = (kp && gate && k >= order_key(thr[0])) ? 1u : 0u;
}

__global__ void __launch_bounds__(256) grad_screen_mean_kernel(const float4* __restrict__ acc, int64_t n,
                                                               float* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const float4 a = acc[i];
  out[i] = a.y > 0.f ? a.x / a.y : 0.f;
}

}  // namespace tgs

using namespace tgs;

extern "C" int32_t tgs_grad_screen_accumulate(const float* g2d, const int32_t* radius, int64_t n, int32_t width,
                                              int32_t height, float* acc, void* stream) {
  TGS_REQUIRE(n >= 0 && n < (1ll << 31), "tgs_grad_screen_accumulate: n out of range");
  TGS_REQUIRE(width > 0 && height > 0, "tgs_grad_screen_accumulate: bad image size %d x %d", width, height);
  if (n == 0) return TGS_OK;
  TGS_REQUIRE(g2d && radius && acc, "tgs_grad_screen_accumulate: null pointer");
  TGS_REQUIRE(((uintptr_t)acc & 15) == 0, "tgs_grad_screen_accumulate: acc must be 16-byte aligned");
  hipLaunchKernelGGL(grad_screen_kernel, dim3((unsigned)ceil_div(n, (int64_t)256)), dim3(256), 0, as_stream(stream),
                     g2d, radius, n, 0.5f * (float)width, 0.5f * (float)height, (float4*)acc);
  return hip_status("tgs_grad_screen_accumulate");
}

extern "C" int32_t tgs_density_masks(const float* scores, const float* gstats, const float* dstats, int64_t n,
                                     const float* thr, float tau_grad, float tau_grad_abs, int32_t prune,
                                     uint8_t* densify, uint8_t* keep, void* stream) {
  TGS_REQUIRE(n >= 0 && n < (1ll << 31), "tgs_density_masks: n out of range");
  if (n == 0) return TGS_OK;
  TGS_REQUIRE(scores && gstats && thr && densify && keep, "tgs_density_masks: null pointer");
  TGS_REQUIRE(((uintptr_t)gstats & 15) == 0 && ((uintptr_t)dstats & 15) == 0,
              "tgs_density_masks: gstats and dstats must be 16-byte aligned");
  hipLaunchKernelGGL(density_masks_kernel, dim3((unsigned)ceil_div(n, (int64_t)256)), dim3(256), 0,
                     as_stream(stream), scores, (const float4*)gstats, (const float4*)dstats, n, thr, tau_grad,
                     tau_grad_abs, (int)prune, densify, keep);
  return hip_status("tgs_density_masks");
}

extern "C" int32_t tgs_grad_screen_mean(const float* acc, int64_t n, float* out, void* stream) {
  TGS_REQUIRE(n >= 0 && n < (1ll << 31), "tgs_grad_screen_mean: n out of range");
  if (n == 0) return TGS_OK;
  TGS_REQUIRE(acc && out, "tgs_grad_screen_mean: null pointer");
  TGS_REQUIRE(((uintptr_t)acc & 15) == 0, "tgs_grad_screen_mean: acc must be 16-byte aligned");
  hipLaunchKernelGGL(grad_screen_mean_kernel, dim3((unsigned)ceil_div(n, (int64_t)256)), dim3(256), 0,
                     as_stream(stream), (const float4*)acc, n, out);
  return hip_status("tgs_grad_screen_mean");
}

extern "C" size_t tgs_density_topology_workspace_size(int64_t n) {
  if (n < 0) return 0;
  return topo_layout(nullptr, n).bytes;
}

extern "C" int32_t tgs_density_topology_count(const uint8_t* keep, const uint8_t* densify, int64_t n,
                                              int64_t* n_keep, int64_t* n_new, void* ws, size_t ws_bytes,
                                              void* stream) {
  TGS_REQUIRE(n > 0 && n < (1ll << 31), "tgs_density_topology_count: n out of range");
  TGS_REQUIRE(keep && densify && n_keep && n_new && ws, "tgs_density_topology_count: null pointer");
  const TopoWs w = topo_layout(ws, n);
  TGS_REQUIRE(ws_bytes >= w.bytes, "tgs_density_topology_count: workspace %zu bytes < %zu", ws_bytes, w.bytes);
  hipStream_t s = as_stream(stream);
  hipLaunchKernelGGL(topo_flags_kernel, dim3((unsigned)ceil_div(n, (int64_t)256)), dim3(256), 0, s, keep, densify,
                     n, w.kflag, w.dflag);
  exclusive_scan_u32(w.kflag, w.koff, n, w.part, s);
  exclusive_scan_u32(w.dflag, w.doff, n, w.part, s);
  uint32_t tot[2] = {0u, 0u};
  if (hipMemcpyAsync(&tot[0], w.koff + n, sizeof(uint32_t), hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipMemcpyAsync(&tot[1], w.doff + n, sizeof(uint32_t), hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return hip_status("tgs_density_topology_count");
  *n_keep = tot[0];
  *n_new = tot[1];
  return hip_status("tgs_density_topology_count");
}

extern "C" int32_t tgs_density_topology_apply(const float* params, const float* m, const float* v, int64_t n,
                                              const float* z, float log_split, const void* ws, size_t ws_bytes,
                                              float* params_out, float* m_out, float* v_out, int64_t n_out,
                                              void* stream) {
  TGS_REQUIRE(n > 0 && n < (1ll << 31), "tgs_density_topology_apply: n out of range");
  TGS_REQUIRE(n_out >= 0 && n_out <= 2 * n, "tgs_density_topology_apply: n_out %lld out of range",
              (long long)n_out);
  TGS_REQUIRE(params && m && v && z && ws, "tgs_density_topology_apply: null pointer");
  const TopoWs w = topo_layout((void*)ws, n);
  TGS_REQUIRE(ws_bytes >= w.bytes, "tgs_density_topology_apply: workspace %zu bytes < %zu", ws_bytes, w.bytes);
  if (n_out == 0) return TGS_OK;
  TGS_REQUIRE(params_out && m_out && v_out, "tgs_density_topology_apply: null output");
  TGS_REQUIRE((((uintptr_t)m | (uintptr_t)v | (uintptr_t)m_out | (uintptr_t)v_out) & 15) == 0,
              "tgs_density_topology_apply: moment arrays must be 16-byte aligned");
  hipStream_t s = as_stream(stream);
  hipLaunchKernelGGL(topo_apply_kernel, dim3((unsigned)ceil_div(n, (int64_t)256)), dim3(256), 0, s, params, m, v,
                     n, w.kflag, w.dflag, w.koff, w.doff, z, log_split, params_out, m_out, v_out, n_out);
  return hip_status("tgs_density_topology_apply");
}

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
