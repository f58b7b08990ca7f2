// Per-(view, splat) preprocess: key stage (depth, screen rectangle, tile count) and the
// blend record (ray-splat homography, projected centre, opacity).
//
// Key stage: a float32 computation with a fixed operation order and no contraction, so that
// the tiling it defines is reproducible bit for bit:
//   pc = ((R_i0 p0 + R_i1 p1) + R_i2 p2) + t_i,  d = pc_z;  cull if !(d > z_near) or o < alpha_min
//   a = R (s_u t_u), b = R (s_v t_v)  (same summation order, no translation)
//   corners q = (pc +- 3.33 a) +- 3.33 b in the order (-,-), (+,-), (-,+), (+,+)
//   any corner with q_z <= z_near (or alpha_min < 1/255): rectangle = whole image; otherwise
//   x = fx (q_x / q_z) + cx, y likewise, c2 = (fx (pc_x / d) + cx, fy (pc_y / d) + cy),
//   xmin = min(x.., c2x - r_lp) - 0.01, xmax = max(x.., c2x + r_lp) + 0.01 (y likewise),
//   i0 = ceil(xmin - 0.5), i1 = floor(xmax - 0.5), clamped to the image, empty -> culled.
// 3.33 bounds the uv radius where o G >= 1/255 (sqrt(2 ln 255) = 3.329) and r_lp the radius of
// the low-pass disk with the same bound, sqrt(2 var ln 255) = 3.329 sqrt(var) px: r_lp = 2.36
// for variances up to 1/2 (the default), else 3.34 sqrt(var) rounded once to float32 (host
// side, in double precision). Every pixel with alpha >= alpha_min then lies inside (Eq. 3-4;
// the 0.01 px margin covers rounding).
#include <cmath>

#include "device_util.h"
#include "gbb_internal.h"
#include "sh_eval.h"

namespace gbb {

namespace {

struct ViewChunk {
  gb_view v[8];
  int32_t tile_base[8];
  int32_t pix_base[8];
  int32_t sat_base[8];
  int32_t count;
  int32_t first;
};

__global__ void upload_views_kernel(ViewChunk c, int tile_w, int tile_h, ViewDev* out) {
  int i = threadIdx.x;
  if (i >= c.count) return;
  const gb_view& v = c.v[i];
  ViewDev d;
  for (int k = 0; k < 9; ++k) d.R[k] = v.R[k];
  for (int k = 0; k < 3; ++k) d.t[k] = v.t[k];
  d.fx = v.fx;
  d.fy = v.fy;
  d.cx = v.cx;
  d.cy = v.cy;
  d.z_near = v.z_near;
  d.W = v.width;
  d.H = v.height;
  d.tiles_x = (v.width + tile_w - 1) / tile_w;
  d.tiles_y = (v.height + tile_h - 1) / tile_h;
  d.tile_base = c.tile_base[i];
  d.pix_base = c.pix_base[i];
  d.sat_base = c.sat_base[i];
  out[c.first + i] = d;
}

__device__ __forceinline__ float p_of(int i, float p0, float p1, float p2) {
  return i == 0 ? p0 : i == 1 ? p1 : p2;
}

__device__ __forceinline__ float ks_min(float a, float b) { return a < b ? a : b; }
__device__ __forceinline__ float ks_max(float a, float b) { return a > b ? a : b; }

__device__ __forceinline__ float rot_row(const float* R, int i, float x0, float x1, float x2) {
#pragma clang fp contract(off)
  return (R[3 * i + 0] * x0 + R[3 * i + 1] * x1) + R[3 * i + 2] * x2;
}

__device__ __forceinline__ f2 rot_row_f2(const float* R, int i, float x0, float x1, float x2,
                                         float t) {
  // exact products, then compensated sums
  f2 s = two_prod(R[3 * i + 0], x0);
  s = f2_add(s, two_prod(R[3 * i + 1], x1));
  s = f2_add(s, two_prod(R[3 * i + 2], x2));
  return f2_add(s, t);
}

// SHD: degree of the view-dependent colour term (-1: none).
template <int SHD>
__global__ void __launch_bounds__(256)
preprocess_kernel(const float* __restrict__ means, const float* __restrict__ tan_u,
                  const float* __restrict__ tan_v, const float* __restrict__ scales,
                  const float* __restrict__ opacity, const ViewDev* __restrict__ views,
                  int64_t P, int64_t VP, float alpha_min, float r_lp, int tile_w, int tile_h,
                  uint32_t* __restrict__ depth_key, uint32_t* __restrict__ sort_key,
                  uint32_t* __restrict__ count,
                  SplatRec* __restrict__ rec, const float* __restrict__ sh,
                  float4* __restrict__ spec, uint32_t* __restrict__ order,
                  uint32_t* __restrict__ zero, int64_t n_zero) {
  int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (order) {
    // the depth sort's initial order (record indices), and words to clear, in the same launch
    if (idx < VP) order[idx] = (uint32_t)idx;
    const int64_t n_threads = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = idx; i < n_zero; i += n_threads) zero[i] = 0u;
  }
  if (idx >= VP) return;
  const int v = (int)(idx / P);
  const int64_t k = idx - (int64_t)v * P;
  const ViewDev& V = views[v];
  float R[9];
#pragma unroll
  for (int i = 0; i < 9; ++i) R[i] = V.R[i];

  const float p0 = means[3 * k + 0], p1 = means[3 * k + 1], p2 = means[3 * k + 2];
  const float u0 = tan_u[3 * k + 0], u1 = tan_u[3 * k + 1], u2 = tan_u[3 * k + 2];
  const float w0 = tan_v[3 * k + 0], w1 = tan_v[3 * k + 1], w2 = tan_v[3 * k + 2];
  const float su = scales[2 * k + 0], sv = scales[2 * k + 1];
  const float o = opacity[k];

  uint32_t key = kCulledKey;
  uint32_t n_tiles = 0;
  int i0 = 0, i1 = -1, j0 = 0, j1 = -1;
  float a[3], b[3];
  {
#pragma clang fp contract(off)
    float pc[3];
    for (int i = 0; i < 3; ++i) pc[i] = rot_row(R, i, p0, p1, p2) + V.t[i];
    const float d = pc[2];
    const float wa0 = su * u0, wa1 = su * u1, wa2 = su * u2;
    const float wb0 = sv * w0, wb1 = sv * w1, wb2 = sv * w2;
    for (int i = 0; i < 3; ++i) {
      a[i] = rot_row(R, i, wa0, wa1, wa2);
      b[i] = rot_row(R, i, wb0, wb1, wb2);
    }
    const float zn = V.z_near;
    const float W1 = (float)(V.W - 1), H1 = (float)(V.H - 1);
    bool whole = !(alpha_min >= (1.0f / 255.0f));
    float ra[3], rb[3];
    for (int i = 0; i < 3; ++i) {
      ra[i] = 3.33f * a[i];
      rb[i] = 3.33f * b[i];
    }
    float xmin = 0.f, xmax = 0.f, ymin = 0.f, ymax = 0.f;
    const float sgn_a[4] = {-1.f, 1.f, -1.f, 1.f};
    const float sgn_b[4] = {-1.f, -1.f, 1.f, 1.f};
    float xs[4], ys[4];
    for (int c = 0; c < 4; ++c) {
      float q[3];
      for (int i = 0; i < 3; ++i) {
        float t0 = sgn_a[c] > 0.f ? pc[i] + ra[i] : pc[i] - ra[i];
        q[i] = sgn_b[c] > 0.f ? t0 + rb[i] : t0 - rb[i];
      }
      if (!(q[2] > zn)) whole = true;
      xs[c] = V.fx * (q[0] / q[2]) + V.cx;
      ys[c] = V.fy * (q[1] / q[2]) + V.cy;
    }
    float fi0, fi1, fj0, fj1;
    if (whole) {
      fi0 = 0.f;
      fi1 = W1;
      fj0 = 0.f;
      fj1 = H1;
    } else {
      const float c2x = V.fx * (pc[0] / d) + V.cx;
      const float c2y = V.fy * (pc[1] / d) + V.cy;
      xmin = ks_min(ks_min(ks_min(ks_min(xs[0], xs[1]), xs[2]), xs[3]), c2x - r_lp) - 0.01f;
      xmax = ks_max(ks_max(ks_max(ks_max(xs[0], xs[1]), xs[2]), xs[3]), c2x + r_lp) + 0.01f;
      ymin = ks_min(ks_min(ks_min(ks_min(ys[0], ys[1]), ys[2]), ys[3]), c2y - r_lp) - 0.01f;
      ymax = ks_max(ks_max(ks_max(ks_max(ys[0], ys[1]), ys[2]), ys[3]), c2y + r_lp) + 0.01f;
      fi0 = ceilf(xmin - 0.5f);
      fi1 = floorf(xmax - 0.5f);
      fj0 = ceilf(ymin - 0.5f);
      fj1 = floorf(ymax - 0.5f);
    }
    bool on = (fi0 <= W1) && (fi1 >= 0.f) && (fj0 <= H1) && (fj1 >= 0.f) && (fi0 <= fi1) &&
              (fj0 <= fj1);
    on = on && (d > zn) && !(o < alpha_min);
    if (on) {
      i0 = (int)ks_max(fi0, 0.f);
      i1 = (int)ks_min(fi1, W1);
      j0 = (int)ks_max(fj0, 0.f);
      j1 = (int)ks_min(fj1, H1);
      const int tx0 = i0 / tile_w, tx1 = i1 / tile_w, ty0 = j0 / tile_h, ty1 = j1 / tile_h;
      n_tiles = (uint32_t)((tx1 - tx0 + 1) * (ty1 - ty0 + 1));
      key = __float_as_uint(d);
    }
  }
  depth_key[idx] = key;
  sort_key[idx] = key;
  count[idx] = n_tiles;

  // ---- blend record (only meaningful for visible records) --------------------------------
  SplatRec r;
  if (n_tiles > 0) {
    // The record is computed in float-pair arithmetic from the float32 inputs: the projected
    // centre must be exact to far below a pixel, and the homography entries of nearly edge-on
    // splats come out of cancelling differences.
    f2 pc2[3], a2[3], b2[3];
    const f2 wa[3] = {two_prod(su, u0), two_prod(su, u1), two_prod(su, u2)};
    const f2 wb[3] = {two_prod(sv, w0), two_prod(sv, w1), two_prod(sv, w2)};
    for (int i = 0; i < 3; ++i) {
      pc2[i] = rot_row_f2(R, i, p0, p1, p2, V.t[i]);
      a2[i] = f2_add(f2_add(f2_mul(wa[0], R[3 * i + 0]), f2_mul(wa[1], R[3 * i + 1])),
                     f2_mul(wa[2], R[3 * i + 2]));
      b2[i] = f2_add(f2_add(f2_mul(wb[0], R[3 * i + 0]), f2_mul(wb[1], R[3 * i + 1])),
                     f2_mul(wb[2], R[3 * i + 2]));
    }
    const f2 iz = f2_div(f2_of(1.0f), pc2[2]);
    const f2 xi = f2_mul(pc2[0], iz), eta = f2_mul(pc2[1], iz);
    const f2 c2x = f2_add(f2_mul(xi, V.fx), V.cx);
    const f2 c2y = f2_add(f2_mul(eta, V.fy), V.cy);
    const f2 m0 = f2_mul(a2[2], iz), m1 = f2_mul(b2[2], iz);
    const f2 X0 = f2_mul(f2_mul(f2_sub(a2[0], f2_mul(xi, a2[2])), iz), V.fx);
    const f2 X1 = f2_mul(f2_mul(f2_sub(b2[0], f2_mul(xi, b2[2])), iz), V.fx);
    const f2 Y0 = f2_mul(f2_mul(f2_sub(a2[1], f2_mul(eta, a2[2])), iz), V.fy);
    const f2 Y1 = f2_mul(f2_mul(f2_sub(b2[1], f2_mul(eta, b2[2])), iz), V.fy);
    const f2 h[7] = {Y1, f2_neg(X1), f2_neg(Y0), X0,
                     f2_sub(f2_mul(m1, Y0), f2_mul(m0, Y1)),
                     f2_sub(f2_mul(X1, m0), f2_mul(X0, m1)),
                     f2_sub(f2_mul(X0, Y1), f2_mul(X1, Y0))};
    for (int i = 0; i < 7; ++i) {
      r.h_hi[i] = h[i].hi;
      r.h_lo[i] = h[i].lo;
    }
    r.c2x_hi = c2x.hi;
    r.c2x_lo = c2x.lo;
    r.c2y_hi = c2y.hi;
    r.c2y_lo = c2y.lo;
  } else {
    for (int i = 0; i < 7; ++i) r.h_hi[i] = r.h_lo[i] = 0.f;
    r.c2x_hi = r.c2x_lo = r.c2y_hi = r.c2y_lo = 0.f;
  }
  r.opacity = o;
  r.rect_x = (i0 & 0xffff) | (i1 << 16);
  r.rect_y = (j0 & 0xffff) | (j1 << 16);
  r.splat = (int32_t)k;
  r.view = v;
  r.pad = 0;
  rec[idx] = r;

  // ---- view-dependent colour (diffuse-specular split): sum_j Y_j(dir) sh[k][j] ---------
  if constexpr (SHD >= 0) {
    if (n_tiles == 0) return;
    // camera centre -R^T t; dir = (p - centre) / |p - centre|
    float d[3];
    for (int i = 0; i < 3; ++i)
      d[i] = p_of(i, p0, p1, p2) + (R[i] * V.t[0] + R[3 + i] * V.t[1] + R[6 + i] * V.t[2]);
    const float inv_len = 1.0f / sqrtf(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    float Y[kShMaxCoef];
    sh_basis(SHD, d[0] * inv_len, d[1] * inv_len, d[2] * inv_len, Y);
    constexpr int n = (SHD + 1) * (SHD + 1);
    const float* c = sh + (int64_t)k * n * 3;
    float s0 = 0.f, s1 = 0.f, s2 = 0.f;
#pragma unroll
    for (int j = 0; j < n; ++j) {
      s0 += Y[j] * c[3 * j + 0];
      s1 += Y[j] * c[3 * j + 1];
      s2 += Y[j] * c[3 * j + 2];
    }
    spec[idx] = make_float4(s0, s1, s2, 0.f);
  }
}

}  // namespace

float lowpass_radius(float lowpass_var) {
  if (lowpass_var <= 0.5f) return 2.36f;
  return (float)(3.34 * std::sqrt((double)lowpass_var));
}

hipError_t launch_upload_views(const gb_view* views, int n_views, int tile_w, int tile_h,
                               ViewDev* d_views, hipStream_t s) {
  int tile_base = 0, pix_base = 0, sat_base = 0;
  for (int first = 0; first < n_views; first += 8) {
    ViewChunk c;
    c.count = n_views - first < 8 ? n_views - first : 8;
    c.first = first;
    for (int i = 0; i < c.count; ++i) {
      const gb_view& v = views[first + i];
      c.v[i] = v;
      c.tile_base[i] = tile_base;
      c.pix_base[i] = pix_base;
      c.sat_base[i] = sat_base;
      const int tx = (v.width + tile_w - 1) / tile_w, ty = (v.height + tile_h - 1) / tile_h;
      sat_base += (tx + 1) * (ty + 1);
      tile_base += ((v.width + tile_w - 1) / tile_w) * ((v.height + tile_h - 1) / tile_h);
      pix_base += v.width * v.height;
    }
    hipLaunchKernelGGL(upload_views_kernel, dim3(1), dim3(8), 0, s, c, tile_w, tile_h, d_views);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_preprocess(const gb_splats& sp, const ViewDev* d_views, int n_views,
                             const gb_options& o, int tile_w, int tile_h, uint32_t* depth_key,
                             uint32_t* sort_key, uint32_t* count, SplatRec* rec, float4* spec,
                             uint32_t* order, uint32_t* zero, int64_t n_zero, hipStream_t s) {
  const int64_t VP = (int64_t)sp.P * n_views;
  const int threads = 256;
  const int64_t blocks = (VP + threads - 1) / threads;
  const float r_lp = lowpass_radius(o.lowpass_var);
  const int shd = sp.sh ? sp.sh_degree : -1;
#define GBB_PRE(D)                                                                            \
  hipLaunchKernelGGL(preprocess_kernel<D>, dim3((unsigned)blocks), dim3(threads), 0, s,        \
                     sp.means, sp.tan_u, sp.tan_v, sp.scales, sp.opacity, d_views,            \
                     (int64_t)sp.P, VP, o.alpha_min, r_lp, tile_w, tile_h, depth_key, sort_key, \
                     count, rec, sp.sh, spec, order, zero, n_zero)
  switch (shd) {
    case 0: GBB_PRE(0); break;
    case 1: GBB_PRE(1); break;
    case 2: GBB_PRE(2); break;
    case 3: GBB_PRE(3); break;
    default: GBB_PRE(-1); break;
  }
#undef GBB_PRE
  return hipGetLastError();
}

}  // namespace gbb
