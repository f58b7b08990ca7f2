// Preprocess backward: per splat, sums over views the chain rule from the record gradients
// (homography entries H, projected centre c2, opacity) to centre p, tangents t_u, t_v and
// scales (s_u, s_v), the primitive parameters of Eq. 3.
//
// Forward relations (camera space, per view):
//   pc = R p + t, a = R (s_u t_u), b = R (s_v t_v), iz = 1 / pc_z,
//   xi = pc_x iz, eta = pc_y iz, c2 = (fx xi + cx, fy eta + cy),
//   m = (a_z, b_z) iz, X = fx (a_x - xi a_z, b_x - xi b_z) iz, Y = fy (a_y - eta a_z, b_y - eta b_z) iz,
//   H = [[Y1, -X1, 0], [-Y0, X0, 0], [m1 Y0 - m0 Y1, X1 m0 - X0 m1, X0 Y1 - X1 Y0]].
// With spherical-harmonic coefficients (diffuse-specular split) the record's colour adjoint
// also gives the coefficients' gradient and, through the view direction, a term of the
// centre's. The gradients are written (not accumulated).
#include "device_util.h"
#include "gbb_internal.h"
#include "sh_eval.h"

namespace gbb {

namespace {

// SHD: degree of the view-dependent colour term (-1: none).
template <int SHD>
__global__ void __launch_bounds__(256)
preprocess_bwd_kernel(const float* __restrict__ means, const float* __restrict__ tan_u,
                      const float* __restrict__ tan_v, const float* __restrict__ scales,
                      const ViewDev* __restrict__ views, int n_views, int64_t P,
                      const uint32_t* __restrict__ count, const float* __restrict__ d_rec,
                      float* __restrict__ d_means, float* __restrict__ d_tan_u,
                      float* __restrict__ d_tan_v, float* __restrict__ d_scales,
                      float* __restrict__ d_opacity, const float* __restrict__ sh,
                      const float4* __restrict__ d_spec, float* __restrict__ d_sh) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= P) return;
  const float p[3] = {means[3 * k + 0], means[3 * k + 1], means[3 * k + 2]};
  const float tu[3] = {tan_u[3 * k + 0], tan_u[3 * k + 1], tan_u[3 * k + 2]};
  const float tv[3] = {tan_v[3 * k + 0], tan_v[3 * k + 1], tan_v[3 * k + 2]};
  const float su = scales[2 * k + 0], sv = scales[2 * k + 1];
  float dp[3] = {0.f, 0.f, 0.f}, dtu[3] = {0.f, 0.f, 0.f}, dtv[3] = {0.f, 0.f, 0.f};
  float dsu = 0.f, dsv = 0.f, dop = 0.f;
  constexpr int n_sh = SHD >= 0 ? (SHD + 1) * (SHD + 1) : 0;
  float dsh[kShMaxCoef][3];
#pragma unroll
  for (int j = 0; j < kShMaxCoef; ++j) dsh[j][0] = dsh[j][1] = dsh[j][2] = 0.f;
  for (int vi = 0; vi < n_views; ++vi) {
    const int64_t idx = (int64_t)vi * P + k;
    if (count[idx] == 0) continue;
    if constexpr (n_sh > 0) {
      // colour term sum_j Y_j(dir) sh_j with dir = (p - centre) / |p - centre|, centre = -R^T t:
      // d sh_j += Y_j ds, and d p += (I - dir dir^T) / |p - centre| grad_dir(sum_j Y_j (sh_j . ds))
      const ViewDev& Vs = views[vi];
      const float4 ds = d_spec[idx];
      float dv[3];
      for (int i = 0; i < 3; ++i)
        dv[i] = p[i] + (Vs.R[i] * Vs.t[0] + Vs.R[3 + i] * Vs.t[1] + Vs.R[6 + i] * Vs.t[2]);
      const float inv_len = 1.0f / sqrtf(dv[0] * dv[0] + dv[1] * dv[1] + dv[2] * dv[2]);
      const float x = dv[0] * inv_len, y = dv[1] * inv_len, z = dv[2] * inv_len;
      float Y[kShMaxCoef], a[kShMaxCoef];
      sh_basis(SHD, x, y, z, Y);
      const float* c = sh + (int64_t)k * n_sh * 3;
#pragma unroll
      for (int j = 0; j < kShMaxCoef; ++j) a[j] = 0.f;
#pragma unroll
      for (int j = 0; j < n_sh; ++j) {
        dsh[j][0] += Y[j] * ds.x;
        dsh[j][1] += Y[j] * ds.y;
        dsh[j][2] += Y[j] * ds.z;
        a[j] = c[3 * j] * ds.x + c[3 * j + 1] * ds.y + c[3 * j + 2] * ds.z;
      }
      float gd[3];
      sh_grad(SHD, x, y, z, a, gd);
      const float radial = gd[0] * x + gd[1] * y + gd[2] * z;
      dp[0] += (gd[0] - radial * x) * inv_len;
      dp[1] += (gd[1] - radial * y) * inv_len;
      dp[2] += (gd[2] - radial * z) * inv_len;
    }
    float g[kRecGrad];
#pragma unroll
    for (int i = 0; i < kRecGrad; ++i) g[i] = d_rec[idx * kRecGrad + i];
    const ViewDev& V = views[vi];
    const float* R = V.R;
    float pc[3], a[3], b[3];
    for (int i = 0; i < 3; ++i) {
      pc[i] = R[3 * i] * p[0] + R[3 * i + 1] * p[1] + R[3 * i + 2] * p[2] + V.t[i];
      a[i] = su * (R[3 * i] * tu[0] + R[3 * i + 1] * tu[1] + R[3 * i + 2] * tu[2]);
      b[i] = sv * (R[3 * i] * tv[0] + R[3 * i + 1] * tv[1] + R[3 * i + 2] * tv[2]);
    }
    const float fx = V.fx, fy = V.fy;
    const float iz = 1.0f / pc[2];
    const float xi = pc[0] * iz, eta = pc[1] * iz;
    const float m0 = a[2] * iz, m1 = b[2] * iz;
    const float ax = a[0] - xi * a[2], bx = b[0] - xi * b[2];
    const float ay = a[1] - eta * a[2], by = b[1] - eta * b[2];
    const float X0 = fx * ax * iz, X1 = fx * bx * iz;
    const float Y0 = fy * ay * iz, Y1 = fy * by * iz;
    // H -> (X, Y, m)
    const float dY1 = g[0] - g[4] * m0 + g[6] * X0;
    const float dX1 = -g[1] + g[5] * m0 - g[6] * Y0;
    const float dY0 = -g[2] + g[4] * m1 - g[6] * X1;
    const float dX0 = g[3] - g[5] * m1 + g[6] * Y1;
    const float dm0 = -g[4] * Y1 + g[5] * X1;
    const float dm1 = g[4] * Y0 - g[5] * X0;
    float da[3] = {0.f, 0.f, 0.f}, db[3] = {0.f, 0.f, 0.f};
    float dxi = fx * g[7], deta = fy * g[8], diz = 0.f;
    // X0 = fx (a_x - xi a_z) iz, X1 = fx (b_x - xi b_z) iz
    da[0] += dX0 * fx * iz;
    da[2] -= dX0 * fx * xi * iz;
    dxi -= dX0 * fx * a[2] * iz;
    diz += dX0 * fx * ax;
    db[0] += dX1 * fx * iz;
    db[2] -= dX1 * fx * xi * iz;
    dxi -= dX1 * fx * b[2] * iz;
    diz += dX1 * fx * bx;
    // Y0 = fy (a_y - eta a_z) iz, Y1 = fy (b_y - eta b_z) iz
    da[1] += dY0 * fy * iz;
    da[2] -= dY0 * fy * eta * iz;
    deta -= dY0 * fy * a[2] * iz;
    diz += dY0 * fy * ay;
    db[1] += dY1 * fy * iz;
    db[2] -= dY1 * fy * eta * iz;
    deta -= dY1 * fy * b[2] * iz;
    diz += dY1 * fy * by;
    // m = (a_z, b_z) iz
    da[2] += dm0 * iz;
    db[2] += dm1 * iz;
    diz += dm0 * a[2] + dm1 * b[2];
    // xi = pc_x iz, eta = pc_y iz, iz = 1 / pc_z
    float dpc[3];
    dpc[0] = dxi * iz;
    dpc[1] = deta * iz;
    diz += dxi * pc[0] + deta * pc[1];
    dpc[2] = -diz * iz * iz;
    // back through R: a = R (s_u t_u), b = R (s_v t_v), pc = R p + t
    for (int j = 0; j < 3; ++j) {
      const float wa = R[j] * da[0] + R[3 + j] * da[1] + R[6 + j] * da[2];
      const float wb = R[j] * db[0] + R[3 + j] * db[1] + R[6 + j] * db[2];
      const float wp = R[j] * dpc[0] + R[3 + j] * dpc[1] + R[6 + j] * dpc[2];
      dtu[j] += su * wa;
      dtv[j] += sv * wb;
      dsu += tu[j] * wa;
      dsv += tv[j] * wb;
      dp[j] += wp;
    }
    dop += g[9];
  }
  for (int j = 0; j < 3; ++j) {
    d_means[3 * k + j] = dp[j];
    d_tan_u[3 * k + j] = dtu[j];
    d_tan_v[3 * k + j] = dtv[j];
  }
  d_scales[2 * k + 0] = dsu;
  d_scales[2 * k + 1] = dsv;
  d_opacity[k] = dop;
#pragma unroll
  for (int j = 0; j < n_sh; ++j) {
    d_sh[((int64_t)k * n_sh + j) * 3 + 0] = dsh[j][0];
    d_sh[((int64_t)k * n_sh + j) * 3 + 1] = dsh[j][1];
    d_sh[((int64_t)k * n_sh + j) * 3 + 2] = dsh[j][2];
  }
}

}  // namespace

hipError_t launch_preprocess_bwd(const gb_splats& sp, const ViewDev* d_views, int n_views,
                                 const uint32_t* count, const float* d_rec,
                                 const float4* d_spec, const gb_grads& g, hipStream_t s) {
  const int64_t P = sp.P;
  const int64_t blocks = (P + 255) / 256;
  const int shd = sp.sh ? sp.sh_degree : -1;
#define GBB_PREB(D)                                                                           \
  hipLaunchKernelGGL(preprocess_bwd_kernel<D>, dim3((unsigned)blocks), dim3(256), 0, s,        \
                     sp.means, sp.tan_u, sp.tan_v, sp.scales, d_views, n_views, P, count,     \
                     d_rec, g.d_means, g.d_tan_u, g.d_tan_v, g.d_scales, g.d_opacity, sp.sh,   \
                     d_spec, g.d_sh)
  switch (shd) {
    case 0: GBB_PREB(0); break;
    case 1: GBB_PREB(1); break;
    case 2: GBB_PREB(2); break;
    case 3: GBB_PREB(3); break;
    default: GBB_PREB(-1); break;
  }
#undef GBB_PREB
  return hipGetLastError();
}

}  // namespace gbb
