// View-dependent colour term of the diffuse-specular split (Sec. 4.2): real spherical
// harmonics of degree <= 3 at a unit direction, and the gradient of a weighted sum of them.
//
// Basis index j = l^2 + l + m. Each function is (-1)^m times the usual real harmonic, i.e.
// sqrt(2) Re Y_l^m (m > 0), sqrt(2) Im Y_l^|m| (m < 0) or Y_l^0 of the complex harmonic with
// the Condon-Shortley phase; written as polynomials in the direction (x, y, z) with the
// normalisations sqrt((2l + 1) (l - |m|)! / (4 pi (l + |m|)!)) folded into the constants:
//   kC0 = 1 / (2 sqrt(pi)), kC1 = sqrt(3 / (4 pi)),
//   kC2a = sqrt(15 / pi) / 2, kC2b = sqrt(5 / pi) / 4, kC2c = sqrt(15 / pi) / 4,
//   kC3a = sqrt(35 / (2 pi)) / 4, kC3b = sqrt(105 / pi) / 2, kC3c = sqrt(21 / (2 pi)) / 4,
//   kC3d = sqrt(7 / pi) / 4, kC3e = sqrt(105 / pi) / 4.
#pragma once

#include <hip/hip_runtime.h>

namespace gbb {

constexpr int kShMaxCoef = 16;  // (3 + 1)^2

constexpr float kC0 = 0.28209479177387814f;
constexpr float kC1 = 0.4886025119029199f;
constexpr float kC2a = 1.0925484305920792f;
constexpr float kC2b = 0.31539156525252005f;
constexpr float kC2c = 0.5462742152960396f;
constexpr float kC3a = 0.5900435899266435f;
constexpr float kC3b = 2.890611442640554f;
constexpr float kC3c = 0.4570457994644658f;
constexpr float kC3d = 0.3731763325901154f;
constexpr float kC3e = 1.445305721320277f;

// Y[0 .. (degree + 1)^2) at the unit direction (x, y, z).
__device__ __forceinline__ void sh_basis(int degree, float x, float y, float z,
                                         float (&Y)[kShMaxCoef]) {
  Y[0] = kC0;
  if (degree < 1) return;
  Y[1] = -kC1 * y;
  Y[2] = kC1 * z;
  Y[3] = -kC1 * x;
  if (degree < 2) return;
  const float xx = x * x, yy = y * y, zz = z * z;
  Y[4] = kC2a * x * y;
  Y[5] = -kC2a * y * z;
  Y[6] = kC2b * (2.f * zz - xx - yy);
  Y[7] = -kC2a * x * z;
  Y[8] = kC2c * (xx - yy);
  if (degree < 3) return;
  Y[9] = -kC3a * y * (3.f * xx - yy);
  Y[10] = kC3b * x * y * z;
  Y[11] = -kC3c * y * (4.f * zz - xx - yy);
  Y[12] = kC3d * z * (2.f * zz - 3.f * xx - 3.f * yy);
  Y[13] = -kC3c * x * (4.f * zz - xx - yy);
  Y[14] = kC3e * z * (xx - yy);
  Y[15] = -kC3a * x * (xx - 3.f * yy);
}

// g = sum_j a_j grad Y_j at (x, y, z), each Y_j taken as the polynomial above in three free
// variables (the caller projects onto the sphere's tangent plane).
__device__ __forceinline__ void sh_grad(int degree, float x, float y, float z,
                                        const float (&a)[kShMaxCoef], float (&g)[3]) {
  g[0] = g[1] = g[2] = 0.f;
  if (degree < 1) return;
  g[0] += -kC1 * a[3];
  g[1] += -kC1 * a[1];
  g[2] += kC1 * a[2];
  if (degree < 2) return;
  const float xx = x * x, yy = y * y, zz = z * z;
  // xy, -yz, 2zz - xx - yy, -xz, xx - yy
  g[0] += kC2a * a[4] * y - kC2a * a[7] * z - 2.f * kC2b * a[6] * x + 2.f * kC2c * a[8] * x;
  g[1] += kC2a * a[4] * x - kC2a * a[5] * z - 2.f * kC2b * a[6] * y - 2.f * kC2c * a[8] * y;
  g[2] += -kC2a * a[5] * y - kC2a * a[7] * x + 4.f * kC2b * a[6] * z;
  if (degree < 3) return;
  // -y(3xx - yy), xyz, -y(4zz - xx - yy), z(2zz - 3xx - 3yy), -x(4zz - xx - yy),
  // z(xx - yy), -x(xx - 3yy)
  g[0] += -kC3a * a[9] * 6.f * x * y + kC3b * a[10] * y * z + kC3c * a[11] * 2.f * x * y -
          kC3d * a[12] * 6.f * x * z - kC3c * a[13] * (4.f * zz - 3.f * xx - yy) +
          kC3e * a[14] * 2.f * x * z - kC3a * a[15] * (3.f * xx - 3.f * yy);
  g[1] += -kC3a * a[9] * (3.f * xx - 3.f * yy) + kC3b * a[10] * x * z -
          kC3c * a[11] * (4.f * zz - xx - 3.f * yy) - kC3d * a[12] * 6.f * y * z +
          kC3c * a[13] * 2.f * x * y - kC3e * a[14] * 2.f * y * z + kC3a * a[15] * 6.f * x * y;
  g[2] += kC3b * a[10] * x * y - kC3c * a[11] * 8.f * y * z +
          kC3d * a[12] * (6.f * zz - 3.f * xx - 3.f * yy) - kC3c * a[13] * 8.f * x * z +
          kC3e * a[14] * (xx - yy);
}

}  // namespace gbb
