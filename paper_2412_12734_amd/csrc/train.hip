// Training glue around the rasterizer. Sec. 3.3 trains the textured splats with an image loss
// and Adam; the parameters are activated as in 2D Gaussian splatting:
//   (w, x, y, z) = q / |q|,  t_u = (1 - 2(y^2 + z^2), 2(xy + wz), 2(xz - wy)),
//                            t_v = (2(xy - wz), 1 - 2(x^2 + z^2), 2(yz + wx))
// (the first two columns of the rotation of the unit quaternion), s = exp(log s),
// o = 1 / (1 + exp(-logit)). The backward applies the Jacobian of those columns with respect to
// the unit quaternion, then the projection (I - q^ q^T) / |q| of the normalisation. The L1 loss
// and Adam are element-wise. Everything here is HBM-bound: per splat or per parameter, one read
// of each input and one write of each output, four elements per thread where the arrays allow.
#include "device_util.h"
#include "gbb_internal.h"

namespace gbb {

namespace {

constexpr int kThreads = 256;
constexpr unsigned kL1MaxBlocks = 1024;

unsigned grid_for(int64_t n, int64_t per_thread) {
  int64_t b = (n + kThreads * per_thread - 1) / (kThreads * per_thread);
  if (b > 65536) b = 65536;
  if (b < 1) b = 1;
  return (unsigned)b;
}

__global__ void __launch_bounds__(kThreads)
activate_fwd_kernel(int P, const float* __restrict__ quats, const float* __restrict__ log_scales,
                    const float* __restrict__ logits, float* __restrict__ tan_u,
                    float* __restrict__ tan_v, float* __restrict__ scales,
                    float* __restrict__ opacity) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= P) return;
  float w = quats[4 * k], x = quats[4 * k + 1], y = quats[4 * k + 2], z = quats[4 * k + 3];
  const float inv = 1.0f / sqrtf(w * w + x * x + y * y + z * z);
  w *= inv;
  x *= inv;
  y *= inv;
  z *= inv;
  tan_u[3 * k + 0] = 1.0f - 2.0f * (y * y + z * z);
  tan_u[3 * k + 1] = 2.0f * (x * y + w * z);
  tan_u[3 * k + 2] = 2.0f * (x * z - w * y);
  tan_v[3 * k + 0] = 2.0f * (x * y - w * z);
  tan_v[3 * k + 1] = 1.0f - 2.0f * (x * x + z * z);
  tan_v[3 * k + 2] = 2.0f * (y * z + w * x);
  scales[2 * k + 0] = expf(log_scales[2 * k + 0]);
  scales[2 * k + 1] = expf(log_scales[2 * k + 1]);
  opacity[k] = 1.0f / (1.0f + expf(-logits[k]));
}

__global__ void __launch_bounds__(kThreads)
activate_bwd_kernel(int P, const float* __restrict__ quats, const float* __restrict__ log_scales,
                    const float* __restrict__ logits, const float* __restrict__ d_tan_u,
                    const float* __restrict__ d_tan_v, const float* __restrict__ d_scales,
                    const float* __restrict__ d_opacity, float* __restrict__ d_quats,
                    float* __restrict__ d_log_scales, float* __restrict__ d_logits) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= P) return;
  float w = quats[4 * k], x = quats[4 * k + 1], y = quats[4 * k + 2], z = quats[4 * k + 3];
  const float inv = 1.0f / sqrtf(w * w + x * x + y * y + z * z);
  w *= inv;
  x *= inv;
  y *= inv;
  z *= inv;
  const float a0 = d_tan_u[3 * k], a1 = d_tan_u[3 * k + 1], a2 = d_tan_u[3 * k + 2];
  const float b0 = d_tan_v[3 * k], b1 = d_tan_v[3 * k + 1], b2 = d_tan_v[3 * k + 2];
  // gradient with respect to the unit quaternion: column derivatives dotted with the adjoints
  const float gw = 2.0f * (a1 * z - a2 * y - b0 * z + b2 * x);
  const float gx = 2.0f * (a1 * y + a2 * z + b0 * y - 2.0f * b1 * x + b2 * w);
  const float gy = 2.0f * (-2.0f * a0 * y + a1 * x - a2 * w + b0 * x + b2 * z);
  const float gz = 2.0f * (-2.0f * a0 * z + a1 * w + a2 * x - b0 * w - 2.0f * b1 * z + b2 * y);
  // through the normalisation
  const float dot = gw * w + gx * x + gy * y + gz * z;
  d_quats[4 * k + 0] = (gw - dot * w) * inv;
  d_quats[4 * k + 1] = (gx - dot * x) * inv;
  d_quats[4 * k + 2] = (gy - dot * y) * inv;
  d_quats[4 * k + 3] = (gz - dot * z) * inv;
  d_log_scales[2 * k + 0] = d_scales[2 * k + 0] * expf(log_scales[2 * k + 0]);
  d_log_scales[2 * k + 1] = d_scales[2 * k + 1] * expf(log_scales[2 * k + 1]);
  const float o = 1.0f / (1.0f + expf(-logits[k]));
  d_logits[k] = d_opacity[k] * o * (1.0f - o);
}

__global__ void zero_kernel(float* p) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *p = 0.0f;
}

__device__ __forceinline__ float l1_term(float r, float t, float scale, float& d) {
  const float diff = r - t;
  d = diff > 0.0f ? scale : (diff < 0.0f ? -scale : 0.0f);
  return fabsf(diff);
}

__device__ __forceinline__ float mse_term(float r, float t, float scale, float& d) {
  const float diff = r - t;
  d = 2.0f * scale * diff;
  return diff * diff;
}

template <bool MSE>
__device__ __forceinline__ float loss_term(float r, float t, float scale, float& d) {
  return MSE ? mse_term(r, t, scale, d) : l1_term(r, t, scale, d);
}

// Image loss (L1, or squared error with MSE): d_rgb = scale sign(rgb - target), or
// 2 scale (rgb - target); the block's sum of the terms goes to *loss with one float atomic
// (the order of those additions is free).
template <bool MSE>
__global__ void __launch_bounds__(kThreads)
loss_kernel(int64_t n, const float* __restrict__ rgb, const float* __restrict__ target,
            float scale, float* __restrict__ loss, float* __restrict__ d_rgb) {
  __shared__ float wave_sum[kThreads / 64];
  float acc = 0.0f;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; 4 * i < n; i += stride) {
    if (4 * i + 3 < n) {
      const float4 r = reinterpret_cast<const float4*>(rgb)[i];
      const float4 t = reinterpret_cast<const float4*>(target)[i];
      float4 d;
      acc += loss_term<MSE>(r.x, t.x, scale, d.x) + loss_term<MSE>(r.y, t.y, scale, d.y) +
             loss_term<MSE>(r.z, t.z, scale, d.z) + loss_term<MSE>(r.w, t.w, scale, d.w);
      reinterpret_cast<float4*>(d_rgb)[i] = d;
    } else {
      for (int64_t j = 4 * i; j < n; ++j) {
        float d;
        acc += loss_term<MSE>(rgb[j], target[j], scale, d);
        d_rgb[j] = d;
      }
    }
  }
  const float s = wave_sum_to_lane63(acc);
  if ((threadIdx.x & 63) == 63) wave_sum[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    float b = 0.0f;
    for (int i = 0; i < kThreads / 64; ++i) b += wave_sum[i];
    atomicAdd(loss, scale * b);
  }
}

__device__ __forceinline__ uint16_t bf16_rne(float x) {
  const uint32_t b = __float_as_uint(x);
  return (uint16_t)((b + 0x7FFFu + ((b >> 16) & 1u)) >> 16);
}

__device__ __forceinline__ float adam_one(float& theta, float g, float& m, float& v, float lr,
                                          float b1, float b2, float c1, float c2, float eps) {
  m = b1 * m + (1.0f - b1) * g;
  v = b2 * v + (1.0f - b2) * g * g;
  theta -= lr * (m * c1) / (sqrtf(v * c2) + eps);
  return theta;
}

// One Adam step; c1 = 1 / (1 - beta1^t), c2 = 1 / (1 - beta2^t) come from the host in double
// precision. With bf16 the updated values are also stored rounded to bfloat16.
__global__ void __launch_bounds__(kThreads)
adam_kernel(int64_t n, float* __restrict__ theta, const float* __restrict__ grad,
            float* __restrict__ m, float* __restrict__ v, float lr, float b1, float b2, float c1,
            float c2, float eps, uint16_t* __restrict__ bf16) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; 4 * i < n; i += stride) {
    if (4 * i + 3 < n) {
      float4 th = reinterpret_cast<float4*>(theta)[i];
      const float4 g = reinterpret_cast<const float4*>(grad)[i];
      float4 mm = reinterpret_cast<float4*>(m)[i];
      float4 vv = reinterpret_cast<float4*>(v)[i];
      adam_one(th.x, g.x, mm.x, vv.x, lr, b1, b2, c1, c2, eps);
      adam_one(th.y, g.y, mm.y, vv.y, lr, b1, b2, c1, c2, eps);
      adam_one(th.z, g.z, mm.z, vv.z, lr, b1, b2, c1, c2, eps);
      adam_one(th.w, g.w, mm.w, vv.w, lr, b1, b2, c1, c2, eps);
      reinterpret_cast<float4*>(theta)[i] = th;
      reinterpret_cast<float4*>(m)[i] = mm;
      reinterpret_cast<float4*>(v)[i] = vv;
      if (bf16) {
        const uint32_t lo = (uint32_t)bf16_rne(th.x) | ((uint32_t)bf16_rne(th.y) << 16);
        const uint32_t hi = (uint32_t)bf16_rne(th.z) | ((uint32_t)bf16_rne(th.w) << 16);
        reinterpret_cast<uint2*>(bf16)[i] = make_uint2(lo, hi);
      }
    } else {
      for (int64_t j = 4 * i; j < n; ++j) {
        float th = theta[j], mm = m[j], vv = v[j];
        adam_one(th, grad[j], mm, vv, lr, b1, b2, c1, c2, eps);
        theta[j] = th;
        m[j] = mm;
        v[j] = vv;
        if (bf16) bf16[j] = bf16_rne(th);
      }
    }
  }
}

__global__ void __launch_bounds__(kThreads)
to_bf16_kernel(int64_t n, const float* __restrict__ src, uint16_t* __restrict__ dst) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
    dst[i] = bf16_rne(src[i]);
}

}  // namespace

hipError_t launch_to_bf16(int64_t n, const float* src, uint16_t* dst, hipStream_t s) {
  hipLaunchKernelGGL(to_bf16_kernel, dim3(grid_for(n, 1)), dim3(kThreads), 0, s, n, src, dst);
  return hipGetLastError();
}

hipError_t launch_activate_fwd(int P, const float* quats, const float* log_scales,
                               const float* logits, float* tan_u, float* tan_v, float* scales,
                               float* opacity, hipStream_t s) {
  hipLaunchKernelGGL(activate_fwd_kernel, dim3(grid_for(P, 1)), dim3(kThreads), 0, s, P, quats,
                     log_scales, logits, tan_u, tan_v, scales, opacity);
  return hipGetLastError();
}

hipError_t launch_activate_bwd(int P, const float* quats, const float* log_scales,
                               const float* logits, const float* d_tan_u, const float* d_tan_v,
                               const float* d_scales, const float* d_opacity, float* d_quats,
                               float* d_log_scales, float* d_logits, hipStream_t s) {
  hipLaunchKernelGGL(activate_bwd_kernel, dim3(grid_for(P, 1)), dim3(kThreads), 0, s, P, quats,
                     log_scales, logits, d_tan_u, d_tan_v, d_scales, d_opacity, d_quats,
                     d_log_scales, d_logits);
  return hipGetLastError();
}

// Box filter of colour grids (the paper's check that the optimised grids carry the image):
// each output texel of the M x M grid is the mean of the k x k input texels it covers, k = N / M.
__global__ void __launch_bounds__(kThreads)
box_filter_kernel(int64_t P, int N, int M, const float* __restrict__ in, float* __restrict__ out) {
  const int64_t total = P * M * M * 3;
  const int k = N / M;
  const float inv = 1.0f / (float)(k * k);
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int c = (int)(e % 3);
    const int64_t t = e / 3;
    const int j = (int)(t % M), i = (int)((t / M) % M);
    const int64_t p = t / ((int64_t)M * M);
    const float* src = in + ((p * N + (int64_t)i * k) * N + (int64_t)j * k) * 3 + c;
    float acc = 0.0f;
    for (int a = 0; a < k; ++a)
      for (int b = 0; b < k; ++b) acc += src[((int64_t)a * N + b) * 3];
    out[e] = acc * inv;
  }
}

// Rotation about the Z axis only: the x and y components of each quaternion's gradient are
// zeroed, so that Adam leaves quaternions of the form (w, 0, 0, z) in that form.
__global__ void __launch_bounds__(kThreads)
rotz_only_kernel(int64_t P, float* __restrict__ d_quats) {
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < P;
       k += (int64_t)gridDim.x * blockDim.x) {
    d_quats[4 * k + 1] = 0.0f;
    d_quats[4 * k + 2] = 0.0f;
  }
}

hipError_t launch_mse_loss(int64_t n, const float* rgb, const float* target, float scale,
                           float* loss, float* d_rgb, hipStream_t s) {
  unsigned blocks = grid_for(n, 4);
  if (blocks > kL1MaxBlocks) blocks = kL1MaxBlocks;
  hipLaunchKernelGGL(zero_kernel, dim3(1), dim3(64), 0, s, loss);
  hipLaunchKernelGGL(loss_kernel<true>, dim3(blocks), dim3(kThreads), 0, s, n, rgb, target,
                     scale, loss, d_rgb);
  return hipGetLastError();
}

hipError_t launch_box_filter(int64_t P, int N, int M, const float* in, float* out,
                             hipStream_t s) {
  hipLaunchKernelGGL(box_filter_kernel, dim3(grid_for(P * M * M * 3, 1)), dim3(kThreads), 0, s,
                     P, N, M, in, out);
  return hipGetLastError();
}

hipError_t launch_rotz_only(int64_t P, float* d_quats, hipStream_t s) {
  hipLaunchKernelGGL(rotz_only_kernel, dim3(grid_for(P, 1)), dim3(kThreads), 0, s, P, d_quats);
  return hipGetLastError();
}

hipError_t launch_l1_loss(int64_t n, const float* rgb, const float* target, float scale,
                          float* loss, float* d_rgb, hipStream_t s) {
  // each block ends with one float atomic on the single loss value, and those serialise:
  // at most 1024 blocks (a grid of one block per 1024 values took 142 us for 11M values,
  // against ~25 us of memory traffic)
  unsigned blocks = grid_for(n, 4);
  if (blocks > kL1MaxBlocks) blocks = kL1MaxBlocks;
  hipLaunchKernelGGL(zero_kernel, dim3(1), dim3(64), 0, s, loss);
  hipLaunchKernelGGL(loss_kernel<false>, dim3(blocks), dim3(kThreads), 0, s, n, rgb, target,
                     scale, loss, d_rgb);
  return hipGetLastError();
}

hipError_t launch_adam(int64_t n, float* theta, const float* grad, float* m, float* v, float lr,
                       float b1, float b2, float c1, float c2, float eps, uint16_t* bf16,
                       hipStream_t s) {
  hipLaunchKernelGGL(adam_kernel, dim3(grid_for(n, 4)), dim3(kThreads), 0, s, n, theta, grad, m,
                     v, lr, b1, b2, c1, c2, eps, bf16);
  return hipGetLastError();
}

}  // namespace gbb
