// Densification and pruning of textured splats (the adaptive density control the paper trains
// its 3D scenes with, Sec. 4.2), as HIP kernels over caller-owned arrays.
//
//   stats:  per splat, over the views where it is visible, the norm of the gradient of the loss
//           with respect to a translation of its footprint in the image (the record gradient
//           of the projected centre at fixed homography) and a view count;
//   decide: per splat, from the raw parameters (log-scales, opacity logit) and the mean
//           statistic: prune, keep, clone (keep + copy) or split (two children); children and
//           copies are pruned like their parents;
//   scan:   exclusive scan of the output counts -> output offsets and the new splat count;
//   map:    one entry per output splat: parent index | kind << 30;
//   apply:  gathers every parameter row from its parent; a split child moves its centre to
//           p + s_u z0 t_u + s_v z1 t_v, divides its scales by the shrink factor and resamples
//           its colour grid from the parent's bilinear, border-clamped field at the child's
//           texel centres (Alg. 2); optimiser rows of copies and children start at zero.
#include "device_util.h"
#include "gbb_internal.h"

namespace gbb {

namespace {

constexpr uint32_t kKeep = 0, kCloneCopy = 1, kChild0 = 2, kChild1 = 3;

__global__ void __launch_bounds__(256)
densify_stats_kernel(const uint32_t* __restrict__ count, const float* __restrict__ d_rec,
                     int64_t P, int n_views, float* __restrict__ accum, float* __restrict__ vis) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= P) return;
  float a = 0.f, c = 0.f;
  for (int v = 0; v < n_views; ++v) {
    const int64_t idx = (int64_t)v * P + k;
    if (count[idx] == 0) continue;
    const float gx = d_rec[idx * kRecGrad + 7], gy = d_rec[idx * kRecGrad + 8];
    a += sqrtf(gx * gx + gy * gy);
    c += 1.f;
  }
  if (c > 0.f) {
    accum[k] += a;
    vis[k] += c;
  }
}

// Thresholds moved to the raw parameters' domain on the host (double precision, rounded once):
//   s_max > dense_scale         <=> max(log s) > ls_dense
//   o < min_opacity             <=> logit < logit_min
//   s_max > max_scale (if > 0)  <=> max(log s) > ls_max      (children: > ls_max_child)
struct DecideParams {
  float grad_threshold, ls_dense, logit_min, ls_max, ls_max_child;
  int32_t use_max_scale;
};

__global__ void __launch_bounds__(256)
densify_decide_kernel(int64_t P, const float* __restrict__ log_scales,
                      const float* __restrict__ logits, const float* __restrict__ accum,
                      const float* __restrict__ vis, DecideParams d,
                      uint32_t* __restrict__ action, uint32_t* __restrict__ n_out) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= P) return;
  const float ls = fmaxf(log_scales[2 * k], log_scales[2 * k + 1]);
  const bool transparent = logits[k] < d.logit_min;
  const float c = vis[k];
  const float mean = c > 0.f ? accum[k] / c : 0.f;
  const bool dense = mean >= d.grad_threshold;
  uint32_t act, n;
  if (dense && ls > d.ls_dense) {  // split: the children carry the shrunk scales
    act = 3;
    n = (transparent || (d.use_max_scale && ls > d.ls_max_child)) ? 0u : 2u;
  } else {
    const bool gone = transparent || (d.use_max_scale && ls > d.ls_max);
    act = dense ? 2 : 1;
    n = gone ? 0u : (dense ? 2u : 1u);
  }
  action[k] = act;
  n_out[k] = n;
}

__global__ void __launch_bounds__(256)
densify_map_kernel(int64_t P, const uint32_t* __restrict__ action,
                   const uint32_t* __restrict__ n_out, const uint32_t* __restrict__ offsets,
                   uint32_t* __restrict__ map) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= P) return;
  const uint32_t n = n_out[k];
  if (n == 0) return;
  const uint32_t at = offsets[k], a = action[k];
  if (a == 1) {
    map[at] = (uint32_t)k | (kKeep << 30);
  } else if (a == 2) {
    map[at] = (uint32_t)k | (kKeep << 30);
    map[at + 1] = (uint32_t)k | (kCloneCopy << 30);
  } else {
    map[at] = (uint32_t)k | (kChild0 << 30);
    map[at + 1] = (uint32_t)k | (kChild1 << 30);
  }
}

// Rows of `width` floats gathered from the parents. zero_new: copies and children get zeros
// (optimiser state), else every output copies its parent's row.
__global__ void __launch_bounds__(256)
gather_rows_kernel(const uint32_t* __restrict__ map, const uint32_t* __restrict__ d_n,
                   int64_t n_cap, int width, const float* __restrict__ src,
                   float* __restrict__ dst, int zero_new) {
  const int64_t n_new = *d_n < n_cap ? *d_n : n_cap;
  const int64_t total = n_new * width;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t j = e / width;
    const int c = (int)(e - j * width);
    const uint32_t m = map[j];
    const uint32_t k = m & 0x3FFFFFFFu, kind = m >> 30;
    dst[e] = (zero_new && kind != kKeep) ? 0.f : src[(int64_t)k * width + c];
  }
}

// First two columns of the rotation of q / |q|, q = (w, x, y, z).
__device__ __forceinline__ void tangents(const float* q, float (&tu)[3], float (&tv)[3]) {
  const float n = 1.0f / sqrtf(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
  const float w = q[0] * n, x = q[1] * n, y = q[2] * n, z = q[3] * n;
  tu[0] = 1.f - 2.f * (y * y + z * z);
  tu[1] = 2.f * (x * y + w * z);
  tu[2] = 2.f * (x * z - w * y);
  tv[0] = 2.f * (x * y - w * z);
  tv[1] = 1.f - 2.f * (x * x + z * z);
  tv[2] = 2.f * (y * z + w * x);
}

__global__ void __launch_bounds__(256)
child_geometry_kernel(const uint32_t* __restrict__ map, const uint32_t* __restrict__ d_n,
                      int64_t n_cap, const float* __restrict__ means,
                      const float* __restrict__ quats, const float* __restrict__ log_scales,
                      const float* __restrict__ noise, float log_shrink,
                      float* __restrict__ means_out, float* __restrict__ log_scales_out) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n_cap || j >= (int64_t)*d_n) return;
  const uint32_t m = map[j];
  const uint32_t k = m & 0x3FFFFFFFu, kind = m >> 30;
  float p[3] = {means[3 * k], means[3 * k + 1], means[3 * k + 2]};
  float l0 = log_scales[2 * k], l1 = log_scales[2 * k + 1];
  if (kind >= kChild0) {
    float tu[3], tv[3];
    tangents(quats + 4 * (int64_t)k, tu, tv);
    const float* z = noise + 4 * (int64_t)k + 2 * (kind - kChild0);
    const float su = expf(l0), sv = expf(l1);
    for (int i = 0; i < 3; ++i) p[i] += su * z[0] * tu[i] + sv * z[1] * tv[i];
    l0 -= log_shrink;
    l1 -= log_shrink;
  }
  means_out[3 * j] = p[0];
  means_out[3 * j + 1] = p[1];
  means_out[3 * j + 2] = p[2];
  log_scales_out[2 * j] = l0;
  log_scales_out[2 * j + 1] = l1;
}

// Colour grids of the outputs: copies of the parent's, or for a child the parent's bilinear
// field at the child's texel centres, z + (-sigma + 2 sigma i / (N - 1)) / shrink.
__global__ void __launch_bounds__(256)
child_texture_kernel(const uint32_t* __restrict__ map, const uint32_t* __restrict__ d_n,
                     int64_t n_cap, int N, const float* __restrict__ tex,
                     const float* __restrict__ noise, float sigma, float inv_shrink,
                     float* __restrict__ tex_out) {
  const int per = 3 * N * N;
  const int64_t n_new = *d_n < n_cap ? *d_n : n_cap;
  const int64_t total = n_new * per;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t j = e / per;
    const int r = (int)(e - j * per);
    const uint32_t m = map[j];
    const uint32_t k = m & 0x3FFFFFFFu, kind = m >> 30;
    const float* C = tex + (int64_t)k * per;
    if (kind < kChild0 || N == 1) {
      tex_out[e] = C[r];
      continue;
    }
    const int c = r % 3, t = r / 3, iu = t / N, iv = t - iu * N;
    const float* z = noise + 4 * (int64_t)k + 2 * (kind - kChild0);
    const float step = 2.f * sigma / (float)(N - 1);
    const float u = z[0] + (-sigma + step * (float)iu) * inv_shrink;
    const float v = z[1] + (-sigma + step * (float)iv) * inv_shrink;
    const float scale = (float)(N - 1) / (2.f * sigma);
    const float up = fminf(fmaxf((u + sigma) * scale, 0.f), (float)(N - 1));
    const float vp = fminf(fmaxf((v + sigma) * scale, 0.f), (float)(N - 1));
    const int i0 = min((int)up, N - 2), j0 = min((int)vp, N - 2);
    const float fu = up - (float)i0, fv = vp - (float)j0;
    const float c00 = C[3 * (i0 * N + j0) + c], c01 = C[3 * (i0 * N + j0 + 1) + c];
    const float c10 = C[3 * ((i0 + 1) * N + j0) + c], c11 = C[3 * ((i0 + 1) * N + j0 + 1) + c];
    tex_out[e] = (1.f - fu) * ((1.f - fv) * c00 + fv * c01) + fu * ((1.f - fv) * c10 + fv * c11);
  }
}

unsigned grid1(int64_t n) { return (unsigned)((n + 255) / 256 < 1 ? 1 : (n + 255) / 256); }

unsigned grid_stride(int64_t n) {
  const int64_t b = (n + 255) / 256;
  return (unsigned)(b < 1 ? 1 : (b > 8192 ? 8192 : b));
}

}  // namespace

hipError_t launch_densify_stats(const uint32_t* count, const float* d_rec, int64_t P,
                                int n_views, float* accum, float* vis, hipStream_t s) {
  hipLaunchKernelGGL(densify_stats_kernel, dim3(grid1(P)), dim3(256), 0, s, count, d_rec, P,
                     n_views, accum, vis);
  return hipGetLastError();
}

hipError_t launch_densify_decide(int64_t P, const float* log_scales, const float* logits,
                                 const float* accum, const float* vis, float grad_threshold,
                                 float ls_dense, float logit_min, float ls_max,
                                 float ls_max_child, bool use_max_scale, uint32_t* action,
                                 uint32_t* n_out, hipStream_t s) {
  DecideParams d{grad_threshold, ls_dense, logit_min, ls_max, ls_max_child,
                 use_max_scale ? 1 : 0};
  hipLaunchKernelGGL(densify_decide_kernel, dim3(grid1(P)), dim3(256), 0, s, P, log_scales,
                     logits, accum, vis, d, action, n_out);
  return hipGetLastError();
}

hipError_t launch_densify_map(int64_t P, const uint32_t* action, const uint32_t* n_out,
                              const uint32_t* offsets, uint32_t* map, hipStream_t s) {
  hipLaunchKernelGGL(densify_map_kernel, dim3(grid1(P)), dim3(256), 0, s, P, action, n_out,
                     offsets, map);
  return hipGetLastError();
}

hipError_t launch_gather_rows(const uint32_t* map, const uint32_t* d_n, int64_t n_new, int width,
                              const float* src, float* dst, bool zero_new, hipStream_t s) {
  if (n_new <= 0 || width <= 0) return hipSuccess;
  hipLaunchKernelGGL(gather_rows_kernel, dim3(grid_stride(n_new * width)), dim3(256), 0, s, map,
                     d_n, n_new, width, src, dst, zero_new ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_child_geometry(const uint32_t* map, const uint32_t* d_n, int64_t n_new,
                                 const float* means, const float* quats, const float* log_scales,
                                 const float* noise, float log_shrink, float* means_out,
                                 float* log_scales_out, hipStream_t s) {
  if (n_new <= 0) return hipSuccess;
  hipLaunchKernelGGL(child_geometry_kernel, dim3(grid1(n_new)), dim3(256), 0, s, map, d_n, n_new,
                     means, quats, log_scales, noise, log_shrink, means_out, log_scales_out);
  return hipGetLastError();
}

hipError_t launch_child_texture(const uint32_t* map, const uint32_t* d_n, int64_t n_new, int N,
                                const float* tex, const float* noise, float sigma,
                                float inv_shrink, float* tex_out, hipStream_t s) {
  if (n_new <= 0) return hipSuccess;
  hipLaunchKernelGGL(child_texture_kernel, dim3(grid_stride(n_new * 3 * N * N)), dim3(256), 0, s,
                     map, d_n, n_new, N, tex, noise, sigma, inv_shrink, tex_out);
  return hipGetLastError();
}

}  // namespace gbb
