// Pieces shared by the forward and backward blend kernels: the launch parameters, the
// XCD-aware tile schedule, LDS staging of splat batches (geometry and texels) and the
// per-pixel evaluation of one splat (ray-splat uv, falloff, opacity, bilinear colour).
#pragma once

#include "device_util.h"
#include "gbb_internal.h"

namespace gbb {

// A float array zeroed by the forward's workgroups: n_head single floats up to the first
// 16-byte boundary, n_body float4s, then n_tail (at most 3) trailing floats.
struct ZeroRange {
  float* head;
  float4* body;
  float* tail;
  int64_t n_body;
  int32_t n_head, n_tail;
};

struct BlendParams {
  float tex_scale;    // (N - 1) / (2 sigma): uv -> grid coordinate slope
  float tex_offset;   // (N - 1) / 2
  float sigma;
  float alpha_min, alpha_max, t_min;
  float cull_alpha;   // 0.99 alpha_min: the per-wave cull's margin below alpha_min
  float lp_scale;     // 1 / (2 lowpass_var)
  float bg[3];
  int32_t tile_w, tile_h;
  int32_t n_views;
  int32_t P;          // splats per view: record v P + k is splat k seen from view v
  int32_t total_tiles;
  int32_t tiles_per_xcd;
  const uint32_t* tile_order;  // nullable: workgroup b takes tile tile_order[b]
  uint32_t* tile_work;         // nullable: per-tile blended span written by the forward
  // view-dependent colour of each record, added to every texel on staging (nullable), and
  // the backward's adjoint of it (nullable; xyz summed over the record's blended pixels)
  const float4* spec;
  float* d_spec;
  // colour grids of several sides (nullable: every grid is N x N): per splat its side and the
  // index of its first texel in the packed texture array
  const int32_t* grid_n;
  const int64_t* grid_at;
  // forward only: arrays that the workgroups zero while they blend (the coming backward's
  // texture and record gradients); an empty range zeroes nothing
  ZeroRange zero[2];
};

BlendParams make_blend_params(const Plan& pl, const gb_options& o, int n_views);

// Without a work order, workgroups (handed to the 8 XCDs round-robin) take one contiguous
// band of tiles per XCD, so that neighbouring tiles (which share splats) hit the same L2.
// With one, the tiles with the most work start first, round-robin over the XCDs, which
// shortens the tail of the launch and balances the XCDs.
__device__ __forceinline__ int tile_of_block(const BlendParams& p) {
  const int b = blockIdx.x;
  if (p.tile_order) return b < p.total_tiles ? (int)p.tile_order[b] : p.total_tiles;
  return (b & 7) * p.tiles_per_xcd + (b >> 3);
}

__device__ __forceinline__ int view_of_tile(const ViewDev* views, int n_views, int tile) {
  int v = 0;
  while (v + 1 < n_views && views[v + 1].tile_base <= tile) ++v;
  return v;
}

// Geometry of one staged splat for one wave's pixel block. With (lx, ly) a pixel's offset from
// the block centre (half-integers of at most 3.5 for 8 x 8 blocks, exact),
// rho = A + (h00 lx + h01 ly, h10 lx + h11 ly, h20 lx + h21 ly), where A is rho at the block
// centre, evaluated in pair precision. The float32 error of rho grows with the offset times
// |h|, so a centre per wave block (rather than per tile) keeps it at the block's size whatever
// the tile shape. The low-pass offset uses the tile centre: (ox, oy) = tile centre minus
// projected centre, so that a pixel's offset from the projected centre is (tx + ox, ty + oy)
// with (tx, ty) its offset from the tile centre.
//   g0 = (A0, A1, A2, opacity), g1 = (h00, h01, h10, h11), g2 = (h20, h21, ox, oy),
//   rect_x, rect_y: the record's pixel rectangle.
struct StagedGeo {
  float4 g0, g1, g2;
  int32_t rect_x, rect_y;
};

// (cx, cy): the block centre, (tx, ty) the tile centre, in pixel coordinates (integers: blocks
// and tiles have even sides).
__device__ __forceinline__ StagedGeo stage_geo(const SplatRec& r, int cx, int cy, int tx,
                                               int ty) {
  const f2 c2x{r.c2x_hi, r.c2x_lo}, c2y{r.c2y_hi, r.c2y_lo};
  const f2 ox = f2_sub(f2_of((float)cx), c2x);
  const f2 oy = f2_sub(f2_of((float)cy), c2y);
  f2 h[7];
#pragma unroll
  for (int i = 0; i < 7; ++i) h[i] = f2{r.h_hi[i], r.h_lo[i]};
  const f2 A0 = f2_add(f2_mul(h[0], ox), f2_mul(h[1], oy));
  const f2 A1 = f2_add(f2_mul(h[2], ox), f2_mul(h[3], oy));
  const f2 A2 = f2_add(f2_add(f2_mul(h[4], ox), f2_mul(h[5], oy)), h[6]);
  StagedGeo s;
  s.g0 = make_float4(f2_round(A0), f2_round(A1), f2_round(A2), r.opacity);
  s.g1 = make_float4(r.h_hi[0], r.h_hi[1], r.h_hi[2], r.h_hi[3]);
  s.g2 = make_float4(r.h_hi[4], r.h_hi[5], f2_round(f2_sub(f2_of((float)tx), c2x)),
                     f2_round(f2_sub(f2_of((float)ty), c2y)));
  s.rect_x = r.rect_x;
  s.rect_y = r.rect_y;
  return s;
}

// LDS copy of a batch's staged geometry for the (at most four) wave blocks of a tile: g1 and
// g2 once per splat, g0 once per (block, splat). 96 bytes per splat; reading one (block,
// splat) takes three 16-byte loads.
template <int B>
struct GeoLds {
  float4 g1[B];
  float4 g2[B];
  float4 g0[4][B];
  static constexpr int kBytesPerSplat = 6 * 16;

  __device__ void store(int b, int j, const StagedGeo& g) {
    if (b == 0) {
      g1[j] = g.g1;
      g2[j] = g.g2;
    }
    g0[b][j] = g.g0;
  }
  __device__ StagedGeo load(int b, int j) const {
    StagedGeo g;
    g.g0 = g0[b][j];
    g.g1 = g1[j];
    g.g2 = g2[j];
    return g;
  }
};

// LDS texel layout per staged splat: N rows of N + 1 float4 (RGB + pad), so that texels
// (i, j) and (i + 1, j) fall into different LDS banks.
template <int N>
struct TexLayout {
  static constexpr int kRow = N + 1;
  static constexpr int kPerSplat = N * (N + 1);
  // a 24-bit multiply (full rate; a 32-bit integer multiply is quarter rate): iu < N
  __device__ static int at(int iu, int iv) { return (int)__umul24((unsigned)iu, kRow) + iv; }
};

// Copies the texels of `nb` staged splats into LDS as float4 (RGB + pad) per texel. The j-th
// splat is pairs[j] - rec_base: a tile's pairs all hold records of the tile's view, so the
// splat follows from the pair list alone and the texel loads need not wait for the staged
// records. For even N a splat's 3 N^2 channel values split into groups of 12 (four texels):
// each thread moves whole groups, three 16-byte (float32) or 8-byte (bfloat16) loads in, four
// LDS stores out.
// With spec != null each texel also gets the record's view-dependent colour spec[pairs[j]]
// (the bilinear weights sum to one, so this adds that colour to the lookup).
template <int N, bool BF16>
__device__ __forceinline__ void stage_texels(const void* __restrict__ textures,
                                             const uint32_t* __restrict__ pairs,
                                             uint32_t rec_base, int nb, float4* s_tex,
                                             const float4* __restrict__ spec) {
  constexpr int per = 3 * N * N;  // channel values per splat
  const int tid = threadIdx.x, nthr = blockDim.x;
  if constexpr ((per % 12) == 0) {
    constexpr int groups = per / 12;  // = N^2 / 4
    for (int gi = tid; gi < nb * groups; gi += nthr) {
      const int j = gi / groups, a = gi - j * groups;
      const int64_t src = ((int64_t)(pairs[j] - rec_base) * groups + a) * 3;
      const float4 sc = spec ? spec[pairs[j]] : make_float4(0.f, 0.f, 0.f, 0.f);
      float v[12];
      if constexpr (BF16) {
        const uint2* t = reinterpret_cast<const uint2*>(textures) + src;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          const uint2 x = t[k];
          v[4 * k + 0] = __uint_as_float(x.x << 16);
          v[4 * k + 1] = __uint_as_float(x.x & 0xffff0000u);
          v[4 * k + 2] = __uint_as_float(x.y << 16);
          v[4 * k + 3] = __uint_as_float(x.y & 0xffff0000u);
        }
      } else {
        const float4* t = reinterpret_cast<const float4*>(textures) + src;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          const float4 x = t[k];
          v[4 * k + 0] = x.x;
          v[4 * k + 1] = x.y;
          v[4 * k + 2] = x.z;
          v[4 * k + 3] = x.w;
        }
      }
      float4* dst = s_tex + j * TexLayout<N>::kPerSplat;
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int t = 4 * a + k, iu = t / N, iv = t - iu * N;
        dst[TexLayout<N>::at(iu, iv)] =
            spec ? make_float4(v[3 * k] + sc.x, v[3 * k + 1] + sc.y, v[3 * k + 2] + sc.z, 0.f)
                 : make_float4(v[3 * k], v[3 * k + 1], v[3 * k + 2], 0.f);
      }
    }
  } else {
    for (int e = tid; e < nb * per; e += nthr) {
      const int j = e / per, r = e - j * per;
      const int64_t k = (int64_t)(pairs[j] - rec_base);
      float x;
      if constexpr (BF16)
        x = bf16_to_f32(reinterpret_cast<const uint16_t*>(textures)[k * per + r]);
      else
        x = reinterpret_cast<const float*>(textures)[k * per + r];
      if (spec) {
        const float4 sc = spec[pairs[j]];
        x += (r % 3) == 0 ? sc.x : (r % 3) == 1 ? sc.y : sc.z;
      }
      const int t = r / 3, iu = t / N, iv = t - iu * N;
      reinterpret_cast<float*>(s_tex + j * TexLayout<N>::kPerSplat + TexLayout<N>::at(iu, iv))[r % 3] = x;
    }
  }
}

// Row and column of texel t (< 256) of an n-texel side (n <= 16): t / n as a multiply by
// ceil(2^16 / n) and a shift, exact in that range (checked for every t and n).
__device__ __forceinline__ int div_side(int t, int n) {
  return (int)(((uint32_t)t * (uint32_t)((65536 + n - 1) / n)) >> 16);
}

// Side of splat k's grid in a call with several sides, clamped to [1, N].
template <int N>
__device__ __forceinline__ int grid_side(const BlendParams& p, uint32_t k) {
  return min(max(p.grid_n[k], 1), N);
}

// Copies the texels of `nb` staged splats whose grids have sides of their own (at most N) into
// the N x N LDS layout: splat j's n x n texels go to rows and columns [0, n). Wave w takes
// splats w, w + nw, ...; lane q of the wave first loads the side, first value and
// view-dependent colour (spec, nullable, added to each texel as in stage_texels) of the wave's
// q-th splat, so that these loads of all the wave's splats are in flight together; then, splat
// by splat, lane i moves texels i, i + 64, ... of the grid (three channel values in, one
// 16-byte LDS store out: a third of the index arithmetic of moving single values). A
// one-texel grid is also copied to (0, 1), (1, 0) and (1, 1), so that the bilinear lookup,
// which reads the four corners of cell (0, 0) with weights (1, 0, 0, 0) there, reads finite
// values.
// FROM_LDS: each grid's side and first texel come from the staged copies s_gn / s_toff (the
// backward, whose geometry pass staged them well before); otherwise they are read from
// p.grid_n / p.grid_at for record pairs[j] - rec_base, so that the forward need not wait at a
// barrier for the copies staged in the same phase.
template <int N, bool BF16, bool FROM_LDS>
__device__ __forceinline__ void stage_texels_mixed(const void* __restrict__ textures,
                                                   const uint32_t* __restrict__ pairs,
                                                   uint32_t rec_base, int nb, float4* s_tex,
                                                   const BlendParams& p, const int32_t* s_gn,
                                                   const int64_t* s_toff) {
  const int lane = threadIdx.x & 63, w = (int)(threadIdx.x >> 6), nw = (int)(blockDim.x >> 6);
  const float4* __restrict__ spec = p.spec;
  // lane q: the wave's q-th splat (nb <= 64 nw, so one lane per splat suffices)
  int my_n = 1;
  int64_t my_base = 0;
  float4 my_sc = make_float4(0.f, 0.f, 0.f, 0.f);
  const int jq = w + lane * nw;
  if (jq < nb) {
    const uint32_t r = pairs[jq];
    if constexpr (FROM_LDS) {
      my_n = s_gn[jq];
      my_base = 3 * s_toff[jq];
    } else {
      my_n = grid_side<N>(p, r - rec_base);
      my_base = 3 * p.grid_at[r - rec_base];
    }
    if (spec) my_sc = spec[r];
  }
  for (int q = 0; w + q * nw < nb; ++q) {
    const int j = w + q * nw;
    const int n = __builtin_amdgcn_readlane(my_n, q);
    const int64_t base =
        (int64_t)(((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(my_base >> 32), q) << 32) |
                  (uint32_t)__builtin_amdgcn_readlane((int)my_base, q));
    float4 sc = make_float4(0.f, 0.f, 0.f, 0.f);
    if (spec)
      sc = make_float4(__int_as_float(__builtin_amdgcn_readlane(__float_as_int(my_sc.x), q)),
                       __int_as_float(__builtin_amdgcn_readlane(__float_as_int(my_sc.y), q)),
                       __int_as_float(__builtin_amdgcn_readlane(__float_as_int(my_sc.z), q)),
                       0.f);
    float4* dst = s_tex + j * TexLayout<N>::kPerSplat;
    // texel at value index i (its three channels), with the view-dependent colour added
    auto texel = [&](int64_t i) {
      float x0, x1, x2;
      if constexpr (BF16) {
        const uint16_t* t = reinterpret_cast<const uint16_t*>(textures) + i;
        x0 = bf16_to_f32(t[0]);
        x1 = bf16_to_f32(t[1]);
        x2 = bf16_to_f32(t[2]);
      } else {
        const float* t = reinterpret_cast<const float*>(textures) + i;
        x0 = t[0];
        x1 = t[1];
        x2 = t[2];
      }
      return make_float4(x0 + sc.x, x1 + sc.y, x2 + sc.z, 0.f);
    };
    if (n == 1) {
      if (lane < 4) dst[TexLayout<N>::at(lane >> 1, lane & 1)] = texel(base);  // corner lane
    } else {
      // one texel per lane and pass: its three channels in, one 16-byte LDS store out
      for (int t = lane; t < n * n; t += 64) {
        const int iu = div_side(t, n), iv = t - iu * n;
        dst[TexLayout<N>::at(iu, iv)] = texel(base + 3 * t);
      }
    }
  }
}

// Slope of the uv -> grid map of an n-texel side, formed as the host forms it for a uniform
// side (a call whose sides all equal N then matches the uniform path bit for bit).
__device__ __forceinline__ float grid_scale(int n, float sigma) {
  return (float)(n - 1) / (2.0f * sigma);
}

// Ray-splat solve and falloff of one splat at one pixel.
struct PixelEval {
  float dx, dy;       // pixel centre minus projected centre (float32; low-pass and gradients)
  float inv;          // 1 / rho2
  float u, v;
  float G;            // exp(-q)
  float alpha;
  bool uv_branch;     // q came from the uv Gaussian (else from the screen low-pass)
  bool hit;           // rho2 != 0 and alpha >= alpha_min
};

// (lx, ly): pixel centre minus the wave block's centre; (tx, ty): minus the tile's centre.
__device__ __forceinline__ PixelEval eval_splat(const StagedGeo& s, float lx, float ly, float tx,
                                                float ty, const BlendParams& p) {
  PixelEval e;
  e.dx = tx + s.g2.z;
  e.dy = ty + s.g2.w;
  const float r0 = __builtin_fmaf(s.g1.y, ly, __builtin_fmaf(s.g1.x, lx, s.g0.x));
  const float r1 = __builtin_fmaf(s.g1.w, ly, __builtin_fmaf(s.g1.z, lx, s.g0.y));
  const float r2 = __builtin_fmaf(s.g2.y, ly, __builtin_fmaf(s.g2.x, lx, s.g0.z));
  e.inv = __builtin_amdgcn_rcpf(r2);
  e.u = r0 * e.inv;
  e.v = r1 * e.inv;
  const float q_uv = 0.5f * (e.u * e.u + e.v * e.v);
  const float q_lp = (e.dx * e.dx + e.dy * e.dy) * p.lp_scale;
  e.uv_branch = q_uv <= q_lp;
  const float q = e.uv_branch ? q_uv : q_lp;
  e.G = __builtin_amdgcn_exp2f(-q * 1.4426950408889634f);
  e.alpha = fminf(p.alpha_max, s.g0.w * e.G);
  e.hit = (r2 != 0.0f) && (e.alpha >= p.alpha_min);
  return e;
}

// Conservative test whether a staged splat can reach alpha >= alpha_min anywhere in a wave's
// bw x bh pixel block, staged for that block: (bx0, by0) is the block's first pixel and (cx, cy)
// its centre relative to the tile centre. rho is affine in the pixel offset, so its range over
// the block is exact; where rho2 keeps its sign, |u| >= min|rho0| / max|rho2| (likewise v), and
// the low-pass term is bounded by the block's distance to the projected centre. A splat is
// skipped only if even the largest possible opacity is clearly below alpha_min, so skipping
// never changes a result.
__device__ __forceinline__ bool block_may_contribute(const StagedGeo& s, float cx, float cy,
                                                     int bx0, int by0, const BlendParams& p,
                                                     int bw = 8, int bh = 8) {
  const int rx = s.rect_x, ry = s.rect_y;
  const int i0 = rx & 0xffff, i1 = rx >> 16, j0 = ry & 0xffff, j1 = ry >> 16;
  if (i1 < bx0 || i0 > bx0 + bw - 1 || j1 < by0 || j0 > by0 + bh - 1) return false;
  // half extents of the block's pixel centres
  const float ex = 0.5f * (float)(bw - 1), ey = 0.5f * (float)(bh - 1);
  const float h00 = s.g1.x, h01 = s.g1.y, h10 = s.g1.z, h11 = s.g1.w, h20 = s.g2.x, h21 = s.g2.y;
  const float r2c = s.g0.z;
  const float r2e = ex * fabsf(h20) + ey * fabsf(h21);
  if (!(fabsf(r2c) > 1.001f * r2e)) return true;  // the vanishing line may cross the block
  const float r0c = s.g0.x;
  const float r1c = s.g0.y;
  const float r0m = fmaxf(fabsf(r0c) - (ex * fabsf(h00) + ey * fabsf(h01)), 0.f);
  const float r1m = fmaxf(fabsf(r1c) - (ex * fabsf(h10) + ey * fabsf(h11)), 0.f);
  const float inv = 1.0f / (fabsf(r2c) + r2e);
  const float um = r0m * inv, vm = r1m * inv;
  const float q_uv = 0.5f * (um * um + vm * vm);
  const float dxm = fmaxf(fabsf(cx + s.g2.z) - ex, 0.f);
  const float dym = fmaxf(fabsf(cy + s.g2.w) - ey, 0.f);
  const float q_lp = (dxm * dxm + dym * dym) * p.lp_scale;
  const float q = fminf(q_uv, q_lp);
  return s.g0.w * __builtin_amdgcn_exp2f(-q * 1.4426950408889634f) >= p.cull_alpha;
}

// Grid coordinate of u on the corner-aligned N-texel grid (Alg. 2 with the cell index taken
// from the remapped coordinate and limited to N - 2 at the clamped top edge).
template <int N>
__device__ __forceinline__ void grid_coord(float u, const BlendParams& p, int& i, float& f) {
  const float up = fminf(fmaxf(__builtin_fmaf(u, p.tex_scale, p.tex_offset), 0.0f), (float)(N - 1));
  const int fi = (int)up;  // up >= 0, so truncation is the floor
  i = fi < N - 2 ? fi : N - 2;
  f = up - (float)i;
}

// Grid coordinate of u on a corner-aligned grid of n texels per side with slope `scale`
// (grid_scale): as grid_coord<N> with n in place of N (a uniform call's grids give the same
// results); one texel gives cell 0 with f = 0.
__device__ __forceinline__ void grid_coord_n(float u, float scale, int n, int& i, float& f) {
  const float hi = (float)(n - 1);
  const float up = fminf(fmaxf(__builtin_fmaf(u, scale, 0.5f * hi), 0.0f), hi);
  const int fi = (int)up;
  const int cmax = n > 2 ? n - 2 : 0;
  i = fi < cmax ? fi : cmax;
  f = up - (float)i;
}

// Constants of grid_coord_c for an n-texel side: slope (grid_scale), offset (n - 1) / 2,
// upper clamp n - 1 and the largest cell index (its int bits in w), staged once per splat so
// that the per-pixel coordinate costs what the uniform grid's does.
__device__ __forceinline__ float4 grid_consts(int n, float sigma) {
  const float hi = (float)(n - 1);
  const int cmax = n > 2 ? n - 2 : 0;
  return make_float4(grid_scale(n, sigma), 0.5f * hi, hi, __int_as_float(cmax));
}

// grid_coord_n from the side's staged constants (the same operations in the same order, so
// the same results).
__device__ __forceinline__ void grid_coord_c(float u, const float4& gc, int& i, float& f) {
  const float up = fminf(fmaxf(__builtin_fmaf(u, gc.x, gc.y), 0.0f), gc.z);
  const int fi = (int)up;
  const int cmax = __float_as_int(gc.w);
  i = fi < cmax ? fi : cmax;
  f = up - (float)i;
}

}  // namespace gbb
