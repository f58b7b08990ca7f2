// Forward blend (Alg. 1 forward with Alg. 2 bilinear): one workgroup per tile, one lane per
// pixel, each wave owning an 8 x 8 pixel block. The tile's depth-sorted splats are staged
// into LDS in batches (geometry plus texels, bfloat16 decoded on staging). A wave skips a
// splat whose screen rectangle misses its block, and stops when all of its pixels have
// terminated; the workgroup stops staging when every wave has.
//
// Per pixel and splat: (u, v) from the centre-relative homography, G = exp(-min(q_uv, q_lp)),
// alpha = min(alpha_max, o G); alpha < alpha_min is skipped; if T (1 - alpha) < t_min the
// pixel ends without blending it; otherwise acc += alpha T bilinear(C, u, v), T *= 1 - alpha.
// Saved for the backward: T_final and one past the index of the last blended pair.
//
// Depth-prefix split: the prefix pass also marks every tile where some pixel is still open
// (not stopped by t_min) in a bitmap and saves those pixels' accumulated colour and done flag;
// the rest pass (REST) runs on marked tiles only and resumes from that state, so each pixel
// sees exactly the sequence of splats and operations of a single pass.
#include "blend_common.h"

namespace gbb {

namespace {

// With STATS the kernel also counts its work into stats[0..3]: blended pairs, pixels stopped
// by t_min, lane evaluations (64 per wave and evaluated splat) and staged (tile, splat) pairs;
// the rest pass also adds its blended pairs to stats[4].
// Occupancy target: eight waves per SIMD, or what the 160 KB of LDS per CU allows (a
// workgroup puts one wave on each of the CU's four SIMDs). Grids of several sides (MIXED) ask
// for at most seven: at eight their 64-VGPR budget spills, and seven measured faster for a
// layout of 16 (sides {4, 8, 16} at 1M splats and 1080p: forward 1.468 against 1.516 ms) and
// the same for a layout of 8.
template <int N, int B, bool MIXED>
constexpr int fwd_min_waves() {
  constexpr int lds = B * (GeoLds<B>::kBytesPerSplat + 4 + TexLayout<N>::kPerSplat * 16);
  constexpr int w = 160 * 1024 / lds < 8 ? 160 * 1024 / lds : 8;
  return MIXED && w > 7 ? 7 : w;
}

// This workgroup's slices of the arrays to zero (the coming backward's texture and record
// gradients). Called when the workgroup has finished blending, so that the stores drain
// while other workgroups blend, and without holding registers during the blend. The stores
// are non-temporal: the zeros are not read again before the backward's atomics, and kept out
// of the caches they do not evict the records and texels other workgroups are reading (at 1M
// splats and 1080p the forward took 0.533 ms with ordinary stores, 0.507 with these).
__device__ __forceinline__ void zero_range(const ZeroRange& z) {
  typedef float v4f __attribute__((ext_vector_type(4)));
  const int64_t per = (z.n_body + (int64_t)gridDim.x - 1) / (int64_t)gridDim.x;
  const int64_t lo = (int64_t)blockIdx.x * per;
  const int64_t hi = lo + per < z.n_body ? lo + per : z.n_body;
  v4f* const q = reinterpret_cast<v4f*>(z.body);
  for (int64_t i = lo + (int64_t)threadIdx.x; i < hi; i += (int64_t)blockDim.x)
    __builtin_nontemporal_store((v4f){0.f, 0.f, 0.f, 0.f}, q + i);
  if (blockIdx.x == 0) {
    if ((int)threadIdx.x < z.n_head) z.head[threadIdx.x] = 0.f;
    if ((int)threadIdx.x < z.n_tail) z.tail[threadIdx.x] = 0.f;
  }
}

__device__ __forceinline__ void zero_slice(const BlendParams& p) {
  zero_range(p.zero[0]);
  zero_range(p.zero[1]);
}

// MIXED: each splat has a grid side of its own (at most N), read from p.grid_n.
template <int N, bool BF16, int B, bool STATS, bool REST, bool MIXED>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(fwd_min_waves<N, B, MIXED>())))
blend_fwd_kernel(const ViewDev* __restrict__ views, const SplatRec* __restrict__ rec,
                 const uint32_t* __restrict__ pair_vals, const uint32_t* __restrict__ ranges,
                 const void* __restrict__ textures, BlendParams p, float* __restrict__ rgb,
                 float* __restrict__ T_final, uint32_t* __restrict__ n_last, SplitState split,
                 unsigned long long* __restrict__ stats) {
  __shared__ GeoLds<B> s_geo;
  __shared__ float4 s_tex[B * TexLayout<N>::kPerSplat];
  __shared__ uint8_t s_reach[4][B];  // [wave block][staged splat]: may reach the block
  // MIXED: side and uv -> grid slope of each staged splat's grid (two words per splat: the 16
  // of grid_consts would take the LDS of a batch of 16 8 x 8 grids past an eighth of the CU's)
  __shared__ int32_t s_gn[MIXED ? B : 1];
  __shared__ float s_gscale[MIXED ? B : 1];
  static_assert((B & (B - 1)) == 0, "batch sizes are powers of two");

  const int tile = tile_of_block(p);
  if (tile >= p.total_tiles) {
    if (!REST) zero_slice(p);
    return;
  }
  if (REST && !((split.open_bits[tile >> 5] >> (tile & 31)) & 1u)) return;
  const int vi = view_of_tile(views, p.n_views, tile);
  const ViewDev& V = views[vi];
  const int lt = tile - V.tile_base;
  const int tile_x0 = (lt % V.tiles_x) * p.tile_w;
  const int tile_y0 = (lt / V.tiles_x) * p.tile_h;

  const int tid = threadIdx.x;
  // the wave index is uniform: keep it (and the wave block's geometry) in scalar registers
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
  const int waves_x = p.tile_w >> 3;
  const int n_waves = (int)(blockDim.x >> 6);
  const int bx = (w % waves_x) * 8, by = (w / waves_x) * 8;
  const int lxi = bx + (lane & 7), lyi = by + (lane >> 3);
  const int px = tile_x0 + lxi, py = tile_y0 + lyi;
  const bool inside = px < V.W && py < V.H;
  // pixel centre relative to the wave block's centre and to the tile's (exact half-integers)
  const float lx = (float)(lane & 7) - 3.5f;
  const float ly = (float)(lane >> 3) - 3.5f;
  const float tx = (float)lxi - 0.5f * (float)(p.tile_w - 1);
  const float ty = (float)lyi - 0.5f * (float)(p.tile_h - 1);
  const int tcx = tile_x0 + (p.tile_w >> 1), tcy = tile_y0 + (p.tile_h >> 1);

  const uint32_t rec_base = (uint32_t)vi * (uint32_t)p.P;  // first record of the tile's view
  const uint32_t start = ranges[2 * tile], end = ranges[2 * tile + 1];
  const int64_t pix = (int64_t)V.pix_base + (int64_t)py * V.W + px;  // valid if inside
  float T = 1.0f;
  float acc0 = 0.f, acc1 = 0.f, acc2 = 0.f;
  uint32_t last = start;
  bool done = !inside;
  if (REST && inside) {
    const float4 sv = split.fwd_state[pix];
    acc0 = sv.x;
    acc1 = sv.y;
    acc2 = sv.z;
    done = sv.w != 0.f;
    T = T_final[pix];
  }
  uint32_t st_blend = 0, st_eval = 0;
  bool st_term = false;

  for (uint32_t b0 = start; b0 < end; b0 += B) {
    const int nb = (int)((end - b0) < (uint32_t)B ? (end - b0) : (uint32_t)B);
    if (STATS && tid == 0) atomicAdd(&stats[3], (unsigned long long)nb);
    {
      // thread c stages splat c mod B for wave block c / B (geometry centred on that block)
      // and tests whether it can reach the block: for a batch of 16 and four waves that is
      // one wave doing every (splat, block) staging and test once
      const int j = tid & (B - 1), b = tid / B;
      if (b < n_waves && j < nb) {
        const uint32_t r = pair_vals[b0 + j];
        const SplatRec R = rec[r];
        const int kbx = tile_x0 + (b % waves_x) * 8, kby = tile_y0 + (b / waves_x) * 8;
        const StagedGeo g = stage_geo(R, kbx + 4, kby + 4, tcx, tcy);
        s_geo.store(b, j, g);
        if (MIXED && b == 0) {
          const int n = grid_side<N>(p, r - rec_base);
          s_gn[j] = n;
          s_gscale[j] = grid_scale(n, p.sigma);
        }
        s_reach[b][j] =
            block_may_contribute(g, (float)(kbx + 4 - tcx), (float)(kby + 4 - tcy), kbx, kby, p)
                ? 1
                : 0;
      }
    }
    if constexpr (MIXED)
      stage_texels_mixed<N, BF16, false>(textures, pair_vals + b0, rec_base, nb, s_tex, p,
                                         nullptr, nullptr);
    else
      stage_texels<N, BF16>(textures, pair_vals + b0, rec_base, nb, s_tex, p.spec);
    __syncthreads();

    if (ballot(!done) != 0) {
      // splats of this batch that can reach the wave's 8 x 8 block (one lane per splat)
      const bool may = lane < nb && s_reach[w][lane] != 0;
      uint64_t todo = ballot(may);
      while (todo != 0) {
        const int j = (int)__builtin_ctzll(todo);
        todo &= todo - 1;
        const StagedGeo g = s_geo.load(w, j);
        const PixelEval e = eval_splat(g, lx, ly, tx, ty, p);
        if (STATS) ++st_eval;
        if (!done && e.hit) {
          const float Tn = T * (1.0f - e.alpha);
          if (Tn < p.t_min) {
            done = true;
            if (STATS) st_term = true;
          } else {
            if (STATS) ++st_blend;
            float c0, c1, c2;
            const float4* tex = s_tex + j * TexLayout<N>::kPerSplat;
            if constexpr (N == 1) {
              const float4 t = tex[0];
              c0 = t.x;
              c1 = t.y;
              c2 = t.z;
            } else {
              int iu, iv;
              float fu, fv;
              if constexpr (MIXED) {
                const int n = s_gn[j];
                const float sc = s_gscale[j];
                grid_coord_n(e.u, sc, n, iu, fu);
                grid_coord_n(e.v, sc, n, iv, fv);
              } else {
                grid_coord<N>(e.u, p, iu, fu);
                grid_coord<N>(e.v, p, iv, fv);
              }
              const int k00 = TexLayout<N>::at(iu, iv), kr = TexLayout<N>::kRow;
              const float4 t00 = tex[k00], t01 = tex[k00 + 1];
              const float4 t10 = tex[k00 + kr], t11 = tex[k00 + kr + 1];
              const float a0 = t00.x + fv * (t01.x - t00.x), b0_ = t10.x + fv * (t11.x - t10.x);
              const float a1 = t00.y + fv * (t01.y - t00.y), b1 = t10.y + fv * (t11.y - t10.y);
              const float a2 = t00.z + fv * (t01.z - t00.z), b2 = t10.z + fv * (t11.z - t10.z);
              c0 = a0 + fu * (b0_ - a0);
              c1 = a1 + fu * (b1 - a1);
              c2 = a2 + fu * (b2 - a2);
            }
            const float wgt = e.alpha * T;
            acc0 += wgt * c0;
            acc1 += wgt * c1;
            acc2 += wgt * c2;
            T = Tn;
            last = b0 + (uint32_t)j + 1u;
          }
        }
        if (ballot(!done) == 0) break;
      }
    }
    if (__syncthreads_and(done)) break;
  }

  if (p.tile_work) {
    // the tile's blended span: from its first pair to one past the last pair any pixel
    // blended (the backward's work on this tile)
    __shared__ uint32_t s_span;
    if (tid == 0) s_span = 0u;
    __syncthreads();
    uint32_t span = last - start;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const uint32_t o = (uint32_t)__shfl_xor((int)span, d, 64);
      span = o > span ? o : span;
    }
    if (lane == 0) atomicMax(&s_span, span);
    __syncthreads();
    if (tid == 0) p.tile_work[tile] = REST ? p.tile_work[tile] + s_span : s_span;
  }
  if (inside) {
    rgb[3 * pix + 0] = acc0 + T * p.bg[0];
    rgb[3 * pix + 1] = acc1 + T * p.bg[1];
    rgb[3 * pix + 2] = acc2 + T * p.bg[2];
    T_final[pix] = T;
    n_last[pix] = last;
  }
  if (!REST && split.mode == kPrefixPass) {
    // a tile with an open pixel takes part in the rest pass
    if (!__syncthreads_and(done)) {
      if (tid == 0) {
        atomicOr(&split.open_bits[tile >> 5], 1u << (tile & 31));
        atomicOr(split.any_open, 1u);
      }
      if (inside) split.fwd_state[pix] = make_float4(acc0, acc1, acc2, done ? 1.f : 0.f);
    }
  }
  if (STATS) {
    // per-wave totals (exact in float32: at most 64 x 2^17 per wave), one atomic each
    float red[2] = {(float)st_blend, st_term ? 1.f : 0.f};
    wave_sum_all<2>(red);
    if (lane == 0) {
      atomicAdd(&stats[0], (unsigned long long)red[0]);
      atomicAdd(&stats[1], (unsigned long long)red[1]);
      atomicAdd(&stats[2], 64ull * st_eval);
      if (REST) atomicAdd(&stats[4], (unsigned long long)red[0]);
    }
  }
  if (!REST) zero_slice(p);
}

template <int N, bool BF16, bool STATS, bool REST, bool MIXED>
hipError_t launch_n(const Plan& pl, const gb_splats& sp, const BlendParams& bp,
                    const ViewDev* views, const SplatRec* rec, const uint32_t* pair_vals,
                    const uint32_t* ranges, float* rgb, float* T_final, uint32_t* n_last,
                    const SplitState& split, unsigned long long* stats, hipStream_t s) {
  const dim3 grid((unsigned)(bp.tile_order ? (int64_t)bp.total_tiles
                                           : 8 * (int64_t)bp.tiles_per_xcd));
  const dim3 block((unsigned)(pl.tile_w * pl.tile_h));
#define GBB_FWD_B(BB)                                                                        \
  hipLaunchKernelGGL((blend_fwd_kernel<N, BF16, BB, STATS, REST, MIXED>), grid, block, 0, s,   \
                     views,                                                                   \
                     rec, pair_vals, ranges, sp.textures, bp, rgb, T_final, n_last, split,    \
                     stats)
  if constexpr (N >= 16) {
    // the only batch built for N = 16: 8 splats of 16 x 16 texels hold 36 KB of LDS (4
    // workgroups per CU); 4 double that, and the forward at 1M splats and 1080p took 1.24 ms
    // against 1.33 (a batch of 2: 1.85 ms)
    GBB_FWD_B(4);
  } else {
    switch (pl.batch_fwd) {
      case 8: GBB_FWD_B(8); break;
      case 16: GBB_FWD_B(16); break;
      case 32: GBB_FWD_B(32); break;
      default: GBB_FWD_B(64); break;
    }
  }
#undef GBB_FWD_B
  return hipGetLastError();
}

template <int N, bool BF16, bool MIXED = false>
hipError_t launch_nb(const Plan& pl, const gb_splats& sp, const BlendParams& bp,
                     const ViewDev* views, const SplatRec* rec, const uint32_t* pair_vals,
                     const uint32_t* ranges, float* rgb, float* T_final, uint32_t* n_last,
                     const SplitState& split, unsigned long long* stats, hipStream_t s) {
  const bool rest = split.mode == kRestPass;
  if (stats)
    return rest ? launch_n<N, BF16, true, true, MIXED>(pl, sp, bp, views, rec, pair_vals,
                                                       ranges, rgb, T_final, n_last, split,
                                                       stats, s)
                : launch_n<N, BF16, true, false, MIXED>(pl, sp, bp, views, rec, pair_vals,
                                                        ranges, rgb, T_final, n_last, split,
                                                        stats, s);
  return rest ? launch_n<N, BF16, false, true, MIXED>(pl, sp, bp, views, rec, pair_vals, ranges,
                                                      rgb, T_final, n_last, split, stats, s)
              : launch_n<N, BF16, false, false, MIXED>(pl, sp, bp, views, rec, pair_vals,
                                                       ranges, rgb, T_final, n_last, split,
                                                       stats, s);
}

}  // namespace

// Split of a 4-byte aligned float array into single floats up to its first 16-byte boundary,
// 16-byte stores, and at most 3 trailing floats.
static ZeroRange zero_range_of(float* p, int64_t n) {
  ZeroRange z{nullptr, nullptr, nullptr, 0, 0, 0};
  if (!p || n <= 0) return z;
  int64_t head = (int64_t)((16 - (reinterpret_cast<uintptr_t>(p) & 15)) & 15) / 4;
  if (head > n) head = n;
  const int64_t body = (n - head) / 4;
  z.head = p;
  z.n_head = (int32_t)head;
  z.body = reinterpret_cast<float4*>(p + head);
  z.n_body = body;
  z.tail = p + head + 4 * body;
  z.n_tail = (int32_t)(n - head - 4 * body);
  return z;
}

BlendParams make_blend_params(const Plan& pl, const gb_options& o, int n_views) {
  BlendParams bp;
  const int N = pl.N;
  bp.tex_scale = (float)(N - 1) / (2.0f * o.sigma);
  bp.tex_offset = 0.5f * (float)(N - 1);
  bp.sigma = o.sigma;
  bp.alpha_min = o.alpha_min;
  bp.cull_alpha = 0.99f * o.alpha_min;
  bp.alpha_max = o.alpha_max;
  bp.t_min = o.t_min;
  bp.lp_scale = 1.0f / (2.0f * o.lowpass_var);
  bp.bg[0] = o.bg[0];
  bp.bg[1] = o.bg[1];
  bp.bg[2] = o.bg[2];
  bp.tile_w = pl.tile_w;
  bp.tile_h = pl.tile_h;
  bp.n_views = n_views;
  bp.P = pl.P;
  bp.total_tiles = (int32_t)pl.total_tiles;
  bp.tiles_per_xcd = (int32_t)((pl.total_tiles + 7) / 8);
  bp.tile_order = nullptr;
  bp.tile_work = nullptr;
  bp.spec = nullptr;
  bp.d_spec = nullptr;
  bp.grid_n = nullptr;
  bp.grid_at = nullptr;
  bp.zero[0] = ZeroRange{nullptr, nullptr, nullptr, 0, 0, 0};
  bp.zero[1] = ZeroRange{nullptr, nullptr, nullptr, 0, 0, 0};
  return bp;
}

hipError_t launch_blend_fwd(const Plan& pl, const gb_splats& sp, const gb_options& o,
                            const ViewDev* views, int n_views, const SplatRec* rec,
                            const uint32_t* pair_vals, const uint32_t* ranges, float* rgb,
                            float* T_final, uint32_t* n_last, const SplitState& split,
                            uint32_t* tile_work, const float4* spec, unsigned long long* stats,
                            float* zero, int64_t zero_n, float* zero2, int64_t zero2_n,
                            hipStream_t s) {
  // the forward keeps the fixed tile bands: ranking its tiles by list length measured no
  // faster on the 1M-splat 1080p workload (0.50 ms either way)
  BlendParams bp = make_blend_params(pl, o, n_views);
  bp.tile_work = tile_work;
  bp.spec = spec;
  if (split.mode != kRestPass) {
    bp.zero[0] = zero_range_of(zero, zero_n);
    bp.zero[1] = zero_range_of(zero2, zero2_n);
  }
  const bool bf = sp.tex_dtype == GB_BF16;
  if (sp.tex_side) {
    // grids of several sides, staged into the N x N layout (N = 8 or 16, checked by the API)
    bp.grid_n = sp.tex_side;
    bp.grid_at = sp.tex_offset;
    if (pl.N == 16)
      return bf ? launch_nb<16, true, true>(pl, sp, bp, views, rec, pair_vals, ranges, rgb,
                                            T_final, n_last, split, stats, s)
                : launch_nb<16, false, true>(pl, sp, bp, views, rec, pair_vals, ranges, rgb,
                                             T_final, n_last, split, stats, s);
    return bf ? launch_nb<8, true, true>(pl, sp, bp, views, rec, pair_vals, ranges, rgb, T_final,
                                         n_last, split, stats, s)
              : launch_nb<8, false, true>(pl, sp, bp, views, rec, pair_vals, ranges, rgb,
                                          T_final, n_last, split, stats, s);
  }
#define GBB_FWD(NN)                                                                          \
  return bf ? launch_nb<NN, true>(pl, sp, bp, views, rec, pair_vals, ranges, rgb, T_final,   \
                                  n_last, split, stats, s)                                   \
            : launch_nb<NN, false>(pl, sp, bp, views, rec, pair_vals, ranges, rgb, T_final,  \
                                   n_last, split, stats, s)
  switch (pl.N) {
    case 1: GBB_FWD(1);
    case 2: GBB_FWD(2);
    case 4: GBB_FWD(4);
    case 8: GBB_FWD(8);
    case 16: GBB_FWD(16);
    default: return hipErrorInvalidValue;
  }
#undef GBB_FWD
}

}  // namespace gbb
