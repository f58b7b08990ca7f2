// Backward blend (Alg. 1 backward with Alg. 2 adj-bilinear): one workgroup per tile walks the
// tile's pairs back to front in LDS batches, starting at the last pair any of its pixels
// blended. Each pixel starts from its saved T_final and S = T_final * bg and, for every splat
// it blended (index below its saved bound, alpha >= alpha_min), in reverse order:
//   T_k = T_{k+1} / (1 - alpha_k), w = alpha_k T_k, colour adjoint w g,
//   adj-bilinear -> texel gradients and (du, dv),
//   d alpha = g . (col T_k - S / (1 - alpha_k)), S += w col,
//   d o = d alpha G, dq = -G o d alpha (both zero where alpha was clamped to alpha_max),
//   uv branch: du += dq u, dv += dq v; low-pass branch: d(dx, dy) += dq 2 (dx, dy) / (2 var),
//   (u, v) = (rho0, rho1) / rho2 -> d rho -> d H (7 entries) and d(dx, dy) -> d c2 = -d(dx, dy).
//
// A lane owns PIX vertically adjacent pixels (the launch uses PIX = 1: waves of 8 x 8 pixels).
// Per splat, a lane first adds up its pixels' contributions; the ten per-splat scalars are
// then summed over the wave by a transposing reduction (permlane swaps across the wave's
// halves and row pairs, then a DPP butterfly inside each row) that leaves each total in one
// lane, which adds it to the splat's LDS slot. Texel gradients are grouped by grid cell (with
// sigma = 0.5 the grid covers only the splat's core, so most blended pixels are border-clamped
// and share a few cells); each group's four corners and three channels are reduced the same
// way, one group after another until every pixel's cell has been taken (a step that blended
// at most kLaneAddMax pixels adds each pixel's corners directly instead). A splat that no
// pixel of the wave blended is skipped after evaluation. After each batch the non-zero LDS
// sums go to global memory with one float atomic each, while the next batch's texels are
// staged; one staging pass prepares the geometry of several batches (bwd_stage_ahead).
#include "blend_common.h"


namespace gbb {

namespace {

// Per-pixel backward state and the outputs of one (pixel, splat) step.
struct PixState {
  float T, S0, S1, S2, g0, g1, g2;
  uint32_t last;
};

struct PixOut {
  bool act;
  int k00;                       // cell (first corner) in the [N][N] gradient grid
  float w[4];                    // corner weights (00, 01, 10, 11)
  float dc0, dc1, dc2;           // colour adjoint alpha T g
  float gh[7], gc2x, gc2y, go;   // record gradients
};

// One (pixel, splat) step of the reverse walk. `act`: the pixel blended this splat. A lane
// that did not runs the same arithmetic with a zero weight and adjoint and a unit
// transmittance factor, so that all of its outputs are zero and its state is unchanged
// without a branch or zeroed outputs; its u, v and 1 / rho2 are replaced by 0 (they are
// infinite where rho2 = 0). Its cell and corner weights are left unspecified.
// MIXED: gc holds the grid-coordinate constants of the splat's grid (grid_consts).
template <int N, bool MIXED = false>
__device__ __forceinline__ void pixel_step(const StagedGeo& g, const float4* tex,
                                           const PixelEval& e, bool act, PixState& ps,
                                           const BlendParams& p, PixOut& o,
                                           float4 gc = make_float4(0.f, 0.f, 0.f, 0.f)) {
  o.act = act;
  const float inv = act ? e.inv : 0.f;
  const float u = act ? e.u : 0.f, v = act ? e.v : 0.f;
  const float inv1m = act ? __builtin_amdgcn_rcpf(1.0f - e.alpha) : 1.0f;
  ps.T = ps.T * inv1m;  // transmittance in front of this splat
  float c0, c1, c2;
  float du = 0.f, dv = 0.f;
  const float wgt = act ? e.alpha * ps.T : 0.f;
  o.dc0 = wgt * ps.g0;
  o.dc1 = wgt * ps.g1;
  o.dc2 = wgt * ps.g2;
  if constexpr (N == 1) {
    const float4 t = tex[0];
    c0 = t.x;
    c1 = t.y;
    c2 = t.z;
    o.k00 = 0;
    o.w[0] = 1.f;
    o.w[1] = o.w[2] = o.w[3] = 0.f;
  } else {
    int iu, iv;
    float fu, fv;
    if constexpr (MIXED) {
      grid_coord_c(u, gc, iu, fu);
      grid_coord_c(v, gc, iv, fv);
    } else {
      grid_coord<N>(u, p, iu, fu);
      grid_coord<N>(v, p, iv, fv);
    }
    o.k00 = iu * N + iv;
    const int l00 = TexLayout<N>::at(iu, iv), kr = TexLayout<N>::kRow;
    const float4 t00 = tex[l00], t01 = tex[l00 + 1], t10 = tex[l00 + kr], t11 = tex[l00 + kr + 1];
    const float a0 = t00.x + fv * (t01.x - t00.x), b0_ = t10.x + fv * (t11.x - t10.x);
    const float a1 = t00.y + fv * (t01.y - t00.y), b1 = t10.y + fv * (t11.y - t10.y);
    const float a2 = t00.z + fv * (t01.z - t00.z), b2 = t10.z + fv * (t11.z - t10.z);
    c0 = a0 + fu * (b0_ - a0);
    c1 = a1 + fu * (b1 - a1);
    c2 = a2 + fu * (b2 - a2);
    o.w[0] = (1.f - fu) * (1.f - fv);
    o.w[1] = (1.f - fu) * fv;
    o.w[2] = fu * (1.f - fv);
    o.w[3] = fu * fv;
    // fractional-position adjoints (Alg. 2), zero where the coordinate is clamped
    const float dfu = o.dc0 * (b0_ - a0) + o.dc1 * (b1 - a1) + o.dc2 * (b2 - a2);
    const float fv0 = (t01.x - t00.x) * (1.f - fu) + (t11.x - t10.x) * fu;
    const float fv1 = (t01.y - t00.y) * (1.f - fu) + (t11.y - t10.y) * fu;
    const float fv2 = (t01.z - t00.z) * (1.f - fu) + (t11.z - t10.z) * fu;
    const float dfv = o.dc0 * fv0 + o.dc1 * fv1 + o.dc2 * fv2;
    const float tsc = MIXED ? gc.x : p.tex_scale;
    du = fabsf(u) < p.sigma ? tsc * dfu : 0.f;  // (-sigma, sigma): one compare with |u|
    dv = fabsf(v) < p.sigma ? tsc * dfv : 0.f;
  }
  const float dalpha_act = ps.g0 * (c0 * ps.T - ps.S0 * inv1m) +
                           ps.g1 * (c1 * ps.T - ps.S1 * inv1m) + ps.g2 * (c2 * ps.T - ps.S2 * inv1m);
  const float dalpha = act ? dalpha_act : 0.f;
  ps.S0 += wgt * c0;
  ps.S1 += wgt * c1;
  ps.S2 += wgt * c2;
  const bool unclamped = g.g0.w * e.G <= p.alpha_max;
  o.go = unclamped ? dalpha * e.G : 0.f;
  const float dq = unclamped ? -e.G * g.g0.w * dalpha : 0.f;
  // the falloff's adjoint goes to (u, v) or to the low-pass offset, selected without a branch
  const float dq_uv = e.uv_branch ? dq : 0.f;
  const float dq_lp = e.uv_branch ? 0.f : dq * 2.f * p.lp_scale;
  du += dq_uv * u;
  dv += dq_uv * v;
  const float dr0 = du * inv, dr1 = dv * inv;
  const float dr2 = -(du * u + dv * v) * inv;
  o.gh[0] = dr0 * e.dx;
  o.gh[1] = dr0 * e.dy;
  o.gh[2] = dr1 * e.dx;
  o.gh[3] = dr1 * e.dy;
  o.gh[4] = dr2 * e.dx;
  o.gh[5] = dr2 * e.dy;
  o.gh[6] = dr2;
  // d c2 collects the low-pass term and the uv term through rho's dependence on the offset
  // (c2 enters both with a minus sign; written as negated products, which fold into the
  // multiply-adds)
  o.gc2x = -(dq_lp * e.dx) - dr0 * g.g1.x - dr1 * g.g1.z - dr2 * g.g2.x;
  o.gc2y = -(dq_lp * e.dy) - dr0 * g.g1.y - dr1 * g.g1.w - dr2 * g.g2.y;
}

// With batches of 8 the LDS allows 7 workgroups per CU (22.6 KB each for 8 x 8 grids, with
// the geometry of 8 batches), but the register allocation (75 VGPRs unconstrained) stops at
// 6 waves per SIMD; asking for 7 (at most 72 VGPRs; the compiler's resource report for
// 8 x 8 FP32 grids gives 71 and no scratch) measured 4 % faster on the 1M-splat 1080p
// workload, 8 (64 VGPRs) slower.
// (N = 16 blocks, at a batch of 4 with a ring of 4 batches' geometry, hold 32 KB of LDS, five
// per CU, so no register target applies there.)
// Wave steps that blended at most this many pixels skip the cell grouping. Measured with the
// multi-batch staging, backward ms for thresholds 16 / 24 / 28 / 32: 1M splats at 1080p 1.41 /
// 1.41 / 1.41 / 1.42 (two runs each), 3M splats at 4 x 1080p 15.32 / 14.77 / 14.63 / 14.61,
// 100k splats at 800x800 0.807 / 0.764 / 0.765 / 0.745.
constexpr int kLaneAddMax = 28;

// Grids of several sides (MIXED) need a few more registers: at 7 waves they spilled 28-40
// bytes, and 6 waves measured faster (sides {2, 4, 8} at 1M splats and 1080p: backward 1.567
// against 1.605 ms).
template <int N, int B, bool MIXED>
constexpr int bwd_min_waves() { return (B <= 8 && N <= 8) ? (MIXED ? 6 : 7) : 1; }

// Batches whose geometry one staging pass prepares: as many as the workgroup's threads can
// stage at once. A workgroup has 64 threads per wave block and a batch needs B per block, so
// that is 64 / B whatever the tile shape. The staging pass is on every wave's path (the waves
// wait for it at the barrier), so fewer, fuller passes shorten the walk: at 1M splats and
// 1080p the backward took 1.540 ms staging every batch on its own (32 of one wave's 64 lanes
// busy), 1.473 / 1.448 / 1.420 ms staging 2 / 4 / 8 batches at once; at 3M splats on four
// 1080p views 16.82 / 15.95 / 15.60 / 15.50 ms. For 16 x 16 grids LDS decides instead: a ring
// of 4 batches (16 splats) rather than 16 takes the workgroup from 37 to 32 KB, five per CU
// rather than four; backward at 1M splats and 1080p 2.59 -> 2.36 ms (sides {4, 8, 16}:
// 2.83 -> 2.62; a ring of 8 batches: 2.65 and 2.91).
template <int N, int B>
constexpr int bwd_stage_ahead() { return N >= 16 ? 4 : 64 / B; }

// Depth-prefix split: on a tile that the prefix left open the block first walks the rest
// pass's list (the later splats) and then, with each pixel's T and S carried over in
// registers, the prefix pass's list; other tiles only walk the prefix list.
// MIXED: each splat has a grid side of its own (at most N), read from p.grid_n; its texel
// gradients go to its own n x n grid at p.grid_at.
template <int N, bool BF16, int B, int PIX, bool MIXED>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(bwd_min_waves<N, B, MIXED>())))
blend_bwd_kernel(const ViewDev* __restrict__ views, const SplatRec* __restrict__ rec,
                 PairList first, PairList rest, const uint32_t* __restrict__ open_bits,
                 const void* __restrict__ textures, BlendParams p,
                 const float* __restrict__ T_final, const float* __restrict__ d_rgb,
                 float* __restrict__ d_rec, float* __restrict__ d_tex) {
  constexpr int TEXG = 3 * N * N;
  constexpr int BH = 8 * PIX;  // wave block: 8 columns x BH rows
  // Per-splat geometry and indices of AHEAD batches (slot k holds [k B, (k + 1) B)): every
  // AHEAD-th batch stages its own and the next AHEAD - 1 batches' geometry in one pass of the
  // staging threads.
  constexpr int AHEAD = bwd_stage_ahead<N, B>();
  __shared__ GeoLds<AHEAD * B> s_geo;
  __shared__ uint8_t s_reach[4][AHEAD * B];  // [wave block][staged splat]: may reach the block
  __shared__ int32_t s_splat[AHEAD * B];
  __shared__ uint32_t s_recid[AHEAD * B];
  __shared__ float4 s_tex[B * TexLayout<N>::kPerSplat];
  __shared__ __attribute__((aligned(16))) float s_gtex[B * TEXG];
  __shared__ float s_grec[B * kRecGrad];  // per splat
  __shared__ uint32_t s_tile_last;
  __shared__ int32_t s_gn[MIXED ? AHEAD * B : 1];
  __shared__ float4 s_gc[MIXED ? AHEAD * B : 1];
  __shared__ int64_t s_toff[MIXED ? AHEAD * B : 1];

  const int tile = tile_of_block(p);
  if (tile >= p.total_tiles) return;
  const bool tile_open = open_bits && ((open_bits[tile >> 5] >> (tile & 31)) & 1u) != 0;
  const int vi = view_of_tile(views, p.n_views, tile);
  const ViewDev& V = views[vi];
  const uint32_t rec_base = (uint32_t)vi * (uint32_t)p.P;  // first record of the tile's view
  const int lt = tile - V.tile_base;
  const int tile_x0 = (lt % V.tiles_x) * p.tile_w;
  const int tile_y0 = (lt / V.tiles_x) * p.tile_h;

  const int tid = threadIdx.x, nthr = blockDim.x;
  // the wave index is uniform: keep it (and the wave block's geometry) in scalar registers
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
  const int waves_x = p.tile_w >> 3;
  const int n_waves = nthr >> 6;
  const int bx = (w % waves_x) * 8, by = (w / waves_x) * BH;
  const int lxi = bx + (lane & 7);
  // pixel centres relative to the wave block's centre (exact half-integers); the block centre
  // relative to the tile's (wave-uniform integers)
  const float lx = (float)(lane & 7) - 3.5f;
  const int tcx = tile_x0 + (p.tile_w >> 1), tcy = tile_y0 + (p.tile_h >> 1);
  const float bcx = (float)(tile_x0 + bx + 4 - tcx), bcy = (float)(tile_y0 + by + BH / 2 - tcy);
  float ly[PIX];
  PixState ps[PIX];
  // packed index of the lane's s-th pixel, or -1 outside the view (recomputed when needed)
  auto pixel_index = [&](int s) -> int64_t {
    const int px = tile_x0 + lxi, py = tile_y0 + by + PIX * (lane >> 3) + s;
    return (px < V.W && py < V.H) ? (int64_t)V.pix_base + (int64_t)py * V.W + px : -1;
  };
#pragma unroll
  for (int s = 0; s < PIX; ++s) {
    ly[s] = (float)(PIX * (lane >> 3) + s) - 0.5f * (float)(BH - 1);
    const int64_t pix = pixel_index(s);
    ps[s].T = 1.0f;
    ps[s].g0 = ps[s].g1 = ps[s].g2 = 0.f;
    if (pix >= 0) {
      ps[s].T = T_final[pix];
      ps[s].g0 = d_rgb[3 * pix + 0];
      ps[s].g1 = d_rgb[3 * pix + 1];
      ps[s].g2 = d_rgb[3 * pix + 2];
    }
    ps[s].S0 = ps[s].T * p.bg[0];
    ps[s].S1 = ps[s].T * p.bg[1];
    ps[s].S2 = ps[s].T * p.bg[2];
  }
  // which wave total each lane receives from the reductions below
  int rec_slot, tex_slot;
  bool rec_owner, tex_owner;
  const SwapSides sides = swap_sides();
  wave_scatter_slot<kRecGrad>(sides, rec_slot, rec_owner);
  // texel sums: the three channels of each of the four cell corners (one corner when N = 1);
  // tex_off is the lane's value's offset from the cell's first channel
  constexpr int KT = N == 1 ? 3 : 12;
  wave_scatter_slot<KT>(sides, tex_slot, tex_owner);
  const int tex_off = 3 * ((tex_slot / 3 & 1) + (tex_slot / 6) * N) + tex_slot % 3;

  // the per-batch LDS sums start at zero; each batch's flush clears what it read
  // (the first barrier of the list loop orders these stores before any add)
  for (int e = tid; e < B * TEXG; e += nthr) s_gtex[e] = 0.f;
  for (int e = tid; e < B * kRecGrad; e += nthr) s_grec[e] = 0.f;

#pragma unroll 1
  for (int li = tile_open ? 0 : 1; li < 2; ++li) {
    const PairList L = li == 0 ? rest : first;
    const uint32_t* __restrict__ pair_vals = L.pair_vals;
    const uint32_t start = L.ranges[2 * tile];
#pragma unroll
    for (int s = 0; s < PIX; ++s) {
      const int64_t pix = pixel_index(s);
      ps[s].last = pix >= 0 ? L.n_last[pix] : start;
    }
    uint32_t lane_last = ps[0].last;
#pragma unroll
    for (int s = 1; s < PIX; ++s) lane_last = ps[s].last > lane_last ? ps[s].last : lane_last;

    __syncthreads();  // every thread has read the previous list's bound
    if (tid == 0) s_tile_last = start;
    __syncthreads();
    atomicMax(&s_tile_last, lane_last);  // largest bound over the tile's pixels
    __syncthreads();
    const uint32_t tile_last = s_tile_last;

    // One staging pass: the geometry of the AHEAD batches that end at pend, into slots
    // [0, AHEAD B).
    auto stage_geometry = [&](uint32_t pend) {
      // thread c stages splat c mod B of batch h = c / (B n_waves) from this one (h = 0 is
      // this batch; h < AHEAD since the workgroup has 64 n_waves threads) for wave block
      // (c / B) mod n_waves (n_waves is 1, 2 or 4), geometry centred on that block, and tests
      // whether it can reach the block
      // (recomputed per pass from an opaque copy of the thread index: hoisted out of the
      // loop, these indices would hold registers across the reverse walk)
      int t = tid;
      __asm__ volatile("" : "+v"(t));
      const int j = t & (B - 1), b = (t / B) & (n_waves - 1),
                h = (t / B) >> __builtin_ctz((unsigned)n_waves);
      // batch h is [pend - min(rem, (h + 1) B), pend - min(rem, h B))
      const uint32_t rem = pend - start;
      const uint32_t o0 = (uint32_t)(h * B) < rem ? (uint32_t)(h * B) : rem;
      const uint32_t o1 = (uint32_t)((h + 1) * B) < rem ? (uint32_t)((h + 1) * B) : rem;
      const uint32_t hstart = pend - o1;
      const int hnb = (int)(o1 - o0);
      if (h < AHEAD && j < hnb) {
        const int jj = h * B + j;
        const uint32_t r = pair_vals[hstart + j];
        const SplatRec R = rec[r];
        const int kbx = tile_x0 + (b % waves_x) * 8, kby = tile_y0 + (b / waves_x) * BH;
        const StagedGeo g = stage_geo(R, kbx + 4, kby + BH / 2, tcx, tcy);
        s_geo.store(b, jj, g);
        s_reach[b][jj] = block_may_contribute(g, (float)(kbx + 4 - tcx),
                                              (float)(kby + BH / 2 - tcy), kbx, kby, p, 8, BH)
                             ? 1
                             : 0;
        if (b == 0) {
          s_splat[jj] = R.splat;
          s_recid[jj] = r;
          if (MIXED) {
            const int n = grid_side<N>(p, r - rec_base);
            s_gn[jj] = n;
            s_gc[jj] = grid_consts(n, p.sigma);
            s_toff[jj] = p.grid_at[r - rec_base];
          }
        }
      }
    };
    // Texels of the batch [bs, bs + n), whose geometry is in slot offset sof (staged by the
    // pass's geometry launch, with a barrier between them).
    auto stage_batch_texels = [&](uint32_t bs, int n, int sof) {
      if constexpr (MIXED)
        stage_texels_mixed<N, BF16, true>(textures, pair_vals + bs, rec_base, n, s_tex, p,
                                          s_gn + sof, s_toff + sof);
      else
        stage_texels<N, BF16>(textures, pair_vals + bs, rec_base, n, s_tex, p.spec);
    };
    // The first batch's geometry pass and texels; later batches stage theirs while the batch
    // before them flushes its sums (below).
    if (tile_last > start) {
      stage_geometry(tile_last);
      if constexpr (MIXED) __syncthreads();  // sides and offsets of the batch's grids
      const uint32_t bs = (tile_last - start) > (uint32_t)B ? tile_last - (uint32_t)B : start;
      stage_batch_texels(bs, (int)(tile_last - bs), 0);
      __syncthreads();
    }
    int slot = 0;  // slot of the batch's geometry: the batch's index in the list mod AHEAD
    for (uint32_t bend = tile_last; bend > start;) {
      const uint32_t bstart = (bend - start) > (uint32_t)B ? bend - (uint32_t)B : start;
      const int nb = (int)(bend - bstart);
      const int so = slot * B;

      // splats of this batch that can reach the wave's block, walked back to front
      const bool may = lane < nb && s_reach[w][so + lane] != 0;
      uint64_t todo = ballot(may);
      while (todo != 0) {
        const int j = 63 - (int)__builtin_clzll(todo);
        todo &= ~(1ull << j);
        const uint32_t jg = bstart + (uint32_t)j;
        if (ballot(jg < lane_last) == 0) continue;
        const StagedGeo g = s_geo.load(w, so + j);
        const float4* tex = s_tex + j * TexLayout<N>::kPerSplat;
        PixelEval e[PIX];
        bool act[PIX];
        // lanes that blended this splat (one mask per pixel slot); the masks serve the skip test
        // below and the texel scatter
        uint64_t pend[PIX], any_act = 0;
#pragma unroll
        for (int s = 0; s < PIX; ++s) {
          e[s] = eval_splat(g, lx, ly[s], lx + bcx, ly[s] + bcy, p);
          act[s] = (jg < ps[s].last) && e[s].hit;
          pend[s] = ballot(act[s]);
          any_act |= pend[s];
        }
        if (any_act == 0) continue;  // no pixel of the wave blended this splat
        PixOut po[PIX];
        if constexpr (MIXED) {
          const float4 gc = s_gc[so + j];
#pragma unroll
          for (int s = 0; s < PIX; ++s)
            pixel_step<N, true>(g, tex, e[s], act[s], ps[s], p, po[s], gc);
        } else {
#pragma unroll
          for (int s = 0; s < PIX; ++s) pixel_step<N>(g, tex, e[s], act[s], ps[s], p, po[s]);
        }

        // Wave sums of the per-splat scalars (a lane first adds its own pixels); the one lane
        // that owns each total adds it to the splat's LDS slot.
        {
          float red[kRecGrad];
#pragma unroll
          for (int k = 0; k < 7; ++k) red[k] = po[0].gh[k];
          red[7] = po[0].gc2x;
          red[8] = po[0].gc2y;
          red[9] = po[0].go;
#pragma unroll
          for (int s = 1; s < PIX; ++s) {
#pragma unroll
            for (int k = 0; k < 7; ++k) red[k] += po[s].gh[k];
            red[7] += po[s].gc2x;
            red[8] += po[s].gc2y;
            red[9] += po[s].go;
          }
          const float tot = wave_reduce_scatter<kRecGrad>(red);
          if (rec_owner) atomicAdd(&s_grec[j * kRecGrad + rec_slot], tot);
        }

        // Texel gradients, grouped by cell over all pixels of the wave.
        float* gt = s_gtex + j * TEXG + tex_off;  // this lane's value in cell 0
        // A wave step that blended few pixels (small or distant splats) adds each pixel's
        // bilinear corners to LDS directly; up to kLaneAddMax lanes this costs less than group
        // passes.
        int n_act = 0;
#pragma unroll
        for (int s = 0; s < PIX; ++s) n_act += __builtin_popcountll(pend[s]);
        if (n_act <= kLaneAddMax) {
          float* gb = s_gtex + j * TEXG;
#pragma unroll
          for (int s = 0; s < PIX; ++s) {
            if (act[s]) {  // this lane's bit of pend[s]
#pragma unroll
              for (int q = 0; q < KT / 3; ++q) {
                const float wq = po[s].w[q];
                if (wq != 0.f) {
                  float* dst = gb + 3 * (po[s].k00 + (q & 1) + (q >> 1) * N);
                  atomicAdd(dst + 0, wq * po[s].dc0);
                  atomicAdd(dst + 1, wq * po[s].dc1);
                  atomicAdd(dst + 2, wq * po[s].dc2);
                }
              }
            }
          }
        } else {
          // Every group takes at least its lead lane, so the loop ends within 64 passes. A bound
          // of four passes with per-lane LDS adds for the remaining lanes measured 1.80 ms at
          // 1M splats and 1080p (10 % of wave steps have more than four cells), eight passes
          // 1.73 ms: the per-lane adds, serialised on shared addresses, cost more than passes.
          // Each pending lane carries its cell as the group key, -1 once its group is taken;
          // non-members contribute through zeroed adjoints. (The lean form of the pass: about
          // four VALU instructions fewer than testing the pending mask bit and selecting the
          // four corner weights; backward 1.41 -> 1.39 ms at 1M splats and 1080p.)
          static_assert(PIX == 1, "one pixel per lane");
          int key = act[0] ? po[0].k00 : -1;  // act[0]: this lane's bit of pend[0]
  #pragma unroll 1
          for (uint64_t left = pend[0]; left != 0;) {
            const int lead_cell = __builtin_amdgcn_readlane(key, (int)__builtin_ctzll(left));
            const bool in = key == lead_cell;
            key = in ? -1 : key;
            left &= ~ballot(in);
            // all corners and channels in one transposing wave reduction, so that one lane per
            // value adds it to LDS: one add instruction per group
            const float d0 = in ? po[0].dc0 : 0.f, d1 = in ? po[0].dc1 : 0.f,
                        d2 = in ? po[0].dc2 : 0.f;
            float red[KT];
  #pragma unroll
            for (int q = 0; q < KT / 3; ++q) {
              red[3 * q] = po[0].w[q] * d0;
              red[3 * q + 1] = po[0].w[q] * d1;
              red[3 * q + 2] = po[0].w[q] * d2;
            }
            const float tot = wave_reduce_scatter<KT>(red);
            if (tex_owner) atomicAdd(gt + 3 * lead_cell, tot);
          }
        }
      }
      __syncthreads();
      // the view-dependent colour of a record is added to every texel of its lookup, so its
      // adjoint over the tile is the sum of the record's texel sums, one per channel: each
      // wave sums the N^2 texels of a (splat, channel) pair at a time
      if (p.d_spec) {
        for (int jc = w; jc < 3 * nb; jc += nthr >> 6) {
          const int j = jc / 3, c = jc - 3 * j;
          float x = 0.f;
          for (int t = lane; t < N * N; t += 64) x += s_gtex[j * TEXG + 3 * t + c];
          x = wave_sum(x);
          if (lane == 0 && x != 0.f) atomicAdd(&p.d_spec[4 * (int64_t)s_recid[so + j] + c], x);
        }
        __syncthreads();  // every texel sum has been read before the flush clears it
      }
      // flush the batch's sums, leaving them zero for the next batch
      if constexpr (MIXED) {
        // the N x N sums hold splat j's n x n grid in rows and columns [0, n): one wave per
        // splat, lane i taking values i, i + 64, ... of the grid's 3 n^2
        for (int j = w; j < nb; j += nthr >> 6) {
          const int n = s_gn[so + j];
          for (int i = lane; i < 3 * n * n; i += 64) {
            const int t = i / 3, c = i - 3 * t, iu = div_side(t, n), iv = t - iu * n;
            float* const sum = &s_gtex[j * TEXG + 3 * (iu * N + iv) + c];
            const float x = *sum;
            *sum = 0.f;
            if (x != 0.f) atomicAdd(&d_tex[3 * s_toff[so + j] + i], x);
          }
        }
      } else if constexpr (TEXG % 4 == 0) {
        // four sums per 16-byte LDS read; one global atomic per non-zero sum
        constexpr int TEXG4 = TEXG / 4;
        float4* g4 = reinterpret_cast<float4*>(s_gtex);
        for (int e = tid; e < nb * TEXG4; e += nthr) {
          const float4 x = g4[e];
          g4[e] = make_float4(0.f, 0.f, 0.f, 0.f);
          if (x.x != 0.f || x.y != 0.f || x.z != 0.f || x.w != 0.f) {
            const int j = e / TEXG4, r = 4 * (e - j * TEXG4);
            float* dst = d_tex + (int64_t)s_splat[so + j] * TEXG + r;
            if (x.x != 0.f) atomicAdd(dst + 0, x.x);
            if (x.y != 0.f) atomicAdd(dst + 1, x.y);
            if (x.z != 0.f) atomicAdd(dst + 2, x.z);
            if (x.w != 0.f) atomicAdd(dst + 3, x.w);
          }
        }
      } else {
        for (int e = tid; e < nb * TEXG; e += nthr) {
          const float x = s_gtex[e];
          s_gtex[e] = 0.f;
          if (x != 0.f) {
            const int j = e / TEXG, r = e - j * TEXG;
            atomicAdd(&d_tex[(int64_t)s_splat[so + j] * TEXG + r], x);
          }
        }
      }
      for (int e = tid; e < nb * kRecGrad; e += nthr) {
        const int j = e / kRecGrad, r = e - j * kRecGrad;
        const float x = s_grec[e];
        s_grec[e] = 0.f;
        if (x != 0.f) atomicAdd(&d_rec[(int64_t)s_recid[so + j] * kRecGrad + r], x);
      }
      // the next batch: its texels (and, when it starts a staging pass, the pass's geometry)
      // load while the atomics above drain
      const int nslot = slot + 1 < AHEAD ? slot + 1 : 0;
      if (bstart > start) {
        const uint32_t nbs = (bstart - start) > (uint32_t)B ? bstart - (uint32_t)B : start;
        if (nslot == 0) {
          __syncthreads();  // the flush above has read the pass's splat and record indices
          stage_geometry(bstart);
          if constexpr (MIXED) __syncthreads();  // sides and offsets of the batch's grids
        }
        stage_batch_texels(nbs, (int)(bstart - nbs), nslot * B);
      }
      __syncthreads();
      bend = bstart;
      slot = nslot;
    }
  }  // lists
}

template <int N, bool BF16, int PIX, bool MIXED = false>
hipError_t launch_np(const Plan& pl, const gb_splats& sp, const BlendParams& bp,
                     const ViewDev* views, const SplatRec* rec, const PairList& first,
                     const PairList& rest, const uint32_t* open_bits, const float* T_final,
                     const float* d_rgb, float* d_rec, float* d_tex, hipStream_t s) {
  const dim3 grid((unsigned)(bp.tile_order ? (int64_t)bp.total_tiles
                                           : 8 * (int64_t)bp.tiles_per_xcd));
  const dim3 block((unsigned)(pl.tile_w * pl.tile_h / PIX));
#define GBB_BWD_B(BB)                                                                         \
  hipLaunchKernelGGL((blend_bwd_kernel<N, BF16, BB, PIX, MIXED>), grid, block, 0, s, views, rec, \
                     first, rest, open_bits, sp.textures, bp, T_final, d_rgb, d_rec, d_tex)
  if constexpr (N >= 16) {
    // the only batch built for N = 16: at 8 splats of 16 x 16 texels (texels and their
    // gradient sums) a workgroup held 67 KB of LDS, two per CU; at 4 the backward at 1M
    // splats and 1080p took 2.58 ms against 3.87 (grids of sides {4, 8, 16}: 2.84 against
    // 4.48); a batch of 2 took 2.47 and 3.25
    GBB_BWD_B(4);
  } else {
    switch (pl.batch_bwd) {
      case 8: GBB_BWD_B(8); break;
      case 32: GBB_BWD_B(32); break;
      default: GBB_BWD_B(16); break;
    }
  }
#undef GBB_BWD_B
  return hipGetLastError();
}

}  // namespace

hipError_t launch_blend_bwd(const Plan& pl, const gb_splats& sp, const gb_options& o,
                            const ViewDev* views, int n_views, const SplatRec* rec,
                            const PairList& first, const PairList& rest,
                            const uint32_t* open_bits, const uint32_t* tile_order,
                            const float* T_final, const float* d_rgb, float* d_rec,
                            float* d_tex, const float4* spec, float* d_spec, hipStream_t s) {
  BlendParams bp = make_blend_params(pl, o, n_views);
  bp.tile_order = tile_order;
  bp.spec = spec;
  bp.d_spec = d_spec;
  const bool bf = sp.tex_dtype == GB_BF16;
  if (sp.tex_side) {
    // grids of several sides in the N x N layout (N = 8 or 16, checked by the API)
    bp.grid_n = sp.tex_side;
    bp.grid_at = sp.tex_offset;
    if (pl.N == 16)
      return bf ? launch_np<16, true, 1, true>(pl, sp, bp, views, rec, first, rest, open_bits,
                                               T_final, d_rgb, d_rec, d_tex, s)
                : launch_np<16, false, 1, true>(pl, sp, bp, views, rec, first, rest, open_bits,
                                                T_final, d_rgb, d_rec, d_tex, s);
    return bf ? launch_np<8, true, 1, true>(pl, sp, bp, views, rec, first, rest, open_bits,
                                            T_final, d_rgb, d_rec, d_tex, s)
              : launch_np<8, false, 1, true>(pl, sp, bp, views, rec, first, rest, open_bits,
                                             T_final, d_rgb, d_rec, d_tex, s);
  }
  // One pixel per lane. Two pixels per lane (8 x 16 wave blocks) measured slower on the
  // 1M-splat 1080p workload (3.0 vs 2.3 ms): LDS limits such blocks to two waves per SIMD and
  // the per-wave cull is coarser.
#define GBB_BWD(NN)                                                                           \
  return bf ? launch_np<NN, true, 1>(pl, sp, bp, views, rec, first, rest, open_bits, T_final, \
                                     d_rgb, d_rec, d_tex, s)                                  \
            : launch_np<NN, false, 1>(pl, sp, bp, views, rec, first, rest, open_bits, T_final,\
                                      d_rgb, d_rec, d_tex, s)
  switch (pl.N) {
    case 1: GBB_BWD(1);
    case 2: GBB_BWD(2);
    case 4: GBB_BWD(4);
    case 8: GBB_BWD(8);
    case 16: GBB_BWD(16);
    default: return hipErrorInvalidValue;
  }
#undef GBB_BWD
}

}  // namespace gbb
