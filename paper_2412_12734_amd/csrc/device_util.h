// Device helpers for gfx950: float-pair ("double-float") arithmetic, wave64 reductions via
// DPP, ballot helpers and bfloat16 decoding.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gbb {

// ---- unevaluated float pairs (hi + lo), error-free transformations ---------------------
// Knuth's TwoSum and the FMA-based TwoProduct; contraction is switched off so that the
// compiler cannot fuse the error terms away.
struct f2 {
  float hi, lo;
};

__device__ __forceinline__ f2 two_sum(float a, float b) {
#pragma clang fp contract(off)
  float s = a + b;
  float bb = s - a;
  float e = (a - (s - bb)) + (b - bb);
  return {s, e};
}

__device__ __forceinline__ f2 fast_two_sum(float a, float b) {
#pragma clang fp contract(off)
  float s = a + b;
  float e = b - (s - a);
  return {s, e};
}

__device__ __forceinline__ f2 two_prod(float a, float b) {
#pragma clang fp contract(off)
  float p = a * b;
  float e = __builtin_fmaf(a, b, -p);
  return {p, e};
}

__device__ __forceinline__ f2 f2_add(f2 a, f2 b) {
#pragma clang fp contract(off)
  f2 s = two_sum(a.hi, b.hi);
  float lo = s.lo + (a.lo + b.lo);
  return fast_two_sum(s.hi, lo);
}

__device__ __forceinline__ f2 f2_add(f2 a, float b) {
#pragma clang fp contract(off)
  f2 s = two_sum(a.hi, b);
  float lo = s.lo + a.lo;
  return fast_two_sum(s.hi, lo);
}

__device__ __forceinline__ f2 f2_mul(f2 a, float b) {
#pragma clang fp contract(off)
  f2 p = two_prod(a.hi, b);
  float lo = __builtin_fmaf(a.lo, b, p.lo);
  return fast_two_sum(p.hi, lo);
}

__device__ __forceinline__ f2 f2_neg(f2 a) { return {-a.hi, -a.lo}; }

__device__ __forceinline__ f2 f2_sub(f2 a, f2 b) { return f2_add(a, f2_neg(b)); }

__device__ __forceinline__ f2 f2_mul(f2 a, f2 b) {
#pragma clang fp contract(off)
  f2 p = two_prod(a.hi, b.hi);
  float lo = __builtin_fmaf(a.hi, b.lo, __builtin_fmaf(a.lo, b.hi, p.lo));
  return fast_two_sum(p.hi, lo);
}

__device__ __forceinline__ f2 f2_of(float a) { return {a, 0.0f}; }

__device__ __forceinline__ float f2_round(f2 a) { return a.hi + a.lo; }

__device__ __forceinline__ f2 f2_div(f2 a, f2 b) {
#pragma clang fp contract(off)
  float q1 = a.hi / b.hi;
  // r = a - q1 * b, exactly enough: q1*b.hi as a pair, then the small terms
  f2 p = two_prod(q1, b.hi);
  float r = ((a.hi - p.hi) - p.lo) + (a.lo - q1 * b.lo);
  float q2 = r / b.hi;
  return fast_two_sum(q1, q2);
}

// ---- wave64 helpers ------------------------------------------------------------------
// The lanes (of the active ones) where p holds. The compiler builtin takes the condition as
// a lane mask in scalar registers; HIP's __ballot(int) widened it to an integer first and
// compared that again (two vector instructions per vote in the blend loops).
__device__ __forceinline__ uint64_t ballot(bool p) { return __builtin_amdgcn_ballot_w64(p); }

__device__ __forceinline__ uint32_t lane_id() {
  return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
}

__device__ __forceinline__ uint32_t popc64(uint64_t m) { return (uint32_t)__popcll(m); }

// Number of set bits of m below this lane.
__device__ __forceinline__ uint32_t mbcnt(uint64_t m) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                   __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

template <int CTRL, int ROW_MASK = 0xf, int BANK_MASK = 0xf, bool BOUND_CTRL = true>
__device__ __forceinline__ float dpp_f(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROW_MASK,
                                                    BANK_MASK, BOUND_CTRL));
}

// Sum over the 64 lanes of a wave; every lane must be active. The total lands in lane 63.
__device__ __forceinline__ float wave_sum_to_lane63(float v) {
  v += dpp_f<0xB1>(v);             // quad_perm [1,0,3,2]
  v += dpp_f<0x4E>(v);             // quad_perm [2,3,0,1]
  v += dpp_f<0x124>(v);            // row_ror:4
  v += dpp_f<0x128>(v);            // row_ror:8   -> every lane holds its row's sum
  v += dpp_f<0x142, 0xa, 0xf, false>(v);  // row_bcast:15 into rows 1 and 3
  v += dpp_f<0x143, 0xc, 0xf, false>(v);  // row_bcast:31 into rows 2 and 3
  return v;
}

// Sums of K values over the 64 lanes, every lane receiving the totals. The K reductions are
// interleaved step by step so that independent DPP operations fill the VALU-to-DPP wait
// states. Within each row of 16 lanes: xor 1 and xor 2 (quad permutes), rotate by 4 and by 8;
// across rows: swap with the neighbouring row (permlane16) and with the other half of the
// wave (permlane32), each followed by an add.
template <int K>
__device__ __forceinline__ void wave_sum_all(float (&v)[K]) {
#pragma unroll
  for (int k = 0; k < K; ++k) v[k] += dpp_f<0xB1>(v[k]);
#pragma unroll
  for (int k = 0; k < K; ++k) v[k] += dpp_f<0x4E>(v[k]);
#pragma unroll
  for (int k = 0; k < K; ++k) v[k] += dpp_f<0x124>(v[k]);
#pragma unroll
  for (int k = 0; k < K; ++k) v[k] += dpp_f<0x128>(v[k]);
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(v[k]), __float_as_uint(v[k]),
                                                    false, false);
    v[k] = __uint_as_float(r[0]) + __uint_as_float(r[1]);
  }
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(v[k]), __float_as_uint(v[k]),
                                                    false, false);
    v[k] = __uint_as_float(r[0]) + __uint_as_float(r[1]);
  }
}

// Sums of K values over each row of 16 lanes (every lane receives its row's totals),
// interleaved like wave_sum_all.
template <int K>
__device__ __forceinline__ void row_sum_all(float (&v)[K]) {
#pragma unroll
  for (int k = 0; k < K; ++k) v[k] += dpp_f<0xB1>(v[k]);
#pragma unroll
  for (int k = 0; k < K; ++k) v[k] += dpp_f<0x4E>(v[k]);
#pragma unroll
  for (int k = 0; k < K; ++k) v[k] += dpp_f<0x124>(v[k]);
#pragma unroll
  for (int k = 0; k < K; ++k) v[k] += dpp_f<0x128>(v[k]);
}

// Row sums of K values (K <= 16) by a transposing butterfly. In each of four steps a lane and
// its partner inside the 16-lane row (lane ^ 15, ^ 7, ^ 3, ^ 1: DPP row_mirror,
// row_half_mirror, quad_perm [3,2,1,0], quad_perm [1,0,3,2]) split their values pairwise:
// each keeps one value of a pair, chosen by one bit of its row position, and adds the
// partner's copy of it; a value left without a pair is added whole on both sides. The masks
// span all 16 positions, so each lane ends with the row total of one value: about 3K/2 + 4
// instructions instead of 4K for plain reductions. row_scatter_slot gives that value's index
// and whether this lane is the one lane of the row that owns it.
template <int CTRL, int KI>
__device__ __forceinline__ void rs_step(const float (&in)[KI], float (&out)[(KI + 1) / 2],
                                        bool hi) {
#pragma unroll
  for (int i = 0; i < KI / 2; ++i) {
    const float keep = hi ? in[2 * i + 1] : in[2 * i];
    const float send = hi ? in[2 * i] : in[2 * i + 1];
    out[i] = keep + dpp_f<CTRL>(send);
  }
  if (KI & 1) out[KI / 2] = in[KI - 1] + dpp_f<CTRL>(in[KI - 1]);
}

template <int K>
__device__ __forceinline__ float row_reduce_scatter(const float (&v)[K]) {
  static_assert(K >= 1 && K <= 16, "at most 16 values per row");
  constexpr int K1 = (K + 1) / 2, K2 = (K1 + 1) / 2, K3 = (K2 + 1) / 2;
  const int l = threadIdx.x & 15;
  float a[K1], b[K2], c[K3], d[1];
  rs_step<0x140>(v, a, (l & 8) != 0);
  rs_step<0x141>(a, b, (l & 4) != 0);
  rs_step<0x1B>(b, c, (l & 2) != 0);
  rs_step<0xB1>(c, d, (l & 1) != 0);
  return d[0];
}

// One swap step across lane groups: v_permlane32_swap pairs each lane of the wave's lower half
// with one of the upper half, v_permlane16_swap each lane of an even row with one of the next
// row. Swapping a value pair (a, b) and adding the two results leaves one side of every lane
// pair with a summed over the pair and the other side with b summed: a transposing step at one
// swap and one add per pair. A value without a pair is summed on both sides.
template <bool HALVES>
__device__ __forceinline__ float swap_sum(float a, float b) {
  if constexpr (HALVES) {
    const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(a), __float_as_uint(b),
                                                    false, false);
    return __uint_as_float(r[0]) + __uint_as_float(r[1]);
  } else {
    const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(a), __float_as_uint(b),
                                                    false, false);
    return __uint_as_float(r[0]) + __uint_as_float(r[1]);
  }
}

template <bool HALVES, int KI>
__device__ __forceinline__ void swap_step(const float (&in)[KI], float (&out)[(KI + 1) / 2]) {
#pragma unroll
  for (int i = 0; i < KI / 2; ++i) out[i] = swap_sum<HALVES>(in[2 * i], in[2 * i + 1]);
  if (KI & 1) out[KI / 2] = swap_sum<HALVES>(in[KI - 1], in[KI - 1]);
}

// Wave sums of K values (K <= 16): two swap steps (wave halves, then row pairs) and the
// transposing row butterfly leave each of the K totals in lanes of one row, at about
// 2 K / 2 + 2 K / 4 + 3 K / 8 + 4 instructions. wave_scatter_slot gives each lane's total.
template <int K>
__device__ __forceinline__ float wave_reduce_scatter(const float (&v)[K]) {
  static_assert(K >= 1 && K <= 16, "at most 16 values per wave");
  constexpr int K1 = (K + 1) / 2, K2 = (K1 + 1) / 2;
  float a[K1], b[K2];
  swap_step<true>(v, a);
  swap_step<false>(a, b);
  return row_reduce_scatter<K2>(b);
}

// The side of each swap step a lane is on: true where it receives the second value of a pair.
// Taken from the swap itself once per kernel, so that the mapping below holds whichever way
// the hardware orders the exchange.
struct SwapSides {
  bool halves, rows;
};

__device__ __forceinline__ SwapSides swap_sides() {
  return {swap_sum<true>(0.f, 1.f) != 0.f, swap_sum<false>(0.f, 1.f) != 0.f};
}

// The value index that wave_reduce_scatter<K> leaves in this lane, and whether the lane owns
// it (a value that went unpaired at some step is held on both sides; only the lane on the low
// side of every such step owns it, so each of the K totals has exactly one owner).
template <int K>
__device__ __forceinline__ void wave_scatter_slot(SwapSides sides, int& idx, bool& owner) {
  const int l = threadIdx.x & 15;
  const bool hi[6] = {sides.halves, sides.rows, (l & 8) != 0, (l & 4) != 0, (l & 2) != 0,
                      (l & 1) != 0};
  int ids[16];
  bool dup[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    ids[i] = i;
    dup[i] = false;
  }
  int n = K;
#pragma unroll
  for (int s = 0; s < 6; ++s) {
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      if (i < n / 2) {
        ids[i] = hi[s] ? ids[2 * i + 1] : ids[2 * i];
        dup[i] = hi[s] ? dup[2 * i + 1] : dup[2 * i];
      }
    }
    if (n & 1) {
#pragma unroll
      for (int i = 0; i < 8; ++i)
        if (i == n / 2) {
          ids[i] = ids[n - 1];
          dup[i] = dup[n - 1] || hi[s];
        }
    }
    n = (n + 1) / 2;
  }
  idx = ids[0];
  owner = !dup[0];
}

__device__ __forceinline__ float wave_sum(float v) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(wave_sum_to_lane63(v)), 63));
}

__device__ __forceinline__ float bf16_to_f32(uint16_t b) {
  return __uint_as_float(((uint32_t)b) << 16);
}

}  // namespace gbb
