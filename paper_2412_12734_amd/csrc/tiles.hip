// Tile duplication and per-tile ranges.
//
// Records arrive in depth order (a stable sort of the float32 depth key over record
// indices). Each visible record covers a rectangle of tiles and owns a run of pair slots (the
// exclusive scan of the tile counts in depth order); the slots are expanded chunk by chunk so
// that consecutive lanes write consecutive pairs. A pair is (global tile index, record index);
// tiles are numbered view by view, row-major within a view. A stable sort of the pairs by tile
// then yields, for each tile, its records in (depth, record index) order.
//
// Depth-prefix split: the first pass takes the longest prefix of the depth order whose pairs
// fit a budget; the second pass pairs each later record only with the tiles that the first
// pass left open (a bitmap over tiles), counting them with a summed-area table of the bitmap
// and locating them by a binary search over the rectangle's rows and a popcount walk along
// one row.
#include "device_util.h"
#include "gbb_internal.h"

namespace gbb {

namespace {

// Largest r in [0, n) with offsets[r] <= x, for non-decreasing offsets with offsets[0] = 0.
__device__ __forceinline__ int64_t last_at_or_below(const uint32_t* __restrict__ offsets,
                                                    int64_t n, uint64_t x) {
  int64_t lo = 0, hi = n - 1;
  while (lo < hi) {
    const int64_t mid = (lo + hi + 1) >> 1;
    if ((uint64_t)offsets[mid] <= x) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// The element whose run [offsets[r], offsets[r] + count) holds slot s (< total, the scan's
// total, with no zero-count element owning a slot): the largest r with offsets[r] <= s. The
// chunk-owner table of the same scan brackets it: the owner of the chunk start at or below s
// is at most r, the owner of the next chunk start (if below total) at least r. One wave
// narrows the bracket by sampling 64 evenly spaced offsets per round (a range of n elements
// takes about log(n) / log(63) dependent loads, against log2(n) for a binary search); all 64
// lanes take part and return the same r.
__device__ int64_t wave_slot_owner(const uint32_t* __restrict__ offsets, int64_t n,
                                   const uint32_t* __restrict__ chunk_owner, uint64_t total,
                                   uint64_t s) {
  const uint64_t c = s / kChunkSlots;
  int64_t lo = chunk_owner[c];
  if (s % kChunkSlots == 0) return lo;
  int64_t hi = (c + 1) * kChunkSlots < total ? (int64_t)chunk_owner[c + 1] : n - 1;
  const int lane = threadIdx.x & 63;
  while (lo < hi) {
    const int64_t span = hi - lo;
    const int64_t pos = lo + span * lane / 63;  // lane 0 samples lo, lane 63 hi
    // offsets do not decrease, so the lanes at or below s form a prefix (lane 0 is in it)
    const uint64_t m = ballot((uint64_t)offsets[pos] <= s);
    const int j = 63 - __builtin_clzll(m);
    const int64_t next = j < 63 ? lo + span * (j + 1) / 63 - 1 : hi;
    lo = lo + span * j / 63;
    hi = next;
  }
  return lo;
}

// One wave.
__global__ void finalize_count_kernel(const uint32_t* __restrict__ offsets, int64_t VP,
                                      Status* st, int64_t capacity, StatusEcho echo,
                                      unsigned long long* mirror, uint32_t* overflow_flag,
                                      int64_t budget, const uint32_t* __restrict__ chunk_owner) {
  // the exact 64-bit total decides: the 32-bit offsets wrap only when it exceeds 2^32,
  // and the capacity is below that
  const unsigned long long K = st->K64;
  const bool over = K > (unsigned long long)capacity;
  uint32_t n = over ? 0u : (uint32_t)K, cut = (uint32_t)VP;
  if (budget > 0) {
    // depth-prefix cut: the largest record count (in depth order) whose pairs fit the budget,
    // i.e. the owner of pair slot `budget`
    if (over) {
      cut = 0u;
    } else if (K > (unsigned long long)budget) {
      cut = (uint32_t)wave_slot_owner(offsets, VP, chunk_owner, K, (uint64_t)budget);
      n = offsets[cut];
    }
  }
  const uint32_t last = n > 0 ? (uint32_t)wave_slot_owner(offsets, VP, chunk_owner, K, n - 1)
                              : 0u;
  if (threadIdx.x == 0) {
    st->overflow = over ? 1u : 0u;
    st->sticky_overflow |= over ? 1u : 0u;
    st->n_views = echo.n_views;
    st->P = echo.P;
    st->off_count = echo.off_count;
    st->off_view_pairs = echo.off_view_pairs;
    // one aligned 8-byte store, so that the host never reads a torn value
    if (mirror) *reinterpret_cast<volatile unsigned long long*>(mirror) = (over ? 1ull << 63 : 0ull) | K;
    if (overflow_flag && over) *overflow_flag = 1u;
    st->any_open = 0u;
    st->cut = cut;
    st->n_sorted = n;
    st->last_first = last;
  }
}

// Sum of one view's per-record tile counts (its pair total), one workgroup per view.
__global__ void __launch_bounds__(256)
view_pairs_kernel(const uint32_t* __restrict__ count, int64_t P, unsigned long long* out) {
  __shared__ unsigned long long s_sum[4];
  const uint32_t* c = count + (int64_t)blockIdx.x * P;
  unsigned long long acc = 0;
  for (int64_t i = threadIdx.x; i < P; i += blockDim.x) acc += c[i];
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_down(acc, o, 64);
  if ((threadIdx.x & 63) == 0) s_sum[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) out[blockIdx.x] = s_sum[0] + s_sum[1] + s_sum[2] + s_sum[3];
}

constexpr int kDupThreads = 256;
constexpr int kDupGrid = 4096;  // workgroups of the duplicate kernels (they loop over chunks)
// Rest pass: a chunk whose owners lie more ranks apart than this searches per slot.
constexpr int64_t kSparseChunkRecords = 4 * kChunkSlots;
static_assert(kChunkSlots == 4 * kDupThreads, "four slots per thread and round");

// Prefix pass: the largest record count (in depth order) whose pairs fit the budget; single
// thread, binary search over the exclusive offsets (offsets[VP] = K).
// Inclusive max-scan over the 64 lanes of a wave.
__device__ __forceinline__ int wave_max_scan(int v) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const int t = __shfl_up(v, d, 64);
    if (lane >= d) v = t > v ? t : v;
  }
  return v;
}

// Tile index of the k-th (from 0) set bit of the tile bitmap in the inclusive range [a, b];
// k must be below the number of set bits there.
__device__ __forceinline__ uint32_t nth_open(const uint32_t* __restrict__ bits, uint32_t a,
                                             uint32_t b, uint32_t k) {
  const uint32_t wa = a >> 5, wb = b >> 5;
  for (uint32_t w = wa; w <= wb; ++w) {
    uint32_t m = bits[w];
    if (w == wa) m &= ~0u << (a & 31);
    if (w == wb) m &= ~0u >> (31 - (b & 31));
    const uint32_t c = (uint32_t)__popc(m);
    if (k < c) {
      // position of the k-th set bit: halve the word five times, keeping the half that
      // holds it (popcount of the low half decides)
      uint32_t pos = 0;
#pragma unroll
      for (int width = 16; width >= 1; width >>= 1) {
        const uint32_t lo = (uint32_t)__popc(m & ((1u << width) - 1u));
        if (k >= lo) {
          k -= lo;
          m >>= width;
          pos += (uint32_t)width;
        }
      }
      return (w << 5) + pos;
    }
    k -= c;
  }
  return b;
}

// Open tiles in the first k + 1 rows of a rectangle w tiles wide, from the summed-area table:
// `at` is the table entry of the rectangle's top-left tile, `stride` = tiles_x + 1.
__device__ __forceinline__ uint32_t open_rows(const uint32_t* __restrict__ sat, int64_t at,
                                              uint32_t stride, uint32_t w, uint32_t k) {
  const int64_t lo = at + (int64_t)(k + 1) * stride;
  return sat[lo + w] - sat[at + w] - sat[lo] + sat[at];
}

// Chunked expansion of pair slots into (tile, record) pairs. Workgroups take chunks of
// kChunkSlots slots in turn, so each does the same amount of output however the slots are
// spread over records. For a chunk [c0, c1) the records of depth ranks chunk_owner[c] (the
// owner of slot c0) to the owner of slot c1 (or of the pass's last slot) are read; each one
// with slots starts a run at position max(offset - c0, 0), marks it and parks its data in LDS
// under that position; a block-wide max-scan of the marks gives every slot its record. Thread
// t writes slots 4t..4t+3 of the chunk (16-byte stores where all four are present).
//   REST = false: the record at rank r is order[r] with count[order[r]] slots; the tile of
//   slot `local` of its rectangle is (local / w, local mod w), the division done exactly as a
//   multiply by ceil(2^40 / w) (for w <= 4096 and local < 2^24 the error stays below 1/w).
//   REST = true: count[r] (by rank) open tiles; slot `local` is the local-th open tile of the
//   rectangle, row by row.
template <bool REST>
__global__ void __launch_bounds__(kDupThreads)
expand_kernel(const uint32_t* __restrict__ order, const uint32_t* __restrict__ count,
              const uint32_t* __restrict__ offsets, const uint32_t* __restrict__ chunk_owner,
              const SplatRec* __restrict__ rec, const ViewDev* __restrict__ views, int tile_w,
              int tile_h, const Status* __restrict__ st, const uint32_t* __restrict__ open_bits,
              const uint32_t* __restrict__ sat, int64_t cap, uint32_t* __restrict__ pair_keys,
              uint32_t* __restrict__ pair_vals, ClearList clear) {
  constexpr int C = kChunkSlots;
  __shared__ int s_own[C];
  __shared__ uint32_t s_start[C];   // first slot of the record
  __shared__ uint32_t s_rec[C];     // record index
  __shared__ uint32_t s_tile0[C];   // first tile of the rectangle's top row
  __shared__ uint32_t s_w[C];       // rectangle width in tiles
  __shared__ uint32_t s_step[C];    // tiles per row of the view; rows of the rectangle (REST)
  __shared__ uint64_t s_magic[REST ? 1 : C];
  __shared__ uint32_t s_h[REST ? C : 1];    // rectangle height in tiles
  __shared__ uint32_t s_sat[REST ? C : 1];  // open-tile table entry of the top-left tile
  __shared__ int s_wave_max[kDupThreads / 64];
  // arrays the later stages of the pass expect zeroed (the pass's tile ranges, the open-tile
  // bitmap), whatever the pair count, so that they need no launches of their own
  for (int k = 0; k < 2; ++k) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < clear.n[k];
         i += (int64_t)gridDim.x * blockDim.x)
      clear.p[k][i] = 0u;
  }
  if (st->overflow) return;
  const int64_t total = (int64_t)(REST ? st->n_rest : st->n_sorted);
  const int64_t last = (int64_t)(REST ? st->last_rest : st->last_first);
  const int64_t slots = total < cap ? total : cap;  // equal unless the status is corrupt
  const int64_t n_chunks = (slots + C - 1) / C;
  const int t = threadIdx.x, w = t >> 6, lane = t & 63;
  for (int64_t c = blockIdx.x; c < n_chunks; c += gridDim.x) {
    const int64_t c0 = c * C;
    const int64_t c1 = (c0 + C < total) ? c0 + C : total;
    const int64_t r0 = chunk_owner[c];
    const int64_t r1 = (c + 1 < n_chunks) ? (int64_t)chunk_owner[c + 1] : last;
    if (REST && r1 - r0 > kSparseChunkRecords) {
      // After the depth cut most records meet no open tile, so a chunk's owners can lie far
      // apart. Such a chunk finds each slot's record by a binary search over the offsets
      // instead of walking every record in between: the last rank whose offset is at or
      // below the slot is its owner (records without slots start where their successor
      // does). The branch is uniform over the workgroup.
      const int64_t q0 = c0 + 4 * t;
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int64_t q = q0 + k;
        if (q >= c1) break;
        const int64_t r = r0 + last_at_or_below(offsets + r0, r1 - r0 + 1, (uint64_t)q);
        const uint32_t id = order[r];
        const SplatRec& R = rec[id];
        const int i0 = R.rect_x & 0xffff, i1 = R.rect_x >> 16;
        const int j0 = R.rect_y & 0xffff, j1 = R.rect_y >> 16;
        const ViewDev& V = views[R.view];
        const uint32_t wt = (uint32_t)(i1 / tile_w - i0 / tile_w + 1);
        const uint32_t ht = (uint32_t)(j1 / tile_h - j0 / tile_h + 1);
        const uint32_t step = (uint32_t)V.tiles_x;
        const uint32_t at = (uint32_t)(V.sat_base + (j0 / tile_h) * (V.tiles_x + 1) + i0 / tile_w);
        uint32_t local = (uint32_t)(q - (int64_t)offsets[r]);
        uint32_t lo = 0, hi = ht - 1;
        while (lo < hi) {
          const uint32_t mid = (lo + hi) >> 1;
          if (open_rows(sat, at, step + 1, wt, mid) > local) hi = mid;
          else lo = mid + 1;
        }
        if (lo > 0) local -= open_rows(sat, at, step + 1, wt, lo - 1);
        const uint32_t a = (uint32_t)(V.tile_base + (j0 / tile_h) * V.tiles_x + i0 / tile_w) +
                           lo * step;
        pair_keys[q] = nth_open(open_bits, a, a + wt - 1, local);
        pair_vals[q] = id;
      }
      continue;
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) s_own[4 * t + k] = -1;
    __syncthreads();
    for (int64_t r = r0 + t; r <= r1; r += kDupThreads) {
      uint32_t id, cnt;
      if constexpr (REST) {
        cnt = count[r];
        if (cnt == 0) continue;
        id = order[r];
      } else {
        id = order[r];
        cnt = count[id];
        if (cnt == 0) continue;
      }
      const int64_t o = offsets[r];
      const int64_t pos = r == r0 ? 0 : o - c0;
      if (pos >= C) continue;  // starts at c1
      s_own[pos] = (int)pos;
      s_start[pos] = (uint32_t)o;
      s_rec[pos] = id;
      const SplatRec& R = rec[id];
      const int i0 = R.rect_x & 0xffff, i1 = R.rect_x >> 16;
      const int j0 = R.rect_y & 0xffff, j1 = R.rect_y >> 16;
      const ViewDev& V = views[R.view];
      const uint32_t wt = (uint32_t)(i1 / tile_w - i0 / tile_w + 1);
      s_w[pos] = wt;
      s_step[pos] = (uint32_t)V.tiles_x;
      s_tile0[pos] = (uint32_t)(V.tile_base + (j0 / tile_h) * V.tiles_x + i0 / tile_w);
      if constexpr (REST) {
        s_h[pos] = (uint32_t)(j1 / tile_h - j0 / tile_h + 1);
        s_sat[pos] = (uint32_t)(V.sat_base + (j0 / tile_h) * (V.tiles_x + 1) + i0 / tile_w);
      } else {
        s_magic[pos] = ((1ull << 40) + wt - 1) / wt;
      }
    }
    __syncthreads();
    int v[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) v[k] = s_own[4 * t + k];
    v[1] = v[1] > v[0] ? v[1] : v[0];
    v[2] = v[2] > v[1] ? v[2] : v[1];
    v[3] = v[3] > v[2] ? v[3] : v[2];
    const int incl = wave_max_scan(v[3]);
    if (lane == 63) s_wave_max[w] = incl;
    int before = __shfl_up(incl, 1, 64);
    if (lane == 0) before = -1;
    __syncthreads();
    for (int ww = 0; ww < w; ++ww) before = s_wave_max[ww] > before ? s_wave_max[ww] : before;
    uint32_t key[4], val[4];
    bool ok[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int64_t q = c0 + 4 * t + k;
      const int own = v[k] > before ? v[k] : before;  // >= 0: position 0 is always marked
      ok[k] = q < c1 && own >= 0;
      key[k] = 0u;
      val[k] = 0u;
      if (ok[k]) {
        uint32_t local = (uint32_t)(q - (int64_t)s_start[own]);
        const uint32_t wt = s_w[own];
        if constexpr (REST) {
          // the row: the first k with more than `local` open tiles in rows [0, k] (binary
          // search on the summed-area table), then the tile inside that row's segment
          const uint32_t step = s_step[own], at = s_sat[own];
          uint32_t lo = 0, hi = s_h[own] - 1;
          while (lo < hi) {
            const uint32_t mid = (lo + hi) >> 1;
            if (open_rows(sat, at, step + 1, wt, mid) > local) hi = mid;
            else lo = mid + 1;
          }
          if (lo > 0) local -= open_rows(sat, at, step + 1, wt, lo - 1);
          const uint32_t a = s_tile0[own] + lo * step;
          key[k] = nth_open(open_bits, a, a + wt - 1, local);
        } else {
          const uint32_t ty = (uint32_t)(((uint64_t)local * s_magic[own]) >> 40);
          key[k] = s_tile0[own] + ty * s_step[own] + (local - ty * wt);
        }
        val[k] = s_rec[own];
      }
    }
    const int64_t q = c0 + 4 * t;
    if (ok[0] && ok[3]) {
      *reinterpret_cast<uint4*>(pair_keys + q) = make_uint4(key[0], key[1], key[2], key[3]);
      *reinterpret_cast<uint4*>(pair_vals + q) = make_uint4(val[0], val[1], val[2], val[3]);
    } else {
#pragma unroll
      for (int k = 0; k < 4; ++k)
        if (ok[k]) {
          pair_keys[q + k] = key[k];
          pair_vals[q + k] = val[k];
        }
    }
    __syncthreads();  // the next chunk reuses the LDS
  }
}

__global__ void __launch_bounds__(256)
count_rest_kernel(const uint32_t* __restrict__ order, const uint32_t* __restrict__ count,
                  const SplatRec* __restrict__ rec, const ViewDev* __restrict__ views, int64_t VP,
                  int tile_w, int tile_h, const Status* __restrict__ st,
                  const uint32_t* __restrict__ sat, uint32_t* __restrict__ count_rest) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= VP) return;
  uint32_t c = 0;
  // with no open tile (the common case when the prefix budget suffices) no record is read
  if (!st->overflow && st->any_open != 0u && r >= (int64_t)st->cut) {
    const uint32_t id = order[r];
    if (count[id] > 0) {
      const SplatRec& R = rec[id];
      const int i0 = R.rect_x & 0xffff, i1 = R.rect_x >> 16;
      const int j0 = R.rect_y & 0xffff, j1 = R.rect_y >> 16;
      const ViewDev& V = views[R.view];
      const int64_t at = V.sat_base + (int64_t)(j0 / tile_h) * (V.tiles_x + 1) + i0 / tile_w;
      c = open_rows(sat, at, (uint32_t)V.tiles_x + 1, (uint32_t)(i1 / tile_w - i0 / tile_w + 1),
                    (uint32_t)(j1 / tile_h - j0 / tile_h));
    }
  }
  count_rest[r] = c;
}

// One workgroup per view: row prefix sums of the open bits (a wave per row, 64 tiles per
// step), then column prefix sums (a thread per column). The table is built in LDS and copied
// out when it fits (any 1080p-class view does), else directly in global memory. With no open
// tile (or an overflow) nothing reads the table, and the kernel returns at once.
constexpr int kSatThreads = 1024;
constexpr int kSatLds = 12288;  // table entries held in LDS (48 KB)

__global__ void __launch_bounds__(kSatThreads)
open_sat_kernel(const ViewDev* __restrict__ views, const uint32_t* __restrict__ open_bits,
                const Status* __restrict__ st, uint32_t* __restrict__ sat) {
  __shared__ uint32_t lds[kSatLds];
  if (st->overflow || st->any_open == 0u) return;
  const ViewDev& V = views[blockIdx.x];
  const int tx = V.tiles_x, ty = V.tiles_y, stride = tx + 1;
  const int64_t entries = (int64_t)stride * (ty + 1);
  uint32_t* S = sat + V.sat_base;
  const bool in_lds = entries <= kSatLds;
  uint32_t* Tb = in_lds ? lds : S;
  const int tid = threadIdx.x, wv = tid >> 6, lane = tid & 63;
  for (int x = tid; x <= tx; x += kSatThreads) Tb[x] = 0;
  for (int y = wv; y < ty; y += kSatThreads / 64) {
    uint32_t* row = Tb + (int64_t)(y + 1) * stride;
    if (lane == 0) row[0] = 0;
    const int64_t t0 = V.tile_base + (int64_t)y * tx;
    uint32_t carry = 0;
    for (int x0 = 0; x0 < tx; x0 += 64) {
      const int x = x0 + lane;
      uint32_t v = 0;
      if (x < tx) {
        const int64_t t = t0 + x;
        v = (open_bits[t >> 5] >> (t & 31)) & 1u;
      }
#pragma unroll
      for (int d = 1; d < 64; d <<= 1) {
        const uint32_t u = __shfl_up(v, d, 64);
        if (lane >= d) v += u;
      }
      if (x < tx) row[x + 1] = carry + v;
      carry += __shfl(v, 63, 64);
    }
  }
  __syncthreads();
  for (int x = tid; x <= tx; x += kSatThreads) {
    uint32_t run = 0;
    for (int y = 1; y <= ty; ++y) {
      run += Tb[(int64_t)y * stride + x];
      Tb[(int64_t)y * stride + x] = run;
    }
  }
  if (in_lds) {
    __syncthreads();
    for (int64_t i = tid; i < entries; i += kSatThreads) S[i] = lds[i];
  }
}

// One wave.
__global__ void finalize_rest_kernel(const uint32_t* __restrict__ offsets_rest, int64_t VP,
                                     Status* st, const uint32_t* __restrict__ chunk_owner) {
  const uint64_t K = st->K_rest64;
  const uint32_t n = st->overflow ? 0u : (uint32_t)K;  // <= K64 <= capacity
  const uint32_t last =
      n > 0 ? (uint32_t)wave_slot_owner(offsets_rest, VP, chunk_owner, K, n - 1) : 0u;
  if (threadIdx.x == 0) {
    st->n_rest = n;
    st->last_rest = last;
  }
}

__global__ void ranges_kernel(const uint32_t* __restrict__ keys, const uint32_t* __restrict__ d_n,
                              uint32_t* __restrict__ ranges) {
  // four consecutive keys per thread; a tile starts where its key differs from the previous
  // one and ends where it differs from the next
  const int64_t n = *d_n;
  for (int64_t i0 = 4 * ((int64_t)blockIdx.x * blockDim.x + threadIdx.x); i0 < n;
       i0 += 4 * (int64_t)gridDim.x * blockDim.x) {
    uint32_t k[6];
    k[0] = i0 > 0 ? keys[i0 - 1] : 0xFFFFFFFFu;
    if (i0 + 4 < n) {
      // i0 is a multiple of four and the key array is 16-byte aligned
      const uint4 q = *reinterpret_cast<const uint4*>(keys + i0);
      k[1] = q.x;
      k[2] = q.y;
      k[3] = q.z;
      k[4] = q.w;
      k[5] = keys[i0 + 4];
    } else {
#pragma unroll
      for (int j = 0; j < 5; ++j) k[j + 1] = i0 + j < n ? keys[i0 + j] : 0xFFFFFFFFu;
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int64_t i = i0 + j;
      if (i < n) {
        if (k[j + 1] != k[j]) ranges[2 * (int64_t)k[j + 1]] = (uint32_t)i;
        if (k[j + 2] != k[j + 1]) ranges[2 * (int64_t)k[j + 1] + 1] = (uint32_t)(i + 1);
      }
    }
  }
}

// Work order of the tiles for the backward launch: a counting sort of the tiles by a
// bucketed cost, most work first, in one workgroup (two passes over the tiles with four
// loads in flight per thread, and a scan of the bucket counts in between).
constexpr int kOrderThreads = 1024;
constexpr int kOrderBuckets = 512;
constexpr int kOrderUnroll = 4;

// Monotone bucket of a cost: exact below 16, then 16 buckets per octave (steps of at most
// 1/16 of the cost); at most 463 for 32-bit costs.
__device__ __forceinline__ uint32_t cost_bucket(uint32_t c) {
  if (c < 16u) return c;
  const uint32_t e = 31u - (uint32_t)__clz(c);  // >= 4
  return 16u * (e - 3u) + ((c >> (e - 4u)) & 15u);
}

__global__ void __launch_bounds__(kOrderThreads)
order_tiles_kernel(const uint32_t* __restrict__ work, int n, uint32_t* __restrict__ order) {
  __shared__ uint32_t s_next[kOrderBuckets];
  __shared__ uint32_t s_wave[kOrderBuckets / 64];
  const int tid = threadIdx.x, lane = tid & 63;
  // slot of tile t: buckets reversed, so that the most work comes first
  auto slots = [&](int t0, uint32_t (&sl)[kOrderUnroll]) {
    uint32_t c[kOrderUnroll];
#pragma unroll
    for (int k = 0; k < kOrderUnroll; ++k) {
      const int t = t0 + k * kOrderThreads;
      c[k] = t < n ? work[t] : 0u;
    }
#pragma unroll
    for (int k = 0; k < kOrderUnroll; ++k)
      sl[k] = (uint32_t)(kOrderBuckets - 1) - cost_bucket(c[k]);
  };
  for (int i = tid; i < kOrderBuckets; i += kOrderThreads) s_next[i] = 0u;
  __syncthreads();
  for (int t0 = tid; t0 < n; t0 += kOrderUnroll * kOrderThreads) {
    uint32_t sl[kOrderUnroll];
    slots(t0, sl);
#pragma unroll
    for (int k = 0; k < kOrderUnroll; ++k)
      if (t0 + k * kOrderThreads < n) atomicAdd(&s_next[sl[k]], 1u);
  }
  __syncthreads();
  // exclusive scan of the bucket counts: threads 0..511 are eight whole waves
  uint32_t v = 0u, incl = 0u;
  if (tid < kOrderBuckets) {
    v = s_next[tid];
    incl = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const uint32_t u = (uint32_t)__shfl_up((int)incl, d, 64);
      if (lane >= d) incl += u;
    }
    if (lane == 63) s_wave[tid >> 6] = incl;
  }
  __syncthreads();
  if (tid < kOrderBuckets) {
    uint32_t base = 0u;
    for (int w = 0; w < (tid >> 6); ++w) base += s_wave[w];
    s_next[tid] = base + incl - v;
  }
  __syncthreads();
  for (int t0 = tid; t0 < n; t0 += kOrderUnroll * kOrderThreads) {
    uint32_t sl[kOrderUnroll];
    slots(t0, sl);
#pragma unroll
    for (int k = 0; k < kOrderUnroll; ++k) {
      const int t = t0 + k * kOrderThreads;
      if (t < n) order[atomicAdd(&s_next[sl[k]], 1u)] = (uint32_t)t;
    }
  }
}

}  // namespace

hipError_t launch_order_tiles(const uint32_t* work, int64_t n_tiles, uint32_t* order,
                              hipStream_t s) {
  if (n_tiles < 1 || n_tiles > kMaxOrderedTiles || !work || !order) return hipErrorInvalidValue;
  hipLaunchKernelGGL(order_tiles_kernel, dim3(1), dim3(kOrderThreads), 0, s, work, (int)n_tiles,
                     order);
  return hipGetLastError();
}

hipError_t launch_finalize_count(const uint32_t* offsets, int64_t VP, Status* st,
                                 int64_t capacity, StatusEcho echo,
                                 unsigned long long* mirror, uint32_t* overflow_flag,
                                 int64_t budget, const uint32_t* chunk_owner, hipStream_t s) {
  hipLaunchKernelGGL(finalize_count_kernel, dim3(1), dim3(64), 0, s, offsets, VP, st, capacity,
                     echo, mirror, overflow_flag, budget, chunk_owner);
  return hipGetLastError();
}

hipError_t launch_view_pairs(const uint32_t* count, int64_t P, int n_views,
                             unsigned long long* out, hipStream_t s) {
  hipLaunchKernelGGL(view_pairs_kernel, dim3((unsigned)n_views), dim3(256), 0, s, count, P, out);
  return hipGetLastError();
}

unsigned dup_grid(int64_t cap) {
  const int64_t chunks = (cap + kChunkSlots - 1) / kChunkSlots;
  return (unsigned)(chunks < 1 ? 1 : (chunks > kDupGrid ? kDupGrid : chunks));
}

hipError_t launch_duplicate(const uint32_t* order, const uint32_t* count,
                            const uint32_t* offsets, const uint32_t* chunk_owner,
                            const SplatRec* rec, const ViewDev* views, int tile_w, int tile_h,
                            const Status* st, int64_t cap, uint32_t* pair_keys,
                            uint32_t* pair_vals, ClearList clear, hipStream_t s) {
  hipLaunchKernelGGL(expand_kernel<false>, dim3(dup_grid(cap)), dim3(kDupThreads), 0, s, order,
                     count, offsets, chunk_owner, rec, views, tile_w, tile_h, st, nullptr, nullptr,
                     cap, pair_keys, pair_vals, clear);
  return hipGetLastError();
}

hipError_t launch_count_rest(const uint32_t* order, const uint32_t* count, const SplatRec* rec,
                             const ViewDev* views, int64_t VP, int tile_w, int tile_h,
                             const Status* st, const uint32_t* sat, uint32_t* count_rest,
                             hipStream_t s) {
  const int64_t blocks = (VP + 255) / 256;
  if (blocks == 0) return hipSuccess;
  hipLaunchKernelGGL(count_rest_kernel, dim3((unsigned)blocks), dim3(256), 0, s, order, count,
                     rec, views, VP, tile_w, tile_h, st, sat, count_rest);
  return hipGetLastError();
}

hipError_t launch_open_sat(const ViewDev* views, int n_views, const uint32_t* open_bits,
                           const Status* st, uint32_t* sat, hipStream_t s) {
  hipLaunchKernelGGL(open_sat_kernel, dim3((unsigned)n_views), dim3(kSatThreads), 0, s, views,
                     open_bits, st, sat);
  return hipGetLastError();
}

hipError_t launch_finalize_rest(const uint32_t* offsets_rest, int64_t VP, Status* st,
                                const uint32_t* chunk_owner, hipStream_t s) {
  hipLaunchKernelGGL(finalize_rest_kernel, dim3(1), dim3(64), 0, s, offsets_rest, VP, st,
                     chunk_owner);
  return hipGetLastError();
}

hipError_t launch_duplicate_rest(const uint32_t* order, const uint32_t* count_rest,
                                 const uint32_t* offsets_rest, const uint32_t* chunk_owner,
                                 const SplatRec* rec, const ViewDev* views, int tile_w,
                                 int tile_h, const Status* st, const uint32_t* open_bits,
                                 const uint32_t* sat, int64_t cap, uint32_t* pair_keys,
                                 uint32_t* pair_vals, ClearList clear, hipStream_t s) {
  hipLaunchKernelGGL(expand_kernel<true>, dim3(dup_grid(cap)), dim3(kDupThreads), 0, s, order,
                     count_rest, offsets_rest, chunk_owner, rec, views, tile_w, tile_h, st,
                     open_bits, sat, cap, pair_keys, pair_vals, clear);
  return hipGetLastError();
}

hipError_t launch_ranges(const uint32_t* pair_keys, const uint32_t* d_n, int64_t n_cap,
                         uint32_t* ranges, hipStream_t s) {
  // grid-stride over the device-side count; the grid only bounds the parallelism
  int64_t blocks = (n_cap + 1023) / 1024;
  if (blocks > 4096) blocks = 4096;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(ranges_kernel, dim3((unsigned)blocks), dim3(256), 0, s, pair_keys, d_n,
                     ranges);
  return hipGetLastError();
}

}  // namespace gbb
