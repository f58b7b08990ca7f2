// Tile duplication and per-tile ranges.
//
// Records arrive in depth order (a stable sort of the float32 depth key over record
// indices). Each visible record covers a rectangle of tiles; the records of one 256-wide
// block of the depth order own one contiguous run of pair slots (exclusive scan of their
// tile counts), and the block's threads expand that run in order, so consecutive lanes write
// consecutive pairs. A pair is (global tile index, record index); tiles are numbered view by
// view, row-major within a view. A stable sort of the pairs by tile then yields, for each
// tile, its records in (depth, record index) order.
#include "device_util.h"
#include "gbb_internal.h"

namespace gbb {

namespace {

__global__ void finalize_count_kernel(Status* st, int64_t capacity) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    // the exact 64-bit total decides: the 32-bit offsets wrap only when it exceeds 2^32,
    // and the capacity is below that
    const unsigned long long K = st->K64;
    const bool over = K > (unsigned long long)capacity;
    st->overflow = over ? 1u : 0u;
    st->n_sorted = over ? 0u : (uint32_t)K;
  }
}

constexpr int kDupThreads = 256;
constexpr int kDupChunk = 4 * kDupThreads;  // pair slots per round, four per thread

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

// Expands the slot run [s_off[0], s_end[n - 1]) of one block of records (thread t owns
// record t, whose slots are [my_off, my_off + my_cnt)) in rounds of kDupChunk slots. In a
// round, every record whose first slot falls in the round marks that slot with its local
// index, and a block-wide max-scan of the marks gives each slot its owner (the last record
// starting at or before it). Thread t writes slots 4t..4t+3 of the round: key tile_of(owner,
// local slot), value s_rec[owner]. Slot indices stay below the capacity (< 2^32); rounds are
// counted in 64 bits so that the last one cannot wrap.
template <typename TileOf>
__device__ __forceinline__ void expand_slots(const uint32_t* s_off, const uint32_t* s_end,
                                             const uint32_t* s_rec, int n, uint32_t my_off,
                                             uint32_t my_cnt, int* s_own, int* s_wave_max,
                                             TileOf tile_of, uint32_t* __restrict__ pair_keys,
                                             uint32_t* __restrict__ pair_vals) {
  const int t = threadIdx.x, w = t >> 6, lane = t & 63;
  const int64_t q0 = s_off[0];
  const int64_t q1 = s_end[n - 1];
  int carry = -1;  // owner of the last slot of the previous round
  for (int64_t cq = q0 & ~(int64_t)3; cq < q1; cq += kDupChunk) {
#pragma unroll
    for (int k = 0; k < 4; ++k) s_own[4 * t + k] = -1;
    __syncthreads();
    if (my_cnt > 0 && (int64_t)my_off >= cq && (int64_t)my_off < cq + kDupChunk)
      s_own[(int64_t)my_off - cq] = t;
    __syncthreads();
    int v[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) v[k] = s_own[4 * t + k];
    v[1] = v[1] > v[0] ? v[1] : v[0];
    v[2] = v[2] > v[1] ? v[2] : v[1];
    v[3] = v[3] > v[2] ? v[3] : v[2];
    const int incl = wave_max_scan(v[3]);
    if (lane == 63) s_wave_max[w] = incl;
    int prev = __shfl_up(incl, 1, 64);
    if (lane == 0) prev = -1;
    __syncthreads();
    int before = carry;
    for (int ww = 0; ww < w; ++ww) before = s_wave_max[ww] > before ? s_wave_max[ww] : before;
    before = prev > before ? prev : before;
    int round_max = carry;
#pragma unroll
    for (int ww = 0; ww < kDupThreads / 64; ++ww)
      round_max = s_wave_max[ww] > round_max ? s_wave_max[ww] : round_max;
    uint32_t key[4], val[4];
    bool ok[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int64_t q = cq + 4 * t + k;
      const int own = v[k] > before ? v[k] : before;
      ok[k] = own >= 0 && q >= q0 && q < q1;
      key[k] = 0u;
      val[k] = 0u;
      if (ok[k]) {
        key[k] = tile_of(own, (uint32_t)(q - (int64_t)s_off[own]));
        val[k] = s_rec[own];
      }
    }
    const int64_t q = cq + 4 * t;
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
    carry = round_max;
    __syncthreads();
  }
}

// One block per 256 records of the depth order (only the first *d_nrec records when d_nrec is
// given). The tile inside the owner's rectangle is local / w and local mod w, with the
// division done exactly as a multiply by ceil(2^40 / w): for w <= 4096 and local < 2^24 the
// product's error stays below 1/w.
__global__ void __launch_bounds__(kDupThreads)
duplicate_kernel(const uint32_t* __restrict__ order, const uint32_t* __restrict__ count,
                 const uint32_t* __restrict__ offsets, const SplatRec* __restrict__ rec,
                 const ViewDev* __restrict__ views, int64_t VP, const uint32_t* __restrict__ d_nrec,
                 int tile_w, int tile_h, const Status* __restrict__ st,
                 uint32_t* __restrict__ pair_keys, uint32_t* __restrict__ pair_vals) {
  __shared__ uint32_t s_off[kDupThreads];
  __shared__ uint32_t s_end[kDupThreads];
  __shared__ uint32_t s_rec[kDupThreads];
  __shared__ uint32_t s_tile0[kDupThreads];  // global id of the rectangle's top-left tile
  __shared__ uint32_t s_w[kDupThreads];      // rectangle width in tiles
  __shared__ uint32_t s_tiles_x[kDupThreads];
  __shared__ uint64_t s_magic[kDupThreads];  // ceil(2^40 / w)
  __shared__ int s_own[kDupChunk];
  __shared__ int s_wave_max[kDupThreads / 64];
  if (st->overflow) return;
  const int64_t nrec = d_nrec ? (int64_t)*d_nrec : VP;
  const int64_t first = (int64_t)blockIdx.x * kDupThreads;
  if (first >= nrec) return;
  const int n = (int)((nrec - first) < kDupThreads ? (nrec - first) : kDupThreads);
  const int t = threadIdx.x;
  uint32_t my_off = 0, my_cnt = 0;
  if (t < n) {
    const uint32_t r = order[first + t];
    my_cnt = count[r];
    my_off = offsets[first + t];
    s_off[t] = my_off;
    s_end[t] = my_off + my_cnt;
    s_rec[t] = r;
    if (my_cnt > 0) {
      const SplatRec& R = rec[r];
      const int i0 = R.rect_x & 0xffff, i1 = R.rect_x >> 16;
      const int j0 = R.rect_y & 0xffff;
      const ViewDev& V = views[R.view];
      const uint32_t wt = (uint32_t)(i1 / tile_w - i0 / tile_w + 1);
      s_w[t] = wt;
      s_tiles_x[t] = (uint32_t)V.tiles_x;
      s_tile0[t] = (uint32_t)(V.tile_base + (j0 / tile_h) * V.tiles_x + i0 / tile_w);
      s_magic[t] = ((1ull << 40) + wt - 1) / wt;
    }
  }
  __syncthreads();
  auto tile_of = [&](int own, uint32_t local) -> uint32_t {
    const uint32_t wt = s_w[own];
    const uint32_t ty = (uint32_t)(((uint64_t)local * s_magic[own]) >> 40);
    const uint32_t tx = local - ty * wt;
    return s_tile0[own] + ty * s_tiles_x[own] + tx;
  };
  expand_slots(s_off, s_end, s_rec, n, my_off, my_cnt, s_own, s_wave_max, tile_of, pair_keys,
               pair_vals);
}

// ---- depth-prefix split -------------------------------------------------------------------

// Largest r in [0, VP] whose pairs (offsets[r], the exclusive scan in depth order, with
// offsets[VP] = K) fit the budget; a single thread, binary search.
__global__ void prefix_cut_kernel(const uint32_t* __restrict__ offsets, int64_t VP,
                                  int64_t budget, Status* st) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  if (st->overflow) {
    st->cut = 0;
    st->n_sorted = 0;
    return;
  }
  const unsigned long long K = st->K64;
  if (K <= (unsigned long long)budget) {
    st->cut = (uint32_t)VP;
    st->n_sorted = (uint32_t)K;
    return;
  }
  int64_t lo = 0, hi = VP - 1;  // offsets[0] = 0 <= budget
  while (lo < hi) {
    const int64_t mid = (lo + hi + 1) >> 1;
    if ((int64_t)offsets[mid] <= budget) lo = mid;
    else hi = mid - 1;
  }
  st->cut = (uint32_t)lo;
  st->n_sorted = offsets[lo];
}

// Set bits of the tile bitmap in the inclusive global tile range [a, b].
__device__ __forceinline__ uint32_t count_open(const uint32_t* __restrict__ bits, uint32_t a,
                                               uint32_t b) {
  const uint32_t wa = a >> 5, wb = b >> 5;
  const uint32_t lo = ~0u << (a & 31), hi = ~0u >> (31 - (b & 31));
  if (wa == wb) return (uint32_t)__popc(bits[wa] & lo & hi);
  uint32_t c = (uint32_t)__popc(bits[wa] & lo) + (uint32_t)__popc(bits[wb] & hi);
  for (uint32_t w = wa + 1; w < wb; ++w) c += (uint32_t)__popc(bits[w]);
  return c;
}

// Tile index of the k-th (from 0) set bit in [a, b]; k must be below count_open(a, b).
__device__ __forceinline__ uint32_t nth_open(const uint32_t* __restrict__ bits, uint32_t a,
                                             uint32_t b, uint32_t k) {
  const uint32_t wa = a >> 5, wb = b >> 5;
  for (uint32_t w = wa; w <= wb; ++w) {
    uint32_t m = bits[w];
    if (w == wa) m &= ~0u << (a & 31);
    if (w == wb) m &= ~0u >> (31 - (b & 31));
    const uint32_t c = (uint32_t)__popc(m);
    if (k < c) {
      for (uint32_t i = 0; i < k; ++i) m &= m - 1;  // drop the k lowest set bits
      return (w << 5) + (uint32_t)__builtin_ctz(m);
    }
    k -= c;
  }
  return b;
}

__global__ void __launch_bounds__(256)
count_rest_kernel(const uint32_t* __restrict__ order, const uint32_t* __restrict__ count,
                  const SplatRec* __restrict__ rec, const ViewDev* __restrict__ views, int64_t VP,
                  int tile_w, int tile_h, const Status* __restrict__ st,
                  const uint32_t* __restrict__ open_bits, uint32_t* __restrict__ count_rest) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= VP) return;
  uint32_t c = 0;
  if (!st->overflow && r >= (int64_t)st->cut) {
    const uint32_t id = order[r];
    if (count[id] > 0) {
      const SplatRec& R = rec[id];
      const int i0 = R.rect_x & 0xffff, i1 = R.rect_x >> 16;
      const int j0 = R.rect_y & 0xffff, j1 = R.rect_y >> 16;
      const ViewDev& V = views[R.view];
      const int tx0 = i0 / tile_w, tx1 = i1 / tile_w;
      uint32_t a = (uint32_t)(V.tile_base + (j0 / tile_h) * V.tiles_x + tx0);
      for (int ty = j0 / tile_h; ty <= j1 / tile_h; ++ty, a += (uint32_t)V.tiles_x)
        c += count_open(open_bits, a, a + (uint32_t)(tx1 - tx0));
    }
  }
  count_rest[r] = c;
}

__global__ void finalize_rest_kernel(Status* st) {
  if (threadIdx.x == 0 && blockIdx.x == 0)
    st->n_rest = st->overflow ? 0u : (uint32_t)st->K_rest64;  // <= K64 <= capacity
}

// Second-pass pairs: the open tiles of each record at rank >= cut, row by row.
__global__ void __launch_bounds__(kDupThreads)
duplicate_rest_kernel(const uint32_t* __restrict__ order, const uint32_t* __restrict__ count_rest,
                      const uint32_t* __restrict__ offsets_rest, const SplatRec* __restrict__ rec,
                      const ViewDev* __restrict__ views, int64_t VP, int tile_w, int tile_h,
                      const Status* __restrict__ st, const uint32_t* __restrict__ open_bits,
                      uint32_t* __restrict__ pair_keys, uint32_t* __restrict__ pair_vals) {
  __shared__ uint32_t s_off[kDupThreads];
  __shared__ uint32_t s_end[kDupThreads];
  __shared__ uint32_t s_rec[kDupThreads];
  __shared__ uint32_t s_tile0[kDupThreads];  // first tile of the rectangle's top row
  __shared__ uint32_t s_w[kDupThreads];      // rectangle width and height in tiles
  __shared__ uint32_t s_h[kDupThreads];
  __shared__ uint32_t s_tiles_x[kDupThreads];
  __shared__ int s_own[kDupChunk];
  __shared__ int s_wave_max[kDupThreads / 64];
  if (st->overflow) return;
  const int64_t first = (int64_t)blockIdx.x * kDupThreads;
  if (first >= VP) return;
  const int n = (int)((VP - first) < kDupThreads ? (VP - first) : kDupThreads);
  const int t = threadIdx.x;
  uint32_t my_off = 0, my_cnt = 0;
  if (t < n) {
    my_cnt = count_rest[first + t];
    my_off = offsets_rest[first + t];
    s_off[t] = my_off;
    s_end[t] = my_off + my_cnt;
    if (my_cnt > 0) {
      const uint32_t r = order[first + t];
      s_rec[t] = r;
      const SplatRec& R = rec[r];
      const int i0 = R.rect_x & 0xffff, i1 = R.rect_x >> 16;
      const int j0 = R.rect_y & 0xffff, j1 = R.rect_y >> 16;
      const ViewDev& V = views[R.view];
      s_w[t] = (uint32_t)(i1 / tile_w - i0 / tile_w + 1);
      s_h[t] = (uint32_t)(j1 / tile_h - j0 / tile_h + 1);
      s_tiles_x[t] = (uint32_t)V.tiles_x;
      s_tile0[t] = (uint32_t)(V.tile_base + (j0 / tile_h) * V.tiles_x + i0 / tile_w);
    }
  }
  __syncthreads();
  if (s_off[0] == s_end[n - 1]) return;  // no second-pass pairs in this block (uniform)
  auto tile_of = [&](int own, uint32_t local) -> uint32_t {
    uint32_t a = s_tile0[own];
    const uint32_t w = s_w[own], h = s_h[own], step = s_tiles_x[own];
    for (uint32_t row = 0; row < h; ++row, a += step) {
      const uint32_t c = count_open(open_bits, a, a + w - 1);
      if (local < c) return nth_open(open_bits, a, a + w - 1, local);
      local -= c;
    }
    return a;  // not reached: local is below the record's open-tile count
  };
  expand_slots(s_off, s_end, s_rec, n, my_off, my_cnt, s_own, s_wave_max, tile_of, pair_keys,
               pair_vals);
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

}  // namespace

hipError_t launch_finalize_count(Status* st, int64_t capacity, hipStream_t s) {
  hipLaunchKernelGGL(finalize_count_kernel, dim3(1), dim3(64), 0, s, st, capacity);
  return hipGetLastError();
}

hipError_t launch_prefix_cut(const uint32_t* offsets, int64_t VP, int64_t budget, Status* st,
                             hipStream_t s) {
  hipLaunchKernelGGL(prefix_cut_kernel, dim3(1), dim3(64), 0, s, offsets, VP, budget, st);
  return hipGetLastError();
}

hipError_t launch_duplicate(const uint32_t* order, const uint32_t* count,
                            const uint32_t* offsets, const SplatRec* rec, const ViewDev* views,
                            int64_t VP, const uint32_t* d_nrec, int tile_w, int tile_h,
                            const Status* st, uint32_t* pair_keys, uint32_t* pair_vals,
                            hipStream_t s) {
  const int64_t blocks = (VP + kDupThreads - 1) / kDupThreads;
  if (blocks == 0) return hipSuccess;
  hipLaunchKernelGGL(duplicate_kernel, dim3((unsigned)blocks), dim3(kDupThreads), 0, s, order,
                     count, offsets, rec, views, VP, d_nrec, tile_w, tile_h, st, pair_keys,
                     pair_vals);
  return hipGetLastError();
}

hipError_t launch_count_rest(const uint32_t* order, const uint32_t* count, const SplatRec* rec,
                             const ViewDev* views, int64_t VP, int tile_w, int tile_h,
                             const Status* st, const uint32_t* open_bits, uint32_t* count_rest,
                             hipStream_t s) {
  const int64_t blocks = (VP + 255) / 256;
  if (blocks == 0) return hipSuccess;
  hipLaunchKernelGGL(count_rest_kernel, dim3((unsigned)blocks), dim3(256), 0, s, order, count,
                     rec, views, VP, tile_w, tile_h, st, open_bits, count_rest);
  return hipGetLastError();
}

hipError_t launch_finalize_rest(Status* st, hipStream_t s) {
  hipLaunchKernelGGL(finalize_rest_kernel, dim3(1), dim3(64), 0, s, st);
  return hipGetLastError();
}

hipError_t launch_duplicate_rest(const uint32_t* order, const uint32_t* count_rest,
                                 const uint32_t* offsets_rest, const SplatRec* rec,
                                 const ViewDev* views, int64_t VP, int tile_w, int tile_h,
                                 const Status* st, const uint32_t* open_bits,
                                 uint32_t* pair_keys, uint32_t* pair_vals, hipStream_t s) {
  const int64_t blocks = (VP + kDupThreads - 1) / kDupThreads;
  if (blocks == 0) return hipSuccess;
  hipLaunchKernelGGL(duplicate_rest_kernel, dim3((unsigned)blocks), dim3(kDupThreads), 0, s,
                     order, count_rest, offsets_rest, rec, views, VP, tile_w, tile_h, st,
                     open_bits, pair_keys, pair_vals);
  return hipGetLastError();
}

hipError_t launch_ranges(const uint32_t* pair_keys, const uint32_t* d_n, int64_t n_cap,
                         uint32_t* ranges, hipStream_t s) {
  int64_t blocks = (n_cap + 1023) / 1024;
  if (blocks > 65536) blocks = 65536;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(ranges_kernel, dim3((unsigned)blocks), dim3(256), 0, s, pair_keys, d_n,
                     ranges);
  return hipGetLastError();
}

}  // namespace gbb
