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

// One block per 256 records of the depth order. The records own the contiguous slot run
// [q0, q1) (exclusive scan of their counts); it is expanded in rounds of kDupChunk slots. In a
// round, every record whose first slot falls in the round marks that slot with its local index,
// and a block-wide max-scan of the marks gives each slot its owner (the last record starting at
// or before it). Thread t writes slots 4t..4t+3 of the round. The tile inside the owner's
// rectangle is local / w and local mod w, with the division done exactly as a multiply by
// ceil(2^40 / w): for w <= 4096 and local < 2^24 the product's error stays below 1/w.
__global__ void __launch_bounds__(kDupThreads)
duplicate_kernel(const uint32_t* __restrict__ order, const uint32_t* __restrict__ count,
                 const uint32_t* __restrict__ offsets, const SplatRec* __restrict__ rec,
                 const ViewDev* __restrict__ views, int64_t VP, int tile_w, int tile_h,
                 const Status* __restrict__ st, uint32_t* __restrict__ pair_keys,
                 uint32_t* __restrict__ pair_vals) {
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
  const int64_t first = (int64_t)blockIdx.x * kDupThreads;
  if (first >= VP) return;
  const int n = (int)((VP - first) < kDupThreads ? (VP - first) : kDupThreads);
  const int t = threadIdx.x, w = t >> 6, lane = t & 63;
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
  // slot indices stay below the capacity (< 2^32); rounds are counted in 64 bits so that the
  // last one cannot wrap
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
        const uint32_t local = (uint32_t)(q - (int64_t)s_off[own]);
        const uint32_t wt = s_w[own];
        const uint32_t ty = (uint32_t)(((uint64_t)local * s_magic[own]) >> 40);
        const uint32_t tx = local - ty * wt;
        key[k] = s_tile0[own] + ty * s_tiles_x[own] + tx;
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

__global__ void ranges_kernel(const uint32_t* __restrict__ keys, const Status* __restrict__ st,
                              uint32_t* __restrict__ ranges) {
  // four consecutive keys per thread; a tile starts where its key differs from the previous
  // one and ends where it differs from the next
  const int64_t n = st->n_sorted;
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

hipError_t launch_duplicate(const uint32_t* order, const uint32_t* count,
                            const uint32_t* offsets, const SplatRec* rec, const ViewDev* views,
                            int64_t VP, int tile_w, int tile_h, const Status* st,
                            uint32_t* pair_keys, uint32_t* pair_vals, hipStream_t s) {
  const int64_t blocks = (VP + kDupThreads - 1) / kDupThreads;
  if (blocks == 0) return hipSuccess;
  hipLaunchKernelGGL(duplicate_kernel, dim3((unsigned)blocks), dim3(kDupThreads), 0, s, order, count,
                     offsets, rec, views, VP, tile_w, tile_h, st, pair_keys, pair_vals);
  return hipGetLastError();
}

hipError_t launch_ranges(const uint32_t* pair_keys, const Status* st, int64_t n_cap,
                         uint32_t* ranges, hipStream_t s) {
  int64_t blocks = (n_cap + 1023) / 1024;
  if (blocks > 65536) blocks = 65536;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(ranges_kernel, dim3((unsigned)blocks), dim3(256), 0, s, pair_keys, st,
                     ranges);
  return hipGetLastError();
}

}  // namespace gbb
