// Tile duplication and per-tile ranges.
//
// Records arrive in depth order (a stable sort of the float32 depth key over record
// indices). Each visible record covers a rectangle of tiles; the records of one 256-wide
// block of the depth order own one contiguous run of pair slots (exclusive scan of their
// tile counts), and the block's threads walk that run slot by slot, so consecutive lanes
// write consecutive pairs. A pair is (global tile index, record index); tiles are numbered
// view by view, row-major within a view. A stable sort of the pairs by tile then yields,
// for each tile, its records in (depth, record index) order.
#include "device_util.h"
#include "gbb_internal.h"

namespace gbb {

namespace {

__global__ void finalize_count_kernel(Status* st, int64_t capacity) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    const uint32_t K = st->K;
    const bool over = (int64_t)K > capacity;
    st->overflow = over ? 1u : 0u;
    st->n_sorted = over ? 0u : K;
  }
}

__global__ void __launch_bounds__(256)
duplicate_kernel(const uint32_t* __restrict__ order, const uint32_t* __restrict__ count,
                 const uint32_t* __restrict__ offsets, const SplatRec* __restrict__ rec,
                 const ViewDev* __restrict__ views, int64_t VP, int tile_w, int tile_h,
                 const Status* __restrict__ st, uint32_t* __restrict__ pair_keys,
                 uint32_t* __restrict__ pair_vals) {
  __shared__ uint32_t s_off[256];
  __shared__ uint32_t s_cnt[256];
  __shared__ uint32_t s_rec[256];
  __shared__ int32_t s_tx0[256];
  __shared__ int32_t s_ty0[256];
  __shared__ int32_t s_w[256];
  __shared__ int32_t s_base[256];
  __shared__ int32_t s_tiles_x[256];
  if (st->overflow) return;
  const int64_t first = (int64_t)blockIdx.x * 256;
  if (first >= VP) return;
  const int n = (int)((VP - first) < 256 ? (VP - first) : 256);
  const int t = threadIdx.x;
  if (t < n) {
    const uint32_t r = order[first + t];
    const uint32_t c = count[r];
    s_off[t] = offsets[first + t];
    s_cnt[t] = c;
    s_rec[t] = r;
    if (c > 0) {
      const SplatRec& R = rec[r];
      const int i0 = R.rect_x & 0xffff, i1 = R.rect_x >> 16;
      const int j0 = R.rect_y & 0xffff;
      const ViewDev& V = views[R.view];
      s_tx0[t] = i0 / tile_w;
      s_ty0[t] = j0 / tile_h;
      s_w[t] = i1 / tile_w - i0 / tile_w + 1;
      s_base[t] = V.tile_base;
      s_tiles_x[t] = V.tiles_x;
    } else {
      s_tx0[t] = s_ty0[t] = 0;
      s_w[t] = 1;
      s_base[t] = 0;
      s_tiles_x[t] = 1;
    }
  }
  __syncthreads();
  const uint32_t q0 = s_off[0];
  const uint32_t q1 = s_off[n - 1] + s_cnt[n - 1];
  // one pair per lane, consecutive lanes on consecutive slots (coalesced stores)
  for (uint32_t q = q0 + t; q < q1; q += 256) {
    // last record of the block whose first slot is <= q (it has a non-zero count)
    int lo = 0, hi = n - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (s_off[mid] <= q) lo = mid;
      else hi = mid - 1;
    }
    const int local = (int)(q - s_off[lo]);
    const int w = s_w[lo];
    const int ty = s_ty0[lo] + local / w;
    const int tx = s_tx0[lo] + local - (local / w) * w;
    pair_keys[q] = (uint32_t)(s_base[lo] + ty * s_tiles_x[lo] + tx);
    pair_vals[q] = s_rec[lo];
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
#pragma unroll
    for (int j = 0; j < 5; ++j) k[j + 1] = i0 + j < n ? keys[i0 + j] : 0xFFFFFFFFu;
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
  const int64_t blocks = (VP + 255) / 256;
  if (blocks == 0) return hipSuccess;
  hipLaunchKernelGGL(duplicate_kernel, dim3((unsigned)blocks), dim3(256), 0, s, order, count,
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
