// Device-wide exclusive scan and stable LSD radix sort of (uint32 key, uint32 value) pairs.
//
// Scan: reduce per 4096-element tile -> scan of tile sums in one workgroup -> per-tile scan.
// Radix pass (a digit of at most 8 bits; a key of b bits takes ceil(b/8) passes with the bits
// spread evenly over them), three launches: per-tile digit histogram, which also adds each
// digit's count to the pass's digit totals -> one workgroup per digit turns its row of the
// digit-major [digit][tile] counts into output offsets (the totals of the smaller digits
// give the row's base) -> scatter. The totals are kept in kTotCopies copies (workgroup b adds
// to copy b mod kTotCopies): device-wide atomics on one address are served one at a time,
// about 55 ns each, so 2048 workgroups adding to a single copy took 35 us. The scatter ranks each element stably among equal digits
// of its tile: each wave takes a contiguous quarter of the tile in rounds of 64; lanes with
// the same digit are found with one ballot per digit bit and counted against the wave's
// running per-digit counters in LDS. Wave offsets and digit starts then place every element
// in LDS in digit order, and the tile is written out so that consecutive lanes store
// consecutive addresses of one digit run.
#include "device_util.h"
#include "gbb_internal.h"

namespace gbb {

namespace {

constexpr int kThreads = 256;
constexpr int kItems = kScanTile / kThreads;  // 16

// Inclusive scan of v over the 256 threads of the block; returns the inclusive value and
// writes the block total to *total. `wave_tot` is LDS scratch of 4 entries.
__device__ __forceinline__ uint32_t block_inclusive_scan(uint32_t v, uint32_t* wave_tot,
                                                         uint32_t* total) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    uint32_t t = __shfl_up(v, d, 64);
    if (lane >= d) v += t;
  }
  if (lane == 63) wave_tot[w] = v;
  __syncthreads();
  uint32_t add = 0, tot = 0;
#pragma unroll
  for (int i = 0; i < kThreads / 64; ++i) {
    uint32_t t = wave_tot[i];
    if (i < w) add += t;
    tot += t;
  }
  __syncthreads();
  *total = tot;
  return v + add;
}

template <bool GATHER>
__device__ __forceinline__ uint32_t scan_load(const uint32_t* in, const uint32_t* gather,
                                              int64_t i) {
  if (GATHER) return in[gather[i]];
  return in[i];
}

__device__ __forceinline__ int64_t scan_len(int64_t n, const ScanLen& L) {
  if (!L.d_count) return n;
  const int64_t m = ((int64_t)*L.d_count + L.per - 1) / L.per * L.mult;
  return m < n ? m : n;
}

template <bool GATHER>
__global__ void __launch_bounds__(kThreads)
scan_reduce_kernel(const uint32_t* __restrict__ in, const uint32_t* __restrict__ gather,
                   int64_t n_cap, ScanLen L, uint32_t* __restrict__ partials,
                   unsigned long long* __restrict__ partials64) {
  __shared__ uint32_t wave_tot[4];
  __shared__ unsigned long long wave_tot64[4];
  const int64_t n = scan_len(n_cap, L);
  const int64_t base = (int64_t)blockIdx.x * kScanTile;
  if (base >= n && base > 0) return;
  uint32_t s = 0;
  unsigned long long s64 = 0;
#pragma unroll 4
  for (int k = 0; k < kItems; ++k) {
    int64_t i = base + k * kThreads + threadIdx.x;
    if (i < n) {
      const uint32_t x = scan_load<GATHER>(in, gather, i);
      s += x;
      s64 += x;
    }
  }
  if (partials64) {
    // exact block sum in 64 bits (the partials kernel adds the blocks up)
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) s64 += __shfl_xor(s64, d, 64);
    if ((threadIdx.x & 63) == 0) wave_tot64[threadIdx.x >> 6] = s64;
  }
  uint32_t total;
  block_inclusive_scan(s, wave_tot, &total);  // its barriers also publish wave_tot64
  if (threadIdx.x == 0) {
    partials[blockIdx.x] = total;
    if (partials64)
      partials64[blockIdx.x] = (wave_tot64[0] + wave_tot64[1]) + (wave_tot64[2] + wave_tot64[3]);
  }
}

// One workgroup: exclusive scan of partials[0..nb) in place, total to partials[nb] and *total.
__global__ void __launch_bounds__(1024)
scan_partials_kernel(uint32_t* __restrict__ partials, int64_t n_cap, ScanLen L,
                     uint32_t* __restrict__ total,
                     const unsigned long long* __restrict__ partials64,
                     unsigned long long* __restrict__ total64) {
  __shared__ uint32_t wave_tot[16];
  __shared__ uint32_t carry_s;
  __shared__ unsigned long long wave_sum64[16];
  const int64_t n = scan_len(n_cap, L);
  const int64_t nb = n > 0 ? (n + kScanTile - 1) / kScanTile : 1;
  if (total64) {
    unsigned long long s64 = 0;
    for (int64_t i = threadIdx.x; i < nb; i += 1024) s64 += partials64[i];
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) s64 += __shfl_xor(s64, d, 64);
    if ((threadIdx.x & 63) == 0) wave_sum64[threadIdx.x >> 6] = s64;
    __syncthreads();
    if (threadIdx.x == 0) {
      unsigned long long t = 0;
      for (int k = 0; k < 16; ++k) t += wave_sum64[k];
      *total64 = t;
    }
  }
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (threadIdx.x == 0) carry_s = 0;
  __syncthreads();
  for (int64_t start = 0; start < nb; start += 1024) {
    int64_t i = start + threadIdx.x;
    uint32_t x = i < nb ? partials[i] : 0u;
    uint32_t v = x;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      uint32_t t = __shfl_up(v, d, 64);
      if (lane >= d) v += t;
    }
    if (lane == 63) wave_tot[w] = v;
    __syncthreads();
    uint32_t add = 0, tot = 0;
    for (int k = 0; k < 16; ++k) {
      uint32_t t = wave_tot[k];
      if (k < w) add += t;
      tot += t;
    }
    const uint32_t carry = carry_s;
    if (i < nb) partials[i] = carry + add + v - x;
    __syncthreads();
    if (threadIdx.x == 0) carry_s = carry + tot;
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    partials[nb] = carry_s;
    if (total) *total = carry_s;
  }
}

// LDS index with one pad word per 32 so that both the striped and the blocked access
// patterns below are free of bank conflicts.
__device__ __forceinline__ int pad_idx(int i) { return i + (i >> 5); }

// With chunk_owner, element i with value x > 0 and exclusive prefix o also records itself as
// the owner of every chunk of kChunkSlots slots that starts inside [o, o + x) (chunk indices
// below n_chunks).
template <bool GATHER>
__global__ void __launch_bounds__(kThreads)
scan_down_kernel(const uint32_t* __restrict__ in, const uint32_t* __restrict__ gather,
                 int64_t n_cap, ScanLen L, const uint32_t* __restrict__ partials,
                 uint32_t* __restrict__ out, uint32_t* __restrict__ chunk_owner,
                 int64_t n_chunks) {
  __shared__ uint32_t tile[kScanTile + kScanTile / 32];
  __shared__ uint32_t wave_tot[4];
  const int64_t n = scan_len(n_cap, L);
  const int64_t base = (int64_t)blockIdx.x * kScanTile;
  if (base >= n) return;
  // coalesced load into LDS, then each thread owns 16 consecutive elements
#pragma unroll 4
  for (int k = 0; k < kItems; ++k) {
    int64_t i = base + k * kThreads + threadIdx.x;
    tile[pad_idx(k * kThreads + threadIdx.x)] = i < n ? scan_load<GATHER>(in, gather, i) : 0u;
  }
  __syncthreads();
  uint32_t loc[kItems];
  uint32_t s = 0;
#pragma unroll
  for (int k = 0; k < kItems; ++k) loc[k] = tile[pad_idx(threadIdx.x * kItems + k)];
#pragma unroll
  for (int k = 0; k < kItems; ++k) s += loc[k];
  uint32_t total;
  uint32_t incl = block_inclusive_scan(s, wave_tot, &total);
  uint32_t run = partials[blockIdx.x] + incl - s;
#pragma unroll
  for (int k = 0; k < kItems; ++k) {
    uint32_t x = loc[k];
    loc[k] = run;
    if (chunk_owner && x > 0) {
      const int64_t i = base + threadIdx.x * kItems + k;
      const uint64_t o = run, e = (uint64_t)run + x;
      for (uint64_t c = (o + kChunkSlots - 1) / kChunkSlots;
           c * kChunkSlots < e && (int64_t)c < n_chunks; ++c)
        chunk_owner[c] = (uint32_t)i;
    }
    run += x;
  }
#pragma unroll
  for (int k = 0; k < kItems; ++k) tile[pad_idx(threadIdx.x * kItems + k)] = loc[k];
  __syncthreads();
#pragma unroll 4
  for (int k = 0; k < kItems; ++k) {
    int64_t i = base + k * kThreads + threadIdx.x;
    if (i < n) out[i] = tile[pad_idx(k * kThreads + threadIdx.x)];
  }
}

// ---- radix sort --------------------------------------------------------------------------
// A pass works on tiles of kRadixTile elements; the tile count follows the device-side
// element count, and workgroups take tiles in turn (at most kRadixGrid workgroups), so a
// short sort in a large buffer costs what its elements cost. Digit counts are stored
// digit-major, one column per tile.
constexpr int kRadixGrid = 2048;

__device__ __forceinline__ int64_t sort_count(const uint32_t* d_n, int64_t n_cap) {
  if (!d_n) return n_cap;
  int64_t n = (int64_t)(*d_n);
  return n < n_cap ? n : n_cap;
}

// Digit counts of one tile. Each wave counts into its own LDS histogram with plain LDS
// atomics (lanes that hit one bin are served one after another by the LDS, which is cheaper
// than grouping equal digits with ballots); each lane loads four consecutive keys at a time.
template <int NBITS>
__global__ void __launch_bounds__(kRadixThreads)
radix_hist_kernel(const uint32_t* __restrict__ keys, const uint32_t* __restrict__ d_n,
                  int64_t n_cap, int shift, uint32_t* __restrict__ hist,
                  uint32_t* __restrict__ digit_tot) {
  constexpr int kBins = 1 << NBITS;
  constexpr uint32_t kMask = (uint32_t)kBins - 1u;
  constexpr int kWaves = kRadixThreads / 64;
  __shared__ uint32_t h[kWaves][kBins];
  const int64_t n = sort_count(d_n, n_cap);
  const int64_t nb = (n + kRadixTile - 1) / kRadixTile;
  const int w = threadIdx.x >> 6;
  static_assert(kBins <= kRadixThreads, "one digit per thread");
  uint32_t acc = 0;  // this thread's digit, summed over the workgroup's tiles
  for (int64_t tile = blockIdx.x; tile < nb; tile += gridDim.x) {
    for (int i = threadIdx.x; i < kWaves * kBins; i += kRadixThreads) (&h[0][0])[i] = 0;
    __syncthreads();
    const int64_t base = tile * kRadixTile;
    {
      const int nvalid = (int)((n - base) < kRadixTile ? (n - base) : kRadixTile);
      const uint32_t* kt = keys + base;
      uint4 q[kRadixItems / 4];
#pragma unroll
      for (int k = 0; k < kRadixItems / 4; ++k) {
        const int i = 4 * (k * kRadixThreads + threadIdx.x);
        if (i + 3 < nvalid) {
          q[k] = *reinterpret_cast<const uint4*>(kt + i);
        } else {
          q[k].x = i < nvalid ? kt[i] : 0u;
          q[k].y = i + 1 < nvalid ? kt[i + 1] : 0u;
          q[k].z = i + 2 < nvalid ? kt[i + 2] : 0u;
          q[k].w = 0u;
        }
      }
#pragma unroll
      for (int k = 0; k < kRadixItems / 4; ++k) {
        const int i = 4 * (k * kRadixThreads + threadIdx.x);
        if (i < nvalid) atomicAdd(&h[w][(q[k].x >> shift) & kMask], 1u);
        if (i + 1 < nvalid) atomicAdd(&h[w][(q[k].y >> shift) & kMask], 1u);
        if (i + 2 < nvalid) atomicAdd(&h[w][(q[k].z >> shift) & kMask], 1u);
        if (i + 3 < nvalid) atomicAdd(&h[w][(q[k].w >> shift) & kMask], 1u);
      }
    }
    __syncthreads();
    const int d = threadIdx.x;
    if (d < kBins) {
      uint32_t c = 0;
#pragma unroll
      for (int ww = 0; ww < kWaves; ++ww) c += h[ww][d];
      hist[(int64_t)d * nb + tile] = c;
      acc += c;
    }
    __syncthreads();  // the next tile reuses the LDS histograms
  }
  if (threadIdx.x < kBins && acc != 0)
    atomicAdd(&digit_tot[(blockIdx.x % kTotCopies) * 256 + threadIdx.x], acc);
}

// Output offsets of one digit (the workgroup's): its row of the [digit][tile] counts becomes
// the exclusive prefix over tiles plus the number of elements with a smaller digit. Each
// thread takes kItems consecutive entries of a chunk.
template <int NBITS>
__global__ void __launch_bounds__(kThreads)
radix_offsets_kernel(const uint32_t* __restrict__ d_n, int64_t n_cap,
                     const uint32_t* __restrict__ digit_tot, uint32_t* __restrict__ hist) {
  static_assert((1 << NBITS) <= kThreads, "one smaller digit per thread");
  __shared__ uint32_t wave_tot[kThreads / 64];
  const int64_t n = sort_count(d_n, n_cap);
  const int64_t nb = (n + kRadixTile - 1) / kRadixTile;
  const int d = blockIdx.x, tid = threadIdx.x;
  uint32_t smaller = 0;  // elements whose digit is tid (< d)
  if (tid < d) {
#pragma unroll 16
    for (int c = 0; c < kTotCopies; ++c) smaller += digit_tot[c * 256 + tid];
  }
  uint32_t base;
  block_inclusive_scan(smaller, wave_tot, &base);
  uint32_t* __restrict__ row = hist + (int64_t)d * nb;
  for (int64_t c0 = 0; c0 < nb; c0 += (int64_t)kThreads * kItems) {
    const int64_t i0 = c0 + (int64_t)tid * kItems;
    uint32_t v[kItems], sum = 0;
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
      v[k] = i0 + k < nb ? row[i0 + k] : 0u;
      sum += v[k];
    }
    uint32_t tot;
    uint32_t run = base + block_inclusive_scan(sum, wave_tot, &tot) - sum;
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
      if (i0 + k < nb) row[i0 + k] = run;
      run += v[k];
    }
    base += tot;
  }
}

template <int NBITS>
__global__ void __launch_bounds__(kRadixThreads)
radix_scatter_kernel(const uint32_t* __restrict__ keys_in, const uint32_t* __restrict__ vals_in,
                     uint32_t* __restrict__ keys_out, uint32_t* __restrict__ vals_out,
                     const uint32_t* __restrict__ d_n, int64_t n_cap, int shift,
                     const uint32_t* __restrict__ hist_scanned, uint32_t* __restrict__ digit_tot) {
  constexpr int kBins = 1 << NBITS;
  constexpr uint32_t kMask = (uint32_t)kBins - 1u;
  constexpr int kWaves = kRadixThreads / 64;
  constexpr int kPerWave = kRadixTile / kWaves;  // contiguous elements ranked by one wave
  __shared__ uint32_t s_keys[kRadixTile];
  __shared__ uint32_t s_vals[kRadixTile];
  __shared__ uint32_t s_cnt[kWaves][256];  // running per-wave digit counts, then wave offsets
  __shared__ uint32_t s_start[256];
  __shared__ uint32_t s_gofs[kBins];  // output index of the tile's element 0 of each digit
  __shared__ uint32_t wave_tot[4];
  const int64_t n = sort_count(d_n, n_cap);
  const int64_t nb = (n + kRadixTile - 1) / kRadixTile;
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
  // the offsets launch has read this pass's digit totals: leave them zero for the next sort
  for (int c = blockIdx.x; c < kTotCopies; c += gridDim.x) digit_tot[c * 256 + tid] = 0u;
  for (int64_t tile = blockIdx.x; tile < nb; tile += gridDim.x) {
    const int64_t base = tile * kRadixTile;
    const int nvalid = (int)((n - base) < kRadixTile ? (n - base) : kRadixTile);
    // where each digit of this tile starts in the output (loaded early, used at the end)
    const uint32_t gstart = tid < kBins ? hist_scanned[(int64_t)tid * nb + tile] : 0u;
#pragma unroll
    for (int k = 0; k < 4; ++k) s_cnt[w][lane + 64 * k] = 0;
    __builtin_amdgcn_wave_barrier();
    // Each wave ranks its own contiguous quarter of the tile in rounds of 64 elements; program
    // order inside the wave keeps equal digits in index order.
    uint32_t key_r[kRadixItems], val_r[kRadixItems], rank_r[kRadixItems];
    // all loads first (memory-level parallelism)
#pragma unroll
    for (int r = 0; r < kRadixItems; ++r) {
      const int i = w * kPerWave + r * 64 + lane;
      const bool valid = i < nvalid;
      key_r[r] = valid ? keys_in[base + i] : 0u;
      val_r[r] = valid ? vals_in[base + i] : 0u;
    }
#pragma unroll
    for (int r = 0; r < kRadixItems; ++r) {
      const int i = w * kPerWave + r * 64 + lane;
      const bool valid = i < nvalid;
      const uint32_t d = (key_r[r] >> shift) & kMask;
      // lanes holding the same digit: one ballot per digit bit
      uint64_t m = ballot(valid);
#pragma unroll
      for (int bit = 0; bit < NBITS; ++bit) {
        const bool set = (d >> bit) & 1u;
        const uint64_t b = ballot(set);
        m &= set ? b : ~b;
      }
      const uint32_t below = mbcnt(m);
      const uint32_t cnt = s_cnt[w][d];
      __builtin_amdgcn_wave_barrier();
      if (valid && below == 0) s_cnt[w][d] = cnt + popc64(m);
      __builtin_amdgcn_wave_barrier();
      rank_r[r] = cnt + below;
    }
    __syncthreads();
    // digit totals of the tile, offsets of each wave inside a digit, digit starts
    uint32_t tot = 0;
#pragma unroll
    for (int ww = 0; ww < kWaves; ++ww) {
      const uint32_t c = s_cnt[ww][tid];
      s_cnt[ww][tid] = tot;
      tot += c;
    }
    uint32_t total;
    const uint32_t incl = block_inclusive_scan(tot, wave_tot, &total);
    s_start[tid] = incl - tot;
    // element counts fit in 32 bits, so output indices do too
    if (tid < kBins) s_gofs[tid] = gstart - (incl - tot);
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kRadixItems; ++r) {
      const int i = w * kPerWave + r * 64 + lane;
      if (i < nvalid) {
        const uint32_t d = (key_r[r] >> shift) & kMask;
        const uint32_t pos = s_start[d] + s_cnt[w][d] + rank_r[r];
        s_keys[pos] = key_r[r];
        s_vals[pos] = val_r[r];
      }
    }
    __syncthreads();
    for (int i = tid; i < nvalid; i += kRadixThreads) {
      const uint32_t key = s_keys[i];
      const uint32_t gpos = s_gofs[(key >> shift) & kMask] + (uint32_t)i;
      keys_out[gpos] = key;
      vals_out[gpos] = s_vals[i];
    }
    __syncthreads();  // the next tile reuses the LDS
  }
}

__global__ void copy_pairs_kernel(const uint32_t* __restrict__ ka, const uint32_t* __restrict__ va,
                                  uint32_t* __restrict__ kb, uint32_t* __restrict__ vb,
                                  const uint32_t* __restrict__ d_n, int64_t n_cap) {
  const int64_t n = sort_count(d_n, n_cap);
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    kb[i] = ka[i];
    vb[i] = va[i];
  }
}

__global__ void fill_u32_kernel(uint32_t* __restrict__ p, uint32_t value, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = value;
}

// The same fill for a 16-byte aligned array: 16-byte stores for the n / 4 full quads, then the
// n % 4 trailing words.
__global__ void fill_u32x4_kernel(uint32_t* __restrict__ p, uint32_t value, int64_t n) {
  const int64_t n4 = n >> 2;
  const uint4 v = make_uint4(value, value, value, value);
  uint4* __restrict__ q = reinterpret_cast<uint4*>(p);
  const int64_t first = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (int64_t i = first; i < n4; i += (int64_t)gridDim.x * blockDim.x) q[i] = v;
  if (first < (n & 3)) p[4 * n4 + first] = value;
}

unsigned grid_for(int64_t n, int threads) {
  int64_t b = (n + threads - 1) / threads;
  if (b > 65536) b = 65536;
  if (b < 1) b = 1;
  return (unsigned)b;
}

}  // namespace

hipError_t launch_fill_u32(uint32_t* p, uint32_t value, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  if ((reinterpret_cast<uintptr_t>(p) & 15) == 0 && n >= 64) {
    hipLaunchKernelGGL(fill_u32x4_kernel, dim3(grid_for((n + 3) / 4, 256)), dim3(256), 0, s, p,
                       value, n);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(fill_u32_kernel, dim3(grid_for(n, 256)), dim3(256), 0, s, p, value, n);
  return hipGetLastError();
}

hipError_t launch_scan_u32(const uint32_t* in, const uint32_t* gather, uint32_t* out, int64_t n,
                           uint32_t* partials, uint32_t* total, unsigned long long* total64,
                           unsigned long long* partials64, hipStream_t s,
                           uint32_t* chunk_owner, int64_t n_chunks, ScanLen len) {
  const int64_t nb = (n + kScanTile - 1) / kScanTile;
  if (nb == 0) return hipSuccess;
  if (!total64) partials64 = nullptr;
  if (total64 && !partials64) return hipErrorInvalidValue;
  if (gather)
    hipLaunchKernelGGL(scan_reduce_kernel<true>, dim3((unsigned)nb), dim3(kThreads), 0, s, in,
                       gather, n, len, partials, partials64);
  else
    hipLaunchKernelGGL(scan_reduce_kernel<false>, dim3((unsigned)nb), dim3(kThreads), 0, s, in,
                       gather, n, len, partials, partials64);
  hipLaunchKernelGGL(scan_partials_kernel, dim3(1), dim3(1024), 0, s, partials, n, len, total,
                     partials64, total64);
  if (gather)
    hipLaunchKernelGGL(scan_down_kernel<true>, dim3((unsigned)nb), dim3(kThreads), 0, s, in,
                       gather, n, len, partials, out, chunk_owner, n_chunks);
  else
    hipLaunchKernelGGL(scan_down_kernel<false>, dim3((unsigned)nb), dim3(kThreads), 0, s, in,
                       gather, n, len, partials, out, chunk_owner, n_chunks);
  return hipGetLastError();
}

template <int NBITS>
hipError_t radix_pass(const uint32_t* ki, const uint32_t* vi, uint32_t* ko, uint32_t* vo,
                      const uint32_t* d_n, int64_t n_cap, int shift, int64_t nb, uint32_t* hist,
                      uint32_t* digit_tot, hipStream_t s) {
  const unsigned grid = (unsigned)(nb < kRadixGrid ? nb : kRadixGrid);
  hipLaunchKernelGGL(radix_hist_kernel<NBITS>, dim3(grid), dim3(kRadixThreads), 0, s, ki, d_n,
                     n_cap, shift, hist, digit_tot);
  hipLaunchKernelGGL(radix_offsets_kernel<NBITS>, dim3(1u << NBITS), dim3(kThreads), 0, s, d_n,
                     n_cap, digit_tot, hist);
  hipLaunchKernelGGL(radix_scatter_kernel<NBITS>, dim3(grid), dim3(kRadixThreads), 0, s, ki, vi,
                     ko, vo, d_n, n_cap, shift, hist, digit_tot);
  return hipGetLastError();
}

hipError_t launch_radix_sort(uint32_t* keys, uint32_t* vals, uint32_t* keys_alt,
                             uint32_t* vals_alt, const uint32_t* d_n, int64_t n_cap, int bits,
                             uint32_t* hist, uint32_t* digit_tot, hipStream_t s) {
  const int64_t nb = (n_cap + kRadixTile - 1) / kRadixTile;
  if (nb == 0 || bits <= 0) return hipSuccess;
  if (bits > 32) return hipErrorInvalidValue;
  // the fewest 8-bit-or-narrower passes, with the key bits spread evenly over them
  const int passes = (bits + 7) / 8;
  hipError_t e = hipSuccess;
  uint32_t *ki = keys, *vi = vals, *ko = keys_alt, *vo = vals_alt;
  int shift = 0;
  for (int p = 0; p < passes; ++p) {
    const int nbits = bits / passes + (p < bits % passes ? 1 : 0);
    uint32_t* const tot = digit_tot + (int64_t)kTotCopies * 256 * p;
    switch (nbits) {
      case 1: e = radix_pass<1>(ki, vi, ko, vo, d_n, n_cap, shift, nb, hist, tot, s); break;
      case 2: e = radix_pass<2>(ki, vi, ko, vo, d_n, n_cap, shift, nb, hist, tot, s); break;
      case 3: e = radix_pass<3>(ki, vi, ko, vo, d_n, n_cap, shift, nb, hist, tot, s); break;
      case 4: e = radix_pass<4>(ki, vi, ko, vo, d_n, n_cap, shift, nb, hist, tot, s); break;
      case 5: e = radix_pass<5>(ki, vi, ko, vo, d_n, n_cap, shift, nb, hist, tot, s); break;
      case 6: e = radix_pass<6>(ki, vi, ko, vo, d_n, n_cap, shift, nb, hist, tot, s); break;
      case 7: e = radix_pass<7>(ki, vi, ko, vo, d_n, n_cap, shift, nb, hist, tot, s); break;
      default: e = radix_pass<8>(ki, vi, ko, vo, d_n, n_cap, shift, nb, hist, tot, s); break;
    }
    if (e != hipSuccess) return e;
    shift += nbits;
    uint32_t* t = ki;
    ki = ko;
    ko = t;
    t = vi;
    vi = vo;
    vo = t;
  }
  if (ki != keys) {
    hipLaunchKernelGGL(copy_pairs_kernel, dim3(grid_for(n_cap, 256)), dim3(256), 0, s, ki, vi,
                       keys, vals, d_n, n_cap);
  }
  return hipGetLastError();
}

}  // namespace gbb
