// Internal declarations shared by the HIP translation units of libgbb.
// Each .hip file defines its kernels together with plain host launchers declared here, so
// the library links without relocatable device code.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/gbb.h"

namespace gbb {

constexpr int kWave = 64;
constexpr uint32_t kCulledKey = 0xFFFFFFFFu;
constexpr int kRecGrad = 10;  // dh00 dh01 dh10 dh11 dh20 dh21 dh22 dc2x dc2y dopacity

// Device copy of one view, with its place in the global tile and pixel numbering.
struct ViewDev {
  float R[9];
  float t[3];
  float fx, fy, cx, cy, z_near;
  int32_t W, H, tiles_x, tiles_y;
  int32_t tile_base;   // first global tile index of this view
  int32_t pix_base;    // first packed pixel index of this view
  int32_t sat_base;    // first entry of this view's (tiles_y + 1) x (tiles_x + 1) open-tile table
};
static_assert(sizeof(ViewDev) == 96, "ViewDev layout");

// Per (view, splat) record read by the blend kernels (96 bytes).
//
// The ray-splat solve is kept as a homography from the pixel offset (dx, dy) to the
// projected centre onto homogeneous uv: (rho0, rho1, rho2) = H (dx, dy, 1) with
// rho0 = h00 dx + h01 dy, rho1 = h10 dx + h11 dy, rho2 = h20 dx + h21 dy + h22,
// u = rho0 / rho2, v = rho1 / rho2. The entries and the projected centre are unevaluated
// float pairs (hi + lo): the blend re-centres the solve on each wave's 8 x 8 pixel block in
// pair precision, so that float32 per-pixel arithmetic only spans offsets within one block.
struct SplatRec {
  float h_hi[7];
  float h_lo[7];
  float c2x_hi, c2x_lo, c2y_hi, c2y_lo;
  float opacity;
  int32_t rect_x;    // i0 | i1 << 16 (pixel columns, inclusive)
  int32_t rect_y;    // j0 | j1 << 16 (pixel rows, inclusive)
  int32_t splat;     // splat index k
  int32_t view;      // view index v
  int32_t pad;
};
static_assert(sizeof(SplatRec) == 96, "SplatRec layout");

struct Status {
  uint32_t K;          // pair total of the 32-bit offset scan (equals K64 when no overflow)
  uint32_t n_sorted;   // pairs emitted and sorted by the first (or only) pass (0 on overflow)
  uint32_t overflow;   // 1 if K64 exceeded the capacity
  uint32_t cut;        // records (in depth order) rendered by the depth-prefix pass
  unsigned long long K64;  // exact total of pairs requested by the key stage
  uint32_t n_rest;     // pairs emitted and sorted by the second pass (open tiles only)
  uint32_t K_rest;     // 32-bit scan total of the second pass
  unsigned long long K_rest64;  // exact total of the second pass
  uint32_t last_first; // depth rank of the record owning the first pass's last pair slot
  uint32_t last_rest;  // the same for the second pass
  uint32_t any_open;   // nonzero if the prefix pass left some tile open
  uint32_t sticky_overflow;  // ORed by every forward's overflow flag; cleared by gb_read_status
  uint32_t n_views;    // views and splats of the last forward, and the byte offsets of its
  uint32_t P;          // per-record tile counts and per-view pair totals in the workspace
  unsigned long long off_count;
  unsigned long long off_view_pairs;
};
static_assert(sizeof(Status) <= 256, "status section");

// Depth-prefix split. The first pass renders the records of a prefix of the depth order
// (as many as fit a pair budget); tiles where some pixel is still open afterwards get a
// second pass over the remaining records, which resumes from the saved per-pixel state. The
// backward walks, on each such tile, the second pass's pairs and then the first's, with the
// per-pixel state kept in registers.
enum BlendMode : int32_t { kSinglePass = 0, kPrefixPass = 1, kRestPass = 2 };

struct SplitState {
  int32_t mode;
  uint32_t* open_bits;  // one bit per global tile: set if the prefix left a pixel open
  float4* fwd_state;    // per pixel after the prefix: accumulated colour, done flag (0 / 1)
  uint32_t* any_open;   // Status::any_open (prefix pass)
};

// The sorted pairs of one pass as the backward reads them.
struct PairList {
  const uint32_t* pair_vals;  // record of each pair, sorted by tile
  const uint32_t* ranges;     // [tile][2]: [start, end) of the tile's pairs
  const uint32_t* n_last;     // per pixel: one past the last pair it blended
};

// Host-side plan of one call: sizes and workspace carve-up.
struct Plan {
  int32_t P, N, V;
  int64_t VP;
  int64_t capacity;
  int64_t total_tiles;
  int64_t total_pixels;
  int32_t tile_w, tile_h, batch_fwd, batch_bwd;
  int32_t tile_bits;
  bool split;            // depth-prefix split enabled
  bool ordered;          // blend workgroups take tiles in work order (else fixed XCD bands)
  int64_t prefix_cap;    // pair slots of the prefix pass (0 without the split)
  int64_t nb_vp;      // radix blocks over V*P records
  int64_t nb_pairs;   // radix blocks over the pair capacity
  // byte offsets
  size_t off_status, off_views, off_depth_key, off_depth_key_alt, off_order, off_order_alt,
      off_count, off_offsets, off_rec, off_partials, off_hist, off_digit_tot, off_pair_keys, off_pair_vals,
      off_pair_keys_alt, off_pair_vals_alt, off_ranges, off_n_last, off_drec, off_stats,
      off_partials64, off_view_pairs, off_spec, off_dspec,
      off_ranges_rest, off_n_last_rest, off_fwd_state, off_open_bits,
      off_count_rest, off_offsets_rest, off_chunk_owner, off_sat, off_tile_order,
      off_tile_work, total;
  int64_t n_chunks;  // entries of the chunk-owner table
  int64_t sat_len;   // entries of the open-tile summed-area tables of all views
  int64_t partials_len, hist_len;
};

constexpr int kRadixItems = 16;
constexpr int kRadixThreads = 256;
constexpr int kRadixTile = kRadixItems * kRadixThreads;  // 4096 elements per block
constexpr int kScanTile = 4096;
// copies of a radix pass's 256 digit totals, and the words of the four passes' totals
constexpr int kTotCopies = 64;
constexpr int64_t kDigitTotWords = 4 * kTotCopies * 256;

// Key-stage radius (px) of the screen-space low-pass disk: 2.36 for variances up to 1/2, else
// 3.34 sqrt(var) (>= sqrt(2 var ln 255)), computed in double and rounded once to float32.
float lowpass_radius(float lowpass_var);

// ---- launchers (all stream-ordered, no synchronisation) --------------------------------
hipError_t launch_upload_views(const gb_view* views, int n_views, int tile_w, int tile_h,
                               ViewDev* d_views, hipStream_t s);
// With sp.sh != null it also writes spec[v P + k] = (view-dependent colour of splat k seen
// from view v, 0) for every visible record. With order != null it also writes order[r] = r
// for every record r and zero[i] = 0 for i < n_zero.
hipError_t launch_preprocess(const gb_splats& sp, const ViewDev* d_views, int n_views,
                             const gb_options& o, int tile_w, int tile_h, uint32_t* depth_key,
                             uint32_t* sort_key, uint32_t* count, SplatRec* rec, float4* spec,
                             uint32_t* order, uint32_t* zero, int64_t n_zero, hipStream_t s);
hipError_t launch_fill_u32(uint32_t* p, uint32_t value, int64_t n, hipStream_t s);
// Pair slots per chunk of the duplicate kernels (one workgroup round).
constexpr int kChunkSlots = 1024;

// Optional device-side length of a scan: ceil(*d_count / per) * mult elements (never more
// than the host-side n, which sizes the launch).
struct ScanLen {
  const uint32_t* d_count = nullptr;
  int64_t per = 1, mult = 1;
};

// Exclusive scan of n u32 values (optionally gathered in[gather[i]]) in 32-bit arithmetic;
// writes out and, if total != nullptr, the sum to *total. If total64 != nullptr the exact
// 64-bit sum is written to *total64 (partials64 then holds per-block sums). With chunk_owner,
// the index of the element whose run [prefix, prefix + value) holds slot c * kChunkSlots is
// written to chunk_owner[c] for c < n_chunks. partials and partials64 need
// ceil(n / kScanTile) + 1 entries.
hipError_t launch_scan_u32(const uint32_t* in, const uint32_t* gather, uint32_t* out, int64_t n,
                           uint32_t* partials, uint32_t* total, unsigned long long* total64,
                           unsigned long long* partials64, hipStream_t s,
                           uint32_t* chunk_owner = nullptr, int64_t n_chunks = 0,
                           ScanLen len = ScanLen());
// Stable LSD radix sort of (key, value) pairs on bits [0, bits). The element count is
// read from *d_n on the device (at most n_cap); the work of every kernel follows that count,
// the launch sizes follow n_cap. Buffers ping-pong; the result is written back to keys/vals.
// hist needs 256 * ceil(n_cap / kRadixTile) entries. digit_tot (kDigitTotWords entries) must
// be zero on entry and is zero again on return.
hipError_t launch_radix_sort(uint32_t* keys, uint32_t* vals, uint32_t* keys_alt,
                             uint32_t* vals_alt, const uint32_t* d_n, int64_t n_cap, int bits,
                             uint32_t* hist, uint32_t* digit_tot, hipStream_t s);
// Overflow decision of a forward: st->overflow from the exact pair count against the capacity,
// ORed into st->sticky_overflow; records the plan echo (views, splats, section offsets) for
// gb_read_status. With mirror != null (host-mapped memory) it also stores
// (overflow << 63) | K64 there, so that the host sees an overflow without synchronising;
// with overflow_flag != null (device memory) it sets *overflow_flag = 1 on overflow.
struct StatusEcho {
  uint32_t n_views, P;
  unsigned long long off_count, off_view_pairs;
};
// With budget > 0 (the depth-prefix split) it also takes the prefix cut: the largest record
// count (in depth order) whose pairs fit the budget, in st->cut, with st->n_sorted the
// prefix's pairs (both zero on overflow); otherwise st->cut = VP and st->n_sorted = K.
// chunk_owner: the table written by the scan that produced `offsets` (searches start there).
hipError_t launch_finalize_count(const uint32_t* offsets, int64_t VP, Status* st,
                                 int64_t capacity, StatusEcho echo,
                                 unsigned long long* mirror, uint32_t* overflow_flag,
                                 int64_t budget, const uint32_t* chunk_owner, hipStream_t s);
// Per-view pair totals: out[v] = sum of count[v P .. (v + 1) P) (one workgroup per view).
hipError_t launch_view_pairs(const uint32_t* count, int64_t P, int n_views,
                             unsigned long long* out, hipStream_t s);
// Pairs of the first pass: the st->n_sorted slots of the depth order's offsets, expanded in
// chunks of kChunkSlots (chunk_owner from the offset scan); cap bounds the slot count.
// Up to two u32 arrays that a duplicate launch also zeroes (p[k] may be null when n[k] = 0).
struct ClearList {
  uint32_t* p[2] = {nullptr, nullptr};
  int64_t n[2] = {0, 0};
};
hipError_t launch_duplicate(const uint32_t* order, const uint32_t* count,
                            const uint32_t* offsets, const uint32_t* chunk_owner,
                            const SplatRec* rec, const ViewDev* views, int tile_w, int tile_h,
                            const Status* st, int64_t cap, uint32_t* pair_keys,
                            uint32_t* pair_vals, ClearList clear, hipStream_t s);
// Second pass: count_rest[r] = open tiles covered by the record at depth rank r >= st->cut.
hipError_t launch_count_rest(const uint32_t* order, const uint32_t* count, const SplatRec* rec,
                             const ViewDev* views, int64_t VP, int tile_w, int tile_h,
                             const Status* st, const uint32_t* sat, uint32_t* count_rest,
                             hipStream_t s);
hipError_t launch_finalize_rest(const uint32_t* offsets_rest, int64_t VP, Status* st,
                                const uint32_t* chunk_owner, hipStream_t s);
// Summed-area tables of the open-tile bitmap, one per view: sat[y][x] = open tiles in rows
// below y and columns below x (row stride tiles_x + 1). Left unwritten when st reports an
// overflow or no open tile.
hipError_t launch_open_sat(const ViewDev* views, int n_views, const uint32_t* open_bits,
                           const Status* st, uint32_t* sat, hipStream_t s);
// Second pass pairs: (open tile, record) for every record at rank >= st->cut, in depth order.
hipError_t launch_duplicate_rest(const uint32_t* order, const uint32_t* count_rest,
                                 const uint32_t* offsets_rest, const uint32_t* chunk_owner,
                                 const SplatRec* rec, const ViewDev* views, int tile_w,
                                 int tile_h, const Status* st, const uint32_t* open_bits,
                                 const uint32_t* sat, int64_t cap, uint32_t* pair_keys,
                                 uint32_t* pair_vals, ClearList clear, hipStream_t s);
// Tile ranges of the first *d_n sorted keys.
hipError_t launch_ranges(const uint32_t* pair_keys, const uint32_t* d_n, int64_t n_cap,
                         uint32_t* ranges, hipStream_t s);
// Work order of the tiles: order[0..n_tiles) is a permutation of the tiles by decreasing
// cost work[t]. Costs are compared in buckets (exact below 16, then 1/16 of the cost wide);
// the order inside a bucket is unspecified. One workgroup; n_tiles <= kMaxOrderedTiles.
constexpr int64_t kMaxOrderedTiles = (int64_t)1 << 20;
hipError_t launch_order_tiles(const uint32_t* work, int64_t n_tiles, uint32_t* order,
                              hipStream_t s);
// Forward blend of one pass (mode in split.mode). REST launches the open-tile kernel.
// tile_work (nullable): per tile, the span of pairs (first pair to one past the last pair any
// pixel blended) is written by the first pass and added to by the rest pass. zero (nullable):
// zero_n floats that the first pass's workgroups set to zero while they blend.
hipError_t launch_blend_fwd(const Plan& pl, const gb_splats& sp, const gb_options& o,
                            const ViewDev* views, int n_views, const SplatRec* rec,
                            const uint32_t* pair_vals, const uint32_t* ranges, float* rgb,
                            float* T_final, uint32_t* n_last, const SplitState& split,
                            uint32_t* tile_work, const float4* spec, unsigned long long* stats,
                            float* zero, int64_t zero_n, float* zero2, int64_t zero2_n,
                            hipStream_t s);
// Backward blend over the prefix (or only) pass's pairs `first`; with open_bits != null the
// tiles marked there first walk `rest` (the rest pass's pairs). tile_order (nullable):
// workgroup b takes tile tile_order[b]. With spec != null the records' view-dependent colours
// are part of the colour and d_spec[4 r + c] (zeroed by the caller) receives their adjoints.
hipError_t launch_blend_bwd(const Plan& pl, const gb_splats& sp, const gb_options& o,
                            const ViewDev* views, int n_views, const SplatRec* rec,
                            const PairList& first, const PairList& rest,
                            const uint32_t* open_bits, const uint32_t* tile_order,
                            const float* T_final, const float* d_rgb, float* d_rec,
                            float* d_tex, const float4* spec, float* d_spec, hipStream_t s);
// Training glue (train.hip).
hipError_t launch_activate_fwd(int P, const float* quats, const float* log_scales,
                               const float* logits, float* tan_u, float* tan_v, float* scales,
                               float* opacity, hipStream_t s);
hipError_t launch_activate_bwd(int P, const float* quats, const float* log_scales,
                               const float* logits, const float* d_tan_u, const float* d_tan_v,
                               const float* d_scales, const float* d_opacity, float* d_quats,
                               float* d_log_scales, float* d_logits, hipStream_t s);
hipError_t launch_l1_loss(int64_t n, const float* rgb, const float* target, float scale,
                          float* loss, float* d_rgb, hipStream_t s);
hipError_t launch_mse_loss(int64_t n, const float* rgb, const float* target, float scale,
                           float* loss, float* d_rgb, hipStream_t s);
hipError_t launch_box_filter(int64_t P, int N, int M, const float* in, float* out,
                             hipStream_t s);
hipError_t launch_rotz_only(int64_t P, float* d_quats, hipStream_t s);
hipError_t launch_to_bf16(int64_t n, const float* src, uint16_t* dst, hipStream_t s);
hipError_t launch_adam(int64_t n, float* theta, const float* grad, float* m, float* v, float lr,
                       float b1, float b2, float c1, float c2, float eps, uint16_t* bf16,
                       hipStream_t s);
// With sp.sh != null, d_spec[v P + k] holds the adjoint of record v P + k's view-dependent
// colour; g.d_sh receives the coefficients' gradient and the centres' gradient includes the
// term through the view direction.
hipError_t launch_preprocess_bwd(const gb_splats& sp, const ViewDev* d_views, int n_views,
                                 const uint32_t* count, const float* d_rec,
                                 const float4* d_spec, const gb_grads& g, hipStream_t s);

// Densification and pruning (densify.hip). The apply launchers are sized by n_new (the
// host's count) and bounded on the device by *d_n (the planned count).
hipError_t launch_densify_stats(const uint32_t* count, const float* d_rec, int64_t P,
                                int n_views, float* accum, float* vis, hipStream_t s);
hipError_t launch_densify_decide(int64_t P, const float* log_scales, const float* logits,
                                 const float* accum, const float* vis, float grad_threshold,
                                 float ls_dense, float logit_min, float ls_max,
                                 float ls_max_child, bool use_max_scale, uint32_t* action,
                                 uint32_t* n_out, hipStream_t s);
hipError_t launch_densify_map(int64_t P, const uint32_t* action, const uint32_t* n_out,
                              const uint32_t* offsets, uint32_t* map, hipStream_t s);
hipError_t launch_gather_rows(const uint32_t* map, const uint32_t* d_n, int64_t n_new, int width,
                              const float* src, float* dst, bool zero_new, hipStream_t s);
hipError_t launch_child_geometry(const uint32_t* map, const uint32_t* d_n, int64_t n_new,
                                 const float* means, const float* quats, const float* log_scales,
                                 const float* noise, float log_shrink, float* means_out,
                                 float* log_scales_out, hipStream_t s);
hipError_t launch_child_texture(const uint32_t* map, const uint32_t* d_n, int64_t n_new, int N,
                                const float* tex, const float* noise, float sigma,
                                float inv_shrink, float* tex_out, hipStream_t s);

}  // namespace gbb
