// C ABI of libgbb: argument validation, workspace plan, stream-ordered launch sequence.
//
// Forward sequence (all on the caller's stream, no host synchronisation):
//   views -> preprocess (key stage + records) -> depth sort of records (stable, 32-bit key)
//   -> exclusive scan of tile counts in depth order (K) -> overflow check
//   -> duplicate into (tile, record) pairs -> stable sort of pairs by tile
//   -> per-tile ranges -> blend forward (with the depth-prefix split: open-tile table -> rest
//   pairs -> sort -> ranges -> blend forward of open tiles); the forward also records each
//   tile's blended span.
// Backward: clear gradient buffers, work order of the tiles from the forward's per-tile spans
//   -> blend backward -> preprocess backward.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>

#include "gbb_internal.h"

namespace gbb {
namespace {

thread_local std::string g_last_error;

gb_status hip_fail(hipError_t e, const char* what) {
  char buf[256];
  snprintf(buf, sizeof(buf), "%s: %s", what, hipGetErrorString(e));
  g_last_error = buf;
  return GB_ERR_HIP;
}

gb_status arg_fail(const char* what) {
  g_last_error = what;
  return GB_ERR_ARG;
}

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }
int64_t align_up_i64(int64_t x, int64_t a) { return (x + a - 1) / a * a; }

bool aligned(const void* p, size_t a) { return ((uintptr_t)p % a) == 0; }

gb_status validate_options(const gb_options* o) {
  if (!o) return arg_fail("options is NULL");
  if (!(o->sigma > 0.f) || !std::isfinite(o->sigma)) return arg_fail("sigma must be > 0");
  if (!(o->alpha_min >= 0.f && o->alpha_min < 1.f)) return arg_fail("alpha_min outside [0,1)");
  if (!(o->alpha_max > 0.f && o->alpha_max <= 1.f)) return arg_fail("alpha_max outside (0,1]");
  if (!(o->t_min >= 0.f && o->t_min < 1.f)) return arg_fail("t_min outside [0,1)");
  if (!(o->lowpass_var > 0.f) || !std::isfinite(o->lowpass_var))
    return arg_fail("lowpass_var must be > 0");
  for (int i = 0; i < 3; ++i)
    if (!std::isfinite(o->bg[i])) return arg_fail("bg must be finite");
  const int tw = o->tile_w == 0 ? 16 : o->tile_w, th = o->tile_h == 0 ? 16 : o->tile_h;
  const bool ok_w = tw == 8 || tw == 16 || tw == 32, ok_h = th == 8 || th == 16 || th == 32;
  if (!ok_w || !ok_h || tw * th > 256) return arg_fail("tile must be 8/16/32 per side, <= 256 px");
  if (o->batch != 0 && o->batch != 4 && o->batch != 8 && o->batch != 16 && o->batch != 32 &&
      o->batch != 64)
    return arg_fail("batch must be 0, 4, 8, 16, 32 or 64");
  if (o->batch_bwd != 0 && o->batch_bwd != 4 && o->batch_bwd != 8 && o->batch_bwd != 16 &&
      o->batch_bwd != 32)
    return arg_fail("batch_bwd must be 0, 4, 8, 16 or 32");
  if (o->prefix_pairs_per_tile < -1 || o->prefix_pairs_per_tile > (1 << 20))
    return arg_fail("prefix_pairs_per_tile must be -1, 0 or in [1, 2^20]");
  if (o->tile_order < -1 || o->tile_order > 1) return arg_fail("tile_order must be -1, 0 or 1");
  return GB_OK;
}

gb_status validate_views(const gb_view* views, int32_t n_views) {
  if (!views) return arg_fail("views is NULL");
  if (n_views < 1 || n_views > GB_MAX_VIEWS) return arg_fail("n_views outside [1, 256]");
  for (int i = 0; i < n_views; ++i) {
    const gb_view& v = views[i];
    if (v.width < 1 || v.height < 1 || v.width > 32767 || v.height > 32767)
      return arg_fail("view size outside [1, 32767]");
    if (!(v.fx > 0.f) || !(v.fy > 0.f) || !std::isfinite(v.fx) || !std::isfinite(v.fy) ||
        !std::isfinite(v.cx) || !std::isfinite(v.cy))
      return arg_fail("view intrinsics invalid");
    if (!(v.z_near >= 0.f) || !std::isfinite(v.z_near)) return arg_fail("z_near must be >= 0");
    for (int k = 0; k < 9; ++k)
      if (!std::isfinite(v.R[k])) return arg_fail("view rotation not finite");
    for (int k = 0; k < 3; ++k)
      if (!std::isfinite(v.t[k])) return arg_fail("view translation not finite");
  }
  return GB_OK;
}

gb_status validate_splats(const gb_splats* s) {
  if (!s) return arg_fail("splats is NULL");
  if (s->P < 1) return arg_fail("P must be >= 1");
  if (!(s->N == 1 || s->N == 2 || s->N == 4 || s->N == 8 || s->N == 16)) {
    g_last_error = "texture side N must be 1, 2, 4, 8 or 16";
    return GB_ERR_UNSUPPORTED;
  }
  if (s->tex_dtype != GB_F32 && s->tex_dtype != GB_BF16) {
    g_last_error = "tex_dtype must be GB_F32 or GB_BF16";
    return GB_ERR_UNSUPPORTED;
  }
  const void* ptrs[] = {s->means, s->tan_u, s->tan_v, s->scales, s->opacity};
  for (const void* p : ptrs)
    if (!p || !aligned(p, 4)) return arg_fail("splat array NULL or not 4-byte aligned");
  if (!s->textures || !aligned(s->textures, 16)) return arg_fail("textures NULL or not 16-byte aligned");
  if (s->tex_side) {
    if (s->N != 8 && s->N != 16) {
      g_last_error = "with tex_side the layout side N must be 8 or 16";
      return GB_ERR_UNSUPPORTED;
    }
    if (!s->tex_offset || !aligned(s->tex_side, 4) || !aligned(s->tex_offset, 8))
      return arg_fail("tex_offset NULL, or tex_side / tex_offset misaligned");
    if (s->n_texels < 1) return arg_fail("n_texels must be >= 1 with tex_side");
  }
  if (s->sh) {
    if (s->sh_degree < 0 || s->sh_degree > 3) {
      g_last_error = "sh_degree must be 0, 1, 2 or 3";
      return GB_ERR_UNSUPPORTED;
    }
    if (!aligned(s->sh, 4)) return arg_fail("sh not 4-byte aligned");
  }
  return GB_OK;
}

gb_status make_plan(int32_t P, int32_t N, const gb_view* views, int32_t n_views,
                    const gb_options* o, int64_t capacity, Plan* pl) {
  if (capacity < 0 || capacity > (int64_t)0xFFFFFFF0) return arg_fail("pair_capacity outside [0, 2^32-16]");
  const int64_t VP = (int64_t)P * n_views;
  if (VP > ((int64_t)1 << 31)) return arg_fail("P * n_views exceeds 2^31");
  pl->P = P;
  pl->N = N;
  pl->V = n_views;
  pl->VP = VP;
  pl->capacity = capacity;
  pl->tile_w = o->tile_w == 0 ? 16 : o->tile_w;
  pl->tile_h = o->tile_h == 0 ? 16 : o->tile_h;
  // defaults: at N = 8 the smaller batches measured faster on the 1M-splat 1080p workload
  // (forward 16 vs 32: 0.50 vs 0.60 ms; backward 8 vs 16: 2.21 vs 2.31 ms), because less LDS
  // per block lets more blocks share a CU; at N = 4 a forward batch of 32 beat 64 and 16 (1M
  // splats at 1080p, forward + backward: 2.06 vs 2.13 ms) and a backward batch of 32 beat
  // 16 and 8 (2.13 vs 2.19 and 2.28 ms)
  pl->batch_fwd = o->batch != 0 ? o->batch : (N >= 16 ? 4 : N >= 8 ? 16 : N >= 4 ? 32 : 64);
  pl->batch_bwd = o->batch_bwd != 0 ? o->batch_bwd : (N >= 16 ? 4 : N >= 8 ? 8 : 32);
  // N = 16: 4.3 KB of staged texels per splat; batches of 4 keep the backward's LDS (texels,
  // their gradient sums and a ring of 4 batches' geometry) near 32 KB per workgroup, five per
  // CU. Batches of 4 are built for N = 16 only, and N = 16 only with them.
  if (N >= 16 && (pl->batch_fwd != 4 || pl->batch_bwd != 4)) {
    g_last_error = "N = 16 takes batch and batch_bwd 4 (or 0)";
    return GB_ERR_UNSUPPORTED;
  }
  if (N < 16 && (pl->batch_fwd == 4 || pl->batch_bwd == 4)) {
    g_last_error = "batches of 4 are built for N = 16 only";
    return GB_ERR_UNSUPPORTED;
  }
  int64_t tiles = 0, pixels = 0, sat = 0;
  for (int i = 0; i < n_views; ++i) {
    const int64_t tx = (views[i].width + pl->tile_w - 1) / pl->tile_w;
    const int64_t ty = (views[i].height + pl->tile_h - 1) / pl->tile_h;
    tiles += tx * ty;
    sat += (tx + 1) * (ty + 1);
    pixels += (int64_t)views[i].width * views[i].height;
  }
  if (sat >= ((int64_t)1 << 31)) return arg_fail("too many tiles");
  // packed pixel and tile indices are int32 on the device
  if (pixels >= ((int64_t)1 << 31)) return arg_fail("total pixels of all views must be < 2^31");
  pl->sat_len = sat;
  pl->total_tiles = tiles;
  pl->total_pixels = pixels;
  // depth-prefix split: pair slots of the prefix pass come on top of the capacity
  pl->split = o->prefix_pairs_per_tile >= 0;
  // default budget: 1024 pairs per tile measured faster than 512 on the 1M-splat 1080p
  // workload (3.12 vs 3.14 ms) and on four 1080p views of it (10.7 vs 12.5 ms), where more
  // tiles stay open after a smaller prefix
  const int64_t per_tile = o->prefix_pairs_per_tile > 0 ? o->prefix_pairs_per_tile : 1024;
  pl->prefix_cap = pl->split ? align_up_i64(per_tile * tiles, 1024) : 0;
  if (capacity + pl->prefix_cap > (int64_t)0xFFFFFFF0)
    return arg_fail("pair capacity plus the prefix pass's slots exceed 2^32-16");
  pl->ordered = o->tile_order >= 0 && tiles <= kMaxOrderedTiles;
  int bits = 1;
  while (((int64_t)1 << bits) < tiles) ++bits;
  pl->tile_bits = bits;
  pl->nb_vp = (VP + kRadixTile - 1) / kRadixTile;
  // radix blocks of the larger pair sort (the prefix's slots can exceed a small capacity)
  const int64_t sort_cap = capacity > pl->prefix_cap ? capacity : pl->prefix_cap;
  pl->nb_pairs = (sort_cap + kRadixTile - 1) / kRadixTile;
  const int64_t nb_max = pl->nb_vp > pl->nb_pairs ? pl->nb_vp : pl->nb_pairs;
  pl->hist_len = 256 * nb_max;
  int64_t part = (VP + kScanTile - 1) / kScanTile;
  const int64_t part_h = (pl->hist_len + kScanTile - 1) / kScanTile;
  if (part_h > part) part = part_h;
  pl->partials_len = part + 2;

  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t at = off;
    off = align_up(off + bytes, 256);
    return at;
  };
  pl->off_status = take(256);
  pl->off_views = take(sizeof(ViewDev) * (size_t)n_views);
  pl->off_depth_key = take(4 * (size_t)VP);
  pl->off_depth_key_alt = take(4 * (size_t)VP);
  pl->off_order = take(4 * (size_t)VP);
  pl->off_order_alt = take(4 * (size_t)VP);
  pl->off_count = take(4 * (size_t)VP);
  pl->off_offsets = take(4 * (size_t)VP);
  pl->off_rec = take(sizeof(SplatRec) * (size_t)VP);
  pl->off_partials = take(4 * (size_t)pl->partials_len);
  pl->off_partials64 = take(8 * (size_t)pl->partials_len);
  pl->off_hist = take(4 * (size_t)pl->hist_len);
  pl->off_digit_tot = take(4 * (size_t)kDigitTotWords);
  // pairs: the prefix pass's [0, prefix_cap), then the capacity (the only pass, or the rest)
  const size_t slots = (size_t)(pl->prefix_cap + capacity);
  pl->off_pair_keys = take(4 * slots);
  pl->off_pair_vals = take(4 * slots);
  pl->off_pair_keys_alt = take(4 * slots);
  pl->off_pair_vals_alt = take(4 * slots);
  pl->off_ranges = take(8 * (size_t)tiles);
  pl->off_n_last = take(4 * (size_t)pixels);
  pl->off_drec = take(4 * (size_t)kRecGrad * (size_t)VP);
  pl->off_stats = take(64);
  const size_t sp = pl->split ? 1 : 0;
  pl->off_ranges_rest = take(sp * 8 * (size_t)tiles);
  pl->off_n_last_rest = take(sp * 4 * (size_t)pixels);
  pl->off_fwd_state = take(sp * 16 * (size_t)pixels);
  pl->off_open_bits = take(sp * 4 * (size_t)((tiles + 31) / 32));
  pl->off_count_rest = take(sp * 4 * (size_t)VP);
  pl->off_offsets_rest = take(sp * 4 * (size_t)VP);
  pl->n_chunks = (sort_cap + kChunkSlots - 1) / kChunkSlots + 1;
  pl->off_chunk_owner = take(4 * (size_t)pl->n_chunks);
  pl->off_sat = take(sp * 4 * (size_t)pl->sat_len);
  // work order of the tiles for the backward, and the forward's per-tile spans it sorts
  const size_t od = pl->ordered ? 1 : 0;
  pl->off_tile_order = take(od * 4 * (size_t)tiles);
  pl->off_tile_work = take(od * 4 * (size_t)tiles);
  pl->off_view_pairs = take(8 * (size_t)n_views);
  // view-dependent colour of each record and its adjoint (used with SH coefficients)
  pl->off_spec = take(16 * (size_t)VP);
  pl->off_dspec = take(16 * (size_t)VP);
  pl->total = off;
  return GB_OK;
}

gb_status check_common(const gb_splats* s, const gb_view* views, int32_t n_views,
                       const gb_options* o, void* ws, size_t ws_bytes, int64_t cap, Plan* pl) {
  gb_status st;
  if ((st = validate_splats(s)) != GB_OK) return st;
  if ((st = validate_views(views, n_views)) != GB_OK) return st;
  if ((st = validate_options(o)) != GB_OK) return st;
  if ((st = make_plan(s->P, s->N, views, n_views, o, cap, pl)) != GB_OK) return st;
  if (!ws || !aligned(ws, 256)) return arg_fail("workspace NULL or not 256-byte aligned");
  if (ws_bytes < pl->total) return arg_fail("workspace too small for this plan");
  return GB_OK;
}

// ---- stage timing (measurement only) ------------------------------------------------------
enum Stage {
  kStPreprocess, kStDepthSort, kStPairScan, kStDuplicate, kStTileSort, kStRanges, kStBlendFwd,
  kStRestTiles, kStBlendFwdRest, kStBwdClear, kStBlendBwd, kStPreprocessBwd, kNumStages
};
const char* const kStageNames[kNumStages] = {
    "preprocess", "depth_sort", "pair_scan", "duplicate", "tile_sort", "ranges", "blend_fwd",
    "rest_tiles", "blend_fwd_rest", "bwd_clear", "blend_bwd", "preprocess_bwd"};

struct Timing {
  bool on = false;
  bool created = false;
  hipEvent_t ev[kNumStages][2];
  bool recorded[kNumStages] = {};
} g_timing;

hipError_t stage_mark(int stage, int end, hipStream_t s) {
  if (!g_timing.on) return hipSuccess;
  if (!g_timing.created) {
    for (int i = 0; i < kNumStages; ++i)
      for (int j = 0; j < 2; ++j) {
        hipError_t e = hipEventCreate(&g_timing.ev[i][j]);
        if (e != hipSuccess) return e;
      }
    g_timing.created = true;
  }
  if (end) g_timing.recorded[stage] = true;
  return hipEventRecord(g_timing.ev[stage][end], s);
}

// ---- host-visible overflow state ---------------------------------------------------------
// Every forward's count finalisation stores (overflow << 63) | K into a slot of host-mapped,
// coherent memory chosen by the workspace address. A later gb_render_fwd on the same
// workspace reads that slot without synchronising: if the last forward that has completed
// overflowed and needed more pairs than the new call's capacity, it returns GB_ERR_CAPACITY
// before launching anything. Slots are reused round-robin beyond kMirrorSlots workspaces.
constexpr int kMirrorSlots = 64;
struct Mirror {
  std::mutex mu;
  bool tried = false;
  unsigned long long* host = nullptr;
  unsigned long long* dev = nullptr;
  const void* key[kMirrorSlots] = {};
  int next = 0;
} g_mirror;

// Slot of `ws`: its host and device addresses (both null if host-mapped memory is
// unavailable). `fresh` is set when the library has not seen this workspace before (or its
// slot was recycled), so that the caller can clear the workspace's sticky overflow word.
void mirror_slot(const void* ws, volatile unsigned long long** host, unsigned long long** dev,
                 bool* fresh) {
  std::lock_guard<std::mutex> lock(g_mirror.mu);
  if (!g_mirror.tried) {
    g_mirror.tried = true;
    void* h = nullptr;
    if (hipHostMalloc(&h, kMirrorSlots * sizeof(unsigned long long),
                      hipHostMallocCoherent | hipHostMallocMapped) == hipSuccess) {
      memset(h, 0, kMirrorSlots * sizeof(unsigned long long));
      void* d = nullptr;
      if (hipHostGetDevicePointer(&d, h, 0) == hipSuccess) {
        g_mirror.host = static_cast<unsigned long long*>(h);
        g_mirror.dev = static_cast<unsigned long long*>(d);
      } else {
        (void)hipHostFree(h);
      }
    }
    (void)hipGetLastError();  // a failure here must not surface in a later call
  }
  int i = 0;
  while (i < kMirrorSlots && g_mirror.key[i] != ws) ++i;
  *fresh = i == kMirrorSlots;
  if (*fresh) {
    i = g_mirror.next;
    g_mirror.next = (g_mirror.next + 1) % kMirrorSlots;
    g_mirror.key[i] = ws;
    if (g_mirror.host) g_mirror.host[i] = 0;
  }
  *host = g_mirror.host ? g_mirror.host + i : nullptr;
  *dev = g_mirror.dev ? g_mirror.dev + i : nullptr;
}

template <typename T>
T* at(void* ws, size_t off) {
  return reinterpret_cast<T*>(reinterpret_cast<char*>(ws) + off);
}

#define GBB_TRY(expr, what)                     \
  do {                                          \
    hipError_t e_ = (expr);                     \
    if (e_ != hipSuccess) return hip_fail(e_, what); \
  } while (0)

// With order != null the preprocess launch also writes the depth sort's initial order and
// clears n_zero words at `zero`.
gb_status run_preprocess(const gb_splats* s, const gb_view* views, int32_t n_views,
                         const gb_options* o, void* ws, const Plan& pl, hipStream_t st,
                         uint32_t* order = nullptr, uint32_t* zero = nullptr,
                         int64_t n_zero = 0) {
  GBB_TRY(stage_mark(kStPreprocess, 0, st), "timing");
  ViewDev* d_views = at<ViewDev>(ws, pl.off_views);
  GBB_TRY(launch_upload_views(views, n_views, pl.tile_w, pl.tile_h, d_views, st), "upload views");
  GBB_TRY(launch_preprocess(*s, d_views, n_views, *o, pl.tile_w, pl.tile_h,
                            at<uint32_t>(ws, pl.off_depth_key),
                            at<uint32_t>(ws, pl.off_depth_key_alt), at<uint32_t>(ws, pl.off_count),
                            at<SplatRec>(ws, pl.off_rec), at<float4>(ws, pl.off_spec), order,
                            zero, n_zero, st),
          "preprocess");
  GBB_TRY(stage_mark(kStPreprocess, 1, st), "timing");
  return GB_OK;
}

}  // namespace
}  // namespace gbb

namespace gbb {
namespace {
struct DensifyWork {
  size_t status, action, n_out, offsets, map, partials, partials64, total;
};

constexpr size_t align256(size_t x) { return (x + 255) / 256 * 256; }

// Work buffer of the densification plan for P splats: per splat its action, output count,
// output offset and two parent-map entries, plus the scan's partial sums.
constexpr DensifyWork densify_work(int64_t P) {
  const size_t parts = (size_t)((P + kScanTile - 1) / kScanTile + 2);
  DensifyWork w{};
  w.status = 0;
  w.action = w.status + align256(256);
  w.n_out = w.action + align256(4 * (size_t)P);
  w.offsets = w.n_out + align256(4 * (size_t)P);
  w.map = w.offsets + align256(4 * (size_t)P);
  w.partials = w.map + align256(8 * (size_t)P);
  w.partials64 = w.partials + align256(4 * parts);
  w.total = w.partials64 + align256(8 * parts);
  return w;
}

gb_status check_raw(const gb_raw_splats* r, const char* what) {
  if (!r) return arg_fail(what);
  if (r->P < 0 || r->N < 1 || r->N > 64 || r->sh_coef < 0 || r->sh_coef > 64)
    return arg_fail("raw splats: P >= 0, 1 <= N <= 64, 0 <= sh_coef <= 64");
  if (r->P == 0) return GB_OK;
  const void* ptrs[] = {r->means, r->quats, r->log_scales, r->opacity_logits, r->textures};
  for (const void* p : ptrs)
    if (!p || !aligned(p, 4)) return arg_fail("raw splat array NULL or misaligned");
  if (r->sh_coef > 0 && (!r->sh || !aligned(r->sh, 4)))
    return arg_fail("raw splats: sh NULL or misaligned with sh_coef > 0");
  return GB_OK;
}

gb_status check_densify_options(const gb_densify_options* o) {
  if (!o) return arg_fail("densify options NULL");
  if (!(o->grad_threshold >= 0.f) || !std::isfinite(o->grad_threshold))
    return arg_fail("grad_threshold must be >= 0");
  if (!(o->dense_scale > 0.f) || !std::isfinite(o->dense_scale))
    return arg_fail("dense_scale must be > 0");
  if (!(o->min_opacity >= 0.f && o->min_opacity < 1.f)) return arg_fail("min_opacity in [0, 1)");
  if (!(o->max_scale >= 0.f) || !std::isfinite(o->max_scale)) return arg_fail("max_scale >= 0");
  if (!(o->split_shrink >= 1.f) || !std::isfinite(o->split_shrink))
    return arg_fail("split_shrink must be >= 1");
  return GB_OK;
}

gb_status check_densify_plan_args(const gb_raw_splats* src, const float* grad_accum,
                                  const float* vis_count, const gb_densify_options* o,
                                  const int64_t* P_new) {
  gb_status st;
  if ((st = check_raw(src, "src NULL")) != GB_OK) return st;
  if ((st = check_densify_options(o)) != GB_OK) return st;
  if (!P_new) return arg_fail("P_new NULL");
  if (src->P > 0 &&
      (!grad_accum || !vis_count || !aligned(grad_accum, 4) || !aligned(vis_count, 4)))
    return arg_fail("grad_accum / vis_count NULL or misaligned");
  return GB_OK;
}

gb_status check_densify_apply_args(const gb_raw_splats* src, const float* noise, float sigma,
                                   const gb_densify_options* o, const gb_raw_splats* dst,
                                   const gb_row_state* states, int32_t n_states) {
  gb_status st;
  if ((st = check_raw(src, "src NULL")) != GB_OK) return st;
  if ((st = check_raw(dst, "dst NULL")) != GB_OK) return st;
  if ((st = check_densify_options(o)) != GB_OK) return st;
  if (dst->N != src->N || dst->sh_coef != src->sh_coef)
    return arg_fail("dst must have the texture side and SH coefficients of src");
  if (!(sigma > 0.f) || !std::isfinite(sigma)) return arg_fail("sigma must be > 0");
  if (n_states < 0 || (n_states > 0 && !states)) return arg_fail("states NULL");
  for (int i = 0; i < n_states; ++i)
    if (!states[i].src || !states[i].dst || states[i].width < 1 || !aligned(states[i].src, 4) ||
        !aligned(states[i].dst, 4))
      return arg_fail("state row arrays NULL, misaligned or of width < 1");
  if (dst->P > 0 && (!noise || !aligned(noise, 4))) return arg_fail("noise NULL or misaligned");
  return GB_OK;
}

// Decide, scan and map of the densification plan into `work` (laid out by densify_work),
// stream-ordered, without waiting.
gb_status densify_plan_launch(const gb_raw_splats* src, const float* grad_accum,
                              const float* vis_count, const gb_densify_options* o, void* work,
                              hipStream_t hs) {
  const DensifyWork w = densify_work(src->P);
  char* b = static_cast<char*>(work);
  // thresholds in the domain of the raw parameters (double precision, rounded once)
  const double shrink = o->split_shrink;
  const float ls_dense = (float)std::log((double)o->dense_scale);
  const float logit_min =
      o->min_opacity > 0.f ? (float)std::log((double)o->min_opacity / (1.0 - o->min_opacity))
                           : -INFINITY;
  const bool use_max = o->max_scale > 0.f;
  const float ls_max = use_max ? (float)std::log((double)o->max_scale) : 0.f;
  const float ls_max_child = use_max ? (float)(std::log((double)o->max_scale) + std::log(shrink))
                                     : 0.f;
  uint32_t* action = reinterpret_cast<uint32_t*>(b + w.action);
  uint32_t* n_out = reinterpret_cast<uint32_t*>(b + w.n_out);
  uint32_t* offsets = reinterpret_cast<uint32_t*>(b + w.offsets);
  uint32_t* d_total = reinterpret_cast<uint32_t*>(b + w.status);
  unsigned long long* d_total64 = reinterpret_cast<unsigned long long*>(b + w.status + 8);
  GBB_TRY(launch_densify_decide(src->P, src->log_scales, src->opacity_logits, grad_accum,
                                vis_count, o->grad_threshold, ls_dense, logit_min, ls_max,
                                ls_max_child, use_max, action, n_out, hs),
          "densify decide");
  GBB_TRY(launch_scan_u32(n_out, nullptr, offsets, src->P,
                          reinterpret_cast<uint32_t*>(b + w.partials), d_total, d_total64,
                          reinterpret_cast<unsigned long long*>(b + w.partials64), hs),
          "densify scan");
  GBB_TRY(launch_densify_map(src->P, action, n_out, offsets,
                             reinterpret_cast<uint32_t*>(b + w.map), hs),
          "densify map");
  return GB_OK;
}

// Waits for the stream and reads the plan's output count from `work`.
gb_status densify_read_count(const void* work, hipStream_t hs, int64_t* P_new) {
  unsigned long long total = 0;
  GBB_TRY(hipMemcpyAsync(&total, static_cast<const char*>(work) + 8, sizeof(total),
                         hipMemcpyDeviceToHost, hs),
          "read densify count");
  GBB_TRY(hipStreamSynchronize(hs), "sync");
  *P_new = (int64_t)total;
  return GB_OK;
}

// Writes the planned outputs (at most n_cap rows, and no more than the plan's count) into dst.
gb_status densify_apply_launch(const gb_raw_splats* src, const void* work, const float* noise,
                               float sigma, const gb_densify_options* o,
                               const gb_raw_splats* dst, int64_t n, const gb_row_state* states,
                               int32_t n_states, hipStream_t hs) {
  const DensifyWork w = densify_work(src->P);
  const char* b = static_cast<const char*>(work);
  const uint32_t* map = reinterpret_cast<const uint32_t*>(b + w.map);
  const uint32_t* d_n = reinterpret_cast<const uint32_t*>(b + w.status);
  const int N = src->N;
  GBB_TRY(launch_child_geometry(map, d_n, n, src->means, src->quats, src->log_scales, noise,
                                (float)std::log((double)o->split_shrink), dst->means,
                                dst->log_scales, hs),
          "densify geometry");
  GBB_TRY(launch_gather_rows(map, d_n, n, 4, src->quats, dst->quats, false, hs), "quats");
  GBB_TRY(launch_gather_rows(map, d_n, n, 1, src->opacity_logits, dst->opacity_logits, false, hs),
          "logits");
  if (src->sh_coef > 0)
    GBB_TRY(launch_gather_rows(map, d_n, n, 3 * src->sh_coef, src->sh, dst->sh, false, hs), "sh");
  GBB_TRY(launch_child_texture(map, d_n, n, N, src->textures, noise, sigma,
                               (float)(1.0 / (double)o->split_shrink), dst->textures, hs),
          "densify textures");
  for (int i = 0; i < n_states; ++i)
    GBB_TRY(launch_gather_rows(map, d_n, n, states[i].width, states[i].src, states[i].dst, true,
                               hs),
            "state rows");
  return GB_OK;
}

// The work area of gb_densify_noalloc: a library-owned device array, one copy per GPU, held
// until the process ends. In host code the array's name is only a host-side handle; its
// device address comes from hipGetSymbolAddress, taken once per device with that device
// current, and only that address is ever passed to kernels.
constexpr size_t kNoallocWorkBytes = densify_work(GB_DENSIFY_NOALLOC_MAX_P).total;
static __device__ __align__(256) unsigned char scratch[kNoallocWorkBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

gb_status static_densify_work(void** out) {
  int dev = 0;
  GBB_TRY(hipGetDevice(&dev), "hipGetDevice");
  if (dev < 0 || dev >= kMaxDevices) return arg_fail("device index beyond the library's table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    GBB_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "address of the static work area");
    if (!p) return hip_fail(hipErrorInvalidSymbol, "address of the static work area");
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return GB_OK;
}
}  // namespace
}  // namespace gbb

using namespace gbb;

extern "C" {

void gb_default_options(gb_options* o) {
  if (!o) return;
  o->sigma = 0.5f;
  o->alpha_min = 1.0f / 255.0f;
  o->alpha_max = 0.99f;
  o->t_min = 1e-4f;
  o->lowpass_var = 0.5f;
  o->bg[0] = o->bg[1] = o->bg[2] = 0.f;
  o->tile_w = 16;
  o->tile_h = 16;
  o->batch = 0;
  o->batch_bwd = 0;
  o->prefix_pairs_per_tile = 0;
  o->tile_order = 0;
}

const char* gb_status_string(gb_status s) {
  switch (s) {
    case GB_OK: return "ok";
    case GB_ERR_ARG: return "invalid argument";
    case GB_ERR_HIP: return "HIP runtime error";
    case GB_ERR_CAPACITY: return "pair capacity exceeded";
    case GB_ERR_UNSUPPORTED: return "unsupported configuration";
  }
  return "unknown status";
}

const char* gb_last_error(void) { return g_last_error.c_str(); }

gb_status gb_workspace_layout(int32_t P, int32_t N, const gb_view* views, int32_t n_views,
                              const gb_options* opts, int64_t pair_capacity, gb_layout* out) {
  if (!out) return arg_fail("out is NULL");
  if (P < 1) return arg_fail("P must be >= 1");
  if (!(N == 1 || N == 2 || N == 4 || N == 8 || N == 16)) {
    g_last_error = "texture side N must be 1, 2, 4, 8 or 16";
    return GB_ERR_UNSUPPORTED;
  }
  gb_status st;
  if ((st = validate_views(views, n_views)) != GB_OK) return st;
  if ((st = validate_options(opts)) != GB_OK) return st;
  Plan pl;
  if ((st = make_plan(P, N, views, n_views, opts, pair_capacity, &pl)) != GB_OK) return st;
  out->total_bytes = pl.total;
  out->status = pl.off_status;
  out->depth_key = pl.off_depth_key;
  out->tile_count = pl.off_count;
  out->records = pl.off_rec;
  out->order = pl.off_order;
  out->pair_keys = pl.off_pair_keys;
  out->pair_vals = pl.off_pair_vals;
  out->ranges = pl.off_ranges;
  out->n_last = pl.off_n_last;
  out->pair_capacity = pl.capacity;
  out->total_tiles = pl.total_tiles;
  out->prefix_capacity = pl.prefix_cap;
  out->pair_keys_rest = pl.off_pair_keys + 4 * (size_t)pl.prefix_cap;
  out->pair_vals_rest = pl.off_pair_vals + 4 * (size_t)pl.prefix_cap;
  out->ranges_rest = pl.off_ranges_rest;
  out->n_last_rest = pl.off_n_last_rest;
  out->open_tiles = pl.off_open_bits;
  out->tile_order = pl.ordered ? pl.off_tile_order : 0;
  out->tile_work = pl.ordered ? pl.off_tile_work : 0;
  return GB_OK;
}

gb_status gb_count_pairs(const gb_splats* s, const gb_view* views, int32_t n_views,
                         const gb_options* o, void* ws, size_t ws_bytes, int64_t cap,
                         int64_t* K_out, void* stream) {
  if (!K_out) return arg_fail("K_out is NULL");
  Plan pl;
  gb_status st = check_common(s, views, n_views, o, ws, ws_bytes, cap, &pl);
  if (st != GB_OK) return st;
  hipStream_t hs = reinterpret_cast<hipStream_t>(stream);
  if ((st = run_preprocess(s, views, n_views, o, ws, pl, hs)) != GB_OK) return st;
  Status* d_st = at<Status>(ws, pl.off_status);
  GBB_TRY(launch_scan_u32(at<uint32_t>(ws, pl.off_count), nullptr, at<uint32_t>(ws, pl.off_offsets),
                          pl.VP, at<uint32_t>(ws, pl.off_partials), &d_st->K, &d_st->K64,
                          at<unsigned long long>(ws, pl.off_partials64), hs),
          "count scan");
  Status h;
  GBB_TRY(hipMemcpyAsync(&h, d_st, sizeof(Status), hipMemcpyDeviceToHost, hs), "read count");
  GBB_TRY(hipStreamSynchronize(hs), "sync");
  *K_out = (int64_t)h.K64;
  // a caller that counts is re-planning: forget an earlier overflow on this workspace
  volatile unsigned long long* m_host = nullptr;
  unsigned long long* m_dev = nullptr;
  bool fresh = false;
  mirror_slot(ws, &m_host, &m_dev, &fresh);
  if (m_host) *m_host = 0ull;
  GBB_TRY(launch_fill_u32(reinterpret_cast<uint32_t*>(reinterpret_cast<char*>(ws) +
                                                      offsetof(Status, sticky_overflow)),
                          0u, 1, hs),
          "clear sticky overflow");
  return GB_OK;
}

// Per workspace: the gradient arrays that its last forward zeroed (kZeroTex: the texture
// gradients, kZeroRec: the per-record gradient accumulators; null if none), so that the
// backward of that forward can skip clearing the same array.
enum { kZeroTex = 0, kZeroRec = 1, kZeroKinds = 2 };
struct ZeroedRecord {
  std::mutex mu;
  const void* key[kMirrorSlots] = {};
  const float* ptr[kMirrorSlots][kZeroKinds] = {};
  int64_t n[kMirrorSlots][kZeroKinds] = {};
  int next = 0;
} g_zeroed;

// Records that the forward on `ws` zeroed ptr [n] (ptr == null: forgets the kind).
void zeroed_set(const void* ws, int kind, const float* ptr, int64_t n) {
  std::lock_guard<std::mutex> lock(g_zeroed.mu);
  int i = 0;
  while (i < kMirrorSlots && g_zeroed.key[i] != ws) ++i;
  if (i == kMirrorSlots) {
    if (!ptr) return;  // nothing recorded for this workspace
    i = g_zeroed.next;
    g_zeroed.next = (g_zeroed.next + 1) % kMirrorSlots;
    g_zeroed.key[i] = ws;
    for (int k = 0; k < kZeroKinds; ++k) g_zeroed.ptr[i][k] = nullptr;
  }
  g_zeroed.ptr[i][kind] = ptr;
  g_zeroed.n[i][kind] = n;
}

// True (and forgets it) if the last forward on `ws` zeroed exactly `ptr` [n] of this kind.
bool zeroed_take(const void* ws, int kind, const float* ptr, int64_t n) {
  std::lock_guard<std::mutex> lock(g_zeroed.mu);
  for (int i = 0; i < kMirrorSlots; ++i) {
    if (g_zeroed.key[i] != ws) continue;
    const bool hit =
        g_zeroed.ptr[i][kind] == ptr && g_zeroed.n[i][kind] == n && ptr != nullptr;
    g_zeroed.ptr[i][kind] = nullptr;
    return hit;
  }
  return false;
}

// Number of floats of the texture-gradient array of these splats.
int64_t tex_grad_values(const gb_splats* s) {
  return s->tex_side ? 3 * s->n_texels : (int64_t)s->P * 3 * s->N * s->N;
}

static gb_status render_fwd_impl(const gb_splats* s, const gb_view* views, int32_t n_views,
                                 const gb_options* o, void* ws, size_t ws_bytes, int64_t cap,
                                 float* rgb, float* T_final, bool stats, void* stream,
                                 bool use_mirror = true, uint32_t* overflow_flag = nullptr,
                                 float* zero_tex = nullptr) {
  Plan pl;
  gb_status st = check_common(s, views, n_views, o, ws, ws_bytes, cap, &pl);
  if (st != GB_OK) return st;
  if (zero_tex && !aligned(zero_tex, 4)) return arg_fail("d_textures to zero misaligned");
  // whatever happens below, the backward must not rely on an older forward's zeroing
  for (int k = 0; k < kZeroKinds; ++k) zeroed_set(ws, k, nullptr, 0);
  const int64_t zero_n = zero_tex ? tex_grad_values(s) : 0;
  if (!rgb || !T_final || !aligned(rgb, 4) || !aligned(T_final, 4))
    return arg_fail("rgb / T_final NULL or misaligned");
  // a completed earlier forward on this workspace that did not fit this capacity
  volatile unsigned long long* m_host = nullptr;
  unsigned long long* m_dev = nullptr;
  bool fresh = false;
  if (use_mirror) mirror_slot(ws, &m_host, &m_dev, &fresh);
  if (m_host) {
    const unsigned long long m = *m_host;
    const unsigned long long need = m & ~(1ull << 63);
    if ((m >> 63) && need > (unsigned long long)cap) {
      char buf[160];
      snprintf(buf, sizeof(buf),
               "an earlier forward on this workspace needed %llu pairs; pair_capacity is %lld",
               need, (long long)cap);
      g_last_error = buf;
      return GB_ERR_CAPACITY;
    }
  }
  hipStream_t hs = reinterpret_cast<hipStream_t>(stream);
  Status* d_st = at<Status>(ws, pl.off_status);
  // a workspace met for the first time holds whatever its memory held: its sticky
  // overflow word starts at zero
  if (fresh)
    GBB_TRY(launch_fill_u32(&d_st->sticky_overflow, 0u, 1, hs), "clear sticky overflow");
  uint32_t* order = at<uint32_t>(ws, pl.off_order);
  uint32_t* digit_tot = at<uint32_t>(ws, pl.off_digit_tot);
  // the preprocess launch also writes the depth sort's initial order (record indices) and
  // clears the radix sorts' digit totals: they start from zero in every forward, and each
  // sort leaves them zero
  if ((st = run_preprocess(s, views, n_views, o, ws, pl, hs, order, digit_tot,
                           kDigitTotWords)) != GB_OK)
    return st;

  uint32_t* dk_a = at<uint32_t>(ws, pl.off_depth_key_alt);
  uint32_t* order_alt = at<uint32_t>(ws, pl.off_order_alt);
  uint32_t* count = at<uint32_t>(ws, pl.off_count);
  uint32_t* offsets = at<uint32_t>(ws, pl.off_offsets);
  uint32_t* partials = at<uint32_t>(ws, pl.off_partials);
  uint32_t* hist = at<uint32_t>(ws, pl.off_hist);
  uint32_t* pk = at<uint32_t>(ws, pl.off_pair_keys);
  uint32_t* pv = at<uint32_t>(ws, pl.off_pair_vals);
  uint32_t* pk_a = at<uint32_t>(ws, pl.off_pair_keys_alt);
  uint32_t* pv_a = at<uint32_t>(ws, pl.off_pair_vals_alt);
  uint32_t* ranges = at<uint32_t>(ws, pl.off_ranges);
  ViewDev* d_views = at<ViewDev>(ws, pl.off_views);
  SplatRec* rec = at<SplatRec>(ws, pl.off_rec);
  unsigned long long* d_stats = at<unsigned long long>(ws, pl.off_stats);

  // depth order of all records: sort the key copy written by the preprocess, carrying
  // record indices (the offsets array is free until the scan and serves as ping-pong space)
  GBB_TRY(stage_mark(kStDepthSort, 0, hs), "timing");
  GBB_TRY(launch_radix_sort(dk_a, order, offsets, order_alt, nullptr, pl.VP, 32, hist, digit_tot,
                            hs),
          "depth sort");
  GBB_TRY(stage_mark(kStDepthSort, 1, hs), "timing");
  // tile counts in depth order -> pair offsets and K; with the split, the prefix cut
  GBB_TRY(stage_mark(kStPairScan, 0, hs), "timing");
  uint32_t* chunk_owner = at<uint32_t>(ws, pl.off_chunk_owner);
  unsigned long long* partials64 = at<unsigned long long>(ws, pl.off_partials64);
  GBB_TRY(launch_scan_u32(count, order, offsets, pl.VP, partials, &d_st->K, &d_st->K64,
                          partials64, hs, chunk_owner, pl.n_chunks),
          "pair scan");
  const StatusEcho echo{(uint32_t)n_views, (uint32_t)pl.P, (unsigned long long)pl.off_count,
                        (unsigned long long)pl.off_view_pairs};
  GBB_TRY(launch_finalize_count(offsets, pl.VP, d_st, pl.capacity, echo, m_dev, overflow_flag,
                                pl.split ? pl.prefix_cap : 0, chunk_owner, hs),
          "finalize count");
  GBB_TRY(stage_mark(kStPairScan, 1, hs), "timing");
  // first (or only) pass: pairs of the depth prefix, sorted by tile, ranges, blend
  const int64_t cap_a = pl.split ? pl.prefix_cap : pl.capacity;
  GBB_TRY(stage_mark(kStDuplicate, 0, hs), "timing");
  // the duplicate launch also zeroes the tile ranges and, with the split, the open-tile bitmap
  ClearList clear_a;
  clear_a.p[0] = ranges;
  clear_a.n[0] = 2 * pl.total_tiles;
  if (pl.split) {
    clear_a.p[1] = at<uint32_t>(ws, pl.off_open_bits);
    clear_a.n[1] = (pl.total_tiles + 31) / 32;
  }
  GBB_TRY(launch_duplicate(order, count, offsets, chunk_owner, rec, d_views, pl.tile_w, pl.tile_h,
                           d_st, cap_a, pk, pv, clear_a, hs),
          "duplicate");
  GBB_TRY(stage_mark(kStDuplicate, 1, hs), "timing");
  GBB_TRY(stage_mark(kStTileSort, 0, hs), "timing");
  GBB_TRY(launch_radix_sort(pk, pv, pk_a, pv_a, &d_st->n_sorted, cap_a, pl.tile_bits, hist,
                            digit_tot, hs),
          "tile sort");
  GBB_TRY(stage_mark(kStTileSort, 1, hs), "timing");
  GBB_TRY(stage_mark(kStRanges, 0, hs), "timing");
  GBB_TRY(launch_ranges(pk, &d_st->n_sorted, cap_a, ranges, hs), "ranges");
  GBB_TRY(stage_mark(kStRanges, 1, hs), "timing");
  // per-tile blended spans for the backward's work order
  uint32_t* tile_work = pl.ordered ? at<uint32_t>(ws, pl.off_tile_work) : nullptr;
  if (stats)
    GBB_TRY(launch_fill_u32(reinterpret_cast<uint32_t*>(d_stats), 0u, 16, hs), "clear stats");
  SplitState split{kSinglePass, nullptr, nullptr, nullptr};
  if (pl.split) {
    split.mode = kPrefixPass;
    split.open_bits = at<uint32_t>(ws, pl.off_open_bits);
    split.fwd_state = at<float4>(ws, pl.off_fwd_state);
    split.any_open = &d_st->any_open;  // cleared by the count's finalisation
  }
  GBB_TRY(stage_mark(kStBlendFwd, 0, hs), "timing");
  const float4* spec = s->sh ? at<float4>(ws, pl.off_spec) : nullptr;
  // the workgroups also zero the coming backward's per-record gradient accumulators (and,
  // with zero_tex, its texture gradients) while they blend
  float* d_rec = at<float>(ws, pl.off_drec);
  const int64_t rec_n = (int64_t)kRecGrad * pl.VP;
  GBB_TRY(launch_blend_fwd(pl, *s, *o, d_views, n_views, rec, pv, ranges, rgb, T_final,
                           at<uint32_t>(ws, pl.off_n_last), split, tile_work, spec,
                           stats ? d_stats : nullptr, zero_tex, zero_n, d_rec, rec_n, hs),
          "blend forward");
  GBB_TRY(stage_mark(kStBlendFwd, 1, hs), "timing");
  if (zero_tex) zeroed_set(ws, kZeroTex, zero_tex, zero_n);
  zeroed_set(ws, kZeroRec, d_rec, rec_n);
  if (!pl.split) return GB_OK;

  // rest pass: the remaining records, paired with the tiles the prefix left open
  uint32_t* count_rest = at<uint32_t>(ws, pl.off_count_rest);
  uint32_t* offsets_rest = at<uint32_t>(ws, pl.off_offsets_rest);
  uint32_t* ranges_rest = at<uint32_t>(ws, pl.off_ranges_rest);
  uint32_t* pk_r = pk + pl.prefix_cap;
  uint32_t* pv_r = pv + pl.prefix_cap;
  uint32_t* pk_ra = pk_a + pl.prefix_cap;
  uint32_t* pv_ra = pv_a + pl.prefix_cap;
  uint32_t* sat = at<uint32_t>(ws, pl.off_sat);
  GBB_TRY(stage_mark(kStRestTiles, 0, hs), "timing");
  GBB_TRY(launch_open_sat(d_views, n_views, split.open_bits, d_st, sat, hs), "open-tile table");
  GBB_TRY(launch_count_rest(order, count, rec, d_views, pl.VP, pl.tile_w, pl.tile_h, d_st, sat,
                            count_rest, hs),
          "rest count");
  GBB_TRY(launch_scan_u32(count_rest, nullptr, offsets_rest, pl.VP, partials, &d_st->K_rest,
                          &d_st->K_rest64, partials64, hs, chunk_owner, pl.n_chunks),
          "rest scan");
  GBB_TRY(launch_finalize_rest(offsets_rest, pl.VP, d_st, chunk_owner, hs), "rest finalize");
  ClearList clear_r;  // the rest pass's tile ranges
  clear_r.p[0] = ranges_rest;
  clear_r.n[0] = 2 * pl.total_tiles;
  GBB_TRY(launch_duplicate_rest(order, count_rest, offsets_rest, chunk_owner, rec, d_views,
                                pl.tile_w, pl.tile_h, d_st, split.open_bits, sat, pl.capacity,
                                pk_r, pv_r, clear_r, hs),
          "rest duplicate");
  GBB_TRY(launch_radix_sort(pk_r, pv_r, pk_ra, pv_ra, &d_st->n_rest, pl.capacity, pl.tile_bits,
                            hist, at<uint32_t>(ws, pl.off_digit_tot), hs),
          "rest tile sort");
  GBB_TRY(launch_ranges(pk_r, &d_st->n_rest, pl.capacity, ranges_rest, hs), "rest ranges");
  GBB_TRY(stage_mark(kStRestTiles, 1, hs), "timing");
  split.mode = kRestPass;
  GBB_TRY(stage_mark(kStBlendFwdRest, 0, hs), "timing");
  GBB_TRY(launch_blend_fwd(pl, *s, *o, d_views, n_views, rec, pv_r, ranges_rest, rgb, T_final,
                           at<uint32_t>(ws, pl.off_n_last_rest), split, tile_work, spec,
                           stats ? d_stats : nullptr, nullptr, 0, nullptr, 0, hs),
          "blend forward (rest)");
  GBB_TRY(stage_mark(kStBlendFwdRest, 1, hs), "timing");
  return GB_OK;
}

gb_status gb_render_fwd(const gb_splats* s, const gb_view* views, int32_t n_views,
                        const gb_options* o, void* ws, size_t ws_bytes, int64_t cap, float* rgb,
                        float* T_final, void* stream) {
  return render_fwd_impl(s, views, n_views, o, ws, ws_bytes, cap, rgb, T_final, false, stream);
}

gb_status gb_render_fwd_zeroing(const gb_splats* s, const gb_view* views, int32_t n_views,
                                const gb_options* o, void* ws, size_t ws_bytes, int64_t cap,
                                float* rgb, float* T_final, float* d_textures, void* stream) {
  if (!d_textures) return arg_fail("d_textures NULL");
  return render_fwd_impl(s, views, n_views, o, ws, ws_bytes, cap, rgb, T_final, false, stream,
                         true, nullptr, d_textures);
}

gb_status gb_blend_stats(const gb_splats* s, const gb_view* views, int32_t n_views,
                         const gb_options* o, void* ws, size_t ws_bytes, int64_t cap, float* rgb,
                         float* T_final, int64_t* counts, void* stream) {
  if (!counts) return arg_fail("counts_out is NULL");
  gb_status st = render_fwd_impl(s, views, n_views, o, ws, ws_bytes, cap, rgb, T_final, true,
                                 stream);
  if (st != GB_OK) return st;
  Plan pl;
  make_plan(s->P, s->N, views, n_views, o, cap, &pl);
  hipStream_t hs = reinterpret_cast<hipStream_t>(stream);
  unsigned long long h[5];
  GBB_TRY(hipMemcpyAsync(h, at<char>(ws, pl.off_stats), sizeof(h), hipMemcpyDeviceToHost, hs),
          "read stats");
  GBB_TRY(hipStreamSynchronize(hs), "sync");
  for (int i = 0; i < 5; ++i) counts[i] = (int64_t)h[i];
  return GB_OK;
}

gb_status gb_timing_enable(int32_t on) {
  g_timing.on = on != 0;
  for (int i = 0; i < kNumStages; ++i) g_timing.recorded[i] = false;
  return GB_OK;
}

gb_status gb_timing_read(float* ms, int32_t n, int32_t* n_written) {
  if (!ms || !n_written) return arg_fail("NULL argument");
  int k = 0;
  for (int i = 0; i < kNumStages && i < n; ++i, ++k) {
    ms[i] = -1.f;
    if (!g_timing.created || !g_timing.recorded[i]) continue;
    GBB_TRY(hipEventSynchronize(g_timing.ev[i][1]), "event sync");
    GBB_TRY(hipEventElapsedTime(&ms[i], g_timing.ev[i][0], g_timing.ev[i][1]), "elapsed");
  }
  *n_written = k;
  return GB_OK;
}

const char* gb_timing_stage_name(int32_t stage) {
  if (stage < 0 || stage >= kNumStages) return "";
  return kStageNames[stage];
}

gb_status gb_render_bwd(const gb_splats* s, const gb_view* views, int32_t n_views,
                        const gb_options* o, void* ws, size_t ws_bytes, int64_t cap,
                        const float* T_final, const float* d_rgb, const gb_grads* g,
                        void* stream) {
  Plan pl;
  gb_status st = check_common(s, views, n_views, o, ws, ws_bytes, cap, &pl);
  if (st != GB_OK) return st;
  if (!T_final || !d_rgb || !g) return arg_fail("T_final / d_rgb / grads NULL");
  const void* gp[] = {g->d_means, g->d_tan_u, g->d_tan_v, g->d_scales, g->d_opacity, g->d_textures};
  for (const void* p : gp)
    if (!p || !aligned(p, 4)) return arg_fail("gradient array NULL or misaligned");
  if (s->sh && (!g->d_sh || !aligned(g->d_sh, 4)))
    return arg_fail("d_sh NULL or misaligned (the splats carry SH coefficients)");
  hipStream_t hs = reinterpret_cast<hipStream_t>(stream);
  float* d_rec = at<float>(ws, pl.off_drec);
  const float4* spec = s->sh ? at<float4>(ws, pl.off_spec) : nullptr;
  float4* d_spec = s->sh ? at<float4>(ws, pl.off_dspec) : nullptr;
  GBB_TRY(stage_mark(kStBwdClear, 0, hs), "timing");
  // skipped when this workspace's forward already zeroed it while it blended
  if (!zeroed_take(ws, kZeroRec, d_rec, (int64_t)kRecGrad * pl.VP))
    GBB_TRY(launch_fill_u32(reinterpret_cast<uint32_t*>(d_rec), 0u, kRecGrad * pl.VP, hs),
            "clear d_rec");
  if (d_spec)
    GBB_TRY(launch_fill_u32(reinterpret_cast<uint32_t*>(d_spec), 0u, 4 * pl.VP, hs),
            "clear d_spec");
  const int64_t tex_values = tex_grad_values(s);
  // skipped when this workspace's forward already zeroed this array while it blended
  if (!zeroed_take(ws, kZeroTex, g->d_textures, tex_values))
    GBB_TRY(launch_fill_u32(reinterpret_cast<uint32_t*>(g->d_textures), 0u, tex_values, hs),
            "clear d_textures");
  // the backward takes the tiles with the longest blended spans (saved by the forward) first
  const uint32_t* tile_order = nullptr;
  if (pl.ordered) {
    uint32_t* ord = at<uint32_t>(ws, pl.off_tile_order);
    GBB_TRY(launch_order_tiles(at<uint32_t>(ws, pl.off_tile_work), pl.total_tiles, ord, hs),
            "tile order");
    tile_order = ord;
  }
  GBB_TRY(stage_mark(kStBwdClear, 1, hs), "timing");
  ViewDev* d_views = at<ViewDev>(ws, pl.off_views);
  const SplatRec* rec = at<SplatRec>(ws, pl.off_rec);
  const uint32_t* pv = at<uint32_t>(ws, pl.off_pair_vals);
  const PairList first{pv, at<uint32_t>(ws, pl.off_ranges), at<uint32_t>(ws, pl.off_n_last)};
  PairList rest{nullptr, nullptr, nullptr};
  const uint32_t* open_bits = nullptr;
  if (pl.split) {
    rest = PairList{pv + pl.prefix_cap, at<uint32_t>(ws, pl.off_ranges_rest),
                    at<uint32_t>(ws, pl.off_n_last_rest)};
    open_bits = at<uint32_t>(ws, pl.off_open_bits);
  }
  GBB_TRY(stage_mark(kStBlendBwd, 0, hs), "timing");
  GBB_TRY(launch_blend_bwd(pl, *s, *o, d_views, n_views, rec, first, rest, open_bits,
                           tile_order, T_final, d_rgb, d_rec, g->d_textures, spec,
                           reinterpret_cast<float*>(d_spec), hs),
          "blend backward");
  GBB_TRY(stage_mark(kStBlendBwd, 1, hs), "timing");
  GBB_TRY(stage_mark(kStPreprocessBwd, 0, hs), "timing");
  GBB_TRY(launch_preprocess_bwd(*s, d_views, n_views, at<uint32_t>(ws, pl.off_count), d_rec,
                                d_spec, *g, hs),
          "preprocess backward");
  GBB_TRY(stage_mark(kStPreprocessBwd, 1, hs), "timing");
  return GB_OK;
}

// ---- densification and pruning --------------------------------------------------------------

size_t gb_densify_work_bytes(int32_t P) { return P < 0 ? 0 : densify_work(P).total; }

gb_status gb_densify_stats(const gb_splats* s, const gb_view* views, int32_t n_views,
                           const gb_options* o, const void* ws, size_t ws_bytes, int64_t cap,
                           float* grad_accum, float* vis_count, void* stream) {
  Plan pl;
  gb_status st = check_common(s, views, n_views, o, const_cast<void*>(ws), ws_bytes, cap, &pl);
  if (st != GB_OK) return st;
  if (!grad_accum || !vis_count || !aligned(grad_accum, 4) || !aligned(vis_count, 4))
    return arg_fail("grad_accum / vis_count NULL or misaligned");
  char* base = const_cast<char*>(static_cast<const char*>(ws));
  GBB_TRY(launch_densify_stats(reinterpret_cast<const uint32_t*>(base + pl.off_count),
                               reinterpret_cast<const float*>(base + pl.off_drec), pl.P, n_views,
                               grad_accum, vis_count, reinterpret_cast<hipStream_t>(stream)),
          "densify stats");
  return GB_OK;
}

gb_status gb_densify_plan(const gb_raw_splats* src, const float* grad_accum,
                          const float* vis_count, const gb_densify_options* o, void* work,
                          size_t work_bytes, int64_t* P_new, void* stream) {
  gb_status st;
  if ((st = check_densify_plan_args(src, grad_accum, vis_count, o, P_new)) != GB_OK) return st;
  const DensifyWork w = densify_work(src->P);
  if (!work || !aligned(work, 256) || work_bytes < w.total)
    return arg_fail("densify work buffer NULL, misaligned or smaller than gb_densify_work_bytes");
  if (src->P == 0) {
    *P_new = 0;
    return GB_OK;
  }
  hipStream_t hs = reinterpret_cast<hipStream_t>(stream);
  if ((st = densify_plan_launch(src, grad_accum, vis_count, o, work, hs)) != GB_OK) return st;
  return densify_read_count(work, hs, P_new);
}

gb_status gb_densify_apply(const gb_raw_splats* src, const void* work, const float* noise,
                           float sigma, const gb_densify_options* o, const gb_raw_splats* dst,
                           const gb_row_state* states, int32_t n_states, void* stream) {
  gb_status st;
  if ((st = check_densify_apply_args(src, noise, sigma, o, dst, states, n_states)) != GB_OK)
    return st;
  if (dst->P > 2 * (int64_t)src->P) return arg_fail("dst->P exceeds twice src->P");
  if (!work || !aligned(work, 256)) return arg_fail("work NULL or misaligned");
  if (dst->P == 0) return GB_OK;
  return densify_apply_launch(src, work, noise, sigma, o, dst, dst->P, states, n_states,
                              reinterpret_cast<hipStream_t>(stream));
}

gb_status gb_densify_noalloc(const gb_raw_splats* src, const float* grad_accum,
                             const float* vis_count, const gb_densify_options* o,
                             const float* noise, float sigma, const gb_raw_splats* dst,
                             const gb_row_state* states, int32_t n_states, int64_t* P_new,
                             void* stream) {
  gb_status st;
  if ((st = check_densify_plan_args(src, grad_accum, vis_count, o, P_new)) != GB_OK) return st;
  if ((st = check_densify_apply_args(src, noise, sigma, o, dst, states, n_states)) != GB_OK)
    return st;
  if (src->P > GB_DENSIFY_NOALLOC_MAX_P)
    return arg_fail("gb_densify_noalloc: src->P exceeds GB_DENSIFY_NOALLOC_MAX_P (use "
                    "gb_densify_plan and gb_densify_apply with a work buffer)");
  if (src->P == 0) {
    *P_new = 0;
    return GB_OK;
  }
  void* work = nullptr;
  if ((st = static_densify_work(&work)) != GB_OK) return st;
  hipStream_t hs = reinterpret_cast<hipStream_t>(stream);
  if ((st = densify_plan_launch(src, grad_accum, vis_count, o, work, hs)) != GB_OK) return st;
  // the apply kernels read the output count from the work area and write at most dst->P rows
  const int64_t n_cap = dst->P < 2 * (int64_t)src->P ? dst->P : 2 * (int64_t)src->P;
  if (n_cap > 0 &&
      (st = densify_apply_launch(src, work, noise, sigma, o, dst, n_cap, states, n_states, hs)) !=
          GB_OK)
    return st;
  if ((st = densify_read_count(work, hs, P_new)) != GB_OK) return st;
  if (*P_new > dst->P) {
    g_last_error = "gb_densify_noalloc: more outputs than dst->P rows (*P_new holds the count)";
    return GB_ERR_CAPACITY;
  }
  return GB_OK;
}

gb_status gb_activate_fwd(int32_t P, const float* quats, const float* log_scales,
                          const float* opacity_logits, float* tan_u, float* tan_v, float* scales,
                          float* opacity, void* stream) {
  if (P < 0) return arg_fail("P must be >= 0");
  if (P == 0) return GB_OK;
  const void* ptrs[] = {quats, log_scales, opacity_logits, tan_u, tan_v, scales, opacity};
  for (const void* p : ptrs)
    if (!p || !aligned(p, 4)) return arg_fail("activation array NULL or misaligned");
  GBB_TRY(launch_activate_fwd(P, quats, log_scales, opacity_logits, tan_u, tan_v, scales, opacity,
                              reinterpret_cast<hipStream_t>(stream)),
          "activate forward");
  return GB_OK;
}

gb_status gb_activate_bwd(int32_t P, const float* quats, const float* log_scales,
                          const float* opacity_logits, const float* d_tan_u,
                          const float* d_tan_v, const float* d_scales, const float* d_opacity,
                          float* d_quats, float* d_log_scales, float* d_opacity_logits,
                          void* stream) {
  if (P < 0) return arg_fail("P must be >= 0");
  if (P == 0) return GB_OK;
  const void* ptrs[] = {quats, log_scales, opacity_logits, d_tan_u, d_tan_v, d_scales,
                        d_opacity, d_quats, d_log_scales, d_opacity_logits};
  for (const void* p : ptrs)
    if (!p || !aligned(p, 4)) return arg_fail("activation array NULL or misaligned");
  GBB_TRY(launch_activate_bwd(P, quats, log_scales, opacity_logits, d_tan_u, d_tan_v, d_scales,
                              d_opacity, d_quats, d_log_scales, d_opacity_logits,
                              reinterpret_cast<hipStream_t>(stream)),
          "activate backward");
  return GB_OK;
}

gb_status gb_l1_loss(int64_t n, const float* rgb, const float* target, float scale, float* loss,
                     float* d_rgb, void* stream) {
  if (n < 0) return arg_fail("n must be >= 0");
  if (!loss || !aligned(loss, 4)) return arg_fail("loss NULL or misaligned");
  const void* ptrs[] = {rgb, target, d_rgb};
  for (const void* p : ptrs)
    if (!p || !aligned(p, 16)) return arg_fail("loss array NULL or not 16-byte aligned");
  GBB_TRY(launch_l1_loss(n, rgb, target, scale, loss, d_rgb, reinterpret_cast<hipStream_t>(stream)),
          "l1 loss");
  return GB_OK;
}

gb_status gb_mse_loss(int64_t n, const float* rgb, const float* target, float scale,
                      float* loss, float* d_rgb, void* stream) {
  if (n < 0) return arg_fail("n must be >= 0");
  if (!loss || !aligned(loss, 4)) return arg_fail("loss NULL or misaligned");
  const void* ptrs[] = {rgb, target, d_rgb};
  for (const void* p : ptrs)
    if (!p || !aligned(p, 16)) return arg_fail("loss array NULL or not 16-byte aligned");
  GBB_TRY(launch_mse_loss(n, rgb, target, scale, loss, d_rgb,
                          reinterpret_cast<hipStream_t>(stream)),
          "mse loss");
  return GB_OK;
}

gb_status gb_box_filter_textures(int32_t P, int32_t N, int32_t M, const float* textures,
                                 float* out, void* stream) {
  if (P < 0) return arg_fail("P must be >= 0");
  if (N < 1 || N > 64 || M < 1 || M > N || N % M != 0)
    return arg_fail("need 1 <= M <= N <= 64 with M dividing N");
  if (P == 0) return GB_OK;
  if (!textures || !out || !aligned(textures, 4) || !aligned(out, 4))
    return arg_fail("texture arrays NULL or misaligned");
  GBB_TRY(launch_box_filter(P, N, M, textures, out, reinterpret_cast<hipStream_t>(stream)),
          "box filter");
  return GB_OK;
}

gb_status gb_rotz_only(int32_t P, float* d_quats, void* stream) {
  if (P < 0) return arg_fail("P must be >= 0");
  if (P == 0) return GB_OK;
  if (!d_quats || !aligned(d_quats, 4)) return arg_fail("d_quats NULL or misaligned");
  GBB_TRY(launch_rotz_only(P, d_quats, reinterpret_cast<hipStream_t>(stream)), "rotz only");
  return GB_OK;
}

gb_status gb_adam_step(int64_t n, float* param, const float* grad, float* m, float* v,
                       int32_t step, float lr, float beta1, float beta2, float eps,
                       uint16_t* bf16_copy, void* stream) {
  if (n < 0) return arg_fail("n must be >= 0");
  if (step < 1) return arg_fail("step must be >= 1");
  if (!(beta1 >= 0.f && beta1 < 1.f) || !(beta2 >= 0.f && beta2 < 1.f))
    return arg_fail("betas must be in [0, 1)");
  if (n == 0) return GB_OK;
  const void* ptrs[] = {param, grad, m, v};
  for (const void* p : ptrs)
    if (!p || !aligned(p, 16)) return arg_fail("Adam array NULL or not 16-byte aligned");
  if (bf16_copy && !aligned(bf16_copy, 8)) return arg_fail("bf16 copy not 8-byte aligned");
  // bias corrections in double precision
  const double c1 = 1.0 / (1.0 - std::pow((double)beta1, (double)step));
  const double c2 = 1.0 / (1.0 - std::pow((double)beta2, (double)step));
  GBB_TRY(launch_adam(n, param, grad, m, v, lr, beta1, beta2, (float)c1, (float)c2, eps, bf16_copy,
                      reinterpret_cast<hipStream_t>(stream)),
          "adam");
  return GB_OK;
}

gb_status gb_to_bf16(int64_t n, const float* src, uint16_t* dst, void* stream) {
  if (n < 0) return arg_fail("n must be >= 0");
  if (n == 0) return GB_OK;
  if (!src || !dst || !aligned(src, 4) || !aligned(dst, 2)) return arg_fail("NULL or misaligned");
  GBB_TRY(launch_to_bf16(n, src, dst, reinterpret_cast<hipStream_t>(stream)), "to bf16");
  return GB_OK;
}

gb_status gb_read_status(const void* ws, int64_t* K_out, int32_t* overflow_out,
                         int64_t* K_per_view, int32_t n_views, void* stream) {
  if (!ws || !K_out || !overflow_out) return arg_fail("NULL argument");
  if (!aligned(ws, 256)) return arg_fail("workspace not 256-byte aligned");
  hipStream_t hs = reinterpret_cast<hipStream_t>(stream);
  Status h;
  GBB_TRY(hipMemcpyAsync(&h, ws, sizeof(Status), hipMemcpyDeviceToHost, hs), "read status");
  GBB_TRY(hipStreamSynchronize(hs), "sync");
  if (K_per_view) {
    if (h.n_views < 1 || h.n_views > GB_MAX_VIEWS) return arg_fail("no forward on this workspace");
    if ((uint32_t)n_views != h.n_views)
      return arg_fail("n_views differs from the last forward on this workspace");
    char* base = const_cast<char*>(static_cast<const char*>(ws));
    unsigned long long* d_kv = reinterpret_cast<unsigned long long*>(base + h.off_view_pairs);
    GBB_TRY(launch_view_pairs(reinterpret_cast<const uint32_t*>(base + h.off_count), h.P,
                              n_views, d_kv, hs),
            "view pairs");
    unsigned long long kv[GB_MAX_VIEWS];
    GBB_TRY(hipMemcpyAsync(kv, d_kv, sizeof(unsigned long long) * (size_t)n_views,
                           hipMemcpyDeviceToHost, hs),
            "read view pairs");
    GBB_TRY(hipStreamSynchronize(hs), "sync");
    for (int v = 0; v < n_views; ++v) K_per_view[v] = (int64_t)kv[v];
  }
  *K_out = (int64_t)h.K64;
  *overflow_out = (int32_t)((h.overflow ? 1 : 0) | (h.sticky_overflow ? 2 : 0));
  // the sticky flag reports every overflow once
  if (h.sticky_overflow) {
    char* base = const_cast<char*>(static_cast<const char*>(ws));
    GBB_TRY(launch_fill_u32(reinterpret_cast<uint32_t*>(base + offsetof(Status, sticky_overflow)),
                            0u, 1, hs),
            "clear sticky overflow");
  }
  return GB_OK;
}

}  // extern "C"
