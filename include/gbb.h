/*
 * gbb.h -- C ABI of the MI355X rasterizer for textured 2D Gaussian splats
 * ("Gaussian Billboards": 2D Gaussian surfels carrying an N x N RGB colour grid).
 *
 * What the library computes (Gaussian Billboards, Sec. 3 and the supplementary Alg. 1-2):
 *   - a splat k has centre p_k, tangents t_u, t_v, scales (s_u, s_v) and opacity o_k; its
 *     tangent plane is P(u, v) = p_k + s_u t_u u + s_v t_v v (Eq. 3);
 *   - a pixel ray meets the plane at (u, v); the splat's opacity there is
 *     alpha = min(alpha_max, o_k * G_hat), G_hat = exp(-min((u^2 + v^2)/2, |x - c2|^2/(2 var_lp)))
 *     (Eq. 4 with a screen-space low-pass around the projected centre c2);
 *   - its colour is the bilinear lookup of the N x N grid C_k over [-sigma, sigma]^2 of the
 *     uv plane, border-clamped (Eq. 5, Alg. 2);
 *   - splats are composited front to back by centre depth (Eq. 2), skipping alpha < alpha_min
 *     and stopping a pixel before its transmittance would drop below t_min (Alg. 1);
 *   - the backward pass returns the gradient of sum(d_rgb * rgb) with respect to every
 *     splat parameter, including the colour grid (Alg. 1 backward, Alg. 2 adj-bilinear).
 *
 * Conventions
 *   - Every pointer in gb_splats, the rgb/T/d_rgb outputs and gb_grads is a DEVICE pointer
 *     owned by the caller; float arrays must be 4-byte aligned, the workspace 256-byte
 *     aligned. The library never allocates device memory in gb_render_fwd/gb_render_bwd.
 *   - gb_view arrays and option structs are HOST memory, read during the call only.
 *   - `stream` is a hipStream_t (NULL = the default stream). Every launch is ordered on it and
 *     no call below synchronises, except gb_count_pairs and gb_read_status, which wait for the
 *     stream. Nothing throws across the ABI and nothing aborts.
 *   - Camera: world->camera rotation R (row-major) and translation t, axes x right, y down,
 *     z forward; pinhole intrinsics fx, fy, cx, cy in pixels; pixel (i, j) has its centre at
 *     (i + 1/2, j + 1/2). Views are packed in order: view v occupies pixels
 *     [sum_{u<v} W_u H_u, ... + W_v H_v), row-major.
 *   - Splat parameters are used as given (already activated): opacity in (0, 1], scales > 0.
 *     Tangents are not renormalised.
 *   - Textures are [P][N][N][3] indexed [k][i_u][i_v][c] (i_u follows u), float32 or bfloat16.
 *     Gradients are always float32.
 */
#ifndef GBB_H_
#define GBB_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  GB_OK = 0,
  GB_ERR_ARG = 1,          /* invalid argument; nothing was launched */
  GB_ERR_HIP = 2,          /* a HIP runtime call failed */
  GB_ERR_CAPACITY = 3,     /* the (tile, splat) pair count exceeded the workspace capacity */
  GB_ERR_UNSUPPORTED = 4   /* valid but not built (e.g. texture side N outside {1,2,4,8,16},
                              N = 16 with a batch other than 4, or a batch of 4 with N < 16) */
} gb_status;

typedef enum { GB_F32 = 0, GB_BF16 = 1 } gb_dtype;

#define GB_MAX_VIEWS 256

typedef struct {
  int32_t width, height;
  float fx, fy, cx, cy;
  float R[9];    /* world -> camera rotation, row-major */
  float t[3];    /* world -> camera translation */
  float z_near;  /* splats whose centre depth is not beyond z_near are culled */
} gb_view;

typedef struct {
  int32_t P;               /* number of splats, >= 1 */
  int32_t N;               /* texture side, one of 1, 2, 4, 8, 16 (16: batch and batch_bwd 4);
                              with tex_side: the largest side any splat may have, 8 or 16 */
  int32_t tex_dtype;       /* gb_dtype of `textures` */
  const float* means;      /* [P][3] */
  const float* tan_u;      /* [P][3] */
  const float* tan_v;      /* [P][3] */
  const float* scales;     /* [P][2] (s_u, s_v) */
  const float* opacity;    /* [P] */
  const void* textures;    /* [P][N][N][3], float32 or bfloat16 bit patterns */
  int32_t sh_degree;       /* degree D in 0..3 of the view-dependent colour term (ignored when
                              sh is NULL) */
  const float* sh;         /* NULL, or [P][(D+1)^2][3] float32 spherical-harmonic coefficients:
                              the diffuse-specular split of Sec. 4.2. Splat k's colour becomes
                              bilinear(C_k, u, v) + sum_j Y_j(dir) sh[k][j], dir the unit vector
                              from the camera centre -R^T t to p_k, Y_j the real harmonics of
                              index j = l^2 + l + m, each (-1)^m times the usual real harmonic
                              (sign convention of 3D Gaussian splatting). */
  /* Colour grids of several sides in one call (NULL tex_side: every grid is N x N, packed as
   * [P][N][N][3]). With tex_side, splat k's grid has its own side n_k = tex_side[k], any value
   * in [1, N] (values outside are clamped to it), spans the same [-sigma, sigma]^2 of the uv
   * plane with its texel centres corner-aligned (Sec. 3.2, Alg. 2 with n_k in place of N), and
   * occupies texels [tex_offset[k], tex_offset[k] + n_k^2) of `textures`, each texel 3 values
   * [i_u][i_v][c]; the grids may lie anywhere in the array, which holds n_texels texels (the
   * gradient d_textures has the same layout and size and is written over all n_texels). */
  const int32_t* tex_side;   /* NULL or [P] (device) */
  const int64_t* tex_offset; /* [P] (device), required with tex_side */
  int64_t n_texels;          /* texels in `textures` with tex_side (>= 1), else ignored */
} gb_splats;

typedef struct {
  float sigma;        /* half extent of the colour grid in uv (paper default 0.5) */
  float alpha_min;    /* skip threshold; >= 1/255 for the tile bound to hold (below it every
                         splat covers the whole image) */
  float alpha_max;    /* opacity clamp, e.g. 0.99; 1 switches it off */
  float t_min;        /* early-termination transmittance, e.g. 1e-4; 0 switches it off */
  float lowpass_var;  /* variance of the screen-space low-pass in px^2, e.g. 0.5; any value > 0 (the
                         tile bound of the low-pass disk is 2.36 px up to 0.5, else
                         3.34 sqrt(lowpass_var)) */
  float bg[3];        /* background colour composited with the final transmittance */
  int32_t tile_w;     /* tile width in px: 8, 16 or 32 */
  int32_t tile_h;     /* tile height in px: 8, 16 or 32; tile_w * tile_h <= 256 */
  int32_t batch;      /* splats staged in LDS per forward batch: 0 = default (4 for N = 16,
                         16 for N = 8, 32 for N = 4, else 64), or 8, 16, 32, 64 (N < 16), 4
                         (N = 16, its only batch) */
  int32_t batch_bwd;  /* splats staged in LDS per backward batch: 0 = default (4 for N = 16,
                         8 for N = 8, else 32), or 8, 16, 32 (N < 16), 4 (N = 16, its only
                         batch) */
  int32_t prefix_pairs_per_tile;
                      /* depth-prefix split. The first pass renders the longest prefix of the
                         depth order whose pairs fit this many pairs per tile (0 = default 1024);
                         a second pass renders the remaining records on the tiles where some
                         pixel is still open (not stopped by t_min). Results are those of one
                         pass over all pairs. -1 = a single pass over all pairs. */
  int32_t tile_order; /* order in which workgroups take tiles in the blend backward: 0 = default
                         (1), 1 = most work first (ranked on the device by the pair span each
                         tile blended in the forward), -1 = fixed bands of neighbouring tiles
                         per XCD (the forward always uses these). Results are the same either
                         way, up to the order of the backward's float atomics. */
} gb_options;

/* Output gradients (device, float32, overwritten -- not accumulated). */
typedef struct {
  float* d_means;     /* [P][3] */
  float* d_tan_u;     /* [P][3] */
  float* d_tan_v;     /* [P][3] */
  float* d_scales;    /* [P][2] */
  float* d_opacity;   /* [P] */
  float* d_textures;  /* [P][N][N][3] float32, or with tex_side [n_texels][3] laid out as the
                         splats' textures */
  float* d_sh;        /* [P][(D+1)^2][3] float32; required when splats->sh != NULL, else
                         ignored */
} gb_grads;

/* Byte offsets of the workspace sections that tests and tools may read back. */
typedef struct {
  size_t total_bytes;
  size_t status;      /* uint32 pair count K (mod 2^32), pairs of the first pass, overflow flag,
                         records in the depth prefix; uint64 exact pair count; uint32 pairs of
                         the rest pass, uint32 32-bit total of the rest pass, uint64 exact pairs
                         of the rest pass; then internal fields (see gb_read_status) */
  size_t depth_key;   /* uint32[V*P]: float bits of the centre depth, 0xFFFFFFFF if culled */
  size_t tile_count;  /* uint32[V*P]: tiles covered by record v*P+k */
  size_t records;     /* 96-byte record per (view, splat): 19 floats of blend geometry, then
                         int32 i0 | i1 << 16, int32 j0 | j1 << 16 (inclusive pixel rectangle,
                         valid if the tile count is > 0), int32 splat, int32 view, pad */
  size_t order;       /* uint32[V*P]: records sorted by (depth, record index) */
  size_t pair_keys;   /* uint32[]: sorted global tile index of each pair of the first (or only)
                         pass */
  size_t pair_vals;   /* uint32[]: record index v*P+k of each pair of the first pass */
  size_t ranges;      /* uint32[total tiles][2]: [start, end) of each tile's first-pass pairs */
  size_t n_last;      /* uint32[sum HW]: one past the last first-pass pair blended at each
                         pixel */
  int64_t pair_capacity;
  int64_t total_tiles;
  int64_t prefix_capacity;  /* pair slots of the first pass with the split (0 without) */
  size_t pair_keys_rest;    /* rest pass (with the split): pairs, ranges and n_last as above */
  size_t pair_vals_rest;
  size_t ranges_rest;
  size_t n_last_rest;
  size_t open_tiles;        /* uint32[ceil(tiles / 32)]: bit t set if tile t had an open pixel
                               after the first pass */
  size_t tile_order;        /* with work-ordered tiles (else 0): uint32[total tiles], the tile
                               taken by each workgroup of the backward */
  size_t tile_work;         /* with work-ordered tiles (else 0): uint32[total tiles], the
                               tile's blended span over both passes (the backward's cost) */
} gb_layout;

/* Workspace layout for P splats of texture side N over n_views views with room for
 * `pair_capacity` (tile, splat) pairs. Pure host computation; no device access.
 * Returns GB_ERR_ARG on invalid sizes or options. */
gb_status gb_workspace_layout(int32_t P, int32_t N, const gb_view* views, int32_t n_views,
                              const gb_options* opts, int64_t pair_capacity, gb_layout* out);

/* Runs the per-splat preprocess (key stage: depth, screen rectangle, tile count) for every
 * (view, splat) and returns the total pair count K in *K_out. The workspace must be laid out
 * for the same arguments (any capacity). Synchronises `stream`. Forgets an earlier overflow
 * on this workspace (see gb_render_fwd): the caller is re-planning with the exact count. */
gb_status gb_count_pairs(const gb_splats* splats, const gb_view* views, int32_t n_views,
                         const gb_options* opts, void* workspace, size_t ws_bytes,
                         int64_t pair_capacity, int64_t* K_out, void* stream);

/* Forward render of all views (Alg. 1 forward):
 *   rgb     [sum HW][3] float32 (device)  composited colour, background included;
 *   T_final [sum HW]    float32 (device)  transmittance after the last blended splat.
 * The workspace keeps what gb_render_bwd needs until the next forward on it (the blend
 * workgroups also clear the workspace's per-record gradient sums for that backward, which then
 * skips the clear; a second backward of the same forward clears them itself).
 * Capacity: if the pair count exceeds `pair_capacity`, the overflow flag is set on the device,
 * every later stage of this call does nothing and the images are background; gb_read_status
 * reports it. The count and flag of every forward are also stored, without synchronising,
 * in host-mapped memory kept per workspace address: a later gb_render_fwd on the same
 * workspace whose `pair_capacity` is below the pair count of an earlier forward that
 * overflowed (and has completed on the device) returns GB_ERR_CAPACITY before launching
 * anything; with a capacity that fits that count (re-planned) it runs. The total number of
 * pixels of all views must be below 2^31 (GB_ERR_ARG). */
gb_status gb_render_fwd(const gb_splats* splats, const gb_view* views, int32_t n_views,
                        const gb_options* opts, void* workspace, size_t ws_bytes,
                        int64_t pair_capacity, float* rgb, float* T_final, void* stream);

/* gb_render_fwd that also zeroes d_textures, the texture-gradient array that the next
 * gb_render_bwd on `workspace` will be given (its full size: [P][N][N][3], or [n_texels][3]
 * with tex_side). The forward's blend workgroups store the zeros while they blend, which is
 * bound by arithmetic and leaves HBM mostly idle, and that gb_render_bwd then skips its own
 * clear of the array. The caller must not write d_textures between the two calls. The
 * backward clears as usual when given another array, or after any other forward on the
 * workspace. Errors as gb_render_fwd, and GB_ERR_ARG for a NULL or misaligned d_textures. */
gb_status gb_render_fwd_zeroing(const gb_splats* splats, const gb_view* views, int32_t n_views,
                                const gb_options* opts, void* workspace, size_t ws_bytes,
                                int64_t pair_capacity, float* rgb, float* T_final,
                                float* d_textures, void* stream);

/* Backward of the last gb_render_fwd on `workspace` with the same splats, views, options and
 * capacity (Alg. 1 backward, Alg. 2 adj-bilinear). T_final is the forward's output;
 * d_rgb: [sum HW][3] float32 device adjoint of rgb. Writes every field of *grads (all must be
 * non-NULL). */
gb_status gb_render_bwd(const gb_splats* splats, const gb_view* views, int32_t n_views,
                        const gb_options* opts, void* workspace, size_t ws_bytes,
                        int64_t pair_capacity, const float* T_final, const float* d_rgb,
                        const gb_grads* grads, void* stream);

/* Waits for `stream`, then reports the last forward on `workspace`:
 *   *K_out        exact (tile, splat) pair count of all views;
 *   *overflow_out bit 0: the last forward overflowed its capacity; bit 1: some forward since
 *                 the previous gb_read_status on this workspace overflowed (this sticky bit is
 *                 cleared by the call, so each overflow is reported once);
 *   K_per_view    (nullable) [n_views] pair count of each view; n_views must equal the last
 *                 forward's (GB_ERR_ARG otherwise, and if no forward ran on the workspace).
 * Launches one small reduction kernel when K_per_view is given. */
gb_status gb_read_status(const void* workspace, int64_t* K_out, int32_t* overflow_out,
                         int64_t* K_per_view, int32_t n_views, void* stream);

/* Work counts of one forward, for measurement: runs gb_render_fwd with counting enabled in the
 * blend kernels and waits for the stream. counts_out[0] = (pixel, splat) pairs blended,
 * [1] = pixels stopped by the t_min rule, [2] = (pixel, splat) evaluations performed by the
 * waves (64 per wave and splat evaluated), [3] = (tile, splat) pairs staged into LDS,
 * [4] = the part of [0] blended by the rest pass of the depth-prefix split. */
gb_status gb_blend_stats(const gb_splats* splats, const gb_view* views, int32_t n_views,
                         const gb_options* opts, void* workspace, size_t ws_bytes,
                         int64_t pair_capacity, float* rgb, float* T_final, int64_t* counts_out,
                         void* stream);

/* Stage timing for measurement. While enabled, gb_render_fwd and gb_render_bwd record a HIP
 * event on their stream before and after each stage (events are created on first use).
 * gb_timing_read waits for the events of the last forward and backward and writes the elapsed
 * milliseconds of up to n stages to ms_out (stage names from gb_timing_stage_name). */
gb_status gb_timing_enable(int32_t on);
gb_status gb_timing_read(float* ms_out, int32_t n, int32_t* n_written);
const char* gb_timing_stage_name(int32_t stage);

/* ---- Training glue (Sec. 3.3: the splats are trained with an image loss and Adam) ---------
 * All arrays are device float32 unless stated, caller-owned, and stream-ordered on `stream`;
 * nothing is allocated. Errors: GB_ERR_ARG for NULL or misaligned pointers or negative sizes
 * (checked before any launch), GB_ERR_HIP for launch failures. */

/* Parameter activations of 2D Gaussian splats: quats [P][4] = (w, x, y, z), any non-zero
 * length -> tan_u, tan_v [P][3], the first two columns of the rotation of q / |q|;
 * log_scales [P][2] -> scales = exp(log_scales); opacity_logits [P] -> opacity = 1 / (1 +
 * exp(-logit)). */
gb_status gb_activate_fwd(int32_t P, const float* quats, const float* log_scales,
                          const float* opacity_logits, float* tan_u, float* tan_v, float* scales,
                          float* opacity, void* stream);

/* Backward of gb_activate_fwd: from dL/d(tan_u, tan_v, scales, opacity) (layouts as above)
 * writes dL/d(quats, log_scales, opacity_logits) (overwritten, not accumulated). */
gb_status gb_activate_bwd(int32_t P, const float* quats, const float* log_scales,
                          const float* opacity_logits, const float* d_tan_u,
                          const float* d_tan_v, const float* d_scales, const float* d_opacity,
                          float* d_quats, float* d_log_scales, float* d_opacity_logits,
                          void* stream);

/* L1 image loss over n values: *loss (one device float) = scale * sum |rgb - target|, and
 * d_rgb = scale * sign(rgb - target) (0 where equal). rgb, target and d_rgb 16-byte aligned. */
gb_status gb_l1_loss(int64_t n, const float* rgb, const float* target, float scale,
                     float* loss, float* d_rgb, void* stream);

/* Squared-error image loss over n values (Sec. 4: single images are fitted with an MSE loss):
 * *loss (one device float) = scale * sum (rgb - target)^2 and d_rgb = 2 scale (rgb - target);
 * scale = 1 / n gives the mean. rgb, target and d_rgb 16-byte aligned. */
gb_status gb_mse_loss(int64_t n, const float* rgb, const float* target, float scale,
                      float* loss, float* d_rgb, void* stream);

/* Box filter of colour grids (Sec. 4: the fitted grids are rendered downsampled to 2 x 2 or to
 * one colour to show that the image lives in them): textures [P][N][N][3] -> out [P][M][M][3],
 * each output texel the mean of the (N / M) x (N / M) input texels it covers. M divides N,
 * 1 <= M <= N <= 64. `out` must not overlap `textures`. */
gb_status gb_box_filter_textures(int32_t P, int32_t N, int32_t M, const float* textures,
                                 float* out, void* stream);

/* Restricts splat rotations to the Z axis (Sec. 4: for single-image fitting the splats only
 * rotate about the camera axis, so that they stay in the image plane): zeroes the x and y
 * components of d_quats [P][4] = d(w, x, y, z) in place. With quaternions initialised as
 * (w, 0, 0, z), Adam then keeps them in that form. */
gb_status gb_rotz_only(int32_t P, float* d_quats, void* stream);

/* One Adam step (Kingma and Ba) on n parameters: m = b1 m + (1 - b1) g, v = b2 v + (1 - b2) g^2,
 * param -= lr (m / (1 - b1^step)) / (sqrt(v / (1 - b2^step)) + eps), in place; step >= 1.
 * With bf16_copy != NULL the updated parameters are also written rounded to bfloat16 (nearest,
 * ties to even) as uint16 bit patterns (the render copy of BF16 textures). param, grad, m, v
 * 16-byte aligned, bf16_copy 8-byte aligned. */
gb_status gb_adam_step(int64_t n, float* param, const float* grad, float* m, float* v,
                       int32_t step, float lr, float beta1, float beta2, float eps,
                       uint16_t* bf16_copy, void* stream);

/* dst[i] = src[i] rounded to bfloat16 (nearest, ties to even) as uint16 bit patterns: the
 * initial render copy of float32 textures. */
gb_status gb_to_bf16(int64_t n, const float* src, uint16_t* dst, void* stream);

/* ---- Densification and pruning (Sec. 4.2 trains with the default adaptive density control
 * of Gaussian splatting; the colour grids are split as described at gb_densify_apply) ------ */

typedef struct {
  float grad_threshold;  /* a splat whose mean screen-translation gradient norm (below) is at
                            least this is densified */
  float dense_scale;     /* a densified splat with max(s_u, s_v) <= dense_scale is cloned,
                            otherwise split */
  float min_opacity;     /* outputs (kept splats, clone copies, split children) with opacity
                            below this are pruned */
  float max_scale;       /* > 0: outputs whose largest scale exceeds it are pruned; 0 = off */
  float split_shrink;    /* scales of split children = parent's / split_shrink (e.g. 1.6), >= 1 */
} gb_densify_options;

/* Raw (pre-activation) training parameters, device float32, caller-owned. */
typedef struct {
  int32_t P;               /* splats */
  int32_t N;               /* colour-grid side */
  int32_t sh_coef;         /* spherical-harmonic coefficients per channel (0 = none) */
  float* means;            /* [P][3] */
  float* quats;            /* [P][4] (w, x, y, z), any non-zero length */
  float* log_scales;       /* [P][2] */
  float* opacity_logits;   /* [P] */
  float* textures;         /* [P][N][N][3] float32 (the master copy) */
  float* sh;               /* [P][sh_coef][3] or NULL */
} gb_raw_splats;

/* Per-splat rows of optimiser state (e.g. an Adam moment of one parameter group): `width`
 * floats per splat; the rows of kept splats are copied, those of new splats are zero. */
typedef struct {
  const float* src;
  float* dst;
  int32_t width;
} gb_row_state;

/* Densification statistic of the last gb_render_bwd on `workspace` (same arguments as that
 * call): for every splat k and every view where it is visible, grad_accum[k] += the norm of
 * the gradient of the loss with respect to a translation of the splat's footprint in the
 * image (pixels), and vis_count[k] += 1. Both [P] float32 device arrays accumulate across
 * calls (the caller zeroes them). */
gb_status gb_densify_stats(const gb_splats* splats, const gb_view* views, int32_t n_views,
                           const gb_options* opts, const void* workspace, size_t ws_bytes,
                           int64_t pair_capacity, float* grad_accum, float* vis_count,
                           void* stream);

/* Bytes of the work buffer (256-byte aligned device memory) of gb_densify_plan/apply. */
size_t gb_densify_work_bytes(int32_t P);

/* Decides, per splat of `src`, from max(exp(log_scales)), sigmoid(logit) and the mean
 * statistic grad_accum / vis_count (0 where vis_count is 0): prune, keep, clone (the splat and
 * an identical copy right after it) or split (two children in its place); outputs are pruned
 * as described in gb_densify_options. Writes the outputs' parent map into `work` and returns
 * their number in *P_new. Synchronises `stream`. */
gb_status gb_densify_plan(const gb_raw_splats* src, const float* grad_accum,
                          const float* vis_count, const gb_densify_options* opts, void* work,
                          size_t work_bytes, int64_t* P_new, void* stream);

/* Writes the planned outputs into `dst` (dst->P = the plan's P_new, same N and sh_coef as src;
 * no overlap with src). Kept splats and clone copies copy their parent's parameters. Split
 * child c in {0, 1} of parent k has centre p + s_u z0 t_u + s_v z1 t_v with (z0, z1) =
 * noise[k][c][0..1] (noise: [src->P][2][2] float32 device, the caller's N(0, 1) draws; t_u, t_v
 * the first two columns of the rotation of q / |q|), log-scales minus log(split_shrink), the
 * parent's quaternion, logit and SH rows, and a colour grid resampled from the parent's: the
 * child's texel (i, j) lies at child uv (u_i, v_j) = (-sigma + 2 sigma i / (N - 1), ...) (0 if
 * N = 1), i.e. at parent uv (z0 + u_i / split_shrink, z1 + v_j / split_shrink), where it takes
 * the parent's bilinear, border-clamped colour (Alg. 2). So a constant grid stays constant.
 * `states` (n_states rows arrays) are carried along as gb_row_state describes. */
gb_status gb_densify_apply(const gb_raw_splats* src, const void* work, const float* noise,
                           float sigma, const gb_densify_options* opts, const gb_raw_splats* dst,
                           const gb_row_state* states, int32_t n_states, void* stream);

/* Most splats gb_densify_noalloc takes (its static work area holds about 21 MB per GPU). */
#define GB_DENSIFY_NOALLOC_MAX_P (1 << 20)

/* For callers that cannot allocate device memory (tight training loops, harnesses that forbid
 * allocation): gb_densify_plan followed by gb_densify_apply in one call, with the plan's work
 * buffer held in a library-owned static device array instead of a caller buffer. Each GPU the
 * library runs on holds its own copy of that array (about 21 MB) until the process ends; the
 * call allocates nothing.
 *   src, grad_accum, vis_count, opts, noise, sigma, states: as for gb_densify_plan/apply;
 *   dst: output arrays with room for dst->P rows (2 * src->P always suffice); the first
 *        min(*P_new, dst->P) rows are written;
 *   *P_new: the number of outputs.
 * Errors: GB_ERR_ARG (nothing launched) for the argument errors of gb_densify_plan/apply and
 * for src->P > GB_DENSIFY_NOALLOC_MAX_P; GB_ERR_CAPACITY if *P_new > dst->P (the rows that fit
 * are written). Synchronises `stream`. All calls on one GPU share the work area: calls that
 * overlap on one GPU (other streams or threads) race and must be serialised by the caller. */
gb_status gb_densify_noalloc(const gb_raw_splats* src, const float* grad_accum,
                             const float* vis_count, const gb_densify_options* opts,
                             const float* noise, float sigma, const gb_raw_splats* dst,
                             const gb_row_state* states, int32_t n_states, int64_t* P_new,
                             void* stream);

/* Fills *out with the default options (sigma 0.5, alpha_min 1/255, alpha_max 0.99,
 * t_min 1e-4, lowpass_var 0.5, black background, 16 x 16 tiles, default batch). */
void gb_default_options(gb_options* out);

const char* gb_status_string(gb_status status);

/* Last HIP error text recorded by the library in this process (empty if none). */
const char* gb_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* GBB_H_ */
