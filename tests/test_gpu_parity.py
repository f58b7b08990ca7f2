"""Parity of the HIP rasterizer (through the C ABI) against the FP64 oracle.

Bars: key stage, pair keys/values and tile ranges bit-exact; images and final transmittance
within 1e-5 max-abs over pixels the oracle does not flag as near a decision threshold; each
gradient tensor within 1e-3 relative L2 of the oracle's analytic gradient.
"""
import math

import numpy as np
import pytest

import scenegen as sg
from oracle import gb_oracle as O

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

IMG_TOL = 1e-5
GRAD_TOL = 1e-3
# Pixels where the oracle finds a decision within its flag threshold (alpha vs alpha_min within
# 1e-5 relative, T(1 - alpha) vs t_min within 1e-4) are not held to the oracle's own outcome:
# each must match one of the outcomes of its in-band decisions taken either way (or stay within
# the oracle's bound for them). Their count is only a sanity check that the flagging does not
# swallow the image: 1 % of the pixels plus a few, since every evaluated splat is one
# alpha-versus-alpha_min decision and the share of flagged pixels grows with depth complexity
# (a 64 x 64 crop of the 1M-splat 1080p scene flags about 8 of 4096 pixels).
MAX_FLAGGED_FRACTION = 1e-2


def _require_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.fixture(scope="module")
def gb():
    _require_gpu()
    import paper_2412_12734_amd as gb
    gb.load()  # fails loudly if the HIP library is missing
    return gb


def gpu_opts(opts: O.Options, batch=0, batch_bwd=0, prefix=0):
    import paper_2412_12734_amd as gb
    return gb.Options(sigma=opts.sigma, alpha_min=opts.alpha_min, alpha_max=opts.alpha_max,
                      t_min=opts.t_min, lowpass_var=opts.lowpass_var, bg=tuple(opts.bg),
                      tile_w=opts.tile_w, tile_h=opts.tile_h, batch=batch, batch_bwd=batch_bwd,
                      prefix_pairs_per_tile=prefix)


def run_gpu(gb, scene, views, opts, tex_bf16=False, batch=0, capacity=None, batch_bwd=0,
            prefix=0):
    sp = gb.Splats.from_numpy(scene, tex_bf16=tex_bf16)
    rast = gb.Rasterizer(views, gpu_opts(opts, batch, batch_bwd, prefix))
    rast.plan(sp, capacity)
    rgb, T = rast.forward(sp)
    torch.cuda.synchronize()
    return rast, sp, rgb, T


def image_crop(arr, base, W, H, crop, ch=3):
    x0, y0, w, h = crop
    a = arr[base:base + W * H].reshape((H, W, ch) if ch else (H, W))
    return a[y0:y0 + h, x0:x0 + w]


def assert_flagged_pixels(g_rgb, g_T, ref: O.RenderResult, flagged, scene, view, opts):
    """Every flagged pixel must equal, within the image bar, one of the outcomes the oracle
    enumerates for its in-band decisions taken either way; with more in-band decisions than
    the enumeration takes, its colour must stay within the oracle's bound for them."""
    worst = 0.0
    for j, i in zip(*np.nonzero(flagged)):
        outs = O.flagged_outcomes(scene, view, opts, ref, int(j), int(i))
        if outs is not None:
            best = min(max(float(np.abs(g_rgb[j, i] - rgb).max()), abs(float(g_T[j, i]) - T))
                       for rgb, T in outs)
            assert best <= IMG_TOL, (f"flagged pixel (x={i + ref.crop[0]}, y={j + ref.crop[1]}) "
                                     f"matches none of {len(outs)} outcomes: {best:.3g}")
            worst = max(worst, best)
        else:
            b = O.flagged_bound(scene, ref, int(j), int(i), opts.bg)
            assert float(np.abs(g_rgb[j, i] - ref.rgb[j, i]).max()) <= b + IMG_TOL
    return worst


def assert_image_parity(rgb_gpu, T_gpu, ref: O.RenderResult, base, W, H, scene, view, opts,
                        max_flagged=MAX_FLAGGED_FRACTION):
    crop = ref.crop
    g_rgb = image_crop(rgb_gpu, base, W, H, crop).astype(np.float64)
    g_T = image_crop(T_gpu, base, W, H, crop, ch=0).astype(np.float64)
    ok = ~O.image_flags(ref)
    flagged = int((~ok).sum())
    assert flagged <= max_flagged * ok.size + 4, f"{flagged} flagged pixels"
    d = np.where(ok[..., None], np.abs(g_rgb - ref.rgb), 0.0)
    dT = np.where(ok, np.abs(g_T - ref.T_final), 0.0)
    if d.max(initial=0) > IMG_TOL or dT.max(initial=0) > IMG_TOL:
        j, i, c = np.unravel_index(np.argmax(d), d.shape)
        print(f"worst pixel (x={i + crop[0]}, y={j + crop[1]}, c={c}): gpu {g_rgb[j, i]} oracle "
              f"{ref.rgb[j, i]} T gpu {g_T[j, i]} oracle {ref.T_final[j, i]} blended "
              f"{ref.n_blended[j, i]} terminated {ref.terminated[j, i]} alpha_gap "
              f"{ref.alpha_gap[j, i]:.3g} t_gap {ref.t_gap[j, i]:.3g}")
    assert d.max(initial=0) <= IMG_TOL, f"max image error {d.max()}"
    assert dT.max(initial=0) <= IMG_TOL, f"max transmittance error {dT.max()}"
    fl_err = assert_flagged_pixels(g_rgb, g_T, ref, ~ok, scene, view, opts)
    return max(float(d.max(initial=0)), fl_err), flagged


# --- key stage, pairs, ranges: bit-exact --------------------------------------------------
def check_tiling(gb, scene, views, opts):
    # one pass over all pairs: the pair arrays then hold every (tile, record) pair
    rast, sp, rgb, T = run_gpu(gb, scene, views, opts, prefix=-1)
    P, V = scene.P, len(views)
    depth = rast.section("depth_key", V * P, torch.int32).cpu().numpy().view(np.uint32)
    count = rast.section("tile_count", V * P, torch.int32).cpu().numpy().view(np.uint32)
    recs = rast.section("records", V * P * 24, torch.int32).cpu().numpy().reshape(V * P, 24)
    for v, view in enumerate(views):
        ks = O.key_stage(scene, view, opts)
        sl = slice(v * P, (v + 1) * P)
        vis = ks["visible"]
        want_key = np.where(vis, ks["depth"].view(np.uint32), np.uint32(0xFFFFFFFF))
        np.testing.assert_array_equal(depth[sl], want_key)
        np.testing.assert_array_equal(count[sl], ks["count"].astype(np.uint32))
        rx, ry = recs[sl, 19], recs[sl, 20]
        i0, i1 = rx & 0xFFFF, rx >> 16
        j0, j1 = ry & 0xFFFF, ry >> 16
        got = np.stack([i0, i1, j0, j1], 1)[vis]
        np.testing.assert_array_equal(got, ks["rect"][vis])
    keys, vals, ranges = O.tile_pairs(scene, views, opts)
    K, over = rast.status()
    assert not over and K == keys.size
    gk = rast.section("pair_keys", K, torch.int32).cpu().numpy().view(np.uint32)
    gv = rast.section("pair_vals", K, torch.int32).cpu().numpy().view(np.uint32)
    np.testing.assert_array_equal(gk, keys)
    np.testing.assert_array_equal(gv, vals)
    gr = rast.section("ranges", 2 * ranges.shape[0], torch.int32).cpu().numpy().view(np.uint32)
    np.testing.assert_array_equal(gr.reshape(-1, 2).astype(np.int64), ranges)
    return rast, rgb, T


def test_tiling_bit_exact_config1(gb):
    scene, views = sg.config("C1")
    check_tiling(gb, scene, views, O.Options())


@pytest.mark.parametrize("tile", [(8, 8), (16, 8), (8, 16), (16, 16)])
def test_tiling_bit_exact_multiview_tile_shapes(gb, tile):
    scene = sg.make_scene(5, 3000, -1.5, 1.5, 0.01, 0.3, 2)
    views = [sg.look_at_view((0.5, 0.3, -3.0), 97, 61), sg.look_at_view((-2.0, 1.0, -2.0), 64, 80),
             sg.look_at_view((0.0, 3.0, 0.1), 33, 17)]
    check_tiling(gb, scene, views, O.Options(tile_w=tile[0], tile_h=tile[1]))


def test_tiling_bit_exact_three_pass_tile_sort(gb):
    """Three 1080p views with 8x8 tiles: 97,200 tiles need 17 key bits (three radix passes)."""
    scene = sg.make_scene(8, 1500, -4.0, 4.0, 0.01, 0.05, 1)
    views = sg.orbit_views(4, 3, 8.0, [(1920, 1080)])
    rast, rgb, T = check_tiling(gb, scene, views, O.Options(tile_w=8, tile_h=8))
    assert rast.layout.total_tiles == 3 * 240 * 135


# --- images -------------------------------------------------------------------------------
def test_image_parity_config1_full_frame(gb):
    scene, views = sg.config("C1")
    opts = O.Options()
    rast, sp, rgb, T = run_gpu(gb, scene, views, opts)
    ref = O.render(scene, views[0], opts)
    err, flagged = assert_image_parity(rgb.cpu().numpy(), T.cpu().numpy(), ref, 0, 128, 128,
                                       scene, views[0], opts)
    print(f"config1 image max err {err:.3g}, flagged {flagged}")


@pytest.mark.parametrize("seed", range(6))
def test_image_parity_tiny_scenes(gb, seed):
    rng = np.random.default_rng(seed)
    P = int(rng.integers(1, 11))
    N = [1, 2, 4, 8][seed % 4]
    scene = sg.make_scene(100 + seed, P, -0.5, 0.5, 0.03, 0.4, N)
    W, H = int(rng.integers(16, 65)), int(rng.integers(16, 65))
    view = sg.look_at_view(rng.standard_normal(3) * 0.5 + np.array([0, 0, -2.5]), W, H)
    tile = [(16, 16), (8, 8), (16, 8), (8, 16)][seed % 4]
    bg = tuple(rng.uniform(0, 1, 3))
    opts = O.Options(tile_w=tile[0], tile_h=tile[1], bg=bg)
    rast, sp, rgb, T = run_gpu(gb, scene, [view], opts)
    ref = O.render(scene, view, opts)
    assert_image_parity(rgb.cpu().numpy(), T.cpu().numpy(), ref, 0, W, H, scene, view, opts)


@pytest.mark.parametrize("W,H", [(1, 1), (1, 37), (41, 2), (7, 5), (17, 9)])
def test_degenerate_view_sizes(gb, W, H):
    """Views narrower or lower than one tile, down to a single pixel: partial tiles, ragged
    wave blocks and lanes outside the view."""
    scene = sg.make_scene(77, 60, -0.4, 0.4, 0.05, 0.5, 4)
    view = sg.look_at_view((0.05, -0.02, -2.0), W, H)
    opts = O.Options()
    rast, sp, rgb, T = run_gpu(gb, scene, [view], opts)
    ref = O.render(scene, view, opts)
    assert_image_parity(rgb.cpu().numpy(), T.cpu().numpy(), ref, 0, W, H, scene, view, opts)
    check_grads(gb, scene, view, opts, (0, 0, W, H), seed=W * 100 + H)


def test_image_parity_thresholds_off(gb):
    scene = sg.make_scene(9, 6, -0.4, 0.4, 0.05, 0.3, 4)
    view = sg.look_at_view((0.1, 0.2, -2.0), 40, 30)
    opts = O.Options(alpha_min=0.0, t_min=0.0, alpha_max=1.0, bg=(0.3, 0.2, 0.1))
    rast, sp, rgb, T = run_gpu(gb, scene, [view], opts)
    ref = O.render(scene, view, opts)
    assert_image_parity(rgb.cpu().numpy(), T.cpu().numpy(), ref, 0, 40, 30, scene, view, opts)


def test_image_parity_config2_crops(gb):
    scene, views = sg.config("C2")
    opts = O.Options()
    rast, sp, rgb, T = run_gpu(gb, scene, views, opts)
    rgb, T = rgb.cpu().numpy(), T.cpu().numpy()
    for crop in [(368, 368, 64, 64), (0, 0, 48, 40), (760, 750, 40, 50)]:
        ref = O.render(scene, views[0], opts, crop=crop)
        assert_image_parity(rgb, T, ref, 0, 800, 800, scene, views[0], opts)


# --- gradients ------------------------------------------------------------------------------
def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30))


def check_grads(gb, scene, view, opts, crop, seed=0, tex_bf16=False, batch=0, batch_bwd=0,
                prefix=0):
    rast, sp, rgb, T = run_gpu(gb, scene, [view], opts, tex_bf16=tex_bf16, batch=batch,
                               batch_bwd=batch_bwd, prefix=prefix)
    ref = O.render(scene, view, opts, crop=crop, keep_saved=True)
    W, H = view.width, view.height
    g_full = sg.make_dl_drgb(seed, [view]).reshape(H, W, 3)
    x0, y0, w, h = crop
    mask = np.zeros((H, W), dtype=bool)
    mask[y0:y0 + h, x0:x0 + w] = ~O.grad_flags(ref)
    g_full = np.where(mask[..., None], g_full, 0.0).astype(np.float32)
    g_crop = g_full[y0:y0 + h, x0:x0 + w].reshape(-1, 3).astype(np.float64)
    ref_g = O.render_backward(scene, view, opts, ref, g_crop)
    d_rgb = torch.from_numpy(g_full.reshape(-1, 3)).cuda()
    grads = rast.backward(sp, T, d_rgb)
    torch.cuda.synchronize()
    errs, p999 = {}, {}
    names = ("means", "tan_u", "tan_v", "scales", "opacity", "textures")
    if scene.sh is not None:
        names = names + ("sh",)
    for name in names:
        got = grads[name].cpu().numpy().astype(np.float64)
        want = getattr(ref_g, name)
        if isinstance(want, list):  # grids of several sides: packed in splat order
            want = np.concatenate([np.asarray(w).reshape(-1, 3) for w in want])
        errs[name] = rel_l2(got, want)
        # element-wise error against the tensor's scale, 99.9th percentile (reported only)
        scale = np.abs(want) + np.sqrt(np.mean(want * want))
        p999[name] = float(np.percentile(np.abs(got - want) / np.maximum(scale, 1e-30), 99.9))
    print("gradient rel L2:", {k: f"{v:.2e}" for k, v in errs.items()})
    print("gradient p99.9 |d|/(|g| + rms g):", {k: f"{v:.2e}" for k, v in p999.items()})
    for k, v in errs.items():
        assert v <= GRAD_TOL, (k, v)
    return errs


def test_gradient_parity_config1_full_frame(gb):
    scene, views = sg.config("C1")
    check_grads(gb, scene, views[0], O.Options(), (0, 0, 128, 128))


@pytest.mark.parametrize("seed", range(4))
def test_gradient_parity_tiny_scenes(gb, seed):
    rng = np.random.default_rng(50 + seed)
    P = int(rng.integers(2, 9))
    N = [2, 4, 8, 1][seed]
    scene = sg.make_scene(200 + seed, P, -0.4, 0.4, 0.05, 0.4, N)
    W, H = int(rng.integers(20, 50)), int(rng.integers(20, 50))
    view = sg.look_at_view(rng.standard_normal(3) * 0.5 + np.array([0, 0, -2.5]), W, H)
    opts = O.Options(bg=tuple(rng.uniform(0, 1, 3)), tile_w=[16, 8, 16, 8][seed],
                     tile_h=[16, 8, 8, 16][seed])
    check_grads(gb, scene, view, opts, (0, 0, W, H), seed=seed)


def test_gradient_parity_config2_crop(gb):
    scene, views = sg.config("C2")
    check_grads(gb, scene, views[0], O.Options(), (368, 368, 64, 64))


# --- full-size workloads: 64 x 64 crops against the oracle ----------------------------------
# The whole workload is rendered in the default launch configuration (depth-prefix split on,
# default batches); the oracle evaluates one crop of one view. dL/drgb is zero outside the crop
# (and at flagged pixels) on both sides, so every splat gradient is comparable: the splats the
# oracle blended inside the crop are compared by relative L2, and the GPU gradient of every
# other splat must carry no more than a 1e-6 share of the energy.
def check_full_size_crop(gb, name, vi, seed=0, sh_degree=None):
    import scenegen as sgm
    scene, views = sg.config(name)
    if sh_degree is not None:
        scene = sg.with_sh(scene, 99, sh_degree)
    bf16 = sgm.CONFIGS[name]["bf16"]
    opts = O.Options()
    sp = gb.Splats.from_numpy(scene, tex_bf16=bf16)
    rast = gb.Rasterizer(views, gpu_opts(opts))
    rast.plan(sp)
    rgb, T = rast.forward(sp)
    torch.cuda.synchronize()
    view = views[vi]
    W, H = view.width, view.height
    base = sum(v.width * v.height for v in views[:vi])
    crop = ((W - 64) // 2, (H - 64) // 2, 64, 64)
    ref = O.render(scene, view, opts, crop=crop, keep_saved=True)
    img_err, flagged = assert_image_parity(rgb.cpu().numpy(), T.cpu().numpy(), ref, base, W, H,
                                           scene, view, opts)
    x0, y0, w, h = crop
    g_view = sg.make_dl_drgb(seed, [view]).reshape(H, W, 3)
    mask = np.zeros((H, W), dtype=bool)
    mask[y0:y0 + h, x0:x0 + w] = ~O.grad_flags(ref)
    g_view = np.where(mask[..., None], g_view, 0.0).astype(np.float32)
    g_crop = g_view[y0:y0 + h, x0:x0 + w].reshape(-1, 3).astype(np.float64)
    ref_g = O.render_backward(scene, view, opts, ref, g_crop)
    d_rgb = torch.zeros((rast.total_pixels, 3), dtype=torch.float32, device="cuda")
    d_rgb[base:base + W * H] = torch.from_numpy(g_view.reshape(-1, 3)).cuda()
    grads = rast.backward(sp, T, d_rgb)
    torch.cuda.synchronize()
    ks = np.unique(np.array([k for k, _, _, _ in ref.saved], dtype=np.int64))
    idx = torch.from_numpy(ks).cuda()
    errs = {}
    gnames = ("means", "tan_u", "tan_v", "scales", "opacity", "textures")
    if scene.sh is not None:
        gnames = gnames + ("sh",)
    for gname in gnames:
        full = grads[gname]
        got = full[idx].double()
        want = getattr(ref_g, gname)[ks]
        errs[gname] = rel_l2(got.cpu().numpy(), want)
        outside = float((full.double() ** 2).sum() - (got ** 2).sum())
        assert outside <= 1e-6 * float((got ** 2).sum()) + 1e-30, (gname, outside)
    print(f"{name} view {vi} crop {crop}: image max err {img_err:.2e}, {flagged} flagged px, "
          f"{ks.size} splats, gradient rel L2", {k: f"{v:.2e}" for k, v in errs.items()})
    for k, v in errs.items():
        assert v <= GRAD_TOL, (k, v)


@pytest.mark.parametrize("name,vi", [("T0", 0), ("C3", 3), ("C3", 12), ("C4", 1)])
def test_full_size_crop_parity(gb, name, vi):
    check_full_size_crop(gb, name, vi)


# --- full-size invariants: properties that hold at any size, checked at 1M splats, 1080p ------
def pixel_tile_index(views, tw=16, th=16):
    """Global tile index of every packed pixel (views in order, row-major)."""
    out, base = [], 0
    for v in views:
        tx = -(-v.width // tw)
        j, i = np.divmod(np.arange(v.width * v.height), v.width)
        out.append(base + (j // th) * tx + i // tw)
        base += tx * -(-v.height // th)
    return np.concatenate(out)


@pytest.mark.parametrize("bf16", [False, True])
def test_full_size_weights_telescope(gb, bf16):
    """Weights plus transmittance sum to one at every pixel whatever was skipped or stopped
    (the weights telescope). With white textures and a black background a pixel shows the sum
    of its weights, so rgb + T_final = 1; and because the bilinear weights of every pixel sum
    to one, the texture gradients of dL/drgb = g summed over all splats and texels equal
    sum_p (1 - T_p) g_p per channel. Checked on the 1M-splat 1920x1080 workload."""
    scene, views = sg.config("T0")
    white = sg.Scene(scene.means, scene.tan_u, scene.tan_v, scene.scales, scene.opacity,
                     np.ones_like(scene.textures))
    sp = gb.Splats.from_numpy(white, tex_bf16=bf16)
    rast = gb.Rasterizer(views)
    rast.plan(sp)
    rgb, T = rast.forward(sp)
    g = torch.from_numpy(sg.make_dl_drgb(0, views)).cuda()
    grads = rast.backward(sp, T, g)
    torch.cuda.synchronize()
    rgb_h = rgb.cpu().numpy().astype(np.float64)
    T_h = T.cpu().numpy().astype(np.float64)
    # pairs each pixel walked (an upper bound of its blended splats); a blended step rounds
    # the weight, the sum, 1 - alpha and T once each: at most 4 units of 2^-24 of acc + T ~ 1
    n = rast.total_pixels
    tiles = rast.layout.total_tiles
    pt = pixel_tile_index(views)
    r1 = rast.section("ranges", 2 * tiles).cpu().numpy().view(np.uint32).reshape(-1, 2)
    steps = rast.section("n_last", n).cpu().numpy().view(np.uint32).astype(np.int64) - r1[pt, 0]
    bits = rast.section("open_tiles", (tiles + 31) // 32).cpu().numpy().view(np.uint32)
    is_open = ((bits[pt >> 5] >> (pt & 31)) & 1).astype(bool)
    r2 = rast.section("ranges_rest", 2 * tiles).cpu().numpy().view(np.uint32).reshape(-1, 2)
    nl2 = rast.section("n_last_rest", n).cpu().numpy().view(np.uint32).astype(np.int64)
    steps = steps + np.where(is_open, nl2 - r2[pt, 0], 0)
    bound = 4.0 * 2.0 ** -24 * (steps + 2)
    err = np.abs(rgb_h + T_h[:, None] - 1.0)
    print(f"max |rgb + T - 1| = {err.max():.3g}, max steps {steps.max()}")
    assert np.all(err <= bound[:, None])
    want = ((1.0 - T_h)[:, None] * sg.make_dl_drgb(0, views).astype(np.float64)).sum(0)
    got = grads["textures"].double().sum(dim=(0, 1, 2)).cpu().numpy()
    np.testing.assert_allclose(got, want, rtol=1e-5)


# --- constant grids: a box-filtered (single-colour) grid renders as one texel -----------------
@pytest.mark.parametrize("N", [4, 8, 16])
def test_constant_grid_renders_as_one_texel(gb, N):
    """A colour grid filled with one colour (the grid box-filtered to 1 x 1, as the paper does
    to show that the grid carries the image) renders exactly like N = 1 with that colour:
    the bilinear lerps of equal values are exact, so images are bit-equal; the grid's
    gradients sum to the single texel's (bilinear weights sum to one), and the geometry
    gradients agree (the uv adjoint from a constant grid is zero)."""
    base = sg.make_scene(23, 2000, -1.0, 1.0, 0.05, 0.4, N)
    mean = base.textures.mean(axis=(1, 2), dtype=np.float64).astype(np.float32)  # [P, 3]
    grid = sg.Scene(base.means, base.tan_u, base.tan_v, base.scales, base.opacity,
                    np.ascontiguousarray(np.broadcast_to(mean[:, None, None, :],
                                                         base.textures.shape)))
    one = sg.Scene(base.means, base.tan_u, base.tan_v, base.scales, base.opacity,
                   np.ascontiguousarray(mean[:, None, None, :]))
    view = sg.look_at_view((0.1, 0.2, -3.0), 80, 64)
    g = torch.from_numpy(sg.make_dl_drgb(4, [view])).cuda()
    out = []
    for sc in (grid, one):
        rast, sp, rgb, T = run_gpu(gb, sc, [view], O.Options())
        out.append((rgb, T, rast.backward(sp, T, g)))
    (rgb_n, T_n, g_n), (rgb_1, T_1, g_1) = out
    assert torch.equal(rgb_n, rgb_1) and torch.equal(T_n, T_1)
    summed = g_n["textures"].double().sum(dim=(1, 2)).cpu().numpy()
    want = g_1["textures"].double().cpu().numpy().reshape(-1, 3)
    # both are float32 sums of terms of both signs: bound the difference by the magnitude of
    # the terms, taken from the same backward with |dL/drgb|
    rast_1, sp_1, _, T_1b = run_gpu(gb, one, [view], O.Options())
    mag = rast_1.backward(sp_1, T_1b, g.abs())["textures"].double().cpu().numpy().reshape(-1, 3)
    assert np.all(np.abs(summed - want) <= 1e-5 * mag + 1e-12)
    for k in ("means", "tan_u", "tan_v", "scales", "opacity"):
        assert rel_l2(g_n[k].cpu().numpy().astype(np.float64),
                      g_1[k].cpu().numpy().astype(np.float64)) <= 1e-5, k


# --- 16 x 16 colour grids (beyond the paper's 8 x 8 shared-memory limit) ----------------------
@pytest.mark.parametrize("bf16", [False, True])
def test_n16_image_and_gradients_match_oracle(gb, bf16):
    scene = sg.make_scene(41, 3000, -1.0, 1.0, 0.05, 0.4, 16, tex_bf16=bf16)
    view = sg.look_at_view((0.2, -0.1, -3.0), 96, 80)
    opts = O.Options()
    rast, sp, rgb, T = run_gpu(gb, scene, [view], opts, tex_bf16=bf16)
    ref = O.render(scene, view, opts, crop=(24, 16, 48, 40))
    assert_image_parity(rgb.cpu().numpy(), T.cpu().numpy(), ref, 0, 96, 80, scene, view, opts)
    check_grads(gb, scene, view, opts, (32, 24, 32, 32), seed=7, tex_bf16=bf16)


# --- LDS batch sizes: same images, gradients within tolerance -------------------------------
@pytest.mark.parametrize("batch,batch_bwd", [(8, 8), (16, 32), (64, 16), (32, 8)])
def test_batch_sizes(gb, batch, batch_bwd):
    scene = sg.make_scene(21, 3000, -1.5, 1.5, 0.02, 0.25, 8)
    view = sg.look_at_view((0.0, 0.0, -4.0), 96, 80)
    opts = O.Options()
    _, _, rgb0, T0 = run_gpu(gb, scene, [view], opts)
    _, _, rgb1, T1 = run_gpu(gb, scene, [view], opts, batch=batch, batch_bwd=batch_bwd)
    assert torch.equal(rgb0, rgb1) and torch.equal(T0, T1)
    check_grads(gb, scene, view, opts, (16, 16, 48, 40), seed=3, batch=batch,
                batch_bwd=batch_bwd)


# --- backward batch sizes on every wave count: one, two and four 8 x 8 wave blocks per tile ----
# (the backward stages the geometry of several batches at once, 64 / batch of them, with the
# staging threads spread over the workgroup's waves; each tile here walks tens of batches)
@pytest.mark.parametrize("tile", [(8, 8), (16, 8), (8, 16), (16, 16)])
@pytest.mark.parametrize("batch_bwd", [8, 16, 32])
def test_backward_batches_on_every_tile_shape(gb, tile, batch_bwd):
    scene = sg.make_scene(23, 3000, -1.5, 1.5, 0.02, 0.25, 4)
    view = sg.look_at_view((0.2, -0.1, -4.0), 88, 72)
    opts = O.Options(tile_w=tile[0], tile_h=tile[1])
    check_grads(gb, scene, view, opts, (8, 8, 64, 56), seed=17, batch_bwd=batch_bwd)


# --- 16 x 16 colour grids (batches of 4) on every wave count: the backward stages 16 batches'
#     geometry per pass, the forward 4 splats per wave block --------------------------------------
@pytest.mark.parametrize("tile", [(8, 8), (16, 8), (8, 16), (16, 16)])
def test_n16_on_every_tile_shape(gb, tile):
    scene = sg.make_scene(29, 1500, -1.5, 1.5, 0.03, 0.3, 16)
    view = sg.look_at_view((0.1, -0.2, -4.0), 80, 64)
    opts = O.Options(tile_w=tile[0], tile_h=tile[1])
    rast, sp, rgb, T = run_gpu(gb, scene, [view], opts)
    ref = O.render(scene, view, opts, crop=(8, 8, 48, 40))
    assert_image_parity(rgb.cpu().numpy(), T.cpu().numpy(), ref, 0, 80, 64, scene, view, opts)
    check_grads(gb, scene, view, opts, (8, 8, 48, 40), seed=19)


# --- depth-prefix split: same images as one pass, exact pair sets ---------------------------
def dense_scene(N=4):
    scene = sg.make_scene(31, 20000, -1.0, 1.0, 0.03, 0.3, N)
    return scene, sg.look_at_view((0.0, 0.0, -3.5), 128, 96)


def global_depth_order(scene, views, opts):
    """Records of all views by (depth key, record index), culled ones last; their counts."""
    bits, idx, counts = [], [], []
    for v, view in enumerate(views):
        ks = O.key_stage(scene, view, opts)
        bits.append(np.where(ks["visible"], ks["depth"].view(np.uint32), np.uint32(0xFFFFFFFF)))
        counts.append(ks["count"].astype(np.int64))
        idx.append(v * scene.P + np.arange(scene.P))
    bits, idx, counts = np.concatenate(bits), np.concatenate(idx), np.concatenate(counts)
    order = idx[np.lexsort((idx, bits))]
    rank = np.empty_like(order)
    rank[order] = np.arange(order.size)
    return order, rank, counts


@pytest.mark.parametrize("per_tile", [0, 1, 8, 64])
def test_split_pairs_are_exact_and_images_equal_one_pass(gb, per_tile):
    scene, view = dense_scene()
    views = [view, sg.look_at_view((0.5, 0.3, -3.0), 72, 50)]
    opts = O.Options()
    rast, sp, rgb, T = run_gpu(gb, scene, views, opts, prefix=per_tile)
    lay = rast.layout
    st = rast.section("status", 10).cpu().numpy().view(np.uint32)
    n_first, overflow, cut, n_rest = int(st[1]), int(st[2]), int(st[3]), int(st[6])
    assert overflow == 0
    # the cut: the longest depth prefix whose pairs fit the prefix pass's slots
    order, rank, counts = global_depth_order(scene, views, opts)
    off = np.concatenate([[0], np.cumsum(counts[order])])
    want_cut = int(np.searchsorted(off, lay.prefix_capacity, side="right")) - 1
    assert cut == want_cut
    keys, vals, _ = O.tile_pairs(scene, views, opts)
    in_first = rank[vals] < cut
    assert n_first == int(in_first.sum())
    gk = rast.section("pair_keys", n_first).cpu().numpy().view(np.uint32)
    gv = rast.section("pair_vals", n_first).cpu().numpy().view(np.uint32)
    np.testing.assert_array_equal(gk, keys[in_first])
    np.testing.assert_array_equal(gv, vals[in_first])
    # the rest: later records on the tiles that the first pass left open
    tiles = lay.total_tiles
    bits = rast.section("open_tiles", (tiles + 31) // 32).cpu().numpy().view(np.uint32)
    is_open = ((bits[keys >> 5] >> (keys & 31)) & 1).astype(bool)
    in_rest = ~in_first & is_open
    assert n_rest == int(in_rest.sum())
    gk = rast.section("pair_keys_rest", n_rest).cpu().numpy().view(np.uint32)
    gv = rast.section("pair_vals_rest", n_rest).cpu().numpy().view(np.uint32)
    np.testing.assert_array_equal(gk, keys[in_rest])
    np.testing.assert_array_equal(gv, vals[in_rest])
    if per_tile in (1, 8):
        assert 0 < cut < len(order) and n_rest > 0  # a real split at this budget
    _, _, rgb1, T1 = run_gpu(gb, scene, views, opts, prefix=-1)
    assert torch.equal(rgb, rgb1) and torch.equal(T, T1)


def test_split_without_termination_equals_one_pass(gb):
    scene, view = dense_scene()
    opts = O.Options(t_min=0.0)
    _, _, rgb0, T0 = run_gpu(gb, scene, [view], opts, prefix=16)
    _, _, rgb1, T1 = run_gpu(gb, scene, [view], opts, prefix=-1)
    assert torch.equal(rgb0, rgb1) and torch.equal(T0, T1)


@pytest.mark.parametrize("per_tile", [1, 16, 0])
def test_split_gradients_match_oracle(gb, per_tile):
    scene, view = dense_scene(N=8)
    check_grads(gb, scene, view, O.Options(), (40, 32, 32, 24), seed=5, prefix=per_tile)


def test_split_image_matches_oracle(gb):
    scene, view = dense_scene(N=8)
    rast, sp, rgb, T = run_gpu(gb, scene, [view], O.Options(), prefix=16)
    ref = O.render(scene, view, O.Options(), crop=(40, 32, 48, 32))
    assert_image_parity(rgb.cpu().numpy(), T.cpu().numpy(), ref, 0, 128, 96, scene, view,
                        O.Options())


# --- work order of the tiles: a schedule, not a change of any result -------------------------
def tile_spans(n_last, ranges, views, tw=16, th=16):
    """Per tile: one past the last pair any of its pixels blended, minus the tile's first pair
    (tiles numbered view by view, row-major)."""
    out, base = [], 0
    for v in views:
        W, H = v.width, v.height
        tx, ty = -(-W // tw), -(-H // th)
        pad = np.zeros((ty * th, tx * tw), np.int64)
        pad[:H, :W] = n_last[base:base + W * H].reshape(H, W)
        out.append(pad.reshape(ty, th, tx, tw).max(axis=(1, 3)).reshape(-1))
        base += W * H
    top = np.concatenate(out)
    return np.maximum(top - ranges[:, 0], 0)


def assert_decreasing_in_buckets(cost):
    # buckets are exact below 16 and 1/16 of the cost wide above: a later tile never costs
    # more than 17/16 of an earlier one
    prev_min = np.minimum.accumulate(cost)[:-1]
    assert np.all(cost[1:] <= prev_min * 17 // 16 + 1)


@pytest.mark.parametrize("prefix", [8, -1])
def test_tile_order_changes_no_result(gb, prefix):
    scene, view = dense_scene(N=8)
    views = [view, sg.look_at_view((0.5, 0.3, -3.0), 72, 50)]
    g = torch.from_numpy(sg.make_dl_drgb(3, views)).cuda()
    runs = {}
    for order in (-1, 1):
        o = gpu_opts(O.Options(), prefix=prefix)
        o.tile_order = order
        sp = gb.Splats.from_numpy(scene)
        rast = gb.Rasterizer(views, o)
        rast.plan(sp)
        rgb, T = rast.forward(sp)
        grads = rast.backward(sp, T, g)
        torch.cuda.synchronize()
        runs[order] = (rast, rgb, T, rast.section("n_last", rast.total_pixels).clone(), grads)
    (r0, rgb0, T0, nl0, g0), (r1, rgb1, T1, nl1, g1) = runs[-1], runs[1]
    assert torch.equal(rgb0, rgb1) and torch.equal(T0, T1) and torch.equal(nl0, nl1)
    for k in g0:  # only the order of the float atomics differs
        assert rel_l2(g1[k].cpu().numpy().astype(np.float64),
                      g0[k].cpu().numpy().astype(np.float64)) <= 1e-5, k
    lay = r1.layout
    n = lay.total_tiles
    assert r0.layout.tile_order == 0 and lay.tile_order != 0
    order = r1.section("tile_order", n).cpu().numpy().view(np.uint32)
    np.testing.assert_array_equal(np.sort(order), np.arange(n))
    ranges = r1.section("ranges", 2 * n).cpu().numpy().view(np.uint32).reshape(n, 2)
    ranges = ranges.astype(np.int64)
    # the backward's cost: the blended span of the first pass plus, on open tiles, the rest's
    work = r1.section("tile_work", n).cpu().numpy().view(np.uint32).astype(np.int64)
    want = tile_spans(nl1.cpu().numpy().view(np.uint32), ranges, views)
    if prefix >= 0:
        bits = r1.section("open_tiles", (n + 31) // 32).cpu().numpy().view(np.uint32)
        t = np.arange(n)
        is_open = ((bits[t >> 5] >> (t & 31)) & 1).astype(bool)
        rr = r1.section("ranges_rest", 2 * n).cpu().numpy().view(np.uint32).reshape(n, 2)
        nlr = r1.section("n_last_rest", r1.total_pixels).cpu().numpy().view(np.uint32)
        want = want + np.where(is_open, tile_spans(nlr, rr.astype(np.int64), views), 0)
    np.testing.assert_array_equal(work, want)
    assert_decreasing_in_buckets(work[order])


# --- autotuner: whatever it picks keeps oracle parity ---------------------------------------
def test_autotuned_options_keep_parity(gb, tmp_path):
    from paper_2412_12734_amd import autotune as at
    scene = sg.make_scene(41, 20000, -1.0, 1.0, 0.02, 0.25, 8)
    view = sg.look_at_view((0.0, 0.0, -3.0), 160, 120)
    sp = gb.Splats.from_numpy(scene)
    knobs = {"tile": [(16, 16), (16, 8), (8, 8)], "batch": [16, 32], "batch_bwd": [8, 16],
             "prefix_pairs_per_tile": [512, -1]}
    path = str(tmp_path / "tune.json")
    opts, rec = at.autotune(sp, [view], base=gpu_opts(O.Options()), cache_path=path,
                            knobs=knobs, steps=2)
    assert rec["ms"] <= rec["default_ms"] and len(rec["candidates"]) >= 6
    rast = gb.Rasterizer([view], opts)
    rast.plan(sp)
    rgb, T = rast.forward(sp)
    ref = O.render(scene, view, O.Options(), crop=(48, 36, 64, 48))
    assert_image_parity(rgb.cpu().numpy(), T.cpu().numpy(), ref, 0, 160, 120, scene, view,
                        O.Options())
    opts2, rec2 = at.autotune(sp, [view], cache_path=path, knobs=knobs)
    assert opts2 == opts  # second call served from the cache


# --- HIP graph: a captured forward + backward replays the eager results ----------------------
def test_graph_replay_matches_eager(gb):
    scene, view = dense_scene(N=8)
    views = [view, sg.look_at_view((0.4, -0.2, -3.2), 72, 50)]
    sp = gb.Splats.from_numpy(scene)
    rast = gb.Rasterizer(views, gpu_opts(O.Options()), check_overflow=False)
    rast.plan(sp)
    rgb, T = rast.forward(sp)
    g = torch.from_numpy(sg.make_dl_drgb(7, views)).cuda()
    grads = rast.backward(sp, T, g)
    torch.cuda.synchronize()
    want_rgb, want_T = rgb.clone(), T.clone()
    want = {k: v.clone() for k, v in grads.items()}
    graph = rast.capture_step(sp, rgb, T, g, grads)
    for rep in range(3):
        # eager work between replays: spoil the outputs, then replay and compare
        rgb.fill_(-1.0)
        T.fill_(-1.0)
        for v in grads.values():
            v.fill_(123.0)
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(rgb, want_rgb) and torch.equal(T, want_T), rep
        for k, v in want.items():
            # gradients accumulate with float atomics: the order may differ between runs
            err = float((grads[k].double() - v.double()).norm() / v.double().norm().clamp_min(1e-30))
            assert err <= 1e-5, (rep, k, err)
        assert not rast.status()[1]


# --- precision: bfloat16 texture storage ---------------------------------------------------
def test_bf16_exact_texels_give_identical_images(gb):
    scene, views = sg.config("C1")
    q = (np.round(scene.textures * 256) / 256).astype(np.float32)  # exact in bfloat16
    s = sg.Scene(scene.means, scene.tan_u, scene.tan_v, scene.scales, scene.opacity, q)
    _, _, rgb32, T32 = run_gpu(gb, s, views, O.Options())
    _, _, rgb16, T16 = run_gpu(gb, s, views, O.Options(), tex_bf16=True)
    assert torch.equal(rgb32, rgb16) and torch.equal(T32, T16)


def test_bf16_textures_match_oracle_on_rounded_texels(gb):
    scene, views = sg.config("C1")
    rast, sp, rgb, T = run_gpu(gb, scene, views, O.Options(), tex_bf16=True)
    rounded = sg.bf16_bits_to_f32(sg.to_bf16_bits(scene.textures)).reshape(scene.textures.shape)
    s = sg.Scene(scene.means, scene.tan_u, scene.tan_v, scene.scales, scene.opacity, rounded)
    ref = O.render(s, views[0], O.Options())
    assert_image_parity(rgb.cpu().numpy(), T.cpu().numpy(), ref, 0, 128, 128, s, views[0],
                        O.Options())


# --- batching: many views in one launch sequence --------------------------------------------
def test_batched_views_equal_single_views(gb):
    scene = sg.make_scene(11, 5000, -2, 2, 0.01, 0.2, 4)
    views = sg.orbit_views(3, 4, 6.0, [(96, 64), (64, 80), (128, 72), (50, 50)],
                           pick_resolution=True)
    opts = O.Options()
    _, _, rgb_b, T_b = run_gpu(gb, scene, views, opts)
    base = 0
    for v in views:
        _, _, rgb1, T1 = run_gpu(gb, scene, [v], opts)
        n = v.width * v.height
        assert torch.equal(rgb_b[base:base + n], rgb1)
        assert torch.equal(T_b[base:base + n], T1)
        base += n


# --- capacity and degenerate inputs ---------------------------------------------------------
def test_capacity_overflow_is_reported_then_replanned(gb):
    scene, views = sg.config("C1")
    sp = gb.Splats.from_numpy(scene)
    rast = gb.Rasterizer(views, gpu_opts(O.Options()), check_overflow=False)
    rast.plan(sp, capacity=100)
    rgb, T = rast.forward(sp)
    K, over = rast.status()
    assert over and K > 100
    assert float(rgb.abs().max()) == 0.0 and float(T.min()) == 1.0
    rast.check_overflow = True
    rgb2, T2 = rast.forward(sp)
    K2, over2 = rast.status()
    assert not over2 and K2 == K
    ref = O.render(scene, views[0], O.Options())
    assert_image_parity(rgb2.cpu().numpy(), T2.cpu().numpy(), ref, 0, 128, 128, scene, views[0],
                        O.Options())


def test_capacity_error_on_a_later_forward_and_per_view_counts(gb):
    """Through the C ABI: a forward that overflows its capacity sets the overflow flag; once
    it has completed, the next forward on the workspace with the same capacity returns
    GB_ERR_CAPACITY without launching, and one with a capacity that fits runs. The status call
    reports the sticky overflow once and the pair count of every view, which must equal the
    oracle's key-stage counts."""
    import ctypes
    from paper_2412_12734_amd import _lib as L
    scene = sg.make_scene(17, 2000, -1.0, 1.0, 0.02, 0.3, 4)
    views = [sg.look_at_view((0.0, 0.0, -3.0), 80, 60), sg.look_at_view((1.5, 0.5, -2.5), 48, 64),
             sg.look_at_view((-2.0, 1.0, -1.0), 33, 21)]
    sp = gb.Splats.from_numpy(scene)
    rast = gb.Rasterizer(views, gpu_opts(O.Options()), check_overflow=False)
    rast.plan(sp, capacity=64)
    lib = L.load()
    rgb, T = rast.forward(sp)
    torch.cuda.synchronize()

    def fwd(cap):
        return lib.gb_render_fwd(ctypes.byref(sp.c()), rast.cviews, rast.nv,
                                 ctypes.byref(rast.copts), rast.ws.data_ptr(), rast.ws.numel(),
                                 cap, rgb.data_ptr(), T.data_ptr(),
                                 torch.cuda.current_stream().cuda_stream)

    assert fwd(64) == L.GB_ERR_CAPACITY
    assert b"needed" in lib.gb_last_error()
    K, over_last, over_any, per_view = rast.status_ex(per_view=True)
    want = [int(O.key_stage(scene, v, O.Options())["count"].sum()) for v in views]
    assert per_view == want and K == sum(want) and over_last and over_any
    # the sticky bit is reported once; the overflow of the last forward stays visible
    assert rast.status_ex() == (K, True, False)
    assert fwd(64) == L.GB_ERR_CAPACITY  # still too small (status calls do not clear it)
    rast.plan(sp, capacity=K)  # fits exactly (same workspace or a larger one)
    assert fwd(K) == L.GB_OK
    torch.cuda.synchronize()
    assert rast.status_ex() == (K, False, False)
    ref = O.render(scene, views[2], O.Options())
    base = 80 * 60 + 48 * 64
    assert_image_parity(rgb.cpu().numpy(), T.cpu().numpy(), ref, base, 33, 21, scene, views[2],
                        O.Options())


def test_all_splats_culled_gives_background(gb):
    scene, _ = sg.config("C1", P=50)
    view = sg.look_at_view((0, 0, 3.0), 32, 24, target=(0, 0, 6.0))  # looking away
    opts = O.Options(bg=(0.25, 0.5, 0.75))
    rast, sp, rgb, T = run_gpu(gb, scene, [view], opts)
    assert rast.status() == (0, False)
    np.testing.assert_array_equal(rgb.cpu().numpy(), np.broadcast_to([0.25, 0.5, 0.75], (32 * 24, 3)).astype(np.float32))
    assert float(T.min()) == 1.0


# --- gradient buffers are cleared by the backward (odd sizes: the fill's tail words) ---------
@pytest.mark.parametrize("N", [1, 2])
def test_backward_overwrites_stale_gradient_buffers(gb, N):
    scene = sg.make_scene(13, 1001, -1.0, 1.0, 0.05, 0.3, N)  # 3 x 1001 texel words for N = 1
    view = sg.look_at_view((0.0, 0.0, -3.0), 67, 45)
    rast, sp, rgb, T = run_gpu(gb, scene, [view], O.Options())
    g = torch.from_numpy(sg.make_dl_drgb(5, [view])).cuda()
    fresh = {k: v.clone() for k, v in rast.backward(sp, T, g).items()}
    stale = {k: torch.full_like(v, 123.0) for k, v in fresh.items()}
    got = rast.backward(sp, T, g, stale)
    torch.cuda.synchronize()
    for k, v in fresh.items():
        assert not bool((got[k] == 123.0).any()), k
        err = float((got[k].double() - v.double()).norm() / v.double().norm().clamp_min(1e-30))
        assert err <= 1e-5, (k, err)


# --- both texel-scatter paths of the backward: few blended lanes per wave step (small splats,
#     direct per-lane adds) and many (large splats, grouped by cell) ---------------------------
@pytest.mark.parametrize("s_lo,s_hi", [(0.004, 0.015), (0.15, 0.5)])
def test_gradients_with_small_and_large_splats(gb, s_lo, s_hi):
    scene = sg.make_scene(41, 3000, -1.0, 1.0, s_lo, s_hi, 8)
    view = sg.look_at_view((0.0, 0.0, -3.0), 96, 80)
    check_grads(gb, scene, view, O.Options(), (0, 0, 96, 80), seed=3)


# --- full-size tiling: every record and every pair of the 1M-splat 1080p workload -------------
def test_tiling_bit_exact_full_size_t0(gb):
    """Depth keys, tile counts and rectangles of all 1M records, then all (tile, record) pairs
    (one pass, about 43M) and every tile's range, against the oracle's key stage and its
    vectorised pair expansion."""
    scene, views = sg.config("T0")
    opts = O.Options()
    rast, sp, rgb, T = run_gpu(gb, scene, views, opts, prefix=-1)
    P = scene.P
    ks = O.key_stage(scene, views[0], opts)
    vis = ks["visible"]
    depth = rast.section("depth_key", P, torch.int32).cpu().numpy().view(np.uint32)
    np.testing.assert_array_equal(depth, np.where(vis, ks["depth"].view(np.uint32),
                                                  np.uint32(0xFFFFFFFF)))
    count = rast.section("tile_count", P, torch.int32).cpu().numpy().view(np.uint32)
    np.testing.assert_array_equal(count, ks["count"].astype(np.uint32))
    recs = rast.section("records", P * 24, torch.int32).cpu().numpy().reshape(P, 24)
    rx, ry = recs[:, 19], recs[:, 20]
    got = np.stack([rx & 0xFFFF, rx >> 16, ry & 0xFFFF, ry >> 16], 1)[vis]
    np.testing.assert_array_equal(got, ks["rect"][vis])
    del recs, got
    keys, vals, ranges = O.tile_pairs_vectorised(scene, views, opts)
    K, over = rast.status()
    print(f"T0: {int(vis.sum())} visible records, {K} pairs")
    assert not over and K == keys.size
    gk = rast.section("pair_keys", K, torch.int32).cpu().numpy().view(np.uint32)
    np.testing.assert_array_equal(gk, keys)
    del gk
    gv = rast.section("pair_vals", K, torch.int32).cpu().numpy().view(np.uint32)
    np.testing.assert_array_equal(gv, vals)
    del gv
    gr = rast.section("ranges", 2 * ranges.shape[0], torch.int32).cpu().numpy().view(np.uint32)
    np.testing.assert_array_equal(gr.reshape(-1, 2).astype(np.int64), ranges)


# --- screen-space low-pass of any variance: tile bound, images and gradients ------------------
@pytest.mark.parametrize("var", [1.0, 2.0])
def test_lowpass_variance_parity(gb, var):
    """Sub-pixel and ordinary splats with a wider low-pass than the default: the tile
    rectangles (whose low-pass radius follows the variance) are bit-exact and the images and
    gradients match the oracle."""
    small = sg.make_scene(61, 1500, -1.0, 1.0, 5e-4, 4e-3, 4)
    big = sg.make_scene(62, 300, -1.0, 1.0, 0.02, 0.2, 4)
    scene = sg.Scene(*(np.ascontiguousarray(np.concatenate([a, b])) for a, b in
                       zip((small.means, small.tan_u, small.tan_v, small.scales, small.opacity,
                            small.textures),
                           (big.means, big.tan_u, big.tan_v, big.scales, big.opacity,
                            big.textures))))
    view = sg.look_at_view((0.1, -0.2, -3.0), 96, 72)
    opts = O.Options(lowpass_var=var)
    check_tiling(gb, scene, [view], opts)
    rast, sp, rgb, T = run_gpu(gb, scene, [view], opts)
    ref = O.render(scene, view, opts)
    assert_image_parity(rgb.cpu().numpy(), T.cpu().numpy(), ref, 0, 96, 72, scene, view, opts)
    check_grads(gb, scene, view, opts, (16, 8, 48, 40), seed=11)


# --- wide and tall tiles (32 x 8, 8 x 32) -------------------------------------------------------
@pytest.mark.parametrize("tile", [(32, 8), (8, 32)])
def test_wide_and_tall_tiles(gb, tile):
    scene = sg.make_scene(5, 3000, -1.5, 1.5, 0.01, 0.3, 8)
    views = [sg.look_at_view((0.5, 0.3, -3.0), 97, 61), sg.look_at_view((-2.0, 1.0, -2.0), 64, 80)]
    opts = O.Options(tile_w=tile[0], tile_h=tile[1])
    check_tiling(gb, scene, views, opts)
    rast, sp, rgb, T = run_gpu(gb, scene, views, opts)
    ref = O.render(scene, views[1], opts)
    assert_image_parity(rgb.cpu().numpy(), T.cpu().numpy(), ref, 97 * 61, 64, 80, scene, views[1],
                        opts)
    check_grads(gb, scene, views[0], opts, (20, 10, 50, 40), seed=13)


# --- 16 x 16 colour grids at full size: a 64 x 64 crop of 1M splats at 1080p -------------------
def test_n16_full_size_crop_parity(gb):
    check_full_size_crop(gb, "T0_N16", 0)


# --- diffuse-specular split (Sec. 4.2): per-splat spherical harmonics ---------------------------
@pytest.mark.parametrize("degree,N", [(0, 4), (1, 2), (3, 8)])
def test_specular_sh_image_and_gradients(gb, degree, N):
    scene = sg.with_sh(sg.make_scene(71, 2000, -1.0, 1.0, 0.02, 0.3, N), 5, degree, scale=0.3)
    view = sg.look_at_view((0.6, -0.4, -2.8), 96, 72)
    opts = O.Options(bg=(0.1, 0.2, 0.3))
    rast, sp, rgb, T = run_gpu(gb, scene, [view], opts)
    ref = O.render(scene, view, opts)
    assert_image_parity(rgb.cpu().numpy(), T.cpu().numpy(), ref, 0, 96, 72, scene, view, opts)
    check_grads(gb, scene, view, opts, (8, 8, 80, 56), seed=degree)


def test_specular_sh_gradients_over_several_views(gb):
    """The view-dependent colour differs per view: the coefficient and centre gradients of a
    batched call must equal the sum of the oracle's per-view gradients."""
    scene = sg.with_sh(sg.make_scene(72, 800, -0.8, 0.8, 0.03, 0.3, 4), 6, 2, scale=0.3)
    views = [sg.look_at_view((0.3, 0.2, -2.6), 64, 48), sg.look_at_view((2.0, -0.6, -1.2), 48, 56)]
    opts = O.Options()
    rast, sp, rgb, T = run_gpu(gb, scene, views, opts)
    g_all = sg.make_dl_drgb(8, views)
    parts, base, total = [], 0, None
    for v in views:
        hw = v.width * v.height
        ref = O.render(scene, v, opts, keep_saved=True)
        ok = ~O.grad_flags(ref).reshape(-1)
        g_all[base:base + hw] = np.where(ok[:, None], g_all[base:base + hw], 0.0)
        gr = O.render_backward(scene, v, opts, ref, g_all[base:base + hw].astype(np.float64))
        total = gr if total is None else O.Grads(*(a + b for a, b in zip(
            (total.means, total.tan_u, total.tan_v, total.scales, total.opacity, total.textures,
             total.sh),
            (gr.means, gr.tan_u, gr.tan_v, gr.scales, gr.opacity, gr.textures, gr.sh))))
        base += hw
    grads = rast.backward(sp, T, torch.from_numpy(g_all).cuda())
    torch.cuda.synchronize()
    for name in ("means", "tan_u", "tan_v", "scales", "opacity", "textures", "sh"):
        err = rel_l2(grads[name].cpu().numpy().astype(np.float64), getattr(total, name))
        print(name, f"{err:.2e}")
        assert err <= GRAD_TOL, (name, err)


def test_specular_sh_full_size_crop(gb):
    """Degree-3 coefficients on the 1M-splat 1080p workload: a 64 x 64 crop against the oracle
    (image and every gradient, coefficients included)."""
    check_full_size_crop(gb, "T0", 0, sh_degree=3)


# --- colour grids of several sides in one call -------------------------------------------------
def _bf16_grids(scene):
    r = lambda g: sg.bf16_bits_to_f32(sg.to_bf16_bits(g)).reshape(g.shape).astype(np.float32)
    return sg.Scene(scene.means, scene.tan_u, scene.tan_v, scene.scales, scene.opacity,
                    [r(g) for g in scene.textures], scene.sh)


@pytest.mark.parametrize("layout,sides,bf16", [(8, (1, 2, 3, 5, 8), False),
                                               (16, (1, 4, 7, 12, 16), False),
                                               (8, (2, 4, 6, 8), True)])
def test_mixed_sides_image_and_gradients(gb, layout, sides, bf16):
    """Splats whose grids have sides of their own (any side up to the layout's 8 or 16, packed
    in one array with per-splat offsets) against the oracle: images, and every gradient
    including each splat's own grid."""
    scene = sg.with_mixed_sides(sg.make_scene(90 + layout, 2500, -1.2, 1.2, 0.01, 0.3, layout),
                                7 + layout, sides)
    if bf16:
        scene = _bf16_grids(scene)
    view = sg.look_at_view((0.4, 0.2, -3.0), 88, 72)
    opts = O.Options(bg=(0.2, 0.1, 0.3))
    rast, sp, rgb, T = run_gpu(gb, scene, [view], opts, tex_bf16=bf16)
    assert sp.mixed and sp.N == layout
    ref = O.render(scene, view, opts)
    assert_image_parity(rgb.cpu().numpy(), T.cpu().numpy(), ref, 0, 88, 72, scene, view, opts)
    check_grads(gb, scene, view, opts, (12, 8, 64, 56), seed=layout, tex_bf16=bf16)


def test_mixed_sides_all_equal_match_the_uniform_path(gb):
    """The same grids given once as a [P, N, N, 3] array and once through per-splat sides (all
    N) render bit for bit alike, and their gradients agree to float32 summation order."""
    base = sg.make_scene(95, 3000, -1.2, 1.2, 0.01, 0.3, 8)
    mixed = sg.Scene(base.means, base.tan_u, base.tan_v, base.scales, base.opacity,
                     [g for g in base.textures])
    view = sg.look_at_view((-0.3, 0.5, -2.8), 96, 80)
    opts = O.Options()
    out = []
    for scene in (base, mixed):
        rast, sp, rgb, T = run_gpu(gb, scene, [view], opts)
        g = torch.from_numpy(sg.make_dl_drgb(2, [view])).cuda()
        grads = rast.backward(sp, T, g)
        torch.cuda.synchronize()
        out.append((rgb.cpu().numpy(), T.cpu().numpy(),
                    {k: v.cpu().numpy().reshape(-1) for k, v in grads.items()}))
    np.testing.assert_array_equal(out[0][0], out[1][0])
    np.testing.assert_array_equal(out[0][1], out[1][1])
    for k in out[0][2]:
        assert rel_l2(out[1][2][k], out[0][2][k]) <= 1e-6, k


# --- texture gradients zeroed by the forward ----------------------------------------------------
def test_forward_zeroing_replaces_the_backward_clear(gb):
    """A forward given the coming backward's gradient arrays zeroes the texture gradients while
    it blends and the backward skips its clear: gradients equal those of the plain path even
    from arrays full of NaN. After a plain forward, or with another array, the backward clears
    again. The images are those of the plain forward, bit for bit."""
    scene = sg.make_scene(97, 3000, -1.2, 1.2, 0.01, 0.3, 8)
    view = sg.look_at_view((0.2, -0.4, -2.9), 96, 72)
    sp = gb.Splats.from_numpy(scene)
    rast = gb.Rasterizer([view], gpu_opts(O.Options()))
    rast.plan(sp)
    g = torch.from_numpy(sg.make_dl_drgb(5, [view])).cuda()
    rgb0, T0 = rast.forward(sp)
    ref = {k: v.clone() for k, v in rast.backward(sp, T0, g).items()}
    rgb0, T0 = rgb0.clone(), T0.clone()
    nan_like = lambda d: {k: torch.full_like(v, float("nan")) for k, v in d.items()}

    def check(grads):
        torch.cuda.synchronize()
        for k, v in ref.items():
            got = grads[k]
            assert bool(torch.isfinite(got).all()), k
            assert rel_l2(got.cpu().numpy().astype(np.float64),
                          v.cpu().numpy().astype(np.float64)) <= 1e-6, k

    grads = nan_like(ref)
    rgb, T = rast.forward(sp, zero_grads=grads)
    torch.cuda.synchronize()
    assert torch.equal(rgb, rgb0) and torch.equal(T, T0)
    rast.backward(sp, T, g, grads)
    check(grads)
    # a plain forward in between: the backward clears by itself
    grads = nan_like(ref)
    rast.forward(sp, zero_grads=grads)
    grads["textures"].fill_(float("nan"))
    rgb, T = rast.forward(sp)
    rast.backward(sp, T, g, grads)
    check(grads)
    # the backward given another array than the one the forward zeroed
    other = nan_like(ref)
    rgb, T = rast.forward(sp, zero_grads=nan_like(ref))
    rast.backward(sp, T, g, other)
    check(other)


def test_forward_zeroing_of_a_texture_gradient_off_a_16_byte_boundary(gb):
    """The forward's zeroing splits its array into single floats up to the first 16-byte
    boundary, 16-byte stores and a tail: a texture-gradient array that starts 4, 8 or 12 bytes
    past a boundary (and so also ends off one) is zeroed whole, so the backward that skips its
    clear still gives the gradients of the plain path from arrays full of NaN."""
    scene = sg.make_scene(98, 2001, -1.2, 1.2, 0.01, 0.3, 8)
    view = sg.look_at_view((0.1, -0.3, -2.9), 80, 64)
    sp = gb.Splats.from_numpy(scene)
    rast = gb.Rasterizer([view], gpu_opts(O.Options()))
    rast.plan(sp)
    g = torch.from_numpy(sg.make_dl_drgb(6, [view])).cuda()
    rgb0, T0 = rast.forward(sp)
    ref = {k: v.clone() for k, v in rast.backward(sp, T0, g).items()}
    for shift in (1, 2, 3):
        grads = {k: torch.full_like(v, float("nan")) for k, v in ref.items()}
        n = ref["textures"].numel()
        big = torch.full((n + 8,), float("nan"), dtype=torch.float32, device="cuda")
        grads["textures"] = big[shift:shift + n].view(ref["textures"].shape)
        assert grads["textures"].data_ptr() % 16 == 4 * shift
        rgb, T = rast.forward(sp, zero_grads=grads)
        rast.backward(sp, T, g, grads)
        torch.cuda.synchronize()
        for k, v in ref.items():
            got = grads[k]
            assert bool(torch.isfinite(got).all()), (shift, k)
            assert rel_l2(got.cpu().numpy().astype(np.float64),
                          v.cpu().numpy().astype(np.float64)) <= 1e-6, (shift, k)
        # the words around the array are not touched
        assert bool(torch.isnan(big[:shift]).all()) and bool(torch.isnan(big[shift + n:]).all())
