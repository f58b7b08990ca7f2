"""Pins of the FP64 oracle against what the paper and the mathematics fix (CPU only).

Each test names the passage it pins. None of them re-types the oracle's own formula: they use
closed forms of special geometries, invariants, symmetries, finite differences and brute force.
"""
import dataclasses
import json
import math
import os

import numpy as np
import pytest

import scenegen as sg
from oracle import gb_oracle as O

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def one_scene(means, tan_u, tan_v, scales, opacity, textures):
    f = lambda a: np.ascontiguousarray(np.asarray(a, dtype=np.float64), dtype=np.float32)
    return sg.Scene(f(means), f(tan_u), f(tan_v), f(scales), f(opacity), f(textures))


def frontal_splat(X, Y, Z, s=(0.1, 0.1), theta=0.0, o=0.8, tex=None, N=4):
    tu = [math.cos(theta), math.sin(theta), 0.0]
    tv = [-math.sin(theta), math.cos(theta), 0.0]
    if tex is None:
        tex = np.full((N, N, 3), 0.5)
    return [X, Y, Z], tu, tv, list(s), o, tex


def scene_of(splats):
    cols = list(zip(*splats))
    return one_scene(*(np.stack([np.asarray(c, dtype=np.float64) for c in col]) for col in cols))


def pixel_to_world(view, x, y, Z):
    """Identity camera: the point at depth Z seen through pixel position (x, y)."""
    return (Z * (x - view.cx) / view.fx, Z * (y - view.cy) / view.fy, Z)


# --- P1: alpha at the splat centre equals opacity ---------------------------------------
def test_alpha_at_center_equals_opacity():
    view = sg.frontal_view(16, 16)
    X, Y, Z = pixel_to_world(view, 8.5, 7.5, 4.0)
    col = np.array([0.25, 0.5, 0.75])
    sc = scene_of([frontal_splat(X, Y, Z, o=0.6, tex=np.broadcast_to(col, (4, 4, 3)))])
    r = O.render(sc, view, O.Options())
    o = float(sc.opacity[0])
    col = sc.textures[0, 0, 0].astype(np.float64)
    assert r.rgb[7, 8] == pytest.approx(o * col, abs=1e-12)
    assert r.T_final[7, 8] == pytest.approx(1.0 - o, abs=1e-12)


# --- P5: image-fitting geometry (Sec. 4.1: camera along +z, rotation about z only) -------
def test_uv_closed_form_for_image_plane_splats():
    rng = np.random.default_rng(1)
    view = sg.frontal_view(64, 48)
    for _ in range(20):
        Z = rng.uniform(1.0, 10.0)
        X, Y = rng.uniform(-1, 1, 2)
        th = rng.uniform(-math.pi, math.pi)
        su, sv = rng.uniform(0.05, 0.5, 2)
        sc = scene_of([frontal_splat(X, Y, Z, s=(su, sv), theta=th)])
        M = O.splat_M(sc, view, 0)
        xs, ys = rng.uniform(0, 64, 50), rng.uniform(0, 48, 50)
        u, v, valid, *_ = O.ray_splat_uv(M, xs, ys)
        assert valid.all()
        # the inputs are float32; use their exact values in the closed form
        X, Y, Z = (float(c) for c in sc.means[0])
        c, s = float(sc.tan_u[0, 0]), float(sc.tan_u[0, 1])
        su, sv = (float(c_) for c_ in sc.scales[0])
        dx = Z * (xs - view.cx) / view.fx - X
        dy = Z * (ys - view.cy) / view.fy - Y
        tvx, tvy = float(sc.tan_v[0, 0]), float(sc.tan_v[0, 1])
        # tangents of a float32 rotation are only nearly orthonormal: solve the 2x2 system
        A = np.array([[su * c, sv * tvx], [su * s, sv * tvy]])
        uv = np.linalg.solve(A, np.stack([dx, dy]))
        np.testing.assert_allclose(u, uv[0], rtol=1e-9, atol=1e-9)
        np.testing.assert_allclose(v, uv[1], rtol=1e-9, atol=1e-9)


# --- P6 + golden: falloff at the grid border (Sec. 3.2 isolines) -------------------------
def test_grid_border_isolines_match_paper():
    with open(os.path.join(GOLDEN, "isolines.json")) as f:
        gold = json.load(f)
    view = sg.frontal_view(200, 200)
    for case in gold["cases"]:
        sig = case["sigma"]
        # a big frontal splat; the pixel whose ray hits (u, v) = (sigma, 0)
        Z, s = 5.0, 2.0
        X, Y, _ = pixel_to_world(view, 100.5, 100.5, Z)
        sc = scene_of([frontal_splat(X, Y, Z, s=(s, s), o=0.9,
                                     tex=np.ones((4, 4, 3)))])
        Xf, Zf, sf = float(sc.means[0, 0]), float(sc.means[0, 2]), float(sc.scales[0, 0])
        x_border = view.cx + view.fx * (Xf + sig * sf) / Zf
        opts = O.Options(sigma=sig)
        M = O.splat_M(sc, view, 0)
        u, v, *_ = O.ray_splat_uv(M, [x_border], [100.5])
        assert u[0] == pytest.approx(sig, rel=1e-9)
        _, _, _, _, _, G, *_ = O._falloff(M, np.array([x_border]), np.array([100.5]), 0.5)
        assert G[0] == pytest.approx(math.exp(-sig * sig / 2), rel=1e-9)
        # "roughly" the quoted isoline: within a factor 1.5 either way
        assert case["approx_falloff_at_border"] / 1.5 < G[0] < case["approx_falloff_at_border"] * 1.5
        # the colour at the border is the edge texel column, and it stays so beyond it (clamp)
        tex = np.zeros((4, 4, 3))
        tex[3, :, :] = 1.0
        col = O.bilinear(tex, [sig, sig * 1.7, sig * 0.99], [0.0, 0.0, 0.0], sig)
        assert col[0] == pytest.approx([1, 1, 1], abs=1e-12)
        assert col[1] == pytest.approx([1, 1, 1], abs=1e-12)
        assert col[2][0] < 1.0


# --- P4: a linear texel field is reproduced exactly (Alg. 2, pins the floor reading) ------
@pytest.mark.parametrize("N", [2, 3, 4, 8, 16])
def test_bilinear_reproduces_linear_fields(N):
    rng = np.random.default_rng(N)
    sig = 0.5
    a, b, c = rng.standard_normal((3, 3))
    i = np.arange(N)[:, None, None]
    j = np.arange(N)[None, :, None]
    C = a + b * i + c * j
    u = rng.uniform(-0.8, 0.8, 500)
    v = rng.uniform(-0.8, 0.8, 500)
    up = np.clip((N - 1) * (u + sig) / (2 * sig), 0, N - 1)
    vp = np.clip((N - 1) * (v + sig) / (2 * sig), 0, N - 1)
    want = a + b * up[:, None] + c * vp[:, None]
    np.testing.assert_allclose(O.bilinear(C, u, v, sig), want, atol=1e-12)
    # texel centres sit at +-sigma: the corners return the corner texels
    got = O.bilinear(C, [-sig, sig, -sig, sig], [-sig, -sig, sig, sig], sig)
    np.testing.assert_allclose(got, [C[0, 0], C[N - 1, 0], C[0, N - 1], C[N - 1, N - 1]], atol=1e-12)


def test_bilinear_N1_is_constant():
    C = np.array([[[0.1, 0.2, 0.3]]])
    got = O.bilinear(C, [-3, 0, 0.2], [1, 0, -0.4], 0.5)
    np.testing.assert_allclose(got, np.broadcast_to([0.1, 0.2, 0.3], (3, 3)))
    dC, du, dv = O.adj_bilinear(C, [0.1, 0.2], [0.0, 0.3], 0.5, np.ones((2, 3)))
    assert (du == 0).all() and (dv == 0).all()
    np.testing.assert_allclose(dC[0, 0], [2, 2, 2])


# --- P10: adj-bilinear against central differences of bilinear (Alg. 2) -------------------
@pytest.mark.parametrize("N", [2, 4, 8, 16])
def test_adj_bilinear_matches_finite_differences(N):
    rng = np.random.default_rng(10 + N)
    sig = 0.5
    C = rng.uniform(0, 1, (N, N, 3))
    for _ in range(40):
        u, v = rng.uniform(-0.9, 0.9, 2)
        dc = rng.standard_normal(3)
        dC, du, dv = O.adj_bilinear(C, [u], [v], sig, dc[None])
        h = 1e-7
        f = lambda uu, vv: float(O.bilinear(C, [uu], [vv], sig)[0] @ dc)
        grid_u = (N - 1) * (u + sig) / (2 * sig)
        grid_v = (N - 1) * (v + sig) / (2 * sig)
        near_kink = lambda g: abs(g - round(g)) < 1e-5
        if not near_kink(grid_u) and abs(abs(u) - sig) > 1e-5:
            assert du[0] == pytest.approx((f(u + h, v) - f(u - h, v)) / (2 * h), rel=1e-6, abs=1e-7)
        if not near_kink(grid_v) and abs(abs(v) - sig) > 1e-5:
            assert dv[0] == pytest.approx((f(u, v + h) - f(u, v - h)) / (2 * h), rel=1e-6, abs=1e-7)
        if abs(u) >= sig:
            assert du[0] == 0.0
        if abs(v) >= sig:
            assert dv[0] == 0.0
        # colour is linear in C: the adjoint is the exact derivative
        for (i, j, c) in [(0, 0, 0), (N - 1, N - 1, 2), (N // 2, 0, 1)]:
            Cp = C.copy()
            Cp[i, j, c] += 1.0
            assert dC[i, j, c] == pytest.approx(
                float(O.bilinear(Cp, [u], [v], sig)[0] @ dc) - f(u, v), abs=1e-12)


# --- P2: constant texture == plain 2DGS (N = 1, Sec. 4.1 ablation) -----------------------
def test_constant_texture_equals_plain_2dgs():
    scene, views = sg.config("C1", P=200)
    view = sg.look_at_view((0, 0, -3.0), 48, 40)
    colors = np.random.default_rng(3).uniform(0, 1, (scene.P, 3)).astype(np.float32)
    tex4 = np.ascontiguousarray(np.broadcast_to(colors[:, None, None, :], (scene.P, 4, 4, 3)))
    tex1 = np.ascontiguousarray(colors[:, None, None, :])
    s4 = sg.Scene(scene.means, scene.tan_u, scene.tan_v, scene.scales, scene.opacity, tex4)
    s1 = sg.Scene(scene.means, scene.tan_u, scene.tan_v, scene.scales, scene.opacity, tex1)
    r4 = O.render(s4, view, O.Options())
    r1 = O.render(s1, view, O.Options())
    np.testing.assert_allclose(r4.rgb, r1.rgb, atol=1e-13)
    np.testing.assert_array_equal(r4.T_final, r1.T_final)
    # and the box-filtered (coarsest level) grid of a varying texture is its mean colour
    C = np.random.default_rng(4).uniform(0, 1, (8, 8, 3))
    np.testing.assert_allclose(O.box_filter_grid(C, 8)[0, 0], C.mean(axis=(0, 1)))


# --- P3: blend weights plus residual transmittance sum to one (Eq. 2 telescopes) ---------
@pytest.mark.parametrize("t_min", [1e-4, 0.0])
def test_weights_plus_transmittance_sum_to_one(t_min):
    scene, _ = sg.config("C1", P=300)
    view = sg.look_at_view((0, 0, -3.0), 40, 32)
    white = sg.Scene(scene.means, scene.tan_u, scene.tan_v, scene.scales, scene.opacity,
                     np.ones_like(scene.textures))
    r = O.render(white, view, O.Options(t_min=t_min))
    np.testing.assert_allclose(r.rgb[..., 0] + r.T_final, 1.0, atol=1e-12)
    rb = O.render(white, view, O.Options(t_min=t_min, bg=(1.0, 1.0, 1.0)))
    np.testing.assert_allclose(rb.rgb, 1.0, atol=1e-12)


# --- P7: symmetries fix the texture axis order ------------------------------------------
def test_swap_uv_axes_with_transposed_grid():
    scene, _ = sg.config("C1", P=150)
    view = sg.look_at_view((0, 0, -3.0), 40, 40)
    swapped = sg.Scene(scene.means, scene.tan_v, scene.tan_u,
                       np.ascontiguousarray(scene.scales[:, ::-1]), scene.opacity,
                       np.ascontiguousarray(scene.textures.transpose(0, 2, 1, 3)))
    a = O.render(scene, view, O.Options())
    b = O.render(swapped, view, O.Options())
    np.testing.assert_allclose(a.rgb, b.rgb, atol=1e-12)


def test_flip_u_with_flipped_grid():
    scene, _ = sg.config("C1", P=150)
    view = sg.look_at_view((0, 0, -3.0), 40, 40)
    flipped = sg.Scene(scene.means, np.ascontiguousarray(-scene.tan_u), scene.tan_v,
                       scene.scales, scene.opacity,
                       np.ascontiguousarray(scene.textures[:, ::-1, :, :]))
    a = O.render(scene, view, O.Options())
    b = O.render(flipped, view, O.Options())
    np.testing.assert_allclose(a.rgb, b.rgb, atol=1e-12)
    # flipping the grid along the other axis is not a symmetry
    wrong = sg.Scene(scene.means, np.ascontiguousarray(-scene.tan_u), scene.tan_v,
                     scene.scales, scene.opacity,
                     np.ascontiguousarray(scene.textures[:, :, ::-1, :]))
    c = O.render(wrong, view, O.Options())
    assert np.abs(a.rgb - c.rgb).max() > 1e-3


# --- P11: stacked layers, transmittance product and early termination --------------------
def test_stacked_layers_terminate_at_t_min():
    view = sg.frontal_view(16, 16)
    cols = np.random.default_rng(5).uniform(0, 1, (6, 3))
    splats = []
    for k in range(6):
        X, Y, Z = pixel_to_world(view, 8.5, 8.5, 2.0 + 0.1 * k)
        splats.append(frontal_splat(X, Y, Z, s=(1.0, 1.0), o=0.95,
                                    tex=np.broadcast_to(cols[k], (2, 2, 3)), N=2))
    sc = scene_of(splats)
    r = O.render(sc, view, O.Options())
    # T: 1 -> .05 -> .0025 -> .000125; the 4th would give 6.25e-6 < 1e-4 and ends the pixel
    o = float(sc.opacity[0])
    tex = sc.textures[:, 0, 0].astype(np.float64)
    assert r.n_blended[8, 8] == 3 and r.terminated[8, 8]
    assert r.T_final[8, 8] == pytest.approx((1 - o) ** 3, rel=1e-12)
    want = sum(o * (1 - o) ** k * tex[k] for k in range(3))
    np.testing.assert_allclose(r.rgb[8, 8], want, rtol=1e-12)
    # without the early stop all six layers blend
    r0 = O.render(sc, view, O.Options(t_min=0.0))
    assert r0.n_blended[8, 8] == 6
    assert r0.T_final[8, 8] == pytest.approx((1 - o) ** 6, rel=1e-12)


# --- P12: equal depths are ordered by splat index ---------------------------------------
def test_equal_depth_orders_by_index():
    view = sg.frontal_view(16, 16)
    X, Y, Z = pixel_to_world(view, 8.5, 8.5, 3.0)
    red, blue = np.array([1.0, 0, 0]), np.array([0, 0, 1.0])
    sc = scene_of([frontal_splat(X, Y, Z, o=0.5, tex=np.broadcast_to(red, (2, 2, 3)), N=2),
                   frontal_splat(X, Y, Z, o=0.5, tex=np.broadcast_to(blue, (2, 2, 3)), N=2)])
    r = O.render(sc, view, O.Options())
    np.testing.assert_allclose(r.rgb[8, 8], 0.5 * red + 0.25 * blue, atol=1e-12)
    ks = O.key_stage(sc, view, O.Options())
    assert list(O.depth_order(ks)) == [0, 1]


# --- Key stage: hand-computed rectangle and brute-force conservativeness ------------------
def test_key_stage_rectangle_of_a_frontal_splat():
    view = sg.frontal_view(200, 100)
    sc = scene_of([frontal_splat(0.1, -0.05, 2.0, s=(0.05, 0.02), o=0.5)])
    ks = O.key_stage(sc, view, O.Options())
    X, Y, Z = (float(c) for c in sc.means[0])
    su, sv = (float(c) for c in sc.scales[0])
    cx, cy = view.cx + view.fx * X / Z, view.cy + view.fy * Y / Z
    rx, ry = view.fx * 3.33 * su / Z, view.fy * 3.33 * sv / Z
    xmin, xmax = min(cx - rx, cx - 2.36) - 0.01, max(cx + rx, cx + 2.36) + 0.01
    ymin, ymax = min(cy - ry, cy - 2.36) - 0.01, max(cy + ry, cy + 2.36) + 0.01
    want = [math.ceil(xmin - 0.5), math.floor(xmax - 0.5), math.ceil(ymin - 0.5),
            math.floor(ymax - 0.5)]
    assert list(ks["rect"][0]) == want
    assert list(ks["tile_rect"][0]) == [want[0] // 16, want[1] // 16, want[2] // 16, want[3] // 16]
    assert ks["count"][0] == (want[1] // 16 - want[0] // 16 + 1) * (want[3] // 16 - want[2] // 16 + 1)
    assert ks["depth"][0] == np.float32(2.0)


def test_key_stage_culls():
    view = sg.frontal_view(64, 64)
    sc = scene_of([frontal_splat(0, 0, -1.0), frontal_splat(0, 0, 2.0, o=0.003),
                   frontal_splat(50.0, 0, 2.0), frontal_splat(0, 0, 2.0)])
    ks = O.key_stage(sc, view, O.Options())
    assert list(ks["visible"]) == [False, False, False, True]
    assert list(ks["count"][:3]) == [0, 0, 0]


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_key_stage_rect_contains_every_contributing_pixel(seed):
    """Brute force: evaluate every visible splat at every pixel; alpha >= alpha_min only
    inside its rectangle (tiny scenes of big and grazing splats)."""
    rng = np.random.default_rng(100 + seed)
    P = 12
    scene = sg.make_scene(seed, P, -0.6, 0.6, 0.05, 0.6, 2)
    view = sg.look_at_view(rng.standard_normal(3) * 0 + np.array([0.3, -0.2, -2.5]), 40, 30)
    opts = O.Options()
    ks = O.key_stage(scene, view, opts)
    x, y = O._pixel_grid((0, 0, 40, 30))
    for k in range(P):
        M = O.splat_M(scene, view, k)
        *_, G, _, _, _ = O._falloff(M, x, y, opts.lowpass_var)
        u, v, valid, *_ = O.ray_splat_uv(M, x, y)
        alpha = np.minimum(opts.alpha_max, float(scene.opacity[k]) * G)
        hit = valid & (alpha >= opts.alpha_min)
        if not ks["visible"][k]:
            continue
        i0, i1, j0, j1 = ks["rect"][k]
        ii, jj = (x - 0.5).astype(int), (y - 0.5).astype(int)
        inside = (ii >= i0) & (ii <= i1) & (jj >= j0) & (jj <= j1)
        assert not (hit & ~inside).any()


def test_tile_pairs_invariants_multi_view():
    scene, _ = sg.config("C1", P=400)
    views = [sg.look_at_view((0, 0, -3.0), 70, 50), sg.look_at_view((2.0, 1.0, -2.0), 33, 47)]
    opts = O.Options()
    keys, vals, ranges = O.tile_pairs(scene, views, opts)
    total = 0
    for v, view in enumerate(views):
        total += O.key_stage(scene, view, opts)["count"].sum()
    assert keys.size == total
    assert (np.diff(keys.astype(np.int64)) >= 0).all()
    covered = ranges[:, 1] - ranges[:, 0]
    assert covered.sum() == keys.size
    for tile in range(ranges.shape[0]):
        s, e = ranges[tile]
        if e > s:
            assert (keys[s:e] == tile).all()
            rec = vals[s:e].astype(np.int64)
            view_id = rec // scene.P
            assert (view_id == view_id[0]).all()
            ks = O.key_stage(scene, views[view_id[0]], opts)
            d = ks["depth"][rec % scene.P].view(np.uint32).astype(np.int64)
            order = np.lexsort((rec, d))
            assert (order == np.arange(order.size)).all()


# --- P8: analytic gradient vs central finite differences (fp64) --------------------------
def _loss(scene, view, opts, g):
    r = O.render(scene, view, opts)
    return float(np.sum(r.rgb.reshape(-1, 3) * g)), r


def _decisions(r):
    return r.n_blended.copy(), r.terminated.copy()


@pytest.mark.parametrize("thresholds", ["default", "off"])
def test_oracle_gradient_matches_central_differences(thresholds):
    rng = np.random.default_rng(7)
    P = 4
    scene = sg.make_scene(21, P, -0.3, 0.3, 0.08, 0.3, 3)
    view = sg.look_at_view((0.2, -0.1, -2.0), 24, 20)
    if thresholds == "off":
        opts = O.Options(alpha_min=0.0, t_min=0.0, alpha_max=1.0, bg=(0.2, 0.3, 0.4))
    else:
        opts = O.Options(bg=(0.1, 0.0, 0.5))
    g = rng.standard_normal((24 * 20, 3))
    r = O.render(scene, view, opts, keep_saved=True)
    gr = O.render_backward(scene, view, opts, r, g)
    fields = ["means", "tan_u", "tan_v", "scales", "opacity", "textures"]
    checked = 0
    for name in fields:
        arr = getattr(scene, name)
        ana = getattr(gr, name)
        flat_idx = rng.choice(arr.size, size=min(arr.size, 10), replace=False)
        for fi in flat_idx:
            idx = np.unravel_index(fi, arr.shape)
            base = float(arr[idx])
            h = 1e-3 * max(1.0, abs(base)) if name == "textures" else 1e-4 * max(0.1, abs(base))
            vals = []
            decs = []
            for sgn in (1, -1):
                s2 = sg.Scene(*(a.astype(np.float64) for a in
                                (scene.means, scene.tan_u, scene.tan_v, scene.scales,
                                 scene.opacity, scene.textures)))
                getattr(s2, name)[idx] = base + sgn * h
                L, rr = _loss(s2, view, opts, g)
                vals.append(L)
                decs.append(_decisions(rr))
            if not all((a == b).all() for a, b in zip(decs[0], decs[1])):
                continue
            fd = (vals[0] - vals[1]) / (2 * h)
            a = float(ana[idx])
            assert a == pytest.approx(fd, rel=2e-5, abs=2e-6 * max(1.0, abs(fd))), (name, idx)
            checked += 1
    assert checked >= 40


# --- Screen-space low-pass: closed form at a known offset from a sub-pixel splat -----------
@pytest.mark.parametrize("var", [0.5, 1.0, 0.25])
def test_lowpass_falloff_closed_form(var):
    """A splat far smaller than a pixel covers no pixel centre in uv (u, v are in the
    thousands there), so only the low-pass acts: at a pixel centre whose distance to the
    projected centre is d, alpha = o exp(-d^2 / (2 var)). With the camera at the origin and the
    splat at depth Z = fx, the projected centre is (X + cx, Y + cy), so d is set exactly."""
    view = sg.frontal_view(48, 40)
    Z = float(np.float32(view.fx))
    o = 0.7
    for dx, dy in [(0.3, 0.0), (1.1, -0.4), (0.0, 2.0), (-1.5, 1.25)]:
        px, py = 20, 17
        X = px + 0.5 + dx - view.cx
        Y = py + 0.5 + dy - view.cy
        sc = scene_of([frontal_splat(X, Y, Z, s=(1e-4, 1e-4), o=o, tex=np.ones((2, 2, 3)),
                                     N=2)])
        Xf, Yf, Zf = (float(c) for c in sc.means[0])
        d2 = (Xf * view.fx / Zf + view.cx - (px + 0.5)) ** 2 + \
             (Yf * view.fy / Zf + view.cy - (py + 0.5)) ** 2
        opts = O.Options(lowpass_var=var)
        r = O.render(sc, view, opts)
        want = float(sc.opacity[0]) * math.exp(-d2 / (2.0 * var))
        if want >= opts.alpha_min:
            assert 1.0 - r.T_final[py, px] == pytest.approx(want, rel=1e-9)
            assert r.rgb[py, px, 0] == pytest.approx(want, rel=1e-9)
        else:
            assert r.T_final[py, px] == 1.0


@pytest.mark.parametrize("var", [0.5, 1.0, 2.0])
def test_key_stage_rect_contains_lowpass_disk(var):
    """Sub-pixel splats contribute only through the low-pass; every pixel where alpha >=
    alpha_min must lie in the key stage's rectangle, for any low-pass variance."""
    rng = np.random.default_rng(int(var * 10))
    view = sg.frontal_view(40, 32)
    Z = 3.0
    splats = []
    for _ in range(20):
        x, y = rng.uniform(2, 38), rng.uniform(2, 30)
        X, Y, _ = pixel_to_world(view, x, y, Z)
        splats.append(frontal_splat(X, Y, Z, s=(1e-4, 2e-4), theta=rng.uniform(0, 3), o=0.95,
                                    tex=np.ones((2, 2, 3)), N=2))
    sc = scene_of(splats)
    opts = O.Options(lowpass_var=var)
    ks = O.key_stage(sc, view, opts)
    x, y = O._pixel_grid((0, 0, 40, 32))
    ii, jj = (x - 0.5).astype(int), (y - 0.5).astype(int)
    widest = 0
    for k in range(len(splats)):
        M = O.splat_M(sc, view, k)
        *_, G, _, _, _ = O._falloff(M, x, y, var)
        hit = np.minimum(opts.alpha_max, float(sc.opacity[k]) * G) >= opts.alpha_min
        assert ks["visible"][k]
        i0, i1, j0, j1 = ks["rect"][k]
        inside = (ii >= i0) & (ii <= i1) & (jj >= j0) & (jj <= j1)
        assert not (hit & ~inside).any()
        widest = max(widest, int(np.ptp(ii[hit])) if hit.any() else 0)
    # the disk really widens with the variance (radius sqrt(2 var ln(255 o)))
    assert widest >= 2 * math.floor(math.sqrt(2 * var * math.log(255 * 0.95))) - 1


# --- Exact pruning changes nothing: crop renders equal the same pixels of a full render -----
@pytest.mark.parametrize("seed", [0, 1])
def test_crop_render_equals_full_render(seed):
    """Pruning is for speed only. Large, grazing and sub-pixel splats straddle the crop
    edges; every crop must reproduce the full render's pixels, with pruning on and off."""
    rng = np.random.default_rng(300 + seed)
    big = sg.make_scene(seed, 40, -0.8, 0.8, 0.1, 0.7, 4)
    tiny = sg.make_scene(seed + 9, 40, -0.8, 0.8, 3e-4, 2e-3, 2)
    # sub-pixel splats keep a 4x4 grid shape (constant rows) so that both sets stack
    tiny_tex = np.repeat(np.repeat(tiny.textures, 2, axis=1), 2, axis=2)
    scene = sg.Scene(*(np.ascontiguousarray(np.concatenate([a, b])) for a, b in
                       zip((big.means, big.tan_u, big.tan_v, big.scales, big.opacity, big.textures),
                           (tiny.means, tiny.tan_u, tiny.tan_v, tiny.scales, tiny.opacity,
                            tiny_tex))))
    view = sg.look_at_view(np.array([0.4, -0.3, -2.4]) + 0.1 * rng.standard_normal(3), 60, 44)
    opts = O.Options(bg=(0.2, 0.1, 0.3), lowpass_var=[0.5, 1.0][seed])
    full = O.render(scene, view, opts)
    for crop in [(0, 0, 13, 9), (17, 11, 20, 14), (41, 30, 19, 14), (29, 0, 3, 44)]:
        x0, y0, w, h = crop
        for prune in (True, False):
            r = O.render(scene, view, opts, crop=crop, prune=prune)
            np.testing.assert_allclose(r.rgb, full.rgb[y0:y0 + h, x0:x0 + w], rtol=0, atol=1e-13)
            np.testing.assert_allclose(r.T_final, full.T_final[y0:y0 + h, x0:x0 + w], rtol=0,
                                       atol=1e-13)
    # pruning did drop splats here (so the test exercises it)
    order = O.depth_order(O.key_stage(scene, view, opts))
    kept = O.prune_for_crop(scene, view, opts, order, (0, 0, 13, 9))
    assert kept.size < order.size


# --- Flagged pixels: the admissible outcomes of a decision inside its flag band ------------
def test_flagged_outcomes_cover_both_sides_of_alpha_min():
    """A splat whose opacity is the float32 value nearest 1/255 is centred on a pixel, so its
    alpha there is within 1e-7 of alpha_min and the pixel is flagged. Rendering with alpha_min
    moved slightly down (the splat blends) and up (it is skipped) must give two of the
    outcomes the oracle enumerates, and every outcome lies within the decision's bound."""
    view = sg.frontal_view(16, 16)
    X, Y, Z = pixel_to_world(view, 8.5, 6.5, 2.0)
    Xb, Yb, Zb = pixel_to_world(view, 8.0, 6.0, 3.0)
    sc = scene_of([frontal_splat(X, Y, Z, o=float(np.float32(1.0 / 255.0)),
                                 tex=np.full((4, 4, 3), 0.9)),
                   frontal_splat(Xb, Yb, Zb, o=0.8, s=(0.3, 0.3),
                                 tex=np.full((4, 4, 3), 0.2))])
    opts = O.Options()
    r = O.render(sc, view, opts)
    assert O.image_flags(r)[6, 8]
    outs = O.flagged_outcomes(sc, view, opts, r, 6, 8)
    assert outs is not None and len(outs) == 2
    for am in (opts.alpha_min * (1 - 1e-6), opts.alpha_min * (1 + 1e-6)):
        rr = O.render(sc, view, O.Options(alpha_min=am))
        assert min(np.abs(rgb - rr.rgb[6, 8]).max() + abs(T - rr.T_final[6, 8])
                   for rgb, T in outs) < 1e-12
    b = O.flagged_bound(sc, r, 6, 8)
    for rgb, T in outs:
        assert np.abs(rgb - r.rgb[6, 8]).max() <= b + 1e-15


def test_flagged_outcomes_cover_both_sides_of_t_min():
    """Stacked layers whose transmittance after the third lands exactly on t_min: the stop
    decision is flagged; t_min moved slightly either way gives two of the enumerated
    outcomes."""
    view = sg.frontal_view(17, 17)  # principal point at the centre of pixel (8, 8)
    o = 0.9
    layers = [frontal_splat(0.0, 0.0, 2.0 + 0.1 * i, o=o, tex=np.full((4, 4, 3), 0.1 * (i + 1)))
              for i in range(5)]
    sc = scene_of(layers)
    of = float(sc.opacity[0])
    t_star = (1.0 - of) ** 3
    opts = O.Options(t_min=t_star)
    r = O.render(sc, view, opts)
    assert O.image_flags(r)[8, 8]
    outs = O.flagged_outcomes(sc, view, opts, r, 8, 8)
    assert outs is not None and len(outs) >= 2
    for tm in (t_star * (1 - 1e-6), t_star * (1 + 1e-6)):
        rr = O.render(sc, view, O.Options(t_min=tm))
        assert min(np.abs(rgb - rr.rgb[8, 8]).max() + abs(T - rr.T_final[8, 8])
                   for rgb, T in outs) < 1e-12
    b = O.flagged_bound(sc, r, 8, 8)
    for rgb, T in outs:
        assert np.abs(rgb - r.rgb[8, 8]).max() <= b + 1e-15


@pytest.mark.parametrize("tile", [(16, 16), (8, 8), (32, 8)])
def test_vectorised_tile_pairs_equal_the_plain_expansion(tile):
    """The array-based pair expansion used at full size gives exactly the pairs of the plain
    per-splat loop (several views, every tile shape)."""
    scene, _ = sg.config("C1", P=600)
    views = [sg.look_at_view((0, 0, -3.0), 70, 50), sg.look_at_view((2.0, 1.0, -2.0), 33, 47),
             sg.look_at_view((0.3, -2.5, -0.4), 64, 64)]
    opts = O.Options(tile_w=tile[0], tile_h=tile[1])
    a = O.tile_pairs(scene, views, opts)
    b = O.tile_pairs_vectorised(scene, views, opts)
    for x, y in zip(a, b):
        np.testing.assert_array_equal(x, y)


# --- Diffuse-specular split (Sec. 4.2): per-splat spherical harmonics -----------------------
def _real_sh_from_scipy(d, degree):
    """The basis built from scipy's complex harmonics (Condon-Shortley phase included):
    sqrt(2) Re Y_l^m for m > 0, sqrt(2) Im Y_l^|m| for m < 0, Y_l^0 for m = 0."""
    from scipy.special import sph_harm_y
    theta = np.arccos(np.clip(d[:, 2], -1.0, 1.0))
    phi = np.arctan2(d[:, 1], d[:, 0])
    cols = []
    for l in range(degree + 1):
        for m in range(-l, l + 1):
            Y = sph_harm_y(l, abs(m), theta, phi)
            if m > 0:
                cols.append(math.sqrt(2.0) * Y.real)
            elif m < 0:
                cols.append(math.sqrt(2.0) * Y.imag)
            else:
                cols.append(Y.real)
    return np.stack(cols, axis=1)


def _unit(n, seed):
    d = np.random.default_rng(seed).standard_normal((n, 3))
    return d / np.linalg.norm(d, axis=1, keepdims=True)


@pytest.mark.parametrize("degree", [0, 1, 2, 3])
def test_sh_basis_matches_scipy_harmonics(degree):
    d = _unit(200, degree)
    np.testing.assert_allclose(O.sh_basis(d, degree), _real_sh_from_scipy(d, degree),
                               rtol=1e-12, atol=1e-13)


def test_sh_basis_is_orthonormal_on_the_sphere():
    """Gauss-Legendre in cos(theta) times a uniform rule in phi integrates every product of
    two degree-3 harmonics (degree 6 in x, y, z) exactly."""
    xs, ws = np.polynomial.legendre.leggauss(8)
    phis = 2.0 * math.pi * np.arange(16) / 16
    ct, ph = np.meshgrid(xs, phis, indexing="ij")
    w = (ws[:, None] * np.full(16, 2.0 * math.pi / 16)[None, :]).reshape(-1)
    st = np.sqrt(1.0 - ct ** 2)
    d = np.stack([st * np.cos(ph), st * np.sin(ph), ct], axis=-1).reshape(-1, 3)
    Y = O.sh_basis(d, 3)
    gram = (Y * w[:, None]).T @ Y
    np.testing.assert_allclose(gram, np.eye(16), atol=1e-12)


def test_sh_basis_on_the_axes():
    """Closed forms on the coordinate axes: on +z only the zonal harmonics survive,
    Y_00 = 1/(2 sqrt(pi)), Y_10 = sqrt(3/(4 pi)), Y_20 = sqrt(5/pi)/2, Y_30 = sqrt(7/pi)/2;
    on +x the order-1 term is -sqrt(3/(4 pi)) (the (-1)^m sign) and Y_22 = sqrt(15/pi)/4."""
    d = np.array([[0.0, 0.0, 1.0], [1.0, 0.0, 0.0], [0.0, -1.0, 0.0]])
    Y = O.sh_basis(d, 3)
    pi = math.pi
    want_z = np.zeros(16)
    want_z[[0, 2, 6, 12]] = [0.5 / math.sqrt(pi), math.sqrt(3 / (4 * pi)), 0.5 * math.sqrt(5 / pi),
                             0.5 * math.sqrt(7 / pi)]
    np.testing.assert_allclose(Y[0], want_z, atol=1e-15)
    assert Y[1, 3] == pytest.approx(-math.sqrt(3 / (4 * pi)), rel=1e-14)
    assert Y[1, 8] == pytest.approx(0.25 * math.sqrt(15 / pi), rel=1e-14)
    assert Y[1, 6] == pytest.approx(-0.25 * math.sqrt(5 / pi), rel=1e-14)
    assert Y[2, 1] == pytest.approx(math.sqrt(3 / (4 * pi)), rel=1e-14)  # -c1 y at y = -1


def test_sh_degree0_is_a_constant_colour_offset():
    """Degree 0 adds sh_0 / (2 sqrt(pi)) to every texel's colour, whatever the view: the same
    image as the grid shifted by that constant, from two viewpoints."""
    base = sg.make_scene(12, 30, -0.5, 0.5, 0.05, 0.3, 4)
    spec = sg.with_sh(base, 5, 0)
    shifted = sg.Scene(base.means, base.tan_u, base.tan_v, base.scales, base.opacity,
                       np.ascontiguousarray(base.textures.astype(np.float64)
                                            + spec.sh[:, 0, None, None, :].astype(np.float64)
                                            * 0.5 / math.sqrt(math.pi)))
    for pos in ((0.2, 0.1, -2.5), (-1.5, 0.8, -1.5)):
        view = sg.look_at_view(pos, 40, 32)
        a = O.render(spec, view, O.Options())
        b = O.render(shifted, view, O.Options())
        np.testing.assert_allclose(a.rgb, b.rgb, atol=1e-12)


def test_specular_term_depends_on_the_view_direction():
    """A degree-1 term with coefficients along z only: a frontal splat seen from directions
    d gets the colour shift -c1 (d . (0, 1, 0)) ... i.e. sum_j Y_j(d) sh_j; seen from straight
    ahead (d = +z) the shift is sqrt(3/(4 pi)) sh_2."""
    view = sg.frontal_view(17, 17)
    sc = scene_of([frontal_splat(0.0, 0.0, 3.0, o=0.5, tex=np.zeros((2, 2, 3)), N=2)])
    sh = np.zeros((1, 4, 3), dtype=np.float32)
    sh[0, 2] = [0.4, -0.2, 0.1]
    sc = sg.Scene(sc.means, sc.tan_u, sc.tan_v, sc.scales, sc.opacity, sc.textures, sh)
    r = O.render(sc, view, O.Options())
    shift = math.sqrt(3 / (4 * math.pi)) * sh[0, 2].astype(np.float64)
    np.testing.assert_allclose(r.rgb[8, 8], float(sc.opacity[0]) * shift, atol=1e-12)


@pytest.mark.parametrize("degree", [1, 3])
def test_specular_gradients_match_central_differences(degree):
    """The analytic gradient with respect to the SH coefficients and the centres (through the
    view direction) against central differences of the render."""
    rng = np.random.default_rng(90 + degree)
    scene = sg.with_sh(sg.make_scene(31, 4, -0.3, 0.3, 0.08, 0.3, 3), 7, degree, scale=0.3)
    view = sg.look_at_view((0.6, -0.4, -1.6), 24, 20)
    opts = O.Options(bg=(0.1, 0.2, 0.3))
    g = rng.standard_normal((24 * 20, 3))
    r = O.render(scene, view, opts, keep_saved=True)
    gr = O.render_backward(scene, view, opts, r, g)
    checked = 0
    for name in ("sh", "means"):
        arr = getattr(scene, name)
        for fi in rng.choice(arr.size, size=10, replace=False):
            idx = np.unravel_index(fi, arr.shape)
            h = 1e-4 * max(0.1, abs(float(arr[idx])))
            vals, decs = [], []
            for sgn in (1, -1):
                parts = [a.astype(np.float64) for a in (scene.means, scene.tan_u, scene.tan_v,
                                                         scene.scales, scene.opacity,
                                                         scene.textures, scene.sh)]
                target = parts[6] if name == "sh" else parts[0]
                target[idx] += sgn * h
                rr = O.render(sg.Scene(*parts), view, opts)
                vals.append(float(np.sum(rr.rgb.reshape(-1, 3) * g)))
                decs.append((rr.n_blended.copy(), rr.terminated.copy()))
            if not all((a == b).all() for a, b in zip(decs[0], decs[1])):
                continue
            fd = (vals[0] - vals[1]) / (2 * h)
            a = float(getattr(gr, name)[idx])
            assert a == pytest.approx(fd, rel=2e-5, abs=2e-6 * max(1.0, abs(fd))), (name, idx)
            checked += 1
    assert checked >= 14


# --- colour grids of several sides in one scene ----------------------------------------------
def _refine_weights(n, L):
    """[L, n] weights of the exact refinement of a corner-aligned n-texel side to L texels,
    where the coarse knots are fine knots ((L - 1) a multiple of (n - 1), or n = 1): fine texel
    i lies at coarse coordinate x = i (n - 1) / (L - 1), between knots floor(x) and floor(x) + 1
    with weights 1 - frac(x) and frac(x) (one knot of weight 1 for n = 1)."""
    W = np.zeros((L, n))
    if n == 1:
        W[:, 0] = 1.0
        return W
    step = (L - 1) // (n - 1)
    assert step * (n - 1) == L - 1
    for i in range(L):
        a, r = divmod(i, step)
        if a == n - 1:
            W[i, a] = 1.0
        else:
            W[i, a] = 1.0 - r / step
            W[i, a + 1] = r / step
    return W


@pytest.mark.parametrize("layout,sides", [(8, (1, 2, 8)), (16, (1, 2, 4, 16))])
def test_mixed_sides_equal_their_exact_refinement(layout, sides):
    """A scene whose grids have several sides renders exactly as the same scene with every
    coarse grid refined to the largest side (a bilinear field on a coarse grid is bilinear on
    every cell of a refinement whose knots include the coarse knots), and the coarse grids'
    gradients are the refinement's transpose applied to the refined grids' gradients; the
    other gradients are equal."""
    base = sg.make_scene(23 + layout, 40, -0.6, 0.6, 0.05, 0.35, layout)
    scene = sg.with_mixed_sides(base, 5, sides)
    assert {g.shape[0] for g in scene.textures} == set(sides)
    fine = [np.einsum("ia,jb,abc->ijc", _refine_weights(g.shape[0], layout),
                      _refine_weights(g.shape[0], layout), g.astype(np.float64))
            for g in scene.textures]
    refined = dataclasses.replace(scene, textures=np.stack(fine))
    view = sg.look_at_view((0.3, -0.2, -2.4), 40, 36)
    opts = O.Options(bg=(0.1, 0.3, 0.2))
    a = O.render(scene, view, opts, keep_saved=True)
    b = O.render(refined, view, opts, keep_saved=True)
    np.testing.assert_allclose(a.rgb, b.rgb, rtol=0, atol=1e-12)
    np.testing.assert_allclose(a.T_final, b.T_final, rtol=0, atol=1e-12)
    g = np.random.default_rng(3).standard_normal((40 * 36, 3))
    ga = O.render_backward(scene, view, opts, a, g)
    gb_ = O.render_backward(refined, view, opts, b, g)
    for name in ("means", "tan_u", "tan_v", "scales", "opacity"):
        np.testing.assert_allclose(getattr(ga, name), getattr(gb_, name), rtol=1e-9, atol=1e-12)
    for k, gk in enumerate(ga.textures):
        W = _refine_weights(gk.shape[0], layout)
        want = np.einsum("ia,jb,ijc->abc", W, W, gb_.textures[k])
        np.testing.assert_allclose(gk, want, rtol=1e-9, atol=1e-12)
    assert sum(float(np.abs(gk).sum()) > 0 for gk in ga.textures) >= 10
