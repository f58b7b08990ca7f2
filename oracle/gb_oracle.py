"""FP64 CPU oracle for the Gaussian Billboards rasterizer (textured 2D Gaussian splats).

TEST INFRASTRUCTURE ONLY. Only the tests, the smoke check and the CPU-baseline leg of the
benchmark may import this module. The product path (the HIP library and its binding) never
imports or calls it, and this module imports nothing from the product path.

What it computes, and where the paper fixes it:

* Primitive (Sec. 3.1, Eq. 3): centre p, tangents t_u, t_v, scales (s_u, s_v); the tangent
  plane P(u, v) = p + s_u t_u u + s_v t_v v.
* Opacity falloff in uv (Sec. 3.1, Eq. 4): G(u, v) = exp(-(u^2 + v^2) / 2).
* Colour (Sec. 3.2, Eq. 5 and Alg. 2): bilinear lookup in the N x N x 3 grid C_k spanning
  [-sigma, sigma]^2 of the uv plane, coordinates border-clamped.
* Compositing (Sec. 3.1, Eq. 2; Alg. 1): front-to-back over splats sorted by centre depth.
* Backward (Alg. 1 backward, Alg. 2 adj-bilinear): hand-derived adjoints.
* Diffuse-specular split (Sec. 4.2): optionally one set of spherical-harmonic coefficients
  per splat adds a view-dependent colour, the same over the splat, to the grid's colour.

Readings where the paper is silent or garbled (each one is also listed in the design notes):

* Alg. 2 writes ``i_u = floor(u)``; it must be the floor of the remapped u' (the fraction
  f_u = u' - i_u only makes sense then). At the clamped top edge u' = N - 1 the cell index is
  limited to N - 2 so that f_u = 1 and no texel past the grid is read. N = 1 returns the one
  texel and no uv gradient.
* Texel centres sit at +-sigma (corner-aligned map [-sigma, sigma] -> [0, N-1], Alg. 2); the
  grid is indexed C[i_u, i_v, c].
* The ray-splat intersection is the homogeneous solve (u, v, 1) ~ h_x x h_y with
  M = K [R s_u t_u | R s_v t_v | R p + t], h_x = x M_2 - M_0, h_y = y M_2 - M_1. rho_2 = 0 means
  no hit; there is no test on the side of the camera.
* A screen-space low-pass of variance var (default 1/2 px^2) bounds the falloff from below:
  G_hat = exp(-min(q_uv, q_lp)), q_uv = (u^2 + v^2)/2, q_lp = |x - c2|^2 / (2 var), c2 the
  projected centre (ties go to the uv branch). The colour still uses the ray's (u, v).
* alpha = min(alpha_max, o * G_hat); alpha < alpha_min is skipped; a splat that would bring the
  transmittance below t_min is not blended and ends the pixel (Alg. 1 is marked simplified;
  these are the conventions of the splatting line of work it extends).
* Splats are ordered by the camera-space depth of their centre, computed by the key stage
  below in float32, ties by splat index.
* Pixel centres are at (i + 1/2, j + 1/2); camera axes x right, y down, z forward.

The key stage (screen rectangle, tile counts, depth key) is defined in float32 with a fixed
operation order so that the tiling is reproducible bit for bit; everything after it is fp64.
Its constants: 3.33 >= sqrt(2 ln 255) bounds the uv radius where o*G >= 1/255 for o <= 1, and
2.36 >= sqrt(ln 255) px bounds the low-pass disk at variance 1/2 (3.34 sqrt(var) above that);
with them the rectangle contains every pixel where alpha >= alpha_min.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

F32 = np.float32


@dataclasses.dataclass
class Options:
    sigma: float = 0.5
    alpha_min: float = 1.0 / 255.0
    alpha_max: float = 0.99
    t_min: float = 1e-4
    lowpass_var: float = 0.5          # sigma_lp^2 in px^2
    bg: Tuple[float, float, float] = (0.0, 0.0, 0.0)
    tile_w: int = 16
    tile_h: int = 16


# ---------------------------------------------------------------------------------------
# Key stage: float32, fixed operation order, no fused multiply-add.
# ---------------------------------------------------------------------------------------
KS_RADIUS_UV = F32(3.33)
KS_RADIUS_LP = F32(2.36)
KS_MARGIN = F32(0.01)

# The rectangle bound above holds for alpha_min >= 1/255; below it the rectangle is the
# whole image (no culling by extent) so that thresholds can be switched off.
KS_ALPHA_FLOOR = F32(1.0 / 255.0)


def ks_lowpass_radius(lowpass_var: float) -> np.float32:
    """Screen radius (px) beyond which the low-pass term alone gives o*G < 1/255 for o <= 1.

    The term is exp(-r^2 / (2 var)), so the bound is sqrt(2 var ln 255) = 3.3290 sqrt(var):
    2.36 covers every variance up to 1/2 (the default); above it the radius is
    3.34 sqrt(var), evaluated in double precision and rounded once to float32.
    """
    var = float(F32(lowpass_var))
    if var <= 0.5:
        return KS_RADIUS_LP
    return F32(3.34 * math.sqrt(var))


def _f(x):
    return np.asarray(x, dtype=F32)


def _rot3(R, x0, x1, x2, i):
    """((R_i0*x0 + R_i1*x1) + R_i2*x2) in float32, every op rounded."""
    return (F32(R[i, 0]) * x0 + F32(R[i, 1]) * x1) + F32(R[i, 2]) * x2


def _fmin(a, b):
    return np.where(a < b, a, b)


def _fmax(a, b):
    return np.where(a > b, a, b)


def key_stage(scene, view, opts: Options) -> Dict[str, np.ndarray]:
    """Per splat: float32 depth, pixel rectangle, tile rectangle and tile count.

    A splat is culled (count 0) if its depth is not beyond z_near, its opacity is below
    alpha_min, or its rectangle misses the image. If any corner of its 3.33-sigma uv square
    is not beyond z_near the rectangle is the whole image.
    """
    p = scene.means.astype(F32)
    R = np.asarray(view.R, dtype=F32)
    t = np.asarray(view.t, dtype=F32)
    p0, p1, p2 = p[:, 0], p[:, 1], p[:, 2]
    pc = [_rot3(R, p0, p1, p2, i) + t[i] for i in range(3)]
    d = pc[2]
    su, sv = scene.scales[:, 0].astype(F32), scene.scales[:, 1].astype(F32)
    wa = [su * scene.tan_u[:, i].astype(F32) for i in range(3)]
    wb = [sv * scene.tan_v[:, i].astype(F32) for i in range(3)]
    a = [_rot3(R, wa[0], wa[1], wa[2], i) for i in range(3)]
    b = [_rot3(R, wb[0], wb[1], wb[2], i) for i in range(3)]
    ra = [KS_RADIUS_UV * a[i] for i in range(3)]
    rb = [KS_RADIUS_UV * b[i] for i in range(3)]
    corners = []
    for sa, sb in ((-1, -1), (1, -1), (-1, 1), (1, 1)):
        q = [((pc[i] + ra[i]) if sa > 0 else (pc[i] - ra[i])) for i in range(3)]
        q = [((q[i] + rb[i]) if sb > 0 else (q[i] - rb[i])) for i in range(3)]
        corners.append(q)
    zn = F32(view.z_near)
    fx, fy, cx, cy = F32(view.fx), F32(view.fy), F32(view.cx), F32(view.cy)
    W, H = int(view.width), int(view.height)
    r_lp = ks_lowpass_radius(opts.lowpass_var)
    with np.errstate(divide="ignore", invalid="ignore", over="ignore"):
        behind = np.zeros(p.shape[0], dtype=bool)
        for q in corners:
            behind |= ~(q[2] > zn)
        if F32(opts.alpha_min) < KS_ALPHA_FLOOR:
            behind[:] = True
        xs = [fx * (q[0] / q[2]) + cx for q in corners]
        ys = [fy * (q[1] / q[2]) + cy for q in corners]
        c2x = fx * (pc[0] / d) + cx
        c2y = fy * (pc[1] / d) + cy
        xmin = _fmin(_fmin(_fmin(_fmin(xs[0], xs[1]), xs[2]), xs[3]), c2x - r_lp) - KS_MARGIN
        xmax = _fmax(_fmax(_fmax(_fmax(xs[0], xs[1]), xs[2]), xs[3]), c2x + r_lp) + KS_MARGIN
        ymin = _fmin(_fmin(_fmin(_fmin(ys[0], ys[1]), ys[2]), ys[3]), c2y - r_lp) - KS_MARGIN
        ymax = _fmax(_fmax(_fmax(_fmax(ys[0], ys[1]), ys[2]), ys[3]), c2y + r_lp) + KS_MARGIN
        half = F32(0.5)
        i0 = np.ceil(xmin - half)
        i1 = np.floor(xmax - half)
        j0 = np.ceil(ymin - half)
        j1 = np.floor(ymax - half)
        i0 = np.where(behind, F32(0), i0)
        j0 = np.where(behind, F32(0), j0)
        i1 = np.where(behind, F32(W - 1), i1)
        j1 = np.where(behind, F32(H - 1), j1)
        on = (i0 <= F32(W - 1)) & (i1 >= F32(0)) & (j0 <= F32(H - 1)) & (j1 >= F32(0))
        on &= (i0 <= i1) & (j0 <= j1)
        on &= (d > zn) & ~(scene.opacity.astype(F32) < F32(opts.alpha_min))
        i0 = np.clip(np.nan_to_num(i0), 0, W - 1)
        i1 = np.clip(np.nan_to_num(i1), 0, W - 1)
        j0 = np.clip(np.nan_to_num(j0), 0, H - 1)
        j1 = np.clip(np.nan_to_num(j1), 0, H - 1)
    i0, i1, j0, j1 = (np.where(on, x, 0).astype(np.int64) for x in (i0, i1, j0, j1))
    tx0, tx1 = i0 // opts.tile_w, i1 // opts.tile_w
    ty0, ty1 = j0 // opts.tile_h, j1 // opts.tile_h
    count = np.where(on, (tx1 - tx0 + 1) * (ty1 - ty0 + 1), 0).astype(np.int64)
    return dict(depth=d.astype(F32), visible=on, rect=np.stack([i0, i1, j0, j1], 1),
                tile_rect=np.stack([tx0, tx1, ty0, ty1], 1), count=count,
                tiles_x=-(-W // opts.tile_w), tiles_y=-(-H // opts.tile_h))


def depth_order(ks) -> np.ndarray:
    """Visible splats sorted ascending by (float32 depth bit pattern, splat index)."""
    idx = np.nonzero(ks["visible"])[0]
    bits = ks["depth"][idx].view(np.uint32)
    return idx[np.lexsort((idx, bits))]


def tile_pairs(scene, views: Sequence, opts: Options):
    """Sorted (tile, record) pairs and per-tile [start, end) ranges over all views.

    Tiles are numbered view by view, row-major within a view; a record is view * P + splat.
    Within a tile the pairs follow the depth order of ``depth_order``.
    """
    P = scene.P
    keys, vals, tiles_per_view = [], [], []
    base = 0
    for v, view in enumerate(views):
        ks = key_stage(scene, view, opts)
        order = depth_order(ks)
        per_tile: Dict[int, List[int]] = {}
        tr = ks["tile_rect"]
        for s in order:
            tx0, tx1, ty0, ty1 = (int(x) for x in tr[s])
            for ty in range(ty0, ty1 + 1):
                for tx in range(tx0, tx1 + 1):
                    per_tile.setdefault(base + ty * ks["tiles_x"] + tx, []).append(v * P + int(s))
        ntiles = ks["tiles_x"] * ks["tiles_y"]
        for tile in range(base, base + ntiles):
            lst = per_tile.get(tile, [])
            keys.extend([tile] * len(lst))
            vals.extend(lst)
        tiles_per_view.append(ntiles)
        base += ntiles
    keys = np.asarray(keys, dtype=np.uint32)
    vals = np.asarray(vals, dtype=np.uint32)
    ranges = np.zeros((base, 2), dtype=np.int64)
    if keys.size:
        starts = np.searchsorted(keys, np.arange(base), side="left")
        ends = np.searchsorted(keys, np.arange(base), side="right")
        ranges[:, 0] = np.where(ends > starts, starts, 0)
        ranges[:, 1] = np.where(ends > starts, ends, 0)
    return keys, vals, ranges


def tile_pairs_vectorised(scene, views: Sequence, opts: Options):
    """The same (tile, record) pairs and ranges as ``tile_pairs``, built with array operations
    so that millions of splats finish in seconds: each visible record, in depth order, is
    repeated once per tile of its rectangle (rows outer, columns inner); a stable sort by
    tile then keeps the depth order inside every tile."""
    P = scene.P
    keys_v, vals_v = [], []
    base = 0
    for v, view in enumerate(views):
        ks = key_stage(scene, view, opts)
        order = depth_order(ks)
        tr = ks["tile_rect"][order]
        tw = tr[:, 1] - tr[:, 0] + 1
        cnt = ks["count"][order]
        rep = np.repeat(np.arange(order.size), cnt)
        first = np.concatenate([[0], np.cumsum(cnt)[:-1]]) if order.size else np.zeros(0, np.int64)
        local = np.arange(rep.size) - first[rep]
        ty = tr[rep, 2] + local // tw[rep]
        tx = tr[rep, 0] + local % tw[rep]
        keys_v.append((base + ty * ks["tiles_x"] + tx).astype(np.int64))
        vals_v.append((v * P + order[rep]).astype(np.int64))
        base += ks["tiles_x"] * ks["tiles_y"]
    keys = np.concatenate(keys_v) if keys_v else np.zeros(0, np.int64)
    vals = np.concatenate(vals_v) if vals_v else np.zeros(0, np.int64)
    srt = np.argsort(keys, kind="stable")
    keys, vals = keys[srt].astype(np.uint32), vals[srt].astype(np.uint32)
    ranges = np.zeros((base, 2), dtype=np.int64)
    if keys.size:
        starts = np.searchsorted(keys, np.arange(base), side="left")
        ends = np.searchsorted(keys, np.arange(base), side="right")
        ranges[:, 0] = np.where(ends > starts, starts, 0)
        ranges[:, 1] = np.where(ends > starts, ends, 0)
    return keys, vals, ranges


# ---------------------------------------------------------------------------------------
# Alg. 2: bilinear colour lookup and its adjoint (fp64, vectorised over lookups).
# ---------------------------------------------------------------------------------------
def _grid_coords(u, N, sigma):
    """u -> (cell index, fraction) on the corner-aligned grid, border-clamped."""
    up = np.clip((N - 1) * (u + sigma) / (2.0 * sigma), 0.0, N - 1)
    i = np.minimum(np.floor(up), N - 2).astype(np.int64)
    return i, up - i


def bilinear(C, u, v, sigma):
    """C: [N,N,3] or [n,N,N,3] (one grid per lookup); u, v: [n]. Returns [n,3]."""
    C = np.asarray(C, dtype=np.float64)
    u = np.atleast_1d(np.asarray(u, dtype=np.float64))
    v = np.atleast_1d(np.asarray(v, dtype=np.float64))
    N = C.shape[-2]
    if C.ndim == 3:
        C = np.broadcast_to(C, (u.shape[0],) + C.shape)
    n = np.arange(u.shape[0])
    if N == 1:
        return C[n, 0, 0, :].copy()
    iu, fu = _grid_coords(u, N, sigma)
    iv, fv = _grid_coords(v, N, sigma)
    fu, fv = fu[:, None], fv[:, None]
    return (C[n, iu, iv] * (1 - fu) * (1 - fv) + C[n, iu + 1, iv] * fu * (1 - fv)
            + C[n, iu, iv + 1] * (1 - fu) * fv + C[n, iu + 1, iv + 1] * fu * fv)


def adj_bilinear(C, u, v, sigma, dc):
    """Adjoint of ``bilinear`` for one grid C [N,N,3] and lookups u, v [n] with output adjoint
    dc [n,3]. Returns (dC [N,N,3] summed over lookups, du [n], dv [n]).

    The uv adjoint is zero where the coordinate is clamped (|u| >= sigma), as in Alg. 2.
    """
    C = np.asarray(C, dtype=np.float64)
    u = np.atleast_1d(np.asarray(u, dtype=np.float64))
    v = np.atleast_1d(np.asarray(v, dtype=np.float64))
    dc = np.asarray(dc, dtype=np.float64).reshape(-1, 3)
    N = C.shape[0]
    dC = np.zeros_like(C)
    if N == 1:
        dC[0, 0] += dc.sum(axis=0)
        return dC, np.zeros_like(u), np.zeros_like(v)
    iu, fu = _grid_coords(u, N, sigma)
    iv, fv = _grid_coords(v, N, sigma)
    fu1, fv1 = fu[:, None], fv[:, None]
    np.add.at(dC, (iu, iv), dc * (1 - fu1) * (1 - fv1))
    np.add.at(dC, (iu + 1, iv), dc * fu1 * (1 - fv1))
    np.add.at(dC, (iu, iv + 1), dc * (1 - fu1) * fv1)
    np.add.at(dC, (iu + 1, iv + 1), dc * fu1 * fv1)
    c00, c10, c01, c11 = C[iu, iv], C[iu + 1, iv], C[iu, iv + 1], C[iu + 1, iv + 1]
    dfu = np.sum(dc * ((c10 - c00) * (1 - fv1) + (c11 - c01) * fv1), axis=1)
    dfv = np.sum(dc * ((c01 - c00) * (1 - fu1) + (c11 - c10) * fu1), axis=1)
    scale = (N - 1) / (2.0 * sigma)
    du = np.where((u > -sigma) & (u < sigma), scale * dfu, 0.0)
    dv = np.where((v > -sigma) & (v < sigma), scale * dfv, 0.0)
    return dC, du, dv


# ---------------------------------------------------------------------------------------
# Ray-splat intersection (Eq. 3 solved for the pixel ray).
# ---------------------------------------------------------------------------------------
def intrinsics(view) -> np.ndarray:
    """Pinhole matrix from the float32 camera values the renderer receives."""
    fx, fy, cx, cy = (float(F32(c)) for c in (view.fx, view.fy, view.cx, view.cy))
    return np.array([[fx, 0.0, cx], [0.0, fy, cy], [0.0, 0.0, 1.0]], dtype=np.float64)


def splat_frame(scene, view, k: int):
    """Camera-space a = R s_u t_u, b = R s_v t_v, pc = R p + t (fp64 from the float32 inputs)."""
    R = np.asarray(view.R, dtype=np.float64)
    t = np.asarray(view.t, dtype=np.float64)
    su, sv = float(scene.scales[k, 0]), float(scene.scales[k, 1])
    a = R @ (su * scene.tan_u[k].astype(np.float64))
    b = R @ (sv * scene.tan_v[k].astype(np.float64))
    pc = R @ scene.means[k].astype(np.float64) + t
    return a, b, pc


def splat_M(scene, view, k: int) -> np.ndarray:
    """M = K [a | b | pc]: homogeneous screen position of the plane point (u, v, 1)."""
    a, b, pc = splat_frame(scene, view, k)
    return intrinsics(view) @ np.stack([a, b, pc], axis=1)


def ray_splat_uv(M, x, y):
    """(u, v) of the plane point seen through pixel position (x, y); rho_2 = 0 -> no hit."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    hx = x[:, None] * M[2][None, :] - M[0][None, :]
    hy = y[:, None] * M[2][None, :] - M[1][None, :]
    rho = np.cross(hx, hy)
    valid = rho[:, 2] != 0.0
    with np.errstate(divide="ignore", invalid="ignore"):
        u = np.where(valid, rho[:, 0] / np.where(valid, rho[:, 2], 1.0), 0.0)
        v = np.where(valid, rho[:, 1] / np.where(valid, rho[:, 2], 1.0), 0.0)
    return u, v, valid, hx, hy, rho


def projected_center(M):
    return M[0, 2] / M[2, 2], M[1, 2] / M[2, 2]


# ---------------------------------------------------------------------------------------
# View-dependent specular term (Sec. 4.2, diffuse-specular split): the colour grid is the
# view-independent part; one set of spherical-harmonic coefficients per splat, the same over
# the whole splat, adds a colour that depends on the direction from the camera to the centre.
# ---------------------------------------------------------------------------------------
def sh_basis(d, degree: int) -> np.ndarray:
    """Real spherical harmonics of degree <= 3 at unit directions d [n, 3] (real or complex),
    [n, (degree + 1)^2], index l^2 + l + m. Each is (-1)^m times the usual real harmonic
    (for m > 0 the cosine part sqrt(2) Re Y_l^m, for m < 0 the sine part sqrt(2) Im Y_l^|m|,
    of the complex harmonic with the Condon-Shortley phase): the sign convention of the
    splatting line of work the paper extends. The polynomials in (x, y, z) and their
    normalisations sqrt((2l + 1) (l - |m|)! / (4 pi (l + |m|)!)) are written out below."""
    d = np.asarray(d)
    x, y, z = d[:, 0], d[:, 1], d[:, 2]
    pi = math.pi
    out = [0.5 * math.sqrt(1.0 / pi) * np.ones_like(x)]
    if degree >= 1:
        c1 = math.sqrt(3.0 / (4.0 * pi))
        out += [-c1 * y, c1 * z, -c1 * x]
    if degree >= 2:
        out += [0.5 * math.sqrt(15.0 / pi) * x * y,
                -0.5 * math.sqrt(15.0 / pi) * y * z,
                0.25 * math.sqrt(5.0 / pi) * (2.0 * z * z - x * x - y * y),
                -0.5 * math.sqrt(15.0 / pi) * x * z,
                0.25 * math.sqrt(15.0 / pi) * (x * x - y * y)]
    if degree >= 3:
        out += [-0.25 * math.sqrt(35.0 / (2.0 * pi)) * y * (3.0 * x * x - y * y),
                0.5 * math.sqrt(105.0 / pi) * x * y * z,
                -0.25 * math.sqrt(21.0 / (2.0 * pi)) * y * (4.0 * z * z - x * x - y * y),
                0.25 * math.sqrt(7.0 / pi) * z * (2.0 * z * z - 3.0 * x * x - 3.0 * y * y),
                -0.25 * math.sqrt(21.0 / (2.0 * pi)) * x * (4.0 * z * z - x * x - y * y),
                0.25 * math.sqrt(105.0 / pi) * z * (x * x - y * y),
                -0.25 * math.sqrt(35.0 / (2.0 * pi)) * x * (x * x - 3.0 * y * y)]
    if degree > 3:
        raise ValueError("spherical harmonics of degree <= 3 only")
    return np.stack(out, axis=1)


def camera_centre(view) -> np.ndarray:
    """World position of the camera, -R^T t (fp64 from the float32 values)."""
    R = np.asarray(view.R, dtype=np.float64)
    t = np.asarray(view.t, dtype=np.float64)
    return -R.T @ t


def specular(scene, view, k: int, mean=None) -> np.ndarray:
    """The view-dependent colour of splat k: sum_j Y_j(dir) sh[k, j], with dir the unit
    vector from the camera centre to the splat centre (``mean`` overrides the centre; it may
    be complex for complex-step derivatives). Zero without coefficients."""
    if scene.sh is None:
        return np.zeros(3)
    p = scene.means[k].astype(np.float64) if mean is None else mean
    v = p - camera_centre(view)
    dvec = v / np.sqrt(np.sum(v * v))
    Y = sh_basis(dvec[None, :], scene.sh_degree)[0]
    return Y @ scene.sh[k].astype(np.float64)


def specular_grads(scene, view, k: int, dspec) -> Tuple[np.ndarray, np.ndarray]:
    """Adjoint of ``specular`` for the colour adjoint dspec [3]: (d sh [(D+1)^2, 3],
    d mean [3]). The centre derivative is taken by the complex step, Im f(p + i h e) / h with
    h = 1e-30, exact to rounding for this analytic map."""
    p = scene.means[k].astype(np.float64)
    v = p - camera_centre(view)
    Y = sh_basis((v / np.linalg.norm(v))[None, :], scene.sh_degree)[0]
    d_sh = np.outer(Y, dspec)
    h = 1e-30
    d_mean = np.zeros(3)
    for i in range(3):
        pc = p.astype(np.complex128)
        pc[i] += 1j * h
        d_mean[i] = float(np.imag(specular(scene, view, k, mean=pc) @ np.asarray(dspec)) / h)
    return d_sh, d_mean


# ---------------------------------------------------------------------------------------
# Exact pruning (speed only): drop splats that provably have alpha < alpha_min on a crop.
# ---------------------------------------------------------------------------------------
def prune_for_crop(scene, view, opts: Options, cand: np.ndarray, crop) -> np.ndarray:
    """Keep the candidates whose alpha >= alpha_min region can reach the crop.

    Bounding sphere of the 3.33-radius uv square: centre p, radius 3.33 (s_u|t_u| + s_v|t_v|).
    A splat is dropped only if that sphere lies beyond z_near, misses the crop's pixel-centre
    frustum, and the low-pass disk around the projected centre (the key stage's radius) misses
    the crop.
    """
    if cand.size == 0 or F32(opts.alpha_min) < KS_ALPHA_FLOOR:
        return cand
    x0, y0, w, h = crop
    R = np.asarray(view.R, dtype=np.float64)
    t = np.asarray(view.t, dtype=np.float64)
    p = scene.means[cand].astype(np.float64)
    c = p @ R.T + t
    rad = 3.33 * (scene.scales[cand, 0] * np.linalg.norm(scene.tan_u[cand], axis=1)
                  + scene.scales[cand, 1] * np.linalg.norm(scene.tan_v[cand], axis=1))
    rad = rad.astype(np.float64) * (1 + 1e-6) + 1e-9
    xl, xr = (x0 + 0.5 - view.cx) / view.fx, (x0 + w - 0.5 - view.cx) / view.fx
    yt, yb = (y0 + 0.5 - view.cy) / view.fy, (y0 + h - 0.5 - view.cy) / view.fy
    planes = [np.array([1.0, 0.0, -xl]), np.array([-1.0, 0.0, xr]),
              np.array([0.0, 1.0, -yt]), np.array([0.0, -1.0, yb])]
    outside = np.zeros(cand.size, dtype=bool)
    for n in planes:
        n = n / np.linalg.norm(n)
        outside |= (c @ n) < -rad
    in_front = c[:, 2] - rad > view.z_near
    with np.errstate(divide="ignore", invalid="ignore"):
        c2x = view.fx * c[:, 0] / c[:, 2] + view.cx
        c2y = view.fy * c[:, 1] / c[:, 2] + view.cy
    dx = np.maximum(np.maximum((x0 + 0.5) - c2x, c2x - (x0 + w - 0.5)), 0.0)
    dy = np.maximum(np.maximum((y0 + 0.5) - c2y, c2y - (y0 + h - 0.5)), 0.0)
    r_lp = float(ks_lowpass_radius(opts.lowpass_var))
    lp_out = dx * dx + dy * dy > r_lp * r_lp
    drop = in_front & outside & lp_out
    return cand[~drop]


# ---------------------------------------------------------------------------------------
# Forward (Alg. 1 forward, Eq. 2) and backward (Alg. 1 backward, Alg. 2 adj-bilinear).
# ---------------------------------------------------------------------------------------
@dataclasses.dataclass
class RenderResult:
    rgb: np.ndarray            # [h, w, 3]
    T_final: np.ndarray        # [h, w]
    n_blended: np.ndarray      # [h, w]   splats blended per pixel
    terminated: np.ndarray     # [h, w]   pixel stopped by the t_min rule
    alpha_gap: np.ndarray      # [h, w]   min relative distance |alpha - alpha_min| / alpha_min
    t_gap: np.ndarray          # [h, w]   min relative distance |T(1-alpha) - t_min| / t_min
    kink_gap: np.ndarray       # [h, w]   min relative distance to a gradient-only kink (alpha_max
                               #          clamp, tie between the two falloff branches)
    crop: Tuple[int, int, int, int]
    # saved for the backward: per blended splat (index, pixel ids, T before, alpha)
    saved: List[Tuple[int, np.ndarray, np.ndarray, np.ndarray]] = dataclasses.field(repr=False,
                                                                                  default_factory=list)
    eval_count: int = 0        # number of (pixel, splat) evaluations (visited pairs)
    # the depth order walked (after pruning) and, per pixel id of the crop, the decisions that
    # fell inside the flag bands: (splat, 'a') for alpha vs alpha_min, (splat, 't') for the
    # t_min stop, with the transmittance in front of the splat and its alpha
    order: List[int] = dataclasses.field(repr=False, default_factory=list)
    straddles: Dict[int, List[Tuple[int, str, float, float]]] = dataclasses.field(
        repr=False, default_factory=dict)


def _pixel_grid(crop):
    x0, y0, w, h = crop
    jj, ii = np.meshgrid(np.arange(y0, y0 + h), np.arange(x0, x0 + w), indexing="ij")
    return (ii.reshape(-1) + 0.5).astype(np.float64), (jj.reshape(-1) + 0.5).astype(np.float64)


def _falloff(M, x, y, lowpass_var):
    """(u, v), validity, q, branch flag (True = uv Gaussian), G_hat, and the projected centre."""
    u, v, valid, hx, hy, rho = ray_splat_uv(M, x, y)
    c2x, c2y = projected_center(M)
    q_uv = 0.5 * (u * u + v * v)
    q_lp = ((x - c2x) ** 2 + (y - c2y) ** 2) / (2.0 * lowpass_var)
    use_uv = q_uv <= q_lp
    q = np.where(use_uv, q_uv, q_lp)
    return u, v, valid, q, use_uv, np.exp(-q), (c2x, c2y), (hx, hy, rho), (q_uv, q_lp)


def _rel_gap(value, threshold):
    """Relative distance of a value to a decision threshold (inf for a switched-off one)."""
    if threshold <= 0.0:
        return np.full(np.shape(value), np.inf)
    return np.abs(value - threshold) / threshold


# Default flag thresholds: a float32 renderer reproduces alpha to ~1e-6 relative and the
# transmittance after ~100 blends to ~1e-5 relative; decisions closer than these to their
# threshold may legitimately go either way.
TAU_ALPHA = 1e-5
TAU_T = 1e-4
TAU_KINK = 1e-4


def render(scene, view, opts: Options, crop=None, keep_saved: bool = False, prune: bool = True,
           order: Optional[Sequence[int]] = None, flip=None, shift=None) -> RenderResult:
    """Composite every key-stage-visible splat at every pixel of ``crop`` (x0, y0, w, h).

    ``prune=False`` walks every visible splat (no exact pruning). ``order`` replaces the
    depth order (it must be the depth order of a superset of the splats that can reach the
    crop, e.g. the ``order`` of a render of an enclosing crop). ``flip`` is a set of
    (splat, kind) decisions taken the other way at every pixel of the crop: kind 'a' inverts
    the alpha >= alpha_min test, 't' inverts the t_min stop (for enumerating the outcomes of
    flagged pixels). ``shift`` maps a splat index to an image translation (dx, dy) in pixels
    of that splat's footprint (for checking the densification statistic; pruning is then off).
    """
    W, H = view.width, view.height
    crop = tuple(crop) if crop is not None else (0, 0, W, H)
    x, y = _pixel_grid(crop)
    npx = x.size
    if order is None:
        ks = key_stage(scene, view, opts)
        order = depth_order(ks)
        if prune and not shift:
            keep = set(prune_for_crop(scene, view, opts, order, crop).tolist())
            order = [int(k) for k in order if int(k) in keep]
    order = [int(k) for k in order]
    flip = set(flip or ())
    T = np.ones(npx)
    acc = np.zeros((npx, 3))
    done = np.zeros(npx, dtype=bool)
    nbl = np.zeros(npx, dtype=np.int64)
    a_gap = np.full(npx, np.inf)
    t_gap = np.full(npx, np.inf)
    k_gap = np.full(npx, np.inf)
    straddles: Dict[int, List[Tuple[int, str, float, float]]] = {}
    saved = []
    evals = 0
    a_min, a_max, t_min = opts.alpha_min, opts.alpha_max, opts.t_min
    for k in order:
        active = ~done
        if not active.any():
            break
        evals += int(active.sum())
        M = splat_M(scene, view, k)
        if shift and k in shift:
            M = M.copy()
            M[0] += shift[k][0] * M[2]
            M[1] += shift[k][1] * M[2]
        u, v, valid, q, use_uv, G, _, _, (q_uv, q_lp) = _falloff(M, x, y, opts.lowpass_var)
        o = float(scene.opacity[k])
        alpha = np.minimum(a_max, o * G)
        live = active & valid
        m = _rel_gap(alpha, a_min)
        contrib = alpha >= a_min
        if (k, "a") in flip:
            contrib = ~contrib
        contrib &= live
        Tn = T * (1.0 - alpha)
        m_t = _rel_gap(Tn, t_min)
        m_c = _rel_gap(o * G, a_max)
        m_b = np.abs(q_uv - q_lp) / np.maximum(np.maximum(q_uv, q_lp), 1e-300)
        a_gap = np.where(live, np.minimum(a_gap, m), a_gap)
        t_gap = np.where(contrib, np.minimum(t_gap, m_t), t_gap)
        k_gap = np.where(contrib, np.minimum(k_gap, np.minimum(m_c, m_b)), k_gap)
        for pid in np.nonzero(live & (m < TAU_ALPHA))[0]:
            straddles.setdefault(int(pid), []).append((k, "a", float(T[pid]), float(alpha[pid])))
        for pid in np.nonzero(contrib & (m_t < TAU_T))[0]:
            straddles.setdefault(int(pid), []).append((k, "t", float(T[pid]), float(alpha[pid])))
        stop = Tn < t_min
        if (k, "t") in flip:
            stop = ~stop
        term = contrib & stop
        blend = contrib & ~term
        if blend.any():
            ids = np.nonzero(blend)[0]
            col = bilinear(scene.textures[k].astype(np.float64), u[ids], v[ids], opts.sigma)
            col = col + specular(scene, view, k)[None, :]
            w = alpha[ids] * T[ids]
            acc[ids] += w[:, None] * col
            if keep_saved:
                saved.append((k, ids, T[ids].copy(), alpha[ids].copy()))
            T[ids] = Tn[ids]
            nbl[ids] += 1
        done |= term
    bg = np.asarray(opts.bg, dtype=np.float64)
    rgb = acc + T[:, None] * bg[None, :]
    h, w = crop[3], crop[2]
    return RenderResult(rgb.reshape(h, w, 3), T.reshape(h, w), nbl.reshape(h, w),
                        done.reshape(h, w), a_gap.reshape(h, w), t_gap.reshape(h, w),
                        k_gap.reshape(h, w), crop, saved, evals, order, straddles)


def image_flags(r: RenderResult, tau_alpha=TAU_ALPHA, tau_t=TAU_T) -> np.ndarray:
    """Pixels whose image may differ between exact and float32 arithmetic by a discrete
    decision (alpha_min skip or t_min stop taken differently)."""
    return (r.alpha_gap < tau_alpha) | (r.t_gap < tau_t)


def grad_flags(r: RenderResult, tau_alpha=TAU_ALPHA, tau_t=TAU_T, tau_kink=TAU_KINK) -> np.ndarray:
    """Image flags plus pixels near a kink of the gradient (alpha_max clamp, branch tie)."""
    return image_flags(r, tau_alpha, tau_t) | (r.kink_gap < tau_kink)


def flagged_outcomes(scene, view, opts: Options, r: RenderResult, row: int, col: int,
                     max_decisions: int = 4):
    """Every admissible result of a flagged pixel (row, col of the crop of ``r``).

    Each decision of the pixel that fell inside a flag band may go either way in a float32
    renderer. The pixel is re-rendered for every subset of those decisions taken the other
    way (2^m renders for m decisions); returns a list of (rgb [3], T) pairs, the first being
    ``r``'s own result. With more than ``max_decisions`` such decisions returns None.
    """
    pid = row * r.crop[2] + col
    dec = sorted({(k, kind) for k, kind, _, _ in r.straddles.get(pid, [])})
    if len(dec) > max_decisions:
        return None
    x0, y0 = r.crop[0] + col, r.crop[1] + row
    out = [(r.rgb[row, col].copy(), float(r.T_final[row, col]))]
    for mask in range(1, 1 << len(dec)):
        fl = {dec[i] for i in range(len(dec)) if (mask >> i) & 1}
        rr = render(scene, view, opts, crop=(x0, y0, 1, 1), order=r.order, flip=fl)
        out.append((rr.rgb[0, 0].copy(), float(rr.T_final[0, 0])))
    return out


def flagged_bound(scene, r: RenderResult, row: int, col: int, bg=(0.0, 0.0, 0.0)) -> float:
    """Bound on how far a flagged pixel's colour can move when its in-band decisions go the
    other way: a skipped or blended splat changes the colour by at most alpha T (|c| + |S|)
    <= 2 alpha T c_max, a stop taken or not by at most T c_max (what lies behind), with
    c_max the largest texel or background magnitude of the scene."""
    pid = row * r.crop[2] + col
    if isinstance(scene.textures, np.ndarray):
        tmax = float(np.abs(scene.textures).max())
    else:  # grids of several sides
        tmax = max(float(np.abs(np.asarray(g)).max()) for g in scene.textures)
    cmax = max(tmax, float(np.abs(np.asarray(bg)).max()), 1e-30)
    b = 0.0
    for k, kind, T_before, alpha in r.straddles.get(pid, []):
        b += (2.0 * alpha * T_before if kind == "a" else T_before) * cmax
    return b


@dataclasses.dataclass
class Grads:
    means: np.ndarray
    tan_u: np.ndarray
    tan_v: np.ndarray
    scales: np.ndarray
    opacity: np.ndarray
    textures: np.ndarray
    sh: Optional[np.ndarray] = None
    # per splat: gradient of the loss with respect to a translation of the splat's footprint
    # in the image by (dx, dy) pixels (the densification statistic), [P, 2]
    screen: Optional[np.ndarray] = None


def render_backward(scene, view, opts: Options, fwd: RenderResult, dl_drgb) -> Grads:
    """Analytic gradient of sum(dl_drgb * rgb) over the crop of ``fwd`` (rendered with
    ``keep_saved=True``) with respect to every splat parameter.

    Walks the blended splats back to front. With S the colour composited behind splat k
    (including T_final * bg), d alpha_k = g . (col_k T_k - S / (1 - alpha_k)); the colour adjoint
    alpha_k T_k g goes through adj-bilinear to the grid and to (u, v); the falloff adjoint goes
    to the opacity and to (u, v) or, on the low-pass branch, to the projected centre; (u, v) go
    through rho = h_x x h_y to M = K [a | b | pc] and from there to p, t_u, t_v, s_u, s_v.
    """
    P, N = scene.P, scene.N
    g_all = np.asarray(dl_drgb, dtype=np.float64).reshape(-1, 3)
    x_all, y_all = _pixel_grid(fwd.crop)
    bg = np.asarray(opts.bg, dtype=np.float64)
    S = fwd.T_final.reshape(-1)[:, None] * bg[None, :]
    S = np.array(S)
    # grids of one side: one [P,N,N,3] array; of several sides: one [n_k,n_k,3] array each
    dtex = (np.zeros((P, N, N, 3)) if isinstance(scene.textures, np.ndarray)
            else [np.zeros(np.shape(g)) for g in scene.textures])
    gr = Grads(np.zeros((P, 3)), np.zeros((P, 3)), np.zeros((P, 3)), np.zeros((P, 2)),
               np.zeros(P), dtex,
               None if scene.sh is None else np.zeros(scene.sh.shape), np.zeros((P, 2)))
    Kmat = intrinsics(view)
    R = np.asarray(view.R, dtype=np.float64)
    for k, ids, Tk, alpha in reversed(fwd.saved):
        x, y, g = x_all[ids], y_all[ids], g_all[ids]
        M = splat_M(scene, view, k)
        u, v, valid, q, use_uv, G, (c2x, c2y), (hx, hy, rho), _ = _falloff(M, x, y,
                                                                           opts.lowpass_var)
        o = float(scene.opacity[k])
        C = scene.textures[k].astype(np.float64)
        col = bilinear(C, u, v, opts.sigma) + specular(scene, view, k)[None, :]
        w = alpha * Tk
        # colour -> grid and uv
        dC, du, dv = adj_bilinear(C, u, v, opts.sigma, w[:, None] * g)
        gr.textures[k] += dC
        # colour -> view-dependent term -> coefficients and centre
        if scene.sh is not None:
            d_sh, d_mean = specular_grads(scene, view, k, np.sum(w[:, None] * g, axis=0))
            gr.sh[k] += d_sh
            gr.means[k] += d_mean
        # alpha
        Sk = S[ids]
        dalpha = np.sum(g * (col * Tk[:, None] - Sk / (1.0 - alpha)[:, None]), axis=1)
        S[ids] = Sk + w[:, None] * col
        unclamped = o * G <= opts.alpha_max
        dalpha = np.where(unclamped, dalpha, 0.0)
        gr.opacity[k] += np.sum(dalpha * G)
        dq = -G * o * dalpha
        # falloff branch: uv Gaussian or screen low-pass
        du = du + np.where(use_uv, dq * u, 0.0)
        dv = dv + np.where(use_uv, dq * v, 0.0)
        dql = np.where(use_uv, 0.0, dq) / (2.0 * opts.lowpass_var)
        dc2x = np.sum(dql * (-2.0) * (x - c2x))
        dc2y = np.sum(dql * (-2.0) * (y - c2y))
        # (u, v) = (rho_0, rho_1) / rho_2
        r2 = rho[:, 2]
        drho = np.stack([du / r2, dv / r2, -(du * u + dv * v) / r2], axis=1)
        # rho = hx x hy
        dhx = np.cross(hy, drho)
        dhy = np.cross(drho, hx)
        dM = np.zeros((3, 3))
        dM[2] += np.sum(x[:, None] * dhx + y[:, None] * dhy, axis=0)
        dM[0] -= np.sum(dhx, axis=0)
        dM[1] -= np.sum(dhy, axis=0)
        # projected centre c2 = (M02 / M22, M12 / M22)
        dM[0, 2] += dc2x / M[2, 2]
        dM[1, 2] += dc2y / M[2, 2]
        dM[2, 2] -= (dc2x * M[0, 2] + dc2y * M[1, 2]) / (M[2, 2] ** 2)
        # an image translation by (dx, dy) maps row 0 of M to M_0 + dx M_2 (row 1 likewise)
        gr.screen[k] += np.array([dM[0] @ M[2], dM[1] @ M[2]])
        # M = K [a b pc]
        dA = Kmat.T @ dM
        da, db, dpc = dA[:, 0], dA[:, 1], dA[:, 2]
        dwa, dwb = R.T @ da, R.T @ db
        su, sv = float(scene.scales[k, 0]), float(scene.scales[k, 1])
        gr.tan_u[k] += su * dwa
        gr.tan_v[k] += sv * dwb
        gr.scales[k, 0] += float(scene.tan_u[k].astype(np.float64) @ dwa)
        gr.scales[k, 1] += float(scene.tan_v[k].astype(np.float64) @ dwb)
        gr.means[k] += R.T @ dpc
    return gr


def render_views(scene, views: Sequence, opts: Options):
    """Full-frame forward of every view; returns packed rgb [sum HW, 3] and T [sum HW]."""
    rgb, T = [], []
    for view in views:
        r = render(scene, view, opts)
        rgb.append(r.rgb.reshape(-1, 3))
        T.append(r.T_final.reshape(-1))
    return np.concatenate(rgb), np.concatenate(T)


def box_filter_grid(C: np.ndarray, factor: int) -> np.ndarray:
    """Average N x N x 3 texel grids over factor x factor blocks (coarser texture levels)."""
    C = np.asarray(C, dtype=np.float64)
    N = C.shape[-3]
    n = N // factor
    shp = C.shape[:-3] + (n, factor, n, factor, 3)
    return C.reshape(shp).mean(axis=(-4, -2))
