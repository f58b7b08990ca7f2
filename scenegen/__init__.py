"""Seeded synthetic inputs for the textured 2D-Gaussian rasterizer.

This module draws scenes, cameras and output adjoints from fixed seeds. It holds none of
the renderer's arithmetic: both the FP64 oracle and the HIP path read the arrays it makes,
and neither is imported here.

A scene is the set of already-activated per-splat parameters of the paper's primitive
(Sec. 3.1, Eq. 3: center p, tangents t_u and t_v from a rotation, scales s_u and s_v,
opacity) plus the per-splat N x N RGB colour grid of Sec. 3.2. Tangents come from a random
unit quaternion as in 2DGS; everything is drawn in float64 and cast to float32 (textures
optionally rounded to bfloat16, round-to-nearest-even).

Cameras are pinholes with a horizontal field of view, axes x right, y down, z forward,
pixel centres at (i + 1/2, j + 1/2), principal point at the image centre.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence, Tuple

import numpy as np

__all__ = [
    "Scene", "View", "make_scene", "look_at_view", "frontal_view", "orbit_views",
    "make_dl_drgb", "to_bf16_bits", "bf16_bits_to_f32", "CONFIGS", "config", "with_sh",
    "with_mixed_sides",
]


@dataclasses.dataclass
class Scene:
    """Per-splat parameters, all C-contiguous float32 (textures float32; see ``tex_bf16``)."""
    means: np.ndarray      # [P,3]
    tan_u: np.ndarray      # [P,3]
    tan_v: np.ndarray      # [P,3]
    scales: np.ndarray     # [P,2]  (s_u, s_v) > 0
    opacity: np.ndarray    # [P]    in (0, 1)
    textures: np.ndarray   # [P,N,N,3] indexed [k, i_u, i_v, c], or a list of P grids
                           # [n_k, n_k, 3] of several sides
    # optional per-splat spherical-harmonic coefficients of the view-dependent colour term,
    # [P, (degree + 1)^2, 3] (None: no such term)
    sh: Optional[np.ndarray] = None

    @property
    def P(self) -> int:
        return int(self.means.shape[0])

    @property
    def N(self) -> int:
        """Texture side (the largest side when the grids have several)."""
        if isinstance(self.textures, np.ndarray):
            return int(self.textures.shape[1])
        return max(int(g.shape[0]) for g in self.textures)

    @property
    def sh_degree(self) -> int:
        """Degree of the spherical harmonics (-1 without them)."""
        return -1 if self.sh is None else int(round(math.sqrt(self.sh.shape[1]))) - 1

    def subset(self, idx) -> "Scene":
        sh = None if self.sh is None else np.ascontiguousarray(self.sh[idx])
        if isinstance(self.textures, np.ndarray):
            tex = np.ascontiguousarray(self.textures[idx])
        else:
            tex = [self.textures[int(i)] for i in np.arange(self.P)[idx]]
        return Scene(*(np.ascontiguousarray(a[idx]) for a in
                       (self.means, self.tan_u, self.tan_v, self.scales, self.opacity)), tex, sh)


@dataclasses.dataclass
class View:
    """Pinhole camera: world->camera rotation R (row-major) and translation t. All values are
    float32-representable (the renderer's C ABI takes float32)."""
    width: int
    height: int
    fx: float
    fy: float
    cx: float
    cy: float
    R: np.ndarray          # [3,3] float32
    t: np.ndarray          # [3] float32
    z_near: float = 0.01


def _f32(x: float) -> float:
    """The value as the float32 the renderer receives (both sides must see the same inputs)."""
    return float(np.float32(x))


def _intrinsics(width: int, height: int, fov_deg: float) -> Tuple[float, float, float, float]:
    f = (width / 2.0) / math.tan(math.radians(fov_deg) / 2.0)
    return _f32(f), _f32(f), _f32(width / 2.0), _f32(height / 2.0)


def look_at_view(pos, width: int, height: int, fov_deg: float = 60.0,
                 target=(0.0, 0.0, 0.0), z_near: float = 0.01) -> View:
    """Camera at ``pos`` looking at ``target``; rows of R are the camera axes in world space."""
    pos = np.asarray(pos, dtype=np.float64)
    f = np.asarray(target, dtype=np.float64) - pos
    f /= np.linalg.norm(f)
    up = np.array([0.0, 1.0, 0.0])
    if abs(float(f @ up)) > 0.99:
        up = np.array([1.0, 0.0, 0.0])
    r = np.cross(f, up)
    r /= np.linalg.norm(r)
    d = np.cross(f, r)
    R = np.stack([r, d, f])
    t = -R @ pos
    fx, fy, cx, cy = _intrinsics(width, height, fov_deg)
    return View(width, height, fx, fy, cx, cy, R.astype(np.float32), t.astype(np.float32),
                _f32(z_near))


def frontal_view(width: int, height: int, fov_deg: float = 60.0, z_near: float = 0.01) -> View:
    """Identity camera at the origin looking down +z (the image-fitting set-up)."""
    fx, fy, cx, cy = _intrinsics(width, height, fov_deg)
    return View(width, height, fx, fy, cx, cy, np.eye(3, dtype=np.float32),
                np.zeros(3, dtype=np.float32), _f32(z_near))


def quat_to_tangents(q: np.ndarray) -> Tuple[np.ndarray, np.ndarray]:
    """Unit quaternions (w,x,y,z) -> first two columns of the rotation matrix."""
    q = q / np.linalg.norm(q, axis=1, keepdims=True)
    w, x, y, z = q[:, 0], q[:, 1], q[:, 2], q[:, 3]
    c0 = np.stack([1 - 2 * (y * y + z * z), 2 * (x * y + w * z), 2 * (x * z - w * y)], axis=1)
    c1 = np.stack([2 * (x * y - w * z), 1 - 2 * (x * x + z * z), 2 * (y * z + w * x)], axis=1)
    return c0, c1


def to_bf16_bits(x: np.ndarray) -> np.ndarray:
    """float32 -> bfloat16 bit patterns (uint16), round to nearest even. NaN kept quiet."""
    b = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32)
    rounding = ((b >> 16) & 1) + np.uint32(0x7FFF)
    out = ((b + rounding) >> 16).astype(np.uint16)
    nan = np.isnan(x)
    if nan.any():
        out[nan] = np.uint16(0x7FC0)
    return out


def bf16_bits_to_f32(b: np.ndarray) -> np.ndarray:
    return (np.asarray(b, dtype=np.uint16).astype(np.uint32) << 16).view(np.float32)


def make_scene(seed: int, P: int, lo: float, hi: float, s_lo: float, s_hi: float, N: int,
               tex_bf16: bool = False, op_lo: float = 0.05, op_hi: float = 0.95) -> Scene:
    """Draw order: means, quaternions, log-scales, opacity, textures (one PCG64 stream).

    With ``tex_bf16`` the texel values are rounded to the nearest bfloat16 and returned as
    float32 holding those exact values (the GPU receives their bit patterns).
    """
    rng = np.random.default_rng(seed)
    means = rng.uniform(lo, hi, (P, 3))
    q = rng.standard_normal((P, 4))
    tu, tv = quat_to_tangents(q)
    scales = np.exp(rng.uniform(math.log(s_lo), math.log(s_hi), (P, 2)))
    opacity = rng.uniform(op_lo, op_hi, P)
    # textures: the same stream values as one (P, N, N, 3) draw, generated and cast in chunks of
    # splats so that millions of splats do not need the full float64 array at once
    tex = np.empty((P, N, N, 3), dtype=np.float32)
    flat = tex.reshape(P, N * N * 3)
    step = max(1, (1 << 22) // (N * N * 3))
    for i in range(0, P, step):
        part = flat[i:i + step]
        part[...] = rng.uniform(0.0, 1.0, part.shape)
        if tex_bf16:
            part[...] = bf16_bits_to_f32(to_bf16_bits(part)).reshape(part.shape)
    f32 = lambda a: np.ascontiguousarray(a, dtype=np.float32)
    return Scene(f32(means), f32(tu), f32(tv), f32(scales), f32(opacity), tex)


def with_mixed_sides(scene: Scene, seed: int, sides) -> Scene:
    """The scene with colour grids of several sides: splat k gets a side drawn uniformly from
    ``sides`` and a grid of that side U(0, 1), from their own stream (float32 values)."""
    rng = np.random.default_rng(seed)
    sides = np.asarray(sides, dtype=np.int64)
    n = sides[rng.integers(0, sides.size, scene.P)]
    # one draw for all texels, in splat order, cut into the grids
    vals = rng.uniform(0.0, 1.0, (int(np.sum(n * n)), 3)).astype(np.float32)
    cuts = np.cumsum(n * n)[:-1]
    grids = [g.reshape(int(m), int(m), 3) for g, m in zip(np.split(vals, cuts), n)]
    return dataclasses.replace(scene, textures=grids)


def with_sh(scene: Scene, seed: int, degree: int, scale: float = 0.2) -> Scene:
    """The scene with per-splat spherical-harmonic coefficients N(0, scale^2) of the given
    degree, [P, (degree + 1)^2, 3] float32, drawn from their own stream."""
    rng = np.random.default_rng(seed)
    n = (degree + 1) ** 2
    sh = np.empty((scene.P, n, 3), dtype=np.float32)
    flat = sh.reshape(scene.P, n * 3)
    step = max(1, (1 << 22) // (n * 3))
    for i in range(0, scene.P, step):
        part = flat[i:i + step]
        part[...] = rng.normal(0.0, scale, part.shape)
    return dataclasses.replace(scene, sh=sh)


def orbit_views(seed: int, n: int, radius: float, resolutions: Sequence[Tuple[int, int]],
                fov_deg: float = 60.0, pick_resolution: bool = False) -> List[View]:
    """``n`` cameras on a sphere of ``radius`` looking at the origin (directions N(0,I))."""
    rng = np.random.default_rng(seed + 1)
    views = []
    for _ in range(n):
        d = rng.standard_normal(3)
        d /= np.linalg.norm(d)
        if pick_resolution:
            w, h = resolutions[int(rng.integers(0, len(resolutions)))]
        else:
            w, h = resolutions[0]
        views.append(look_at_view(radius * d, w, h, fov_deg))
    return views


def make_dl_drgb(seed: int, views: Sequence[View]) -> np.ndarray:
    """Output adjoint dL/drgb ~ N(0,1), views packed in order, each [H][W][3] (float32)."""
    total = sum(v.width * v.height for v in views)
    rng = np.random.default_rng(seed + 2)
    return np.ascontiguousarray(rng.standard_normal((total, 3)), dtype=np.float32)


# ---------------------------------------------------------------------------------------
# Named workloads. Sizes and distributions follow the benchmark configurations; where a
# detail is open (orientation of config 2, centres and cameras of config 4) it follows the
# nearest configuration that states it.
# ---------------------------------------------------------------------------------------
CONFIGS = {
    # 1k splats, 4x4 FP32 textures, one 128x128 view at distance 3, forward only
    "C1": dict(P=1000, lo=-1.0, hi=1.0, s_lo=0.02, s_hi=0.2, N=4, bf16=False,
               views=("front", 3.0, [(128, 128)], 1)),
    # 100k splats, 8x8 FP32 textures, one 800x800 view at distance 5, fwd+bwd
    "C2": dict(P=100_000, lo=-2.0, hi=2.0, s_lo=0.005, s_hi=0.1, N=8, bf16=False,
               views=("front", 5.0, [(800, 800)], 1)),
    # 1M splats, 4x4 FP32 textures, 16 uneven views on a radius-8 sphere
    "C3": dict(P=1_000_000, lo=-4.0, hi=4.0, s_lo=0.02, s_hi=0.2, N=4, bf16=False,
               views=("orbit", 8.0, [(640, 480), (1024, 768), (1280, 720), (1600, 1060)], 16)),
    # 3M splats, 8x8 BF16 textures, 4 views 1920x1080 on a radius-8 sphere
    "C4": dict(P=3_000_000, lo=-4.0, hi=4.0, s_lo=0.002, s_hi=0.05, N=8, bf16=True,
               views=("orbit", 8.0, [(1920, 1080)], 4)),
    # 1M splats, 8x8 textures, one 1920x1080 view at distance 8 (FP32 and BF16 variants)
    "T0": dict(P=1_000_000, lo=-4.0, hi=4.0, s_lo=0.02, s_hi=0.2, N=8, bf16=False,
               views=("front", 8.0, [(1920, 1080)], 1)),
    "T0_BF16": dict(P=1_000_000, lo=-4.0, hi=4.0, s_lo=0.02, s_hi=0.2, N=8, bf16=True,
                    views=("front", 8.0, [(1920, 1080)], 1)),
    # the same with 16 x 16 colour grids (FP32)
    "T0_N16": dict(P=1_000_000, lo=-4.0, hi=4.0, s_lo=0.02, s_hi=0.2, N=16, bf16=False,
                   views=("front", 8.0, [(1920, 1080)], 1)),
}


def config(name: str, seed: int = 0, P: Optional[int] = None) -> Tuple[Scene, List[View]]:
    """Build the scene and views of a named workload (optionally with fewer splats)."""
    c = CONFIGS[name]
    scene = make_scene(seed, P if P is not None else c["P"], c["lo"], c["hi"], c["s_lo"],
                       c["s_hi"], c["N"], tex_bf16=c["bf16"])
    kind, dist, res, nv = c["views"]
    if kind == "front":
        views = [look_at_view((0.0, 0.0, -dist), res[0][0], res[0][1])]
    else:
        views = orbit_views(seed, nv, dist, res, pick_resolution=len(res) > 1)
    return scene, views


# ---- training workload (raw parameters) ------------------------------------------------------
@dataclasses.dataclass
class RawScene:
    """Raw (pre-activation) splat parameters, float32: means [P][3], quats [P][4] (w, x, y, z,
    not normalised), log_scales [P][2], opacity_logits [P], textures [P][N][N][3] in [0, 1]."""
    means: np.ndarray
    quats: np.ndarray
    log_scales: np.ndarray
    opacity_logits: np.ndarray
    textures: np.ndarray

    @property
    def P(self) -> int:
        return self.means.shape[0]

    @property
    def N(self) -> int:
        return self.textures.shape[1]


def make_raw_scene(seed: int, P: int, lo: float, hi: float, s_lo: float, s_hi: float, N: int,
                   op_lo: float = 0.05, op_hi: float = 0.95) -> RawScene:
    """The draws of ``make_scene`` (same order and stream) kept as raw parameters: the quaternion
    draws, the log-scales, the logits of the opacities and float32 textures."""
    rng = np.random.default_rng(seed)
    means = rng.uniform(lo, hi, (P, 3))
    q = rng.standard_normal((P, 4))
    log_s = rng.uniform(math.log(s_lo), math.log(s_hi), (P, 2))
    o = rng.uniform(op_lo, op_hi, P)
    tex = np.empty((P, N, N, 3), dtype=np.float32)
    flat = tex.reshape(P, N * N * 3)
    step = max(1, (1 << 22) // (N * N * 3))
    for i in range(0, P, step):
        part = flat[i:i + step]
        part[...] = rng.uniform(0.0, 1.0, part.shape)
    f32 = lambda a: np.ascontiguousarray(a, dtype=np.float32)
    return RawScene(f32(means), f32(q), f32(log_s), f32(np.log(o / (1.0 - o))), tex)


def perturb_raw(raw: RawScene, seed: int) -> RawScene:
    """Target scene of the training workload: means + N(0, 0.02), log-scales + N(0, 0.1),
    quaternions + N(0, 0.05) then renormalised, logits + N(0, 0.2), textures + N(0, 0.05)
    clipped to [0, 1]; one stream, in that order."""
    rng = np.random.default_rng(seed)
    P = raw.P
    means = raw.means + rng.normal(0.0, 0.02, (P, 3))
    log_s = raw.log_scales + rng.normal(0.0, 0.1, (P, 2))
    q = raw.quats + rng.normal(0.0, 0.05, (P, 4))
    q = q / np.linalg.norm(q, axis=1, keepdims=True)
    logits = raw.opacity_logits + rng.normal(0.0, 0.2, P)
    tex = np.empty_like(raw.textures)
    src, dst = raw.textures.reshape(P, -1), tex.reshape(P, -1)
    step = max(1, (1 << 22) // src.shape[1])
    for i in range(0, P, step):
        dst[i:i + step] = np.clip(src[i:i + step] + rng.normal(0.0, 0.05, src[i:i + step].shape),
                                  0.0, 1.0)
    f32 = lambda a: np.ascontiguousarray(a, dtype=np.float32)
    return RawScene(f32(means), f32(q), f32(log_s), f32(logits), tex)


# 500k splats, 8x8 textures (BF16 render copy of FP32 masters), 32 views 1280x720 on a radius-8
# sphere, batches of 4 views per iteration, targets from a perturbed copy of the scene
TRAIN_CONFIG = dict(P=500_000, lo=-4.0, hi=4.0, s_lo=0.02, s_hi=0.2, N=8, n_views=32,
                    res=(1280, 720), radius=8.0, batch=4)


def train_config(seed: int = 0, P: Optional[int] = None, n_views: Optional[int] = None,
                 res: Optional[Tuple[int, int]] = None):
    """Raw scene, raw target scene, views and a batch schedule generator of the training
    workload. ``batches(k)`` gives k batches of view indices: each a slice of a fresh
    permutation of the views (seed + 4 stream), batch size TRAIN_CONFIG['batch']."""
    c = TRAIN_CONFIG
    P = P if P is not None else c["P"]
    nv = n_views if n_views is not None else c["n_views"]
    res = res if res is not None else c["res"]
    raw = make_raw_scene(seed, P, c["lo"], c["hi"], c["s_lo"], c["s_hi"], c["N"])
    target = perturb_raw(raw, seed + 3)
    views = orbit_views(seed, nv, c["radius"], [res])
    rng = np.random.default_rng(seed + 4)
    b = c["batch"]

    def batches(k: int) -> List[List[int]]:
        out: List[List[int]] = []
        while len(out) < k:
            perm = rng.permutation(nv)
            out.extend([list(map(int, perm[i:i + b])) for i in range(0, nv - b + 1, b)])
        return out[:k]

    return raw, target, views, batches



def synthetic_image(seed: int, width: int, height: int) -> np.ndarray:
    """A seeded RGB image [H * W, 3] in [0, 1] standing in for the paper's photographs: smooth
    colour gradients, a few sinusoidal stripes (fine texture) and 24 flat-coloured discs (sharp
    edges)."""
    rng = np.random.default_rng(seed)
    y, x = np.mgrid[0:height, 0:width].astype(np.float64)
    u, v = x / max(width - 1, 1), y / max(height - 1, 1)
    img = np.stack([0.2 + 0.6 * u, 0.3 + 0.5 * v, 0.5 + 0.3 * (1.0 - u) * v], axis=-1)
    for _ in range(3):
        k = rng.uniform(20.0, 120.0, 2)
        ph = rng.uniform(0.0, 2.0 * math.pi)
        img += 0.08 * np.sin(k[0] * u + k[1] * v + ph)[..., None] * rng.uniform(-1.0, 1.0, 3)
    for _ in range(24):
        cx, cy = rng.uniform(0, width), rng.uniform(0, height)
        r = rng.uniform(0.02, 0.12) * min(width, height)
        img[(x - cx) ** 2 + (y - cy) ** 2 < r * r] = rng.uniform(0.0, 1.0, 3)
    return np.ascontiguousarray(np.clip(img, 0.0, 1.0).reshape(-1, 3), dtype=np.float32)


def image_fit_config(seed: int, P: int, width: int, height: int, N: int,
                     depth: float = 1.0, fov_deg: float = 60.0):
    """The single-image fitting set-up (Sec. 4): one camera at the origin looking down +z, the
    splats on the plane z = depth inside the view, rotated about z only (quaternions
    (cos a/2, 0, 0, sin a/2), a uniform), scales of 0.5 to 1.5 times sqrt(W H / P) pixels at
    that depth (so the splats together cover the image about once),
    opacities uniform in [0.3, 0.9], colour grids uniform in [0, 1], and a synthetic target
    image. Returns (raw scene, view, target [H * W, 3])."""
    view = frontal_view(width, height, fov_deg)
    rng = np.random.default_rng(seed)
    half_w = (width / 2.0) / float(view.fx) * depth
    half_h = (height / 2.0) / float(view.fy) * depth
    means = np.stack([rng.uniform(-half_w, half_w, P), rng.uniform(-half_h, half_h, P),
                      np.full(P, depth)], axis=1)
    a = rng.uniform(0.0, 2.0 * math.pi, P)
    q = np.stack([np.cos(a / 2), np.zeros(P), np.zeros(P), np.sin(a / 2)], axis=1)
    px = depth / float(view.fx)  # world size of one pixel at that depth
    log_s = np.log(rng.uniform(0.5, 1.5, (P, 2)) * math.sqrt(width * height / P) * px)
    o = rng.uniform(0.3, 0.9, P)
    tex = rng.uniform(0.0, 1.0, (P, N, N, 3))
    f32 = lambda arr: np.ascontiguousarray(arr, dtype=np.float32)
    raw = RawScene(f32(means), f32(q), f32(log_s), f32(np.log(o / (1.0 - o))), f32(tex))
    return raw, view, synthetic_image(seed + 1, width, height)
