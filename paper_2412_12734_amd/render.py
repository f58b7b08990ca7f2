"""Torch-facing binding of libgbb: device buffers, streams and autograd.

PyTorch only provides memory and the stream here; every computation runs in the HIP library
through the C ABI of include/gbb.h.
"""
from __future__ import annotations

import ctypes
import dataclasses
from typing import Optional, Sequence, Tuple

import numpy as np
import torch

from . import _lib as L


@dataclasses.dataclass
class Options:
    sigma: float = 0.5
    alpha_min: float = 1.0 / 255.0
    alpha_max: float = 0.99
    t_min: float = 1e-4
    lowpass_var: float = 0.5
    bg: Tuple[float, float, float] = (0.0, 0.0, 0.0)
    tile_w: int = 16
    tile_h: int = 16
    batch: int = 0
    batch_bwd: int = 0
    # depth-prefix split: pairs per tile of the first pass (0 = default), -1 = one pass
    prefix_pairs_per_tile: int = 0
    # order of the tiles over the blend workgroups: 0 = default, 1 = most work first,
    # -1 = fixed bands of neighbouring tiles per XCD
    tile_order: int = 0

    def c(self) -> L.GbOptions:
        return L.make_options(self.sigma, self.alpha_min, self.alpha_max, self.t_min,
                              self.lowpass_var, tuple(self.bg), self.tile_w, self.tile_h,
                              self.batch, self.batch_bwd, self.prefix_pairs_per_tile,
                              self.tile_order)


def _ptr(t: Optional[torch.Tensor]) -> Optional[int]:
    return None if t is None else t.data_ptr()


def _stream(device) -> int:
    return torch.cuda.current_stream(device).cuda_stream


class Splats:
    """Device views of the per-splat arrays in the layout the library expects. ``sh``
    (optional, [P, (D+1)^2, 3] float32) holds the spherical-harmonic coefficients of the
    view-dependent colour term.

    Colour grids of several sides: with ``tex_side`` ([P] int32, each side in [1, layout_side])
    and ``tex_offset`` ([P] int64, the first texel of each grid), ``textures`` is the packed
    [n_texels, 3] array of all grids, each [n][n][3] row-major, and ``layout_side`` (8 or 16)
    is the largest side allowed; texture gradients then come back in the same packed layout."""

    def __init__(self, means, tan_u, tan_v, scales, opacity, textures, sh=None, tex_side=None,
                 tex_offset=None, layout_side=None):
        self.means, self.tan_u, self.tan_v = means, tan_u, tan_v
        self.scales, self.opacity, self.textures = scales, opacity, textures
        self.sh = sh
        self.tex_side, self.tex_offset = tex_side, tex_offset
        for name in ("means", "tan_u", "tan_v", "scales", "opacity"):
            t = getattr(self, name)
            if t.dtype != torch.float32 or not t.is_contiguous() or not t.is_cuda:
                raise ValueError(f"{name} must be a contiguous float32 CUDA tensor")
        if textures.dtype not in (torch.float32, torch.bfloat16) or not textures.is_contiguous():
            raise ValueError("textures must be contiguous float32 or bfloat16")
        self.P = int(means.shape[0])
        if tex_side is None:
            self.N = int(textures.shape[1])
            self.n_texels = self.P * self.N * self.N
        else:
            if (tex_side.dtype != torch.int32 or tex_offset is None
                    or tex_offset.dtype != torch.int64 or not tex_side.is_contiguous()
                    or not tex_offset.is_contiguous() or tex_side.shape[0] != self.P
                    or tex_offset.shape[0] != self.P or layout_side not in (8, 16)
                    or textures.dim() != 2 or textures.shape[1] != 3):
                raise ValueError("mixed grids take tex_side int32 [P], tex_offset int64 [P], "
                                 "layout_side 8 or 16 and packed textures [n_texels, 3]")
            self.N = int(layout_side)
            self.n_texels = int(textures.shape[0])
        self.sh_degree = -1
        if sh is not None:
            n = int(sh.shape[1])
            d = int(round(n ** 0.5)) - 1
            if (sh.dtype != torch.float32 or not sh.is_contiguous() or sh.dim() != 3
                    or (d + 1) ** 2 != n or not 0 <= d <= 3 or sh.shape[0] != self.P):
                raise ValueError("sh must be contiguous float32 [P, (D+1)^2, 3] with D <= 3")
            self.sh_degree = d

    @property
    def mixed(self) -> bool:
        return self.tex_side is not None

    @staticmethod
    def from_numpy(scene, device="cuda", tex_bf16: bool = False) -> "Splats":
        """From a scene whose textures are one [P,N,N,3] array, or a list of per-splat [n,n,3]
        grids of several sides (packed here in splat order)."""
        f = lambda a: torch.from_numpy(a).to(device)
        sh = getattr(scene, "sh", None)
        side = off = layout = None
        if isinstance(scene.textures, np.ndarray):
            tex = torch.from_numpy(scene.textures).to(device)
        else:
            sides = np.array([g.shape[0] for g in scene.textures], dtype=np.int32)
            offsets = np.zeros(len(sides), dtype=np.int64)
            offsets[1:] = np.cumsum(sides.astype(np.int64) ** 2)[:-1]
            packed = np.concatenate([np.asarray(g, dtype=np.float32).reshape(-1, 3)
                                     for g in scene.textures])
            tex = torch.from_numpy(np.ascontiguousarray(packed)).to(device)
            side, off = f(sides), f(offsets)
            layout = 8 if int(sides.max()) <= 8 else 16
        if tex_bf16:
            tex = tex.to(torch.bfloat16)
        return Splats(f(scene.means), f(scene.tan_u), f(scene.tan_v), f(scene.scales),
                      f(scene.opacity), tex, None if sh is None else f(sh), side, off, layout)

    def c(self) -> L.GbSplats:
        dt = L.GB_BF16 if self.textures.dtype == torch.bfloat16 else L.GB_F32
        return L.GbSplats(self.P, self.N, dt, _ptr(self.means), _ptr(self.tan_u),
                          _ptr(self.tan_v), _ptr(self.scales), _ptr(self.opacity),
                          _ptr(self.textures), max(self.sh_degree, 0), _ptr(self.sh),
                          _ptr(self.tex_side), _ptr(self.tex_offset),
                          self.n_texels if self.mixed else 0)


class Rasterizer:
    """Renders splats into a fixed set of views, owning the workspace between calls.

    ``plan`` counts the (tile, splat) pairs on the device (one synchronisation) and sizes
    the workspace with ``headroom``; ``forward``/``backward`` then run without host
    synchronisation. With ``check_overflow`` the forward reads the device status after each
    call and re-plans if the pair capacity was exceeded.
    """

    def __init__(self, views: Sequence, options: Optional[Options] = None, device="cuda",
                 headroom: float = 1.25, check_overflow: bool = True):
        self.lib = L.load()
        self.views = list(views)
        self.cviews = L.make_views(self.views)
        self.nv = len(self.views)
        self.opts = options or Options()
        self.copts = self.opts.c()
        self.device = torch.device(device)
        self.headroom = headroom
        self.check_overflow = check_overflow
        self.capacity = 0
        self.ws: Optional[torch.Tensor] = None
        self.layout = L.GbLayout()
        self.total_pixels = sum(int(v.width) * int(v.height) for v in self.views)
        # bumped by every forward and view change: a backward must follow the forward whose
        # workspace contents it reads
        self.generation = 0

    # -- workspace -------------------------------------------------------------------------
    def _layout(self, P: int, N: int, capacity: int) -> L.GbLayout:
        lay = L.GbLayout()
        L.check(self.lib.gb_workspace_layout(P, N, self.cviews, self.nv, ctypes.byref(self.copts),
                                             capacity, ctypes.byref(lay)), "gb_workspace_layout")
        return lay

    def _alloc(self, P: int, N: int, capacity: int) -> None:
        lay = self._layout(P, N, capacity)
        if self.ws is None or self.ws.numel() < lay.total_bytes:
            self.ws = torch.empty(int(lay.total_bytes), dtype=torch.uint8, device=self.device)
        self.capacity = capacity
        self.layout = lay
        self._plan_key = (P, N)

    def count_pairs(self, sp: Splats) -> int:
        if self.ws is None or getattr(self, "_plan_key", None) != (sp.P, sp.N):
            self._alloc(sp.P, sp.N, 0)
        K = ctypes.c_int64(0)
        L.check(self.lib.gb_count_pairs(ctypes.byref(sp.c()), self.cviews, self.nv,
                                        ctypes.byref(self.copts), self.ws.data_ptr(),
                                        self.ws.numel(), self.capacity, ctypes.byref(K),
                                        _stream(self.device)), "gb_count_pairs")
        return int(K.value)

    def plan(self, sp: Splats, capacity: Optional[int] = None) -> int:
        if capacity is None:
            K = self.count_pairs(sp)
            capacity = int(K * self.headroom) + 4096
        self._alloc(sp.P, sp.N, capacity)
        return capacity

    def status(self) -> Tuple[int, bool]:
        """(pair count, overflow) of the last forward (synchronises)."""
        K, over, _ = self.status_ex()
        return K, over

    def status_ex(self, per_view: bool = False):
        """(pair count, last forward overflowed, some forward since the previous status call
        overflowed) and, with ``per_view``, the list of per-view pair counts."""
        K = ctypes.c_int64(0)
        ov = ctypes.c_int32(0)
        kv = (ctypes.c_int64 * self.nv)() if per_view else None
        L.check(self.lib.gb_read_status(self.ws.data_ptr(), ctypes.byref(K), ctypes.byref(ov),
                                        kv, self.nv, _stream(self.device)), "gb_read_status")
        out = (int(K.value), bool(ov.value & 1), bool(ov.value & 2))
        return out + (list(kv),) if per_view else out

    # -- raw calls -------------------------------------------------------------------------
    def forward(self, sp: Splats, rgb: Optional[torch.Tensor] = None,
                T_final: Optional[torch.Tensor] = None, zero_grads: Optional[dict] = None):
        """Forward render. ``zero_grads`` (optional): the gradient dict that the next
        ``backward`` will be given; the forward then zeroes its texture gradients while it
        blends, and that backward skips its own clear (the dict must not be written in
        between)."""
        if self.ws is None or getattr(self, "_plan_key", None) != (sp.P, sp.N) or self.capacity == 0:
            self.plan(sp)
        if rgb is None:
            rgb = torch.empty((self.total_pixels, 3), dtype=torch.float32, device=self.device)
        if T_final is None:
            T_final = torch.empty((self.total_pixels,), dtype=torch.float32, device=self.device)
        self.generation += 1
        zt = None if zero_grads is None else zero_grads["textures"]
        if zt is not None and (zt.dtype != torch.float32 or not zt.is_contiguous()
                               or zt.numel() != 3 * sp.n_texels):
            raise ValueError("zero_grads['textures'] must be the contiguous float32 texture "
                             "gradient of these splats")
        for _ in range(3):
            if zt is None:
                st = self.lib.gb_render_fwd(ctypes.byref(sp.c()), self.cviews, self.nv,
                                            ctypes.byref(self.copts), self.ws.data_ptr(),
                                            self.ws.numel(), self.capacity, rgb.data_ptr(),
                                            T_final.data_ptr(), _stream(self.device))
            else:
                st = self.lib.gb_render_fwd_zeroing(
                    ctypes.byref(sp.c()), self.cviews, self.nv, ctypes.byref(self.copts),
                    self.ws.data_ptr(), self.ws.numel(), self.capacity, rgb.data_ptr(),
                    T_final.data_ptr(), zt.data_ptr(), _stream(self.device))
            if st == L.GB_ERR_CAPACITY and self.check_overflow:
                # an earlier forward on this workspace overflowed: count again and re-size
                self.plan(sp)
                continue
            L.check(st, "gb_render_fwd")
            if not self.check_overflow:
                break
            K, over = self.status()
            if not over:
                break
            self._alloc(sp.P, sp.N, int(K * self.headroom) + 4096)
        return rgb, T_final

    def backward(self, sp: Splats, T_final: torch.Tensor, d_rgb: torch.Tensor, grads=None):
        if grads is None:
            z = lambda *s: torch.empty(s, dtype=torch.float32, device=self.device)
            grads = dict(means=z(sp.P, 3), tan_u=z(sp.P, 3), tan_v=z(sp.P, 3),
                         scales=z(sp.P, 2), opacity=z(sp.P),
                         textures=(z(sp.n_texels, 3) if sp.mixed else z(sp.P, sp.N, sp.N, 3)))
        if sp.sh is not None and grads.get("sh") is None:
            grads["sh"] = torch.empty_like(sp.sh)
        d_rgb = d_rgb.contiguous().float()
        g = L.GbGrads(_ptr(grads["means"]), _ptr(grads["tan_u"]), _ptr(grads["tan_v"]),
                      _ptr(grads["scales"]), _ptr(grads["opacity"]), _ptr(grads["textures"]),
                      _ptr(grads.get("sh")) if sp.sh is not None else None)
        L.check(self.lib.gb_render_bwd(ctypes.byref(sp.c()), self.cviews, self.nv,
                                       ctypes.byref(self.copts), self.ws.data_ptr(),
                                       self.ws.numel(), self.capacity, T_final.data_ptr(),
                                       d_rgb.data_ptr(), ctypes.byref(g), _stream(self.device)),
                "gb_render_bwd")
        return grads

    def set_views(self, views: Sequence) -> None:
        """Renders into another set of views from now on. If the views have the same sizes as
        before, the workspace layout is unchanged and is kept (the capacity is re-planned on
        overflow when check_overflow is set); otherwise the next forward plans again."""
        views = list(views)
        self.generation += 1
        same = [(v.width, v.height) for v in views] == [(v.width, v.height) for v in self.views]
        self.views = views
        self.cviews = L.make_views(views)
        self.nv = len(views)
        if not same:
            self.total_pixels = sum(v.width * v.height for v in views)
            self.ws, self.capacity, self._plan_key = None, 0, None

    def capture_step(self, sp: Splats, rgb: torch.Tensor, T_final: torch.Tensor,
                     d_rgb: torch.Tensor, grads: dict) -> "torch.cuda.CUDAGraph":
        """Records one forward + backward over the given preallocated tensors into a HIP graph
        (torch.cuda.CUDAGraph); ``replay()`` reruns it. Every launch reads the pair count from
        the workspace, so nothing in the step returns to the host; the capacity must fit the
        scene (plan first; inside a graph an overflow is not re-planned: check ``status()``
        after a replay). The library clears memory with kernels, never hipMemsetAsync."""
        if self.ws is None or getattr(self, "_plan_key", None) != (sp.P, sp.N):
            self.plan(sp)
        if d_rgb.dtype != torch.float32 or not d_rgb.is_contiguous():
            raise ValueError("d_rgb must be a contiguous float32 tensor")
        keep = self.check_overflow
        self.check_overflow = False
        try:
            side = torch.cuda.Stream(self.device)
            side.wait_stream(torch.cuda.current_stream(self.device))
            with torch.cuda.stream(side):  # warm-up outside the capture
                self.forward(sp, rgb, T_final, zero_grads=grads)
                self.backward(sp, T_final, d_rgb, grads)
            torch.cuda.current_stream(self.device).wait_stream(side)
            graph = torch.cuda.CUDAGraph()
            with torch.cuda.graph(graph):
                self.forward(sp, rgb, T_final, zero_grads=grads)
                self.backward(sp, T_final, d_rgb, grads)
        finally:
            self.check_overflow = keep
        return graph

    # -- measurement ---------------------------------------------------------------------------
    def blend_stats(self, sp: Splats, rgb: torch.Tensor, T_final: torch.Tensor) -> dict:
        """Forward with work counting (synchronises): blended pairs, t_min stops, lane
        evaluations, staged (tile, splat) pairs and the blended pairs of the rest pass."""
        c = (ctypes.c_int64 * 5)()
        L.check(self.lib.gb_blend_stats(ctypes.byref(sp.c()), self.cviews, self.nv,
                                        ctypes.byref(self.copts), self.ws.data_ptr(),
                                        self.ws.numel(), self.capacity, rgb.data_ptr(),
                                        T_final.data_ptr(), c, _stream(self.device)),
                "gb_blend_stats")
        return dict(blended=c[0], terminated=c[1], lane_evals=c[2], staged=c[3],
                    rest_blended=c[4])

    def timing(self, on: bool) -> None:
        L.check(self.lib.gb_timing_enable(1 if on else 0), "gb_timing_enable")

    def stage_times(self) -> dict:
        ms = (ctypes.c_float * 16)()
        n = ctypes.c_int32(0)
        L.check(self.lib.gb_timing_read(ms, 16, ctypes.byref(n)), "gb_timing_read")
        return {self.lib.gb_timing_stage_name(i).decode(): float(ms[i]) for i in range(n.value)
                if ms[i] >= 0.0}

    # -- workspace read-back (inspection and tests) ------------------------------------------
    def section(self, name: str, count: int, dtype=torch.int32) -> torch.Tensor:
        off = getattr(self.layout, name)
        nbytes = count * torch.tensor([], dtype=dtype).element_size()
        return self.ws[off:off + nbytes].view(dtype)


class _RenderFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, rast: Rasterizer, means, tan_u, tan_v, scales, opacity, textures, sh):
        sp = Splats(means.detach(), tan_u.detach(), tan_v.detach(), scales.detach(),
                    opacity.detach(), textures.detach(), None if sh is None else sh.detach())
        rgb, T = rast.forward(sp)
        ctx.rast, ctx.sp = rast, sp
        # the backward reads the pair lists and per-pixel state this forward left in the
        # rasterizer's workspace: remember which forward that was
        ctx.generation = rast.generation
        ctx.ws_ptr = rast.ws.data_ptr()
        ctx.total_pixels = rast.total_pixels
        ctx.save_for_backward(T)
        ctx.mark_non_differentiable(T)
        return rgb, T

    @staticmethod
    def backward(ctx, d_rgb, d_T):
        (T,) = ctx.saved_tensors
        rast = ctx.rast
        if (rast.generation != ctx.generation or rast.ws is None
                or rast.ws.data_ptr() != ctx.ws_ptr or rast.total_pixels != ctx.total_pixels):
            raise RuntimeError(
                "render(): the Rasterizer ran another forward (or changed views) after this "
                "render and before its backward, so the workspace no longer holds this render's "
                "state; call backward first or give each pending render its own Rasterizer")
        if d_rgb is None:
            d_rgb = torch.zeros((ctx.total_pixels, 3), dtype=torch.float32, device=T.device)
        g = rast.backward(ctx.sp, T, d_rgb)
        dtex = g["textures"]
        if ctx.sp.textures.dtype != torch.float32:
            dtex = dtex.to(ctx.sp.textures.dtype)
        return (None, g["means"], g["tan_u"], g["tan_v"], g["scales"], g["opacity"], dtex,
                g.get("sh"))


def render(rast: Rasterizer, means, tan_u, tan_v, scales, opacity, textures, sh=None):
    """Differentiable render of all of ``rast``'s views: returns rgb [sum HW, 3] and T_final.
    ``sh`` (optional, [P, (D+1)^2, 3]) adds the per-splat view-dependent colour term.

    The backward reads state that the forward leaves in ``rast``'s workspace, so each render
    must be differentiated before ``rast`` renders again (a later forward raises in the
    earlier render's backward)."""
    return _RenderFn.apply(rast, means, tan_u, tan_v, scales, opacity, textures, sh)
