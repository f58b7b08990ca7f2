"""Training step around the rasterizer: activations, image loss (L1 or MSE) and Adam.

The paper optimises the splats' positions, rotations, scales, opacities and colour grids
against images (Sec. 3.3). This module keeps raw float32 parameters with their Adam moments
on the device, activates them (quaternion -> tangents, exp scales, sigmoid opacity), renders a
batch of views, takes the L1 loss against target images, backpropagates through the
rasterizer and the activations and applies Adam to every parameter group. With bfloat16
textures the Adam step also rewrites the bfloat16 render copy of the float32 master textures.
For fitting a single image (Sec. 4) the loss is the mean squared error and the splats rotate
about the camera's Z axis only (``rotz_only``); ``box_filter_textures`` downsamples fitted
colour grids as the paper does to show that they carry the image. ``TrainState.densify``
applies densification and pruning (clone, split with resampled colour grids, opacity and size
pruning) from the screen-space gradient statistic the Trainer accumulates after each backward.
Every step runs in libgbb kernels; torch supplies memory and the stream. The SSIM term is not
part of it.
"""
from __future__ import annotations

import ctypes
from typing import Dict, Optional, Sequence

import torch

from . import _lib as L
from ._lib import GbbError
from .render import Options, Rasterizer, Splats, _stream

# learning rates per parameter group (not given by the paper; only their cost matters here)
DEFAULT_LR = dict(means=1.6e-4, quats=1e-3, log_scales=5e-3, opacity_logits=5e-2,
                  textures=2.5e-3)
GROUPS = ("means", "quats", "log_scales", "opacity_logits", "textures")


def _p(t: Optional[torch.Tensor]):
    return None if t is None else t.data_ptr()


class TrainState:
    """Raw parameters (float32 masters), Adam moments and activated copies on the device."""

    def __init__(self, raw, bf16: bool = True, device="cuda",
                 lr: Optional[Dict[str, float]] = None, betas=(0.9, 0.999), eps: float = 1e-15,
                 rotz_only: bool = False):
        self.lib = L.load()
        self.rotz_only = rotz_only
        self.device = torch.device(device)
        f = lambda a: torch.from_numpy(a).to(self.device).contiguous()
        self.params = {g: f(getattr(raw, g)) for g in GROUPS}
        self.m = {g: torch.zeros_like(t) for g, t in self.params.items()}
        self.v = {g: torch.zeros_like(t) for g, t in self.params.items()}
        self.raw_grads = {g: torch.zeros_like(t) for g, t in self.params.items()}
        P = self.P = int(self.params["means"].shape[0])
        self.N = int(self.params["textures"].shape[1])
        z = lambda *s: torch.empty(s, dtype=torch.float32, device=self.device)
        self.tan_u, self.tan_v, self.scales, self.opacity = z(P, 3), z(P, 3), z(P, 2), z(P)
        self.bf16 = bf16
        self.tex_bits = None
        if bf16:
            tex = self.params["textures"]
            self.tex_bits = torch.empty(tex.shape, dtype=torch.int16, device=self.device)
            L.check(self.lib.gb_to_bf16(tex.numel(), _p(tex), _p(self.tex_bits),
                                        self.stream()), "gb_to_bf16")
        self.lr = dict(DEFAULT_LR, **(lr or {}))
        self.betas, self.eps = betas, eps
        self.step_count = 0

    def stream(self) -> int:
        return _stream(self.device)

    def activate(self) -> Splats:
        p = self.params
        L.check(self.lib.gb_activate_fwd(self.P, _p(p["quats"]), _p(p["log_scales"]),
                                         _p(p["opacity_logits"]), _p(self.tan_u),
                                         _p(self.tan_v), _p(self.scales), _p(self.opacity),
                                         self.stream()), "gb_activate_fwd")
        tex = self.tex_bits.view(torch.bfloat16) if self.bf16 else p["textures"]
        return Splats(p["means"], self.tan_u, self.tan_v, self.scales, self.opacity, tex)

    def backward_activations(self, grads: Dict[str, torch.Tensor]) -> Dict[str, torch.Tensor]:
        """Rasterizer gradients (activated parameters) -> gradients of the raw parameters."""
        p, r = self.params, self.raw_grads
        L.check(self.lib.gb_activate_bwd(self.P, _p(p["quats"]), _p(p["log_scales"]),
                                         _p(p["opacity_logits"]), _p(grads["tan_u"]),
                                         _p(grads["tan_v"]), _p(grads["scales"]),
                                         _p(grads["opacity"]), _p(r["quats"]),
                                         _p(r["log_scales"]), _p(r["opacity_logits"]),
                                         self.stream()), "gb_activate_bwd")
        if self.rotz_only:
            L.check(self.lib.gb_rotz_only(self.P, _p(r["quats"]), self.stream()), "gb_rotz_only")
        r["means"] = grads["means"]
        r["textures"] = grads["textures"]
        return r

    def raw(self, params: Optional[Dict[str, torch.Tensor]] = None) -> L.GbRawSplats:
        p = params or self.params
        P = int(p["means"].shape[0])
        return L.GbRawSplats(P, self.N, 0, _p(p["means"]), _p(p["quats"]), _p(p["log_scales"]),
                             _p(p["opacity_logits"]), _p(p["textures"]), None)

    def densify(self, grad_accum: torch.Tensor, vis_count: torch.Tensor,
                options: Optional["DensifyOptions"] = None, noise: Optional[torch.Tensor] = None,
                sigma: float = 0.5, generator: Optional[torch.Generator] = None) -> int:
        """Densification and pruning from the accumulated statistic (one host synchronisation
        for the new count). Replaces the parameters, their Adam moments (kept rows copied, new
        rows zero), the activated copies and the bfloat16 texture copy. ``noise`` ([P, 2, 2]
        N(0, 1), the split children's offsets in units of the parent's scales) is drawn on the
        device when not given. Returns the new number of splats."""
        o = (options or DensifyOptions()).c()
        P = self.P
        work = torch.empty(int(self.lib.gb_densify_work_bytes(P)), dtype=torch.uint8,
                           device=self.device)
        P_new = ctypes.c_int64(0)
        src = self.raw()
        L.check(self.lib.gb_densify_plan(ctypes.byref(src), _p(grad_accum), _p(vis_count),
                                         ctypes.byref(o), _p(work), work.numel(),
                                         ctypes.byref(P_new), self.stream()), "gb_densify_plan")
        n = int(P_new.value)
        if noise is None:
            noise = torch.randn((P, 2, 2), dtype=torch.float32, device=self.device,
                                generator=generator)
        new = {g: torch.empty((n,) + tuple(t.shape[1:]), dtype=torch.float32, device=self.device)
               for g, t in self.params.items()}
        new_m = {g: torch.empty_like(t) for g, t in new.items()}
        new_v = {g: torch.empty_like(t) for g, t in new.items()}
        rows = []
        for g in GROUPS:
            w = int(self.params[g][0].numel()) if P > 0 else 1
            rows.append(L.GbRowState(_p(self.m[g]), _p(new_m[g]), w))
            rows.append(L.GbRowState(_p(self.v[g]), _p(new_v[g]), w))
        states = (L.GbRowState * len(rows))(*rows)
        dst = self.raw(new)
        L.check(self.lib.gb_densify_apply(ctypes.byref(src), _p(work), _p(noise.contiguous()),
                                          float(sigma), ctypes.byref(o), ctypes.byref(dst),
                                          states, len(rows), self.stream()), "gb_densify_apply")
        self.params, self.m, self.v = new, new_m, new_v
        self.raw_grads = {g: torch.zeros_like(t) for g, t in new.items()}
        self.P = n
        z = lambda *s: torch.empty(s, dtype=torch.float32, device=self.device)
        self.tan_u, self.tan_v, self.scales, self.opacity = z(n, 3), z(n, 3), z(n, 2), z(n)
        if self.bf16:
            tex = self.params["textures"]
            self.tex_bits = torch.empty(tex.shape, dtype=torch.int16, device=self.device)
            L.check(self.lib.gb_to_bf16(tex.numel(), _p(tex), _p(self.tex_bits), self.stream()),
                    "gb_to_bf16")
        return n

    def adam(self, raw_grads: Dict[str, torch.Tensor]) -> None:
        self.step_count += 1
        b1, b2 = self.betas
        for g in GROUPS:
            t = self.params[g]
            bits = self.tex_bits if (g == "textures" and self.bf16) else None
            L.check(self.lib.gb_adam_step(t.numel(), _p(t), _p(raw_grads[g]), _p(self.m[g]),
                                          _p(self.v[g]), self.step_count, self.lr[g], b1, b2,
                                          self.eps, _p(bits), self.stream()), "gb_adam_step")


def l1_loss(rgb: torch.Tensor, target: torch.Tensor, scale: float, loss: torch.Tensor,
            d_rgb: torch.Tensor) -> None:
    """loss[0] = scale * sum |rgb - target|, d_rgb = scale * sign(rgb - target)."""
    lib = L.load()
    L.check(lib.gb_l1_loss(rgb.numel(), _p(rgb), _p(target), float(scale), _p(loss), _p(d_rgb),
                           _stream(rgb.device)), "gb_l1_loss")


def mse_loss(rgb: torch.Tensor, target: torch.Tensor, scale: float, loss: torch.Tensor,
             d_rgb: torch.Tensor) -> None:
    """loss[0] = scale * sum (rgb - target)^2, d_rgb = 2 scale (rgb - target)."""
    lib = L.load()
    L.check(lib.gb_mse_loss(rgb.numel(), _p(rgb), _p(target), float(scale), _p(loss),
                            _p(d_rgb), _stream(rgb.device)), "gb_mse_loss")


def box_filter_textures(textures: torch.Tensor, M: int) -> torch.Tensor:
    """[P, N, N, 3] float32 colour grids -> [P, M, M, 3], each texel the mean of the N / M
    square of texels it covers (M divides N)."""
    lib = L.load()
    textures = textures.contiguous()
    P, N = int(textures.shape[0]), int(textures.shape[1])
    out = torch.empty((P, M, M, 3), dtype=torch.float32, device=textures.device)
    L.check(lib.gb_box_filter_textures(P, N, M, _p(textures), _p(out), _stream(textures.device)),
            "gb_box_filter_textures")
    return out


class DensifyOptions:
    """Densification and pruning thresholds (gb_densify_options): the statistic threshold,
    the clone/split scale, the pruning opacity and scale (0: off) and the split shrink."""

    def __init__(self, grad_threshold=0.0002, dense_scale=0.01, min_opacity=0.005,
                 max_scale=0.0, split_shrink=1.6):
        self.grad_threshold, self.dense_scale = grad_threshold, dense_scale
        self.min_opacity, self.max_scale, self.split_shrink = min_opacity, max_scale, split_shrink

    def c(self) -> L.GbDensifyOptions:
        return L.GbDensifyOptions(self.grad_threshold, self.dense_scale, self.min_opacity,
                                  self.max_scale, self.split_shrink)


class Trainer:
    """One optimisation step per call on a batch of views with target images.

    targets: [n_views, H * W, 3] float32 on the device, one image per view (views of
    different sizes use the first width * height rows of theirs)."""

    def __init__(self, state: TrainState, views: Sequence, targets: torch.Tensor,
                 options: Optional[Options] = None, loss: str = "l1"):
        if loss not in ("l1", "mse"):
            raise ValueError("loss must be 'l1' or 'mse'")
        self.loss_fn = l1_loss if loss == "l1" else mse_loss
        self.state, self.views, self.targets = state, list(views), targets
        self.rast: Optional[Rasterizer] = None
        self.options = options or Options()
        self.loss = torch.zeros(1, dtype=torch.float32, device=state.device)
        self.bufs = None
        self.grads = None
        # densification statistic, accumulated after every backward once enabled
        self.grad_accum: Optional[torch.Tensor] = None
        self.vis_count: Optional[torch.Tensor] = None

    def track_densify(self, on: bool = True) -> None:
        """Start (or stop) accumulating the densification statistic of every step."""
        if on:
            self.grad_accum = torch.zeros(self.state.P, dtype=torch.float32,
                                          device=self.state.device)
            self.vis_count = torch.zeros_like(self.grad_accum)
        else:
            self.grad_accum = self.vis_count = None

    def densify(self, options: Optional[DensifyOptions] = None,
                noise: Optional[torch.Tensor] = None, generator=None) -> int:
        """Densify and prune from the statistic accumulated since the last call, reset it and
        drop the buffers sized for the old splat count. Returns the new count."""
        if self.grad_accum is None:
            raise RuntimeError("call track_densify() before training steps to densify")
        n = self.state.densify(self.grad_accum, self.vis_count, options, noise,
                               generator=generator)
        self.grads = None
        self.track_densify(True)
        return n

    def _use(self, batch: Sequence[int]) -> None:
        views = [self.views[i] for i in batch]
        if self.rast is None:
            self.rast = Rasterizer(views, self.options, device=self.state.device, headroom=1.5)
        else:
            self.rast.set_views(views)

    def plan(self, batches: Sequence[Sequence[int]], headroom: float = 1.5) -> int:
        """Sizes the pair capacity for the largest of the given batches at the current
        parameters (one device count per distinct batch) and turns the per-step overflow
        check off, so that steps never wait on the host. The headroom covers the drift of the
        parameters during training; ``overflowed()`` tells whether the last step fitted."""
        sp = self.state.activate()
        K = 0
        for b in sorted({tuple(b) for b in batches}):
            self._use(b)
            K = max(K, self.rast.count_pairs(sp))
        cap = self.rast.plan(sp, int(K * headroom) + 4096)
        self.rast.check_overflow = False
        return cap

    def overflowed(self) -> bool:
        """Whether some step since the previous call overflowed its pair capacity (such a
        step rendered background and took no gradient). Synchronises."""
        return self.rast is not None and self.rast.status_ex()[2]

    def step(self, batch: Sequence[int]) -> torch.Tensor:
        st = self.state
        self._use(batch)
        sp = st.activate()
        n_px = sum(self.views[i].width * self.views[i].height for i in batch)
        if self.bufs is None or self.bufs[0].shape[0] != n_px:
            z = lambda *s: torch.empty(s, dtype=torch.float32, device=st.device)
            self.bufs = (z(n_px, 3), z(n_px), z(n_px, 3), z(n_px, 3))
        rgb, T, target, d_rgb = self.bufs
        # the forward zeroes the texture gradients of the backward below while it blends
        zg = self.grads if (self.grads is not None
                            and self.grads["textures"].numel() == 3 * sp.n_texels) else None
        try:
            rgb, T = self.rast.forward(sp, rgb, T, zero_grads=zg)
        except GbbError as e:
            if e.status != L.GB_ERR_CAPACITY:
                raise
            # a completed earlier step overflowed: re-size for this batch and render again
            self.rast.plan(sp, int(self.rast.count_pairs(sp) * 1.5) + 4096)
            rgb, T = self.rast.forward(sp, rgb, T, zero_grads=zg)
        at = 0
        for i in batch:  # device-to-device copies of the batch's target images
            hw = self.views[i].width * self.views[i].height
            target[at:at + hw].copy_(self.targets[i].view(-1, 3)[:hw])
            at += hw
        self.loss_fn(rgb, target, 1.0 / (3 * n_px), self.loss, d_rgb)
        self.grads = self.rast.backward(sp, T, d_rgb, self.grads)
        if self.grad_accum is not None:
            r = self.rast
            L.check(r.lib.gb_densify_stats(ctypes.byref(sp.c()), r.cviews, r.nv,
                                           ctypes.byref(r.copts), r.ws.data_ptr(), r.ws.numel(),
                                           r.capacity, self.grad_accum.data_ptr(),
                                           self.vis_count.data_ptr(), st.stream()),
                    "gb_densify_stats")
        st.adam(st.backward_activations(self.grads))
        return self.loss
