"""FP64 reference of densification and pruning of textured splats (test infrastructure only).

Only tests, the package's smoke check and the benchmark's CPU baseline use this module; the
product path never imports it, and it shares no code with the HIP kernels.

The paper trains its 3D scenes "with default densification and pruning" (Sec. 4.2), i.e. the
adaptive density control of Gaussian splatting that 2DGS inherits; it does not say how a split
divides a splat's colour grid. The readings written out here (each also in the design notes):

* Statistic: for every view in which a splat is visible (it covers at least one tile), the
  norm of the gradient of the loss with respect to a translation of the splat's footprint in
  the image (pixels) is added to accum[k] and 1 to count[k]; the mean is accum / count (0 for
  count 0).
* Decision, per splat, from the raw parameters: s_max = max(exp(log_scales)), o =
  sigmoid(logit). A splat whose mean is >= grad_threshold is densified: cloned if
  s_max <= dense_scale, split otherwise.
* Clone: the splat is kept and an identical copy follows it.
* Split: the splat is replaced by two children c = 0, 1. Child c's centre is
  p + s_u z_c0 t_u + s_v z_c1 t_v (z drawn N(0, 1) by the caller and passed in; t_u, t_v the
  first two columns of the rotation of q / |q|), its scales are s / shrink, and quaternion,
  opacity logit and SH coefficients are the parent's. Its colour grid resamples the parent's
  colour field: texel (i, j) sits at uv (u_i, v_j) of the child (u_i = -sigma + 2 sigma
  i / (N - 1), or 0 when N = 1), which is the parent's uv (z_c0 + u_i / shrink,
  z_c1 + v_j / shrink), and takes the parent's bilinear, border-clamped colour there
  (Alg. 2). A constant grid stays constant; the parent's field is reproduced where the
  child covers it.
* Pruning: every output splat (kept, clone copy or child) with opacity below min_opacity, or
  with max_scale > 0 and its largest scale above max_scale, is removed.
* Order: outputs follow their parents' order; a clone copy right after its parent, the two
  children in the parent's place.
* Optimiser state: kept splats (and a clone's original) keep their rows; clone copies and
  children start from zero.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence, Tuple

import numpy as np

from .gb_oracle import bilinear
from .train_oracle import rotation

KEEP, CLONE_COPY, CHILD0, CHILD1 = 0, 1, 2, 3


@dataclasses.dataclass
class DensifyOptions:
    grad_threshold: float = 0.0002
    dense_scale: float = 0.01
    min_opacity: float = 0.005
    max_scale: float = 0.0
    split_shrink: float = 1.6
    sigma: float = 0.5


def accumulate(accum, count, screen_grads: Sequence[np.ndarray], visible: Sequence[np.ndarray]):
    """accum += |screen gradient| and count += 1 for every view where the splat is visible."""
    accum = np.array(accum, dtype=np.float64, copy=True)
    count = np.array(count, dtype=np.float64, copy=True)
    for g, vis in zip(screen_grads, visible):
        accum += np.where(vis, np.linalg.norm(np.asarray(g, dtype=np.float64), axis=1), 0.0)
        count += vis.astype(np.float64)
    return accum, count


def plan(log_scales, opacity_logits, accum, count, opts: DensifyOptions):
    """Per output splat: (parent index, kind) in output order."""
    ls = np.asarray(log_scales, dtype=np.float64)
    s_max = np.exp(ls.max(axis=1))
    o = 1.0 / (1.0 + np.exp(-np.asarray(opacity_logits, dtype=np.float64)))
    accum = np.asarray(accum, dtype=np.float64)
    count = np.asarray(count, dtype=np.float64)
    mean = np.where(count > 0, accum / np.where(count > 0, count, 1.0), 0.0)

    def survives(smax):
        bad = o_k < opts.min_opacity
        if opts.max_scale > 0:
            bad = bad or smax > opts.max_scale
        return not bad

    out: List[Tuple[int, int]] = []
    for k in range(ls.shape[0]):
        o_k = o[k]
        if mean[k] >= opts.grad_threshold and s_max[k] > opts.dense_scale:
            if survives(s_max[k] / opts.split_shrink):
                out += [(k, CHILD0), (k, CHILD1)]
        elif mean[k] >= opts.grad_threshold:
            if survives(s_max[k]):
                out += [(k, KEEP), (k, CLONE_COPY)]
        elif survives(s_max[k]):
            out.append((k, KEEP))
    return out


def apply(outputs, means, quats, log_scales, opacity_logits, textures, noise,
          opts: DensifyOptions, sh=None, states: Sequence[np.ndarray] = ()):
    """New parameter arrays (float64) for the planned outputs; ``states`` are per-splat
    optimiser rows (kept rows copied, new rows zero)."""
    means = np.asarray(means, dtype=np.float64)
    quats = np.asarray(quats, dtype=np.float64)
    log_scales = np.asarray(log_scales, dtype=np.float64)
    textures = np.asarray(textures, dtype=np.float64)
    noise = np.asarray(noise, dtype=np.float64).reshape(-1, 2, 2)
    N = textures.shape[1]
    sig = opts.sigma
    R = rotation(quats)
    t_u, t_v = R[:, :, 0], R[:, :, 1]
    s = np.exp(log_scales)
    grid = np.array([0.0]) if N == 1 else -sig + 2.0 * sig * np.arange(N) / (N - 1)
    gu, gv = np.meshgrid(grid, grid, indexing="ij")
    new = {"means": [], "quats": [], "log_scales": [], "opacity_logits": [], "textures": [],
           "sh": [], "states": [[] for _ in states]}
    for k, kind in outputs:
        m = means[k]
        ls = log_scales[k]
        tex = textures[k]
        if kind in (CHILD0, CHILD1):
            z = noise[k, kind - CHILD0]
            m = m + s[k, 0] * z[0] * t_u[k] + s[k, 1] * z[1] * t_v[k]
            ls = ls - math.log(opts.split_shrink)
            pu = z[0] + gu.reshape(-1) / opts.split_shrink
            pv = z[1] + gv.reshape(-1) / opts.split_shrink
            tex = bilinear(textures[k], pu, pv, sig).reshape(N, N, 3)
        new["means"].append(m)
        new["quats"].append(quats[k])
        new["log_scales"].append(ls)
        new["opacity_logits"].append(float(opacity_logits[k]))
        new["textures"].append(tex)
        if sh is not None:
            new["sh"].append(np.asarray(sh[k], dtype=np.float64))
        for i, st in enumerate(states):
            row = np.asarray(st[k], dtype=np.float64)
            new["states"][i].append(row if kind == KEEP else np.zeros_like(row))
    out = {key: np.array(val) for key, val in new.items() if key not in ("sh", "states")}
    out["sh"] = np.array(new["sh"]) if sh is not None else None
    out["states"] = [np.array(v) for v in new["states"]]
    return out
