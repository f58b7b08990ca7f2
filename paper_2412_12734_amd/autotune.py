"""Launch-parameter autotuner for the rasterizer.

The fixed choices of the paper's kernels (16 x 16 tiles, dropping to 8 x 8 for 8 x 8 colour
grids because of shared-memory limits) are replaced by a measured choice per workload class:
tile shape, splats staged per LDS batch in the forward and in the backward, and the pair budget
of the depth-prefix pass. Every candidate computes the same image up to float32 rounding (tile
shape moves the centre the per-pixel solve is re-centred on; batch sizes and the prefix budget
do not change any arithmetic).

The search is coordinate descent from the library defaults: each knob in turn takes the value
with the lowest measured cost while the others stay fixed; two sweeps at most. The cost of a
candidate is the median forward + backward time of a few steps, measured with HIP events on the
launch stream. Results are cached in a JSON file keyed by the workload class: texture side and
dtype, splat count (rounded to a power of two) and the sorted view sizes.
"""
from __future__ import annotations

import dataclasses
import json
import math
import os
from typing import Callable, Dict, Iterable, List, Optional, Sequence, Tuple

KNOBS: Dict[str, List] = {
    "tile": [(16, 16), (16, 8), (8, 8)],
    "batch": [8, 16, 32, 64],
    "batch_bwd": [8, 16, 32],
    "prefix_pairs_per_tile": [256, 512, 1024, 2048, -1],
    "tile_order": [1, -1],
}


def resolve_defaults(opts, N: int):
    """The options with the library's defaults written out (batch 0 -> 8, 16, 32 or 64,
    batch_bwd 0 -> 8 or 32, prefix budget 0 -> 1024 pairs per tile, tile order 0 -> 1), so that
    search results are explicit."""
    return dataclasses.replace(
        opts,
        batch=opts.batch or (4 if N >= 16 else 16 if N >= 8 else 32 if N >= 4 else 64),
        batch_bwd=opts.batch_bwd or (4 if N >= 16 else 8 if N >= 8 else 32),
        prefix_pairs_per_tile=opts.prefix_pairs_per_tile or 1024,
        tile_order=opts.tile_order or 1)


def workload_key(N: int, bf16: bool, P: int, view_sizes: Iterable[Tuple[int, int]]) -> str:
    p2 = 1 << max(0, int(math.ceil(math.log2(max(P, 1)))))
    sizes = ",".join(f"{w}x{h}" for w, h in sorted(view_sizes))
    return f"N{N}-{'bf16' if bf16 else 'f32'}-P{p2}-{sizes}"


def _apply(opts, knob: str, value):
    if knob == "tile":
        return dataclasses.replace(opts, tile_w=value[0], tile_h=value[1])
    return dataclasses.replace(opts, **{knob: value})


def _value(opts, knob: str):
    if knob == "tile":
        return (opts.tile_w, opts.tile_h)
    return getattr(opts, knob)


def search(base, cost: Callable[[object], float], knobs: Optional[Dict[str, List]] = None,
           sweeps: int = 2):
    """Coordinate descent over `knobs` from the options `base`. Returns (best options, best
    cost, log of (options dict, cost) for every candidate measured)."""
    knobs = knobs or KNOBS
    seen: Dict[str, float] = {}
    log = []

    def measure(o):
        key = json.dumps(dataclasses.asdict(o), sort_keys=True)
        if key not in seen:
            seen[key] = float(cost(o))
            log.append((dataclasses.asdict(o), seen[key]))
        return seen[key]

    best, best_cost = base, measure(base)
    for _ in range(sweeps):
        changed = False
        for knob, values in knobs.items():
            for v in values:
                if v == _value(best, knob):
                    continue
                cand = _apply(best, knob, v)
                c = measure(cand)
                if c < best_cost:
                    best, best_cost, changed = cand, c, True
        if not changed:
            break
    return best, best_cost, log


def gpu_cost(splats, views, steps: int = 3, warmup: int = 1) -> Callable[[object], float]:
    """Cost function: median forward + backward milliseconds of `steps` steps (HIP events on
    the launch stream, read back through the library's stage timers)."""
    import torch

    from .render import Rasterizer

    def cost(opts) -> float:
        rast = Rasterizer(views, opts, check_overflow=True)
        rast.plan(splats)
        rgb, T = rast.forward(splats)
        g = torch.ones((rast.total_pixels, 3), dtype=torch.float32, device=rgb.device)
        grads = rast.backward(splats, T, g)
        # the forward zeroes the texture gradients the backward accumulates into, as in a
        # training step
        for _ in range(warmup):
            rast.forward(splats, rgb, T, zero_grads=grads)
            rast.backward(splats, T, g, grads)
        times = []
        rast.timing(True)
        for _ in range(steps):
            rast.forward(splats, rgb, T, zero_grads=grads)
            rast.backward(splats, T, g, grads)
            times.append(sum(rast.stage_times().values()))
        rast.timing(False)
        del rast, rgb, T, g, grads
        torch.cuda.empty_cache()
        times.sort()
        return times[len(times) // 2]

    return cost


def autotune(splats, views, base=None, cache_path: Optional[str] = None,
             knobs: Optional[Dict[str, List]] = None, steps: int = 3,
             cost: Optional[Callable[[object], float]] = None):
    """Best options for this workload class, from the cache or by measuring. Returns
    (options, record) where record holds the cost of every candidate measured."""
    from .render import Options

    base = resolve_defaults(base or Options(), splats.N)
    bf16 = "bfloat16" in str(getattr(splats.textures, "dtype", ""))
    key = workload_key(splats.N, bf16, splats.P, [(v.width, v.height) for v in views])
    cache = {}
    if cache_path and os.path.exists(cache_path):
        with open(cache_path) as f:
            cache = json.load(f)
    if key in cache:
        fields = dict(cache[key]["options"])
        fields["bg"] = tuple(fields["bg"])  # JSON keeps tuples as lists
        return Options(**fields), cache[key]
    cost = cost or gpu_cost(splats, views, steps=steps)
    if knobs is None and splats.N >= 16:  # the library builds only batches of 4 for N = 16
        knobs = dict(KNOBS, batch=[4], batch_bwd=[4])
    best, best_cost, log = search(base, cost, knobs)
    record = {"options": dataclasses.asdict(best), "ms": best_cost,
              "default_ms": log[0][1], "candidates": log}
    if cache_path:
        cache[key] = record
        tmp = cache_path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(cache, f, indent=1)
        os.replace(tmp, cache_path)
    return best, record
