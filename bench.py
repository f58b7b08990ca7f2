#!/usr/bin/env python3
"""Benchmark: forward + backward of the textured 2D-Gaussian rasterizer on one MI355X.

Workload (default): 1,000,000 splats with 8x8 FP32 textures (centres U[-4,4]^3, random
orientations, scales log-U[0.02,0.2], opacity U(0.05,0.95)), one 1920x1080 view at distance 8,
dL/drgb ~ N(0,1), seed 0. One step = one forward + one backward over the whole image. The
inputs are resident in device memory before the timed region starts.

Prints one JSON line: whole-job throughput in Mpixels/s (fwd+bwd), the roofline of the dominant
kernel (blend backward, measured with HIP events on its launch stream), variants (bfloat16
textures; four 1080p views in one batched call; a full optimisation step with L1 loss and Adam
over batches of four 1280x720 views) and the FP64 oracle's rate on a bounded crop of
the same workload on the host CPU.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Peaks of one MI355X (gfx950): 256 CUs x 4 SIMD16 x 2.4 GHz = 39.3 T FP32 lane-ops/s
# without packed FP32 (this build never emits packed FP32), i.e. 78.6 TFLOP/s counting an
# FMA as two flops; HBM3E 8 TB/s.
PEAK_FP32_TFLOPS = 256 * 4 * 16 * 2.4e9 * 2 / 1e12
PEAK_LANE_SLOTS_T = 256 * 4 * 16 * 2.4e9 / 1e12  # FP32 VALU issue slots, T lane-ops/s
PEAK_HBM_GBS = 8000.0

# Algorithmic FP32 flops of the blend kernels per unit of work, counted from the formulas
# (add/mul/min 1, FMA 2, rcp/exp 1; compares and integer ops not counted). The unit counts
# come from the forward's work counters.
#  forward, per evaluated (pixel, splat): offsets 2, uv solve 3x2 FMA 12, rcp 1, u and v 2,
#    q_uv 4, q_lp 4, min 1, exp with scale 2, alpha 2 = 30
#  forward, per blended (pixel, splat), in addition: T(1-alpha) 2, grid coordinates 2x6 12,
#    bilinear 9 lerps 27, weight 1, accumulation 3 FMA 6 = 48
#  backward, per blended (pixel, splat): recompute 30 + 12 + 27, T recovery 2, weight and
#    colour adjoint 4, corner weights 6, texel adjoints 12, fraction adjoints 27, uv adjoints 2,
#    alpha adjoint 15, S update 6, opacity and falloff adjoints 4, uv branch 4, rho adjoint 6,
#    dH 6, dc2 12 + 2 = 177
FLOPS_FWD_EVAL = 30
FLOPS_FWD_BLEND = 48
FLOPS_BWD_BLEND = 177

# The roofline unit of the blend backward: VALU issue slots the method needs per contributing
# (pixel, splat) pair (blended pairs plus the pair that stops each terminated pixel), about
# 200 full-rate lane-ops and 3 quarter-rate ones (4 slots each). The adjoint of Alg. 1's
# per-pixel blend and of the bilinear fetch of Alg. 2 take that many, before any reduction
# of the per-splat gradients over pixels.
SLOTS_BWD_CONTRIB = 212

# Size of the plain device-to-device copy issued once at start-up. Its FETCH_SIZE and
# WRITE_SIZE readings under rocprofv3 --pmc calibrate those counters to bytes.
COPY_BYTES = 256 << 20

# HBM traffic of one blend_bwd launch on the default workload: FETCH_SIZE and WRITE_SIZE of
# the kernel (KiB per dispatch, two rocprofv3 --pmc runs of this script), each scaled by
# COPY_BYTES over the same counter's reading for the start-up copy. It is reported only while
# the kernel's sources hash to the value they had when the counters were taken.
BWD_SOURCES = ["blend_bwd.hip", "blend_common.h", "device_util.h"]
BWD_TRAFFIC = {"sources_sha1": "e341ef8444e9d94cf8d93b6e9812f80a98f609be",
               "fetch_bytes": 979876712, "write_bytes": 305112074}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def sources_sha1(names):
    h = hashlib.sha1()
    for n in names:
        with open(os.path.join(ROOT, "paper_2412_12734_amd", "csrc", n), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def copy_probe(torch):
    """One plain device copy of COPY_BYTES (counter calibration) and its bandwidth."""
    n = COPY_BYTES // 4
    a = torch.empty(n, dtype=torch.float32, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(5):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / 5
    del a, b
    return 2 * COPY_BYTES / (ms * 1e-3) / 1e9


def assert_no_overflow(rast, what):
    """Fails the run if any forward since the previous status read overflowed its pair
    capacity (such a forward renders background and skips its stages, which would make the
    timed steps faster)."""
    K, over_last, over_any = rast.status_ex()
    if over_last or over_any:
        raise RuntimeError(f"{what}: a timed forward overflowed its pair capacity (K={K})")


def time_steps(rast, sp, rgb, T, g, grads, steps, torch):
    rast.status_ex()  # clears the sticky overflow flag of the warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        # the forward zeroes the texture gradients that the backward then accumulates into
        rast.forward(sp, rgb, T, zero_grads=grads)
        rast.backward(sp, T, g, grads)
    torch.cuda.synchronize()
    sec = (time.perf_counter() - t0) / steps
    assert_no_overflow(rast, "timed steps")
    return sec


def setup(gb, sg, torch, name, views=None, transform=None):
    scene, v = sg.config(name)
    views = views or v
    if transform is not None:
        scene = transform(scene)
    sp = gb.Splats.from_numpy(scene, tex_bf16=sg.CONFIGS[name]["bf16"])
    rast = gb.Rasterizer(views, gb.Options(), check_overflow=False)
    rast.plan(sp)
    g = torch.from_numpy(sg.make_dl_drgb(0, views)).cuda()
    rgb, T = rast.forward(sp)
    grads = rast.backward(sp, T, g)
    K, over = rast.status()
    if over:
        raise RuntimeError("pair capacity exceeded after planning")
    return scene, views, sp, rast, g, rgb, T, grads, K


def train_variant(gb, sg, torch, warmup=20, iters=200):
    """Full optimisation step: activations, render of a batch of 4 of 32 views, L1 loss,
    backward through the rasterizer and the activations, Adam on every parameter group with
    the bfloat16 texture copy rewritten. Per-iteration durations from HIP events on the
    launch stream; the targets are the perturbed scene rendered once by the FP32 path."""
    from paper_2412_12734_amd import train as TR
    raw, tgt, views, batches = sg.train_config()
    hw = views[0].width * views[0].height
    targets = torch.empty((len(views), hw, 3), dtype=torch.float32, device="cuda")
    tst = TR.TrainState(tgt, bf16=False)
    sp_t = tst.activate()
    rt = gb.Rasterizer(views[:4])
    for i in range(0, len(views), 4):
        rt.set_views(views[i:i + 4])
        rgb_t, _ = rt.forward(sp_t)
        targets[i:i + 4].copy_(rgb_t.view(4, hw, 3))
    del rt, tst, sp_t, rgb_t
    st = TR.TrainState(raw, bf16=True)
    trainer = TR.Trainer(st, views, targets)
    sched = batches(warmup + iters)
    cap = trainer.plan(sched)
    for b in sched[:warmup]:
        trainer.step(b)
    trainer.overflowed()  # clears the sticky overflow flag of the warm-up
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(iters + 1)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev[0].record()
    for i, b in enumerate(sched[warmup:]):
        trainer.step(b)
        ev[i + 1].record()
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / iters
    ms = sorted(ev[i].elapsed_time(ev[i + 1]) for i in range(iters))
    q = lambda f: ms[min(iters - 1, int(round(f * (iters - 1))))]
    loss = float(trainer.loss)
    over = trainer.overflowed()  # any of the timed steps
    if over:
        raise RuntimeError("training step: a timed step overflowed its pair capacity")
    n_par = sum(t.numel() for t in st.params.values())
    out = {"ms_per_iter_median": round(q(0.5), 3), "ms_per_iter_p10": round(q(0.1), 3),
           "ms_per_iter_p90": round(q(0.9), 3), "ms_per_iter_wall": round(wall * 1e3, 3),
           "iters": iters, "warmup": warmup, "parameters": n_par, "pair_capacity": cap,
           "final_l1": round(loss, 6), "overflow_any_timed_step": over,
           "workload": "500k splats, 8x8 BF16 textures (FP32 master), batch of 4 of 32 "
                       "1280x720 views, L1 + Adam"}
    del trainer, st, targets
    torch.cuda.empty_cache()
    return out


def image_fit_variant(gb, sg, torch, P, N, warmup=10, iters=100):
    """Single-image fitting (Sec. 4): P splats with N x N FP32 colour grids in the plane of a
    1920 x 871 synthetic image (the size of the paper's first test image), rotation about Z
    only, MSE loss, Adam. Per-iteration durations from HIP events on the launch stream."""
    from paper_2412_12734_amd import train as TR
    raw, view, target = sg.image_fit_config(0, P, 1920, 871, N)
    st = TR.TrainState(raw, bf16=False, rotz_only=True)
    trainer = TR.Trainer(st, [view], torch.from_numpy(target).cuda().view(1, -1, 3), loss="mse")
    sched = [[0]] * (warmup + iters)
    trainer.plan(sched[:1], headroom=2.0)
    first = float(trainer.step([0]))
    for b in sched[1:warmup]:
        trainer.step(b)
    trainer.overflowed()  # clears the sticky overflow flag of the warm-up
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(iters + 1)]
    torch.cuda.synchronize()
    ev[0].record()
    for i, b in enumerate(sched[warmup:]):
        trainer.step(b)
        ev[i + 1].record()
    torch.cuda.synchronize()
    ms = sorted(ev[i].elapsed_time(ev[i + 1]) for i in range(iters))
    out = {"ms_per_iter_median": round(ms[iters // 2], 3), "iters": iters, "warmup": warmup,
           "mse_first": round(first, 6), "mse_last": round(float(trainer.loss), 6),
           "overflow_any_timed_step": trainer.overflowed(),
           "workload": f"{P} splats, {N}x{N} FP32 grids, 1920x871 synthetic image, MSE, "
                       "rotation about Z, Adam"}
    del trainer, st
    torch.cuda.empty_cache()
    return out


def c3_variant(gb, sg, torch, warmup, steps):
    """1M splats with 4x4 FP32 textures, 16 views of uneven size on a radius-8 sphere: forward
    + backward of all views as one batched step replayed from a HIP graph, against the same
    views rendered one view per call (16 rasterizers, launched back to back)."""
    scene, views = sg.config("C3")
    sp = gb.Splats.from_numpy(scene)
    g = torch.from_numpy(sg.make_dl_drgb(0, views)).cuda()
    px = sum(v.width * v.height for v in views)
    rast = gb.Rasterizer(views, gb.Options(), check_overflow=False)
    rast.plan(sp)
    rgb, T = rast.forward(sp)
    grads = rast.backward(sp, T, g)
    K, over = rast.status()
    if over:
        raise RuntimeError("pair capacity exceeded after planning")
    graph = rast.capture_step(sp, rgb, T, g, grads)
    for _ in range(warmup):
        graph.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        graph.replay()
    torch.cuda.synchronize()
    s_batch = (time.perf_counter() - t0) / steps
    assert_no_overflow(rast, "C3 graph replays")
    del graph, rast
    torch.cuda.empty_cache()
    singles, at = [], 0
    for v in views:  # one rasterizer per view; the gradient buffers are shared (overwritten)
        r = gb.Rasterizer([v], gb.Options(), check_overflow=False)
        r.plan(sp)
        hw = v.width * v.height
        singles.append((r, rgb[at:at + hw], T[at:at + hw], g[at:at + hw]))
        at += hw

    def single_step():
        for r, rgb_i, T_i, g_i in singles:
            r.forward(sp, rgb_i, T_i, zero_grads=grads)
            r.backward(sp, T_i, g_i, grads)

    for _ in range(warmup):
        single_step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        single_step()
    torch.cuda.synchronize()
    s_single = (time.perf_counter() - t0) / steps
    del singles, grads, rgb, T, g, sp
    torch.cuda.empty_cache()
    return {"batched_graph_ms": round(s_batch * 1e3, 3),
            "single_view_calls_ms": round(s_single * 1e3, 3),
            "speedup_batched": round(s_single / s_batch, 3),
            "mpix_per_s_batched": round(px / s_batch / 1e6, 1), "pixels": px, "pairs": K}


CONFIG_PASSES = (("C1", False), ("C2", True), ("C4", True))


def config_times(gb, sg, torch, warmup, steps, only=None):
    """Step times of the smaller named workloads (their parity is checked by the tests):
    1k splats at 128x128 forward only, 100k splats at 800x800 forward + backward, 3M splats
    with bfloat16 textures at 4 x 1080p forward + backward. ``only`` names one of them; its
    entry then also holds the per-stage times (HIP events) of one further step."""
    out = {}
    for name, bwd in CONFIG_PASSES:
        if only is not None and name != only:
            continue
        scene, views, sp, rast, g, rgb, T, grads, K = setup(gb, sg, torch, name)
        px = sum(v.width * v.height for v in views)
        for _ in range(warmup):
            rast.forward(sp, rgb, T, zero_grads=grads if bwd else None)
            if bwd:
                rast.backward(sp, T, g, grads)
        rast.status_ex()  # clears the sticky overflow flag of the warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            rast.forward(sp, rgb, T, zero_grads=grads if bwd else None)
            if bwd:
                rast.backward(sp, T, g, grads)
        torch.cuda.synchronize()
        sec = (time.perf_counter() - t0) / steps
        assert_no_overflow(rast, name)
        out[name] = {"ms_per_step": round(sec * 1e3, 3), "mpix_per_s": round(px / sec / 1e6, 1),
                     "pass": "fwd+bwd" if bwd else "fwd", "splats": scene.P, "pixels": px,
                     "pairs": K}
        if only is not None:
            rast.timing(True)
            rast.forward(sp, rgb, T, zero_grads=grads if bwd else None)
            if bwd:
                rast.backward(sp, T, g, grads)
            out[name]["stage_ms"] = {k: round(v, 4) for k, v in rast.stage_times().items()}
            rast.timing(False)
        del scene, sp, rast, g, rgb, T, grads
        torch.cuda.empty_cache()
    return out


def cpu_baseline(scene, view, crop):
    """FP64 oracle (one process) on a crop of the workload: forward + analytic backward."""
    import numpy as np
    from oracle import gb_oracle as O
    from threadpoolctl import threadpool_limits
    with threadpool_limits(limits=1):  # one core: BLAS and OpenMP pools held to one thread
        t0 = time.perf_counter()
        r = O.render(scene, view, O.Options(), crop=crop, keep_saved=True)
        g = np.random.default_rng(0).standard_normal((crop[2] * crop[3], 3))
        O.render_backward(scene, view, O.Options(), r, g)
        dt = time.perf_counter() - t0
    return crop[2] * crop[3] / dt / 1e6, dt


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-variants", action="store_true")
    ap.add_argument("--train-iters", type=int, default=200)
    ap.add_argument("--train-only", action="store_true",
                    help="time only the optimisation-step variant (for kernel traces of it)")
    ap.add_argument("--image-fit-only", action="store_true",
                    help="time only the 100k-splat single-image fitting variant")
    ap.add_argument("--config-only", choices=[n for n, _ in CONFIG_PASSES],
                    help="time only this named workload (for kernel traces of it)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); the rasterizer has no "
              "multi-GPU path in this build", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2412_12734_amd as gb
    import scenegen as sg

    gb.load()
    if args.train_only:
        tr = train_variant(gb, sg, torch, warmup=args.warmup, iters=args.train_iters)
        print(json.dumps({"train_step_500k_4x720p": tr}), flush=True)
        return
    if args.image_fit_only:
        fit = image_fit_variant(gb, sg, torch, 100_000, 4, warmup=args.warmup,
                                iters=args.train_iters)
        print(json.dumps({"image_fit_100k": fit}), flush=True)
        return
    if args.config_only:
        out = config_times(gb, sg, torch, args.warmup, args.steps, only=args.config_only)
        print(json.dumps(out), flush=True)
        return
    copy_gbs = copy_probe(torch)
    log(f"plain device copy of {COPY_BYTES >> 20} MiB: {copy_gbs:.0f} GB/s (read + write)")
    log("setting up T0 (1M splats, 8x8 FP32 textures, 1920x1080)")
    scene, views, sp, rast, g, rgb, T, grads, K = setup(gb, sg, torch, "T0")
    pixels = sum(v.width * v.height for v in views)
    for _ in range(args.warmup):
        rast.forward(sp, rgb, T, zero_grads=grads)
        rast.backward(sp, T, g, grads)
    sec = time_steps(rast, sp, rgb, T, g, grads, args.steps, torch)
    value = pixels / sec / 1e6
    log(f"T0 fp32: {sec * 1e3:.3f} ms/step, {value:.1f} Mpx/s, K={K}")

    # the same step captured once into a HIP graph and replayed
    graph = rast.capture_step(sp, rgb, T, g, grads)
    for _ in range(args.warmup):
        graph.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        graph.replay()
    torch.cuda.synchronize()
    sec_graph = (time.perf_counter() - t0) / args.steps
    assert_no_overflow(rast, "graph replays")
    del graph
    log(f"T0 fp32, HIP graph replay: {sec_graph * 1e3:.3f} ms/step")

    # per-stage durations from HIP events recorded on the launch stream
    stage_sum = {}
    rast.timing(True)
    for _ in range(args.steps):
        rast.forward(sp, rgb, T, zero_grads=grads)
        rast.backward(sp, T, g, grads)
        for k, v in rast.stage_times().items():
            stage_sum[k] = stage_sum.get(k, 0.0) + v
    rast.timing(False)
    stages = {k: v / args.steps for k, v in stage_sum.items()}
    log("stages (ms): " + ", ".join(f"{k}={v:.3f}" for k, v in stages.items()))

    st = rast.blend_stats(sp, rgb, T)
    # tiling overhead: pixel slots of the staged (tile, splat) pairs over the (pixel, splat)
    # pairs the method needs (blended ones plus the one that stops each terminated pixel)
    tile_px = rast.opts.tile_w * rast.opts.tile_h
    st["e_contrib"] = st["blended"] + st["terminated"]
    st["e_tile"] = st["staged"] * tile_px
    st["tiling_overhead"] = round(st["e_tile"] / max(st["e_contrib"], 1), 3)
    # the dominant kernel is the blend backward: one launch walks the pairs of both passes of
    # the depth-prefix split, so its units are all blended pairs
    e_eval, e_blend = st["lane_evals"], st["blended"]
    e_blend_bwd = e_blend
    bwd_ms = stages["blend_bwd"]
    fwd_ms = stages["blend_fwd"] + stages.get("blend_fwd_rest", 0.0)
    bwd_flops = e_blend_bwd * FLOPS_BWD_BLEND
    fwd_flops = e_eval * FLOPS_FWD_EVAL + e_blend * FLOPS_FWD_BLEND
    achieved_tf = bwd_flops / (bwd_ms * 1e-3) / 1e12
    # issue slots the method needs over the launch's contributing pairs, per second
    achieved = st["e_contrib"] * SLOTS_BWD_CONTRIB / (bwd_ms * 1e-3) / 1e12
    traffic = None
    if BWD_TRAFFIC and BWD_TRAFFIC["sources_sha1"] == sources_sha1(BWD_SOURCES):
        traffic = BWD_TRAFFIC["fetch_bytes"] + BWD_TRAFFIC["write_bytes"]
    roofline = {"bound": "alu", "kernel": "blend_bwd", "achieved": round(achieved, 3),
                "peak": round(PEAK_LANE_SLOTS_T, 2), "unit": "T VALU lane-slots/s",
                "frac": round(achieved / PEAK_LANE_SLOTS_T, 4), "traffic": traffic,
                "units_per_launch": {"contributing_pairs": st["e_contrib"]},
                "slots_per_unit": SLOTS_BWD_CONTRIB, "avg_ms": round(bwd_ms, 4),
                "flops": {"achieved_tflops": round(achieved_tf, 3),
                          "peak_tflops": round(PEAK_FP32_TFLOPS, 1),
                          "frac": round(achieved_tf / PEAK_FP32_TFLOPS, 4),
                          "flops_per_blended_pair": FLOPS_BWD_BLEND,
                          "blended_pairs": e_blend_bwd}}
    fwd_tf = fwd_flops / (fwd_ms * 1e-3) / 1e12

    variants = {}
    if not args.no_variants:
        del rast
        torch.cuda.empty_cache()
        log("variant: bf16 textures, one view")
        _, views_b, sp_b, rast_b, g_b, rgb_b, T_b, grads_b, _ = setup(gb, sg, torch, "T0_BF16")
        for _ in range(args.warmup):
            rast_b.forward(sp_b, rgb_b, T_b, zero_grads=grads_b)
            rast_b.backward(sp_b, T_b, g_b, grads_b)
        s_b = time_steps(rast_b, sp_b, rgb_b, T_b, g_b, grads_b, args.steps, torch)
        # storage error of bfloat16 textures: the same scene rendered from FP32 textures
        rgb_b, T_b = rast_b.forward(sp_b, rgb_b, T_b)
        grads_b = rast_b.backward(sp_b, T_b, g_b, grads_b)
        d_img = (rgb_b - rgb).abs()
        rel = lambda a, b: float((a - b).double().norm() / b.double().norm().clamp_min(1e-30))
        variants["bf16_single_view"] = {
            "ms_per_step": round(s_b * 1e3, 3), "mpix_per_s": round(pixels / s_b / 1e6, 1),
            "storage_error_vs_fp32_textures": {
                "image_max_abs": float(d_img.max()), "image_rms": float(d_img.pow(2).mean().sqrt()),
                "grad_rel_l2": {k: round(rel(grads_b[k], grads[k]), 7) for k in grads}}}
        del rast_b
        torch.cuda.empty_cache()
        log("variant: 16 x 16 colour grids, one view")
        _, _, sp_16, rast_16, g_16, rgb_16, T_16, grads_16, _ = setup(gb, sg, torch, "T0_N16")
        for _ in range(args.warmup):
            rast_16.forward(sp_16, rgb_16, T_16, zero_grads=grads_16)
            rast_16.backward(sp_16, T_16, g_16, grads_16)
        s_16 = time_steps(rast_16, sp_16, rgb_16, T_16, g_16, grads_16, args.steps, torch)
        variants["n16_single_view"] = {"ms_per_step": round(s_16 * 1e3, 3),
                                       "mpix_per_s": round(pixels / s_16 / 1e6, 1),
                                       "texels_per_splat": 256}
        del rast_16, sp_16, rgb_16, T_16, grads_16, g_16
        torch.cuda.empty_cache()
        for label, sides in (("mixed_sides_2_4_8_single_view", (2, 4, 8)),
                             ("mixed_sides_4_8_16_single_view", (4, 8, 16))):
            log(f"variant: colour grids of sides {sides} in one call, one view")
            _, _, sp_m, rast_m, g_m, rgb_m, T_m, grads_m, _ = setup(
                gb, sg, torch, "T0", transform=lambda sc: sg.with_mixed_sides(sc, 1, sides))
            for _ in range(args.warmup):
                rast_m.forward(sp_m, rgb_m, T_m, zero_grads=grads_m)
                rast_m.backward(sp_m, T_m, g_m, grads_m)
            s_m = time_steps(rast_m, sp_m, rgb_m, T_m, g_m, grads_m, args.steps, torch)
            variants[label] = {"ms_per_step": round(s_m * 1e3, 3),
                               "mpix_per_s": round(pixels / s_m / 1e6, 1),
                               "layout_side": sp_m.N, "texels": sp_m.n_texels}
            del rast_m, sp_m, rgb_m, T_m, grads_m, g_m
            torch.cuda.empty_cache()
        log("variant: bf16 textures, four 1080p views batched in one call")
        views4 = sg.orbit_views(0, 4, 8.0, [(1920, 1080)])
        _, _, sp4, rast4, g4, rgb4, T4, grads4, K4 = setup(gb, sg, torch, "T0_BF16", views=views4)
        for _ in range(args.warmup):
            rast4.forward(sp4, rgb4, T4, zero_grads=grads4)
            rast4.backward(sp4, T4, g4, grads4)
        s_4 = time_steps(rast4, sp4, rgb4, T4, g4, grads4, args.steps, torch)
        px4 = 4 * 1920 * 1080
        variants["bf16_batched_4x1080p"] = {"ms_per_step": round(s_4 * 1e3, 3),
                                            "mpix_per_s": round(px4 / s_4 / 1e6, 1),
                                            "pairs": K4}
        variants["speedup_bf16_batched_vs_fp32_single"] = round((px4 / s_4) / (pixels / sec), 3)
        del rast4, rgb4, T4, grads4
        torch.cuda.empty_cache()
        log("variant: the same, with autotuned tile shape, batch sizes and prefix budget")
        from paper_2412_12734_amd import autotune as at
        opts_t, rec = at.autotune(sp4, views4, steps=3)
        rast_t = gb.Rasterizer(views4, opts_t, check_overflow=False)
        rast_t.plan(sp4)
        rgb_t, T_t = rast_t.forward(sp4)
        grads_t = rast_t.backward(sp4, T_t, g4)
        for _ in range(args.warmup):
            rast_t.forward(sp4, rgb_t, T_t, zero_grads=grads_t)
            rast_t.backward(sp4, T_t, g4, grads_t)
        s_t = time_steps(rast_t, sp4, rgb_t, T_t, g4, grads_t, args.steps, torch)
        variants["bf16_batched_4x1080p_autotuned"] = {
            "ms_per_step": round(s_t * 1e3, 3), "mpix_per_s": round(px4 / s_t / 1e6, 1),
            "options": {k: v for k, v in rec["options"].items()
                        if k in ("tile_w", "tile_h", "batch", "batch_bwd",
                                 "prefix_pairs_per_tile")},
            "candidates_timed": len(rec["candidates"])}
        variants["speedup_autotuned_bf16_batched_vs_fp32_single"] = round(
            (px4 / s_t) / (pixels / sec), 3)
        del rast_t, rgb_t, T_t, grads_t, sp4, g4
        torch.cuda.empty_cache()
        log("variant: 16 uneven views (1M splats, 4x4 textures) in one graph vs one at a time")
        variants["c3_16_views"] = c3_variant(gb, sg, torch, args.warmup, args.steps)
        log(f"c3: {variants['c3_16_views']}")
        log("variant: the smaller named workloads (1k, 100k and 3M splats)")
        variants["configs"] = config_times(gb, sg, torch, args.warmup, args.steps)
        log(f"configs: {variants['configs']}")
        log("variant: full optimisation step (500k splats, batch of 4 of 32 views at 1280x720)")
        variants["train_step_500k_4x720p"] = train_variant(gb, sg, torch,
                                                           iters=args.train_iters)
        log(f"train step: {variants['train_step_500k_4x720p']}")
        for P in (10_000, 100_000):
            log(f"variant: single-image fitting, {P} splats, 4x4 grids, 1920x871")
            variants[f"image_fit_{P // 1000}k"] = image_fit_variant(gb, sg, torch, P, 4)
            log(f"image fit: {variants[f'image_fit_{P // 1000}k']}")

    cpu = None
    if not args.no_cpu_baseline:
        crop = (832, 412, 256, 256)
        log("cpu baseline: FP64 oracle on a 256x256 centre crop (fwd + bwd)")
        mpx, dt = cpu_baseline(scene, views[0], crop)
        cpu = {"value": round(mpx, 6), "unit": "Mpixels/s", "cores": 1, "kind": "oracle",
               "sample": "256x256 centre crop of the 1920x1080 view, forward + analytic "
                         f"backward, one process ({dt:.1f} s)"}

    out = {
        "metric": "fwd+bwd Mpixels/s & ms/iter at 1M textured splats, 1080p; batched BF16 vs FP32",
        "value": round(value, 2), "unit": "Mpixels/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(sec * 1e3, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "T0: 1M splats, 8x8 FP32 textures, one 1920x1080 view, fwd+bwd",
                   "pixels": pixels, "pairs": K, "parallelism": "single GPU"},
        "roofline": roofline,
        "stage_ms": {k: round(v, 4) for k, v in stages.items()},
        "blend_fwd_tflops": round(fwd_tf, 3),
        "hbm_copy_gbs": round(copy_gbs, 1),
        "graph_replay_ms_per_step": round(sec_graph * 1e3, 3),
        "work": st,
        "variants": variants,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
