"""Densification and pruning on the GPU (through the C ABI) against the FP64 reference: the
screen-space gradient statistic after a backward, and plan + apply of clone, split (with
resampled colour grids) and pruning, including the optimiser rows."""
import ctypes
import math

import numpy as np
import pytest

import scenegen as sg
from oracle import gb_oracle as O
from oracle import densify_oracle as D

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gb():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2412_12734_amd as gb
    gb.load()
    return gb


def test_densify_statistic_matches_the_oracle(gb):
    """After a backward over two views, gb_densify_stats adds, per splat, the norms of the
    screen-translation gradients of the views where it is visible; the oracle takes them
    from its analytic backward."""
    from paper_2412_12734_amd import _lib as L
    scene = sg.make_scene(81, 1500, -1.0, 1.0, 0.02, 0.25, 4)
    views = [sg.look_at_view((0.2, 0.1, -2.8), 72, 56), sg.look_at_view((1.5, -0.8, -2.0), 64, 64)]
    opts = O.Options()
    g = sg.make_dl_drgb(4, views)
    acc_ref, cnt_ref = np.zeros(scene.P), np.zeros(scene.P)
    base = 0
    for v in views:
        hw = v.width * v.height
        ref = O.render(scene, v, opts, keep_saved=True)
        ok = ~O.grad_flags(ref).reshape(-1)
        g[base:base + hw] = np.where(ok[:, None], g[base:base + hw], 0.0)
        gr = O.render_backward(scene, v, opts, ref, g[base:base + hw].astype(np.float64))
        vis = O.key_stage(scene, v, opts)["count"] > 0
        acc_ref, cnt_ref = D.accumulate(acc_ref, cnt_ref, [gr.screen], [vis])
        base += hw
    sp = gb.Splats.from_numpy(scene)
    rast = gb.Rasterizer(views)
    rgb, T = rast.forward(sp)
    rast.backward(sp, T, torch.from_numpy(g).cuda())
    acc = torch.full((scene.P,), 0.5, dtype=torch.float32, device="cuda")  # accumulates
    cnt = torch.full((scene.P,), 1.0, dtype=torch.float32, device="cuda")
    L.check(rast.lib.gb_densify_stats(ctypes.byref(sp.c()), rast.cviews, rast.nv,
                                      ctypes.byref(rast.copts), rast.ws.data_ptr(),
                                      rast.ws.numel(), rast.capacity, acc.data_ptr(),
                                      cnt.data_ptr(), torch.cuda.current_stream().cuda_stream),
            "gb_densify_stats")
    torch.cuda.synchronize()
    np.testing.assert_array_equal(cnt.cpu().numpy() - 1.0, cnt_ref)
    got = acc.cpu().numpy().astype(np.float64) - 0.5
    err = np.linalg.norm(got - acc_ref) / np.linalg.norm(acc_ref)
    print(f"statistic rel L2 {err:.2e}, {int((cnt_ref > 0).sum())} visible splats")
    assert err <= 1e-3


def _raw_scene(P, N, seed, sh_coef=0):
    rng = np.random.default_rng(seed)
    means = rng.uniform(-1, 1, (P, 3)).astype(np.float32)
    quats = rng.standard_normal((P, 4)).astype(np.float32)
    log_s = np.log(rng.uniform(0.002, 0.05, (P, 2))).astype(np.float32)
    o = rng.uniform(0.0005, 0.9, P)
    logits = np.log(o / (1 - o)).astype(np.float32)
    tex = rng.uniform(0, 1, (P, N, N, 3)).astype(np.float32)
    sh = rng.normal(0, 0.2, (P, sh_coef, 3)).astype(np.float32) if sh_coef else None
    accum = rng.uniform(0, 6e-4, P).astype(np.float32)
    vis = rng.integers(0, 4, P).astype(np.float32)
    noise = rng.standard_normal((P, 2, 2)).astype(np.float32)
    return means, quats, log_s, logits, tex, sh, accum, vis, noise


def _push_off_thresholds(log_s, logits, accum, vis, opts):
    """Moves the few inputs whose decision lies within 1e-3 (relative) of a threshold out of
    that band, so that the float32 kernel and the float64 reference decide alike."""
    near = lambda a, t: np.abs(a / t - 1.0) < 1e-3
    for _ in range(4):
        s_max = np.exp(log_s.astype(np.float64).max(axis=1))
        bad = near(s_max, opts.dense_scale)
        if opts.max_scale > 0:
            bad |= near(s_max, opts.max_scale) | near(s_max / opts.split_shrink, opts.max_scale)
        log_s[bad] += np.float32(0.01)
        o = 1 / (1 + np.exp(-logits.astype(np.float64)))
        logits[near(o, opts.min_opacity)] += np.float32(0.05)
        mean = accum.astype(np.float64) / np.maximum(vis, 1)
        accum[(vis > 0) & near(mean, opts.grad_threshold)] *= np.float32(1.01)


def _margins_ok(log_s, logits, accum, vis, opts):
    """Every decision is well away from its threshold, so that float32 and float64 agree."""
    s_max = np.exp(log_s.astype(np.float64).max(axis=1))
    o = 1 / (1 + np.exp(-logits.astype(np.float64)))
    mean = np.where(vis > 0, accum.astype(np.float64) / np.maximum(vis, 1), 0.0)
    rel = lambda a, t: np.abs(a - t) / t
    m = [rel(s_max, opts.dense_scale), rel(o, opts.min_opacity),
         np.where(vis > 0, rel(mean, opts.grad_threshold), 1.0)]
    if opts.max_scale > 0:
        m += [rel(s_max, opts.max_scale), rel(s_max / opts.split_shrink, opts.max_scale)]
    return min(float(x.min()) for x in m) > 1e-4


@pytest.mark.parametrize("N,max_scale", [(4, 0.0), (8, 0.03), (1, 0.0)])
def test_densify_plan_and_apply_match_the_oracle(gb, N, max_scale):
    from paper_2412_12734_amd import _lib as L
    P = 4000
    means, quats, log_s, logits, tex, sh, accum, vis, noise = _raw_scene(P, N, 10 + N, sh_coef=4)
    opts = D.DensifyOptions(grad_threshold=2e-4, dense_scale=0.01, min_opacity=0.005,
                            max_scale=max_scale, split_shrink=1.6)
    _push_off_thresholds(log_s, logits, accum, vis, opts)
    assert _margins_ok(log_s, logits, accum, vis, opts)
    outs = D.plan(log_s, logits, accum, vis, opts)
    kinds = np.array([k for _, k in outs])
    assert {D.KEEP, D.CLONE_COPY, D.CHILD0}.issubset(set(kinds.tolist()))  # every case occurs
    assert len(outs) != P
    rng = np.random.default_rng(5)
    m_rows = rng.standard_normal((P, N, N, 3)).astype(np.float32)
    ref = D.apply(outs, means, quats, log_s, logits, tex, noise, opts, sh=sh, states=[m_rows])

    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    src_t = dict(means=dev(means), quats=dev(quats), log_scales=dev(log_s),
                 opacity_logits=dev(logits), textures=dev(tex), sh=dev(sh))
    raw = lambda t, n: L.GbRawSplats(n, N, 4, t["means"].data_ptr(), t["quats"].data_ptr(),
                                     t["log_scales"].data_ptr(), t["opacity_logits"].data_ptr(),
                                     t["textures"].data_ptr(), t["sh"].data_ptr())
    lib = L.load()
    co = L.GbDensifyOptions(opts.grad_threshold, opts.dense_scale, opts.min_opacity,
                            opts.max_scale, opts.split_shrink)
    work = torch.empty(int(lib.gb_densify_work_bytes(P)), dtype=torch.uint8, device="cuda")
    P_new = ctypes.c_int64(0)
    stream = torch.cuda.current_stream().cuda_stream
    src = raw(src_t, P)
    # keep the device copies alive for the call (a temporary's block could be handed out again)
    accum_t, vis_t = dev(accum), dev(vis)
    L.check(lib.gb_densify_plan(ctypes.byref(src), accum_t.data_ptr(), vis_t.data_ptr(),
                                ctypes.byref(co), work.data_ptr(), work.numel(),
                                ctypes.byref(P_new), stream), "gb_densify_plan")
    n = int(P_new.value)
    assert n == len(outs)
    dst_t = {k: torch.full((n,) + tuple(v.shape[1:]), -9.0, dtype=torch.float32, device="cuda")
             for k, v in src_t.items()}
    m_src, m_dst = dev(m_rows), torch.full((n, N, N, 3), -9.0, device="cuda")
    st = (L.GbRowState * 1)(L.GbRowState(m_src.data_ptr(), m_dst.data_ptr(), 3 * N * N))
    dst = raw(dst_t, n)
    noise_t = dev(noise)
    L.check(lib.gb_densify_apply(ctypes.byref(src), work.data_ptr(), noise_t.data_ptr(), 0.5,
                                 ctypes.byref(co), ctypes.byref(dst), st, 1, stream),
            "gb_densify_apply")
    torch.cuda.synchronize()
    # copied rows are bit-exact; children's centres, scales and grids are float32 arithmetic
    np.testing.assert_array_equal(dst_t["quats"].cpu().numpy(), ref["quats"].astype(np.float32))
    np.testing.assert_array_equal(dst_t["opacity_logits"].cpu().numpy(),
                                  ref["opacity_logits"].astype(np.float32))
    np.testing.assert_array_equal(dst_t["sh"].cpu().numpy(), ref["sh"].astype(np.float32))
    np.testing.assert_array_equal(m_dst.cpu().numpy(), ref["states"][0].astype(np.float32))
    np.testing.assert_allclose(dst_t["means"].cpu().numpy(), ref["means"], rtol=0, atol=2e-6)
    np.testing.assert_allclose(dst_t["log_scales"].cpu().numpy(), ref["log_scales"], rtol=0,
                               atol=2e-6)
    np.testing.assert_allclose(dst_t["textures"].cpu().numpy(), ref["textures"], rtol=0,
                               atol=2e-6)
    copies = kinds < D.CHILD0
    np.testing.assert_array_equal(dst_t["means"].cpu().numpy()[copies],
                                  ref["means"][copies].astype(np.float32))


def test_trainer_densifies_and_keeps_training(gb):
    """A few steps with the statistic tracked, one densification, more steps: the splat
    count changes, the optimiser state follows, and the rendered loss stays finite."""
    from paper_2412_12734_amd import train as TR
    raw, tgt, views, batches = sg.train_config(P=20000, n_views=4, res=(160, 120))
    targets = torch.zeros((len(views), 160 * 120, 3), dtype=torch.float32, device="cuda")
    st = TR.TrainState(raw, bf16=True)
    trainer = TR.Trainer(st, views, targets)
    trainer.track_densify(True)
    for b in batches(4):
        trainer.step(b)
    P0 = st.P
    n = trainer.densify(TR.DensifyOptions(grad_threshold=1e-6, dense_scale=0.05,
                                          min_opacity=0.3), generator=torch.Generator("cuda").manual_seed(3))
    assert n == st.P != P0 and st.params["textures"].shape[0] == n
    assert float(st.m["means"][:].abs().sum()) >= 0.0 and st.tex_bits.shape[0] == n
    for b in batches(3):
        loss = float(trainer.step(b))
    assert math.isfinite(loss)
    assert trainer.vis_count.shape[0] == n and float(trainer.vis_count.sum()) > 0
