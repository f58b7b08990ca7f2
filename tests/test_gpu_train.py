"""GPU parity of the training glue (activations, L1 loss, Adam, bfloat16 copies) against the
FP64 oracle, and of the raw-parameter gradients of a render + L1 loss."""
import numpy as np
import pytest

import scenegen as sg
from oracle import gb_oracle as O
from oracle import train_oracle as TO

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gb():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2412_12734_amd as gb
    gb.load()  # fails loudly if the HIP library is missing
    return gb


def cuda(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def rel(a, b):
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30))


def test_activations_match_the_oracle(gb):
    from paper_2412_12734_amd import _lib as L
    lib = L.load()
    rng = np.random.default_rng(11)
    P = 3001
    q = rng.standard_normal((P, 4)) * rng.uniform(0.2, 3.0, (P, 1))
    ls, ol = rng.uniform(-5, 0, (P, 2)), rng.normal(0, 3, P)
    gq, gls, gol = cuda(q), cuda(ls), cuda(ol)
    out = [torch.empty(s, device="cuda") for s in ((P, 3), (P, 3), (P, 2), (P,))]
    assert lib.gb_activate_fwd(P, gq.data_ptr(), gls.data_ptr(), gol.data_ptr(),
                               *[t.data_ptr() for t in out], None) == 0
    want = TO.activate(q.astype(np.float32), ls.astype(np.float32), ol.astype(np.float32))
    # tangent entries have magnitude <= 1 and pass through about eight float32 roundings
    # (square root, division, the four products and two sums scaled by 2): 8 units of 2^-24
    for got, w in zip(out[:2], want[:2]):
        np.testing.assert_allclose(got.cpu().numpy(), w, rtol=0, atol=8 * 2.0 ** -24)
    for got, w in zip(out[2:], want[2:]):
        np.testing.assert_allclose(got.cpu().numpy(), w, rtol=2e-6, atol=0)
    adj = [rng.standard_normal(s) for s in ((P, 3), (P, 3), (P, 2), (P,))]
    gadj = [cuda(a) for a in adj]
    dq, dls, dol = torch.empty(P, 4, device="cuda"), torch.empty(P, 2, device="cuda"), \
        torch.empty(P, device="cuda")
    assert lib.gb_activate_bwd(P, gq.data_ptr(), gls.data_ptr(), gol.data_ptr(),
                               *[t.data_ptr() for t in gadj], dq.data_ptr(), dls.data_ptr(),
                               dol.data_ptr(), None) == 0
    wq, wls, wol = TO.activate_backward(q.astype(np.float32), ls.astype(np.float32),
                                        ol.astype(np.float32), *[a.astype(np.float32) for a in adj])
    assert rel(dq.cpu().numpy(), wq) < 1e-5
    assert rel(dls.cpu().numpy(), wls) < 1e-6
    assert rel(dol.cpu().numpy(), wol) < 1e-6


@pytest.mark.parametrize("n", [1, 7, 4096, 100003])
def test_l1_loss_matches_the_oracle(gb, n):
    from paper_2412_12734_amd import train as T
    rng = np.random.default_rng(n)
    a, b = rng.uniform(0, 1, n).astype(np.float32), rng.uniform(0, 1, n).astype(np.float32)
    b[::5] = a[::5]  # exact ties give a zero gradient
    loss = torch.zeros(1, device="cuda")
    d = torch.empty(n, device="cuda")
    T.l1_loss(cuda(a), cuda(b), 1.0 / n, loss, d)
    wl, wd = TO.l1_loss(a, b, np.float32(1.0 / n))
    assert float(loss) == pytest.approx(wl, rel=1e-5)
    np.testing.assert_array_equal(d.cpu().numpy(), wd.astype(np.float32))


@pytest.mark.parametrize("n", [5, 4099, 200000])
def test_adam_and_bf16_copy_match_the_oracle(gb, n):
    from paper_2412_12734_amd import _lib as L
    lib = L.load()
    rng = np.random.default_rng(n + 1)
    theta = rng.standard_normal(n).astype(np.float32)
    m, v, m_mag = np.zeros(n), np.zeros(n), np.zeros(n)
    gt, gm, gv = cuda(theta), cuda(m), cuda(v)
    bits = torch.empty(n + 4, dtype=torch.int16, device="cuda")
    want = theta.astype(np.float64)
    # the entry point takes float32 hyperparameters: the oracle gets exactly those values
    lr, b1, b2, eps = (float(np.float32(x)) for x in (1e-2, 0.9, 0.999, 1e-15))
    for step in range(1, 4):
        g = (rng.standard_normal(n) * 10.0 ** rng.uniform(-3, 1, n)).astype(np.float32)
        assert lib.gb_adam_step(n, gt.data_ptr(), cuda(g).data_ptr(), gm.data_ptr(),
                                gv.data_ptr(), step, lr, b1, b2, eps, bits.data_ptr(),
                                None) == 0
        want, m, v = TO.adam_step(want, g, m, v, step, lr, b1, b2, eps)
        # m can cancel (gradients of opposite signs): its float32 error scales with the
        # magnitudes that were summed, not with |m|; v sums non-negative terms only
        m_mag = b1 * m_mag + (1.0 - b1) * np.abs(g)
        got = gt.cpu().numpy()
        # each step moves a parameter by at most about lr; compare the movement
        np.testing.assert_allclose(got - theta, want - theta, rtol=0, atol=2e-6)
        assert np.all(np.abs(gm.cpu().numpy() - m) <= 1e-6 * m_mag)
        np.testing.assert_allclose(gv.cpu().numpy(), v, rtol=1e-5, atol=1e-12)
        # the bfloat16 copy: nearest-even rounding of the GPU's own float32 result
        np.testing.assert_array_equal(bits[:n].cpu().numpy().view(np.uint16),
                                      TO.bf16_round(got))


def test_to_bf16_is_nearest_even(gb):
    from paper_2412_12734_amd import _lib as L
    lib = L.load()
    rng = np.random.default_rng(3)
    x = np.concatenate([rng.standard_normal(10000) * 10.0 ** rng.uniform(-30, 30, 10000),
                        [1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, -0.0, 0.0]]).astype(np.float32)
    out = torch.empty(x.size, dtype=torch.int16, device="cuda")
    assert lib.gb_to_bf16(x.size, cuda(x).data_ptr(), out.data_ptr(), None) == 0
    np.testing.assert_array_equal(out.cpu().numpy().view(np.uint16), TO.bf16_round(x))


def test_raw_parameter_gradients_of_render_and_l1(gb):
    from paper_2412_12734_amd import train as T
    raw = sg.make_raw_scene(17, 400, -1.0, 1.0, 0.05, 0.3, 4)
    view = sg.look_at_view((0.0, 0.0, -3.0), 64, 48)
    n_px = 64 * 48
    # a target that no rendered colour (always in [0, 1]) comes near: every sign is certain
    chk = ((np.arange(n_px)[:, None] + np.arange(3)[None, :]) % 2).astype(np.float32)
    target = np.where(chk > 0, 2.0, -1.0).astype(np.float32)
    scale = 1.0 / (3 * n_px)
    # GPU: activate, render, L1, backward through the rasterizer and the activations
    st = T.TrainState(raw, bf16=False)
    sp = st.activate()
    rast = gb.Rasterizer([view])
    rast.plan(sp)
    rgb, Tf = rast.forward(sp)
    loss = torch.zeros(1, device="cuda")
    d_rgb = torch.empty_like(rgb)
    T.l1_loss(rgb, cuda(target), scale, loss, d_rgb)
    # oracle: the same chain in float64 from the raw parameters
    t_u, t_v, s, o = TO.activate(raw.quats, raw.log_scales, raw.opacity_logits)
    scene = sg.Scene(raw.means, t_u.astype(np.float32), t_v.astype(np.float32),
                     s.astype(np.float32), o.astype(np.float32), raw.textures)
    ref = O.render(scene, view, O.Options(), keep_saved=True)
    wl, wd = TO.l1_loss(ref.rgb.reshape(-1, 3), target, scale)
    assert float(loss) == pytest.approx(wl, rel=1e-5)
    keep = ~O.grad_flags(ref).reshape(-1)
    d_rgb[torch.from_numpy(~keep).cuda()] = 0.0
    grads = rast.backward(sp, Tf, d_rgb)
    raw_g = st.backward_activations(grads)
    ref_g = O.render_backward(scene, view, O.Options(), ref, np.where(keep[:, None], wd, 0.0))
    wq, wls, wol = TO.activate_backward(raw.quats, raw.log_scales, raw.opacity_logits,
                                        ref_g.tan_u, ref_g.tan_v, ref_g.scales, ref_g.opacity)
    for name, want in (("means", ref_g.means), ("textures", ref_g.textures), ("quats", wq),
                       ("log_scales", wls), ("opacity_logits", wol)):
        err = rel(raw_g[name].cpu().numpy(), want)
        assert err <= 1e-3, (name, err)


def test_trainer_steps_run_and_move_the_parameters(gb):
    from paper_2412_12734_amd import train as T
    raw, tgt, views, batches = sg.train_config(P=3000, n_views=8, res=(96, 64))
    # targets: the perturbed scene rendered by the library
    tst = T.TrainState(tgt, bf16=False)
    rast = gb.Rasterizer(views)
    rgb, _ = rast.forward(tst.activate())
    targets = rgb.view(len(views), -1, 3).clone()
    st = T.TrainState(raw, bf16=True)
    before = {k: v.clone() for k, v in st.params.items()}
    trainer = T.Trainer(st, views, targets)
    losses = [float(trainer.step(b)) for b in batches(6)]
    assert all(np.isfinite(losses)) and st.step_count == 6
    for k in before:
        assert not torch.equal(before[k], st.params[k]), k
    # the bfloat16 render copy follows the float32 master textures
    np.testing.assert_array_equal(
        st.tex_bits.cpu().numpy().view(np.uint16).reshape(-1),
        TO.bf16_round(st.params["textures"].cpu().numpy().reshape(-1)))


def test_planned_trainer_matches_the_checked_one(gb):
    """Trainer.plan sizes the capacity up front and drops the per-step host check; the
    losses must follow those of the trainer that checks (and re-plans) every step."""
    from paper_2412_12734_amd import train as T
    raw, tgt, views, batches = sg.train_config(seed=2, P=4000, n_views=8, res=(80, 48))
    tst = T.TrainState(tgt, bf16=False)
    rast = gb.Rasterizer(views)
    targets = rast.forward(tst.activate())[0].view(len(views), -1, 3).clone()
    sched = batches(5)
    runs = []
    for planned in (False, True):
        tr = T.Trainer(T.TrainState(raw, bf16=True), views, targets)
        if planned:
            assert tr.plan(sched) > 0 and not tr.rast.check_overflow
        runs.append([float(tr.step(b)) for b in sched])
        assert not tr.overflowed()
    np.testing.assert_allclose(runs[1], runs[0], rtol=1e-5)


# --- single-image fitting set-up (Sec. 4): MSE loss, box-filtered grids, rotation about z ---
@pytest.mark.parametrize("n", [1, 7, 4096, 100003])
def test_mse_loss_matches_the_oracle(gb, n):
    from paper_2412_12734_amd import train as T
    rng = np.random.default_rng(n + 7)
    a, b = rng.uniform(0, 1, n).astype(np.float32), rng.uniform(0, 1, n).astype(np.float32)
    loss = torch.zeros(1, device="cuda")
    d = torch.empty(n, device="cuda")
    T.mse_loss(cuda(a), cuda(b), 1.0 / n, loss, d)
    wl, wd = TO.mse_loss(a, b, np.float32(1.0 / n))
    assert float(loss) == pytest.approx(wl, rel=1e-5)
    # d = 2 scale (a - b): two float32 roundings (the difference, the product)
    np.testing.assert_allclose(d.cpu().numpy(), wd, rtol=3 * 2.0 ** -24, atol=1e-30)


@pytest.mark.parametrize("N,M", [(8, 2), (8, 1), (4, 4), (16, 4), (2, 1)])
def test_box_filter_matches_the_oracle(gb, N, M):
    from paper_2412_12734_amd import train as T
    rng = np.random.default_rng(N * 10 + M)
    tex = rng.uniform(0, 1, (1001, N, N, 3)).astype(np.float32)
    got = T.box_filter_textures(cuda(tex), M).cpu().numpy()
    want = TO.box_filter(tex, M)
    k = N // M
    # k^2 float32 additions of values in [0, 1], then an exact scaling by 1 / k^2
    np.testing.assert_allclose(got, want, rtol=0, atol=k * k * 2.0 ** -24)


def test_image_fit_gradients_with_mse_and_rotation_about_z(gb):
    from paper_2412_12734_amd import train as T
    raw, view, target = sg.image_fit_config(21, 600, 80, 56, 4)
    n_px = view.width * view.height
    scale = 1.0 / (3 * n_px)
    st = T.TrainState(raw, bf16=False, rotz_only=True)
    sp = st.activate()
    rast = gb.Rasterizer([view])
    rast.plan(sp)
    rgb, Tf = rast.forward(sp)
    loss = torch.zeros(1, device="cuda")
    d_rgb = torch.empty_like(rgb)
    T.mse_loss(rgb, cuda(target), scale, loss, d_rgb)
    t_u, t_v, s, o = TO.activate(raw.quats, raw.log_scales, raw.opacity_logits)
    scene = sg.Scene(raw.means, t_u.astype(np.float32), t_v.astype(np.float32),
                     s.astype(np.float32), o.astype(np.float32), raw.textures)
    ref = O.render(scene, view, O.Options(), keep_saved=True)
    wl, wd = TO.mse_loss(ref.rgb.reshape(-1, 3), target, scale)
    assert float(loss) == pytest.approx(wl, rel=1e-4)
    keep = ~O.grad_flags(ref).reshape(-1)
    # both sides take the oracle's pixel adjoint, so that the comparison is of the chain
    d_rgb.copy_(cuda(np.where(keep[:, None], wd, 0.0)))
    raw_g = st.backward_activations(rast.backward(sp, Tf, d_rgb))
    ref_g = O.render_backward(scene, view, O.Options(), ref, np.where(keep[:, None], wd, 0.0))
    wq, wls, wol = TO.activate_backward(raw.quats, raw.log_scales, raw.opacity_logits,
                                        ref_g.tan_u, ref_g.tan_v, ref_g.scales, ref_g.opacity)
    wq = TO.rotz_only(wq)
    got_q = raw_g["quats"].cpu().numpy()
    assert np.all(got_q[:, 1:3] == 0.0)
    for name, want in (("means", ref_g.means), ("textures", ref_g.textures), ("quats", wq),
                       ("log_scales", wls), ("opacity_logits", wol)):
        err = rel(raw_g[name].cpu().numpy(), want)
        assert err <= 1e-3, (name, err)


def test_image_fit_trainer_keeps_rotations_about_z_and_lowers_the_loss(gb):
    from paper_2412_12734_amd import train as T
    raw, view, target = sg.image_fit_config(3, 3000, 128, 96, 4)
    st = T.TrainState(raw, bf16=False, rotz_only=True)
    tr = T.Trainer(st, [view], cuda(target).view(1, -1, 3), loss="mse")
    losses = [float(tr.step([0])) for _ in range(12)]
    assert all(np.isfinite(losses)) and losses[-1] < losses[0]
    q = st.params["quats"].cpu().numpy()
    assert np.all(q[:, 1:3] == 0.0)
    # the box-filtered grids render with N = 2 and N = 1 (the paper's check of the grids)
    for M in (2, 1):
        small = T.box_filter_textures(st.params["textures"], M)
        sp = st.activate()
        sp2 = gb.Splats(sp.means, sp.tan_u, sp.tan_v, sp.scales, sp.opacity, small)
        rast = gb.Rasterizer([view])
        rast.plan(sp2)
        rgb, _ = rast.forward(sp2)
        assert bool(torch.isfinite(rgb).all())
