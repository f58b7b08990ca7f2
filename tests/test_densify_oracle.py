"""Pins of the densification and pruning reference (CPU only): the screen-space statistic by
finite differences of an image translation, split and clone by closed forms and special
cases, pruning by construction."""
import math

import numpy as np
import pytest

import scenegen as sg
from oracle import gb_oracle as O
from oracle import densify_oracle as D
from oracle import train_oracle as TO


def test_screen_gradient_is_the_derivative_of_an_image_translation():
    """gr.screen[k] against central differences of the loss when splat k's footprint is
    translated in the image by +-h pixels along x and y."""
    rng = np.random.default_rng(3)
    scene = sg.make_scene(14, 6, -0.3, 0.3, 0.05, 0.3, 3)
    view = sg.look_at_view((0.2, 0.1, -2.0), 26, 22)
    opts = O.Options(bg=(0.2, 0.1, 0.0))
    g = rng.standard_normal((26 * 22, 3))
    r = O.render(scene, view, opts, keep_saved=True)
    gr = O.render_backward(scene, view, opts, r, g)
    checked = 0
    for k in range(scene.P):
        for axis in range(2):
            h = 1e-5
            vals, decs = [], []
            for sgn in (1.0, -1.0):
                d = [0.0, 0.0]
                d[axis] = sgn * h
                rr = O.render(scene, view, opts, shift={k: tuple(d)})
                vals.append(float(np.sum(rr.rgb.reshape(-1, 3) * g)))
                decs.append((rr.n_blended.copy(), rr.terminated.copy()))
            if not all((a == b).all() for a, b in zip(decs[0], decs[1])):
                continue
            fd = (vals[0] - vals[1]) / (2 * h)
            assert gr.screen[k, axis] == pytest.approx(fd, rel=1e-5, abs=1e-7), (k, axis)
            checked += 1
    assert checked >= 10
    # the statistic is zero for a splat no pixel blends
    assert np.all(gr.screen[[k for k in range(scene.P) if not any(s[0] == k for s in r.saved)]] == 0)


def _raw(P, N, seed=0):
    rng = np.random.default_rng(seed)
    means = rng.uniform(-1, 1, (P, 3))
    quats = rng.standard_normal((P, 4))
    log_s = np.log(rng.uniform(0.005, 0.05, (P, 2)))
    logits = rng.uniform(-2, 3, P)
    tex = rng.uniform(0, 1, (P, N, N, 3))
    return means, quats, log_s, logits, tex


def test_split_of_a_constant_grid_keeps_its_colour():
    means, quats, log_s, logits, tex = _raw(5, 4)
    tex[:] = np.array([0.2, 0.7, 0.4])
    noise = np.random.default_rng(1).standard_normal((5, 2, 2)) * 2.0
    outs = [(k, kind) for k in range(5) for kind in (D.CHILD0, D.CHILD1)]
    new = D.apply(outs, means, quats, log_s, logits, tex, noise, D.DensifyOptions())
    np.testing.assert_allclose(new["textures"], np.broadcast_to([0.2, 0.7, 0.4], (10, 4, 4, 3)),
                               atol=1e-15)


@pytest.mark.parametrize("N", [2, 4, 8])
def test_split_reproduces_a_linear_colour_field(N):
    """A grid holding a linear field C[i, j] = a + b i + c j: where a child's texel positions
    stay inside the parent's [-sigma, sigma]^2 the resampled texel is the field's value at the
    parent grid coordinate, a + b u' + c v' with u' = (N - 1)(u + sigma) / (2 sigma)."""
    rng = np.random.default_rng(N)
    means, quats, log_s, logits, tex = _raw(3, N, seed=N)
    a, b, c = rng.standard_normal((3, 3))
    i = np.arange(N)[:, None, None]
    j = np.arange(N)[None, :, None]
    tex[:] = a + b * i + c * j
    opts = D.DensifyOptions()
    sig, shrink = opts.sigma, opts.split_shrink
    lim = sig - sig / shrink  # |z| below this keeps the child's grid inside the parent's
    noise = rng.uniform(-lim, lim, (3, 2, 2)) * 0.99
    outs = [(k, D.CHILD0) for k in range(3)] + [(k, D.CHILD1) for k in range(3)]
    new = D.apply(outs, means, quats, log_s, logits, tex, noise, opts)
    grid = -sig + 2 * sig * np.arange(N) / (N - 1)
    for o, (k, kind) in enumerate(outs):
        z = noise[k, kind - D.CHILD0]
        up = (N - 1) * (z[0] + grid / shrink + sig) / (2 * sig)
        vp = (N - 1) * (z[1] + grid / shrink + sig) / (2 * sig)
        want = a + b * up[:, None, None] + c * vp[None, :, None]
        np.testing.assert_allclose(new["textures"][o], want, atol=1e-12)


def test_split_at_the_centre_without_shrinking_is_the_identity():
    means, quats, log_s, logits, tex = _raw(4, 8)
    noise = np.zeros((4, 2, 2))
    opts = D.DensifyOptions(split_shrink=1.0)
    new = D.apply([(k, D.CHILD0) for k in range(4)], means, quats, log_s, logits, tex, noise, opts)
    np.testing.assert_allclose(new["textures"], tex, atol=1e-15)
    np.testing.assert_allclose(new["means"], means, atol=0)
    np.testing.assert_allclose(new["log_scales"], log_s, atol=0)


def test_split_child_centres_and_scales():
    """Identity rotation: t_u = x, t_v = y, so child c sits at p + (s_u z_c0, s_v z_c1, 0) with
    scales s / 1.6; a rotation by 90 degrees about z swaps the axes (t_u = y, t_v = -x)."""
    means = np.array([[0.1, -0.2, 0.3], [0.5, 0.5, 0.5]])
    quats = np.array([[1.0, 0.0, 0.0, 0.0], [math.cos(math.pi / 4), 0, 0, math.sin(math.pi / 4)]])
    log_s = np.log(np.array([[0.02, 0.05], [0.04, 0.01]]))
    noise = np.array([[[0.3, -1.0], [2.0, 0.5]], [[1.0, 1.0], [-0.5, 0.2]]])
    tex = np.zeros((2, 2, 2, 3))
    outs = [(0, D.CHILD0), (0, D.CHILD1), (1, D.CHILD0)]
    new = D.apply(outs, means, quats, log_s, np.zeros(2), tex, noise, D.DensifyOptions())
    np.testing.assert_allclose(new["means"][0], [0.1 + 0.02 * 0.3, -0.2 - 0.05, 0.3], atol=1e-15)
    np.testing.assert_allclose(new["means"][1], [0.1 + 0.02 * 2.0, -0.2 + 0.05 * 0.5, 0.3],
                               atol=1e-15)
    np.testing.assert_allclose(new["means"][2], [0.5 - 0.01 * 1.0, 0.5 + 0.04 * 1.0, 0.5],
                               atol=1e-15)
    np.testing.assert_allclose(np.exp(new["log_scales"][0]), [0.02 / 1.6, 0.05 / 1.6], rtol=1e-14)


def test_decisions_clone_split_prune_and_order():
    """Six splats, one per case; the outputs follow the parents' order."""
    sig = lambda o: math.log(o / (1 - o))
    log_s = np.log(np.array([[0.005, 0.004], [0.05, 0.02], [0.005, 0.005], [0.05, 0.05],
                             [0.2, 0.1], [0.3, 0.3]]))
    logits = np.array([sig(0.5), sig(0.5), sig(0.5), sig(0.003), sig(0.6), sig(0.6)])
    accum = np.array([1e-3, 1e-3, 1e-5, 1e-3, 1e-3, 0.0])
    count = np.array([2.0, 1.0, 1.0, 1.0, 2.0, 0.0])
    opts = D.DensifyOptions(grad_threshold=2e-4, dense_scale=0.01, min_opacity=0.005,
                            max_scale=0.15)
    outs = D.plan(log_s, logits, accum, count, opts)
    # 0: clone; 1: split; 2: kept (small gradient); 3: pruned (opacity) although its gradient
    # asks for a split; 4: split, and the children (0.2 / 1.6 = 0.125) pass the scale limit;
    # 5: never visible (count 0) and too large: pruned
    assert outs == [(0, D.KEEP), (0, D.CLONE_COPY), (1, D.CHILD0), (1, D.CHILD1), (2, D.KEEP),
                    (4, D.CHILD0), (4, D.CHILD1)]


def test_decisions_at_the_thresholds():
    """Each decision taken on both sides of its threshold, 1 % away: the split/clone size
    (max scale against dense_scale), the gradient mean (accum / count against grad_threshold,
    equality densifies), the opacity floor and the children's scale limit."""
    sig = lambda o: math.log(o / (1 - o))
    ds, gt, mo, ms, sh = 0.01, 2e-4, 0.005, 0.05, 1.6
    rows = [  # (s_u, s_v, opacity, accum, count)
        (1.01 * ds, 0.5 * ds, 0.5, 1e-3, 1.0),  # 0: just above dense_scale: split
        (0.99 * ds, 0.5 * ds, 0.5, 1e-3, 1.0),  # 1: just below: clone
        (0.5 * ds, 1.01 * ds, 0.5, 1e-3, 1.0),  # 2: the larger scale is s_v: split
        (0.5 * ds, 0.5 * ds, 0.5, 2 * gt, 2.0),  # 3: mean exactly at the threshold: clone
        (0.5 * ds, 0.5 * ds, 0.5, 0.99 * 2 * gt, 2.0),  # 4: mean just below: kept
        (0.5 * ds, 0.5 * ds, 1.01 * mo, 0.0, 0.0),  # 5: opacity just above the floor: kept
        (0.5 * ds, 0.5 * ds, 0.99 * mo, 0.0, 0.0),  # 6: just below: pruned
        (0.99 * sh * ms, ds, 0.5, 1e-3, 1.0),  # 7: children just under max_scale: split
        (1.01 * sh * ms, ds, 0.5, 1e-3, 1.0),  # 8: children just over: pruned
        (1.01 * ms, ds, 0.5, 0.0, 1.0),  # 9: kept splat just over max_scale: pruned
    ]
    r = np.array(rows)
    outs = D.plan(np.log(r[:, :2]), np.array([sig(o) for o in r[:, 2]]), r[:, 3], r[:, 4],
                  D.DensifyOptions(grad_threshold=gt, dense_scale=ds, min_opacity=mo,
                                   max_scale=ms, split_shrink=sh))
    assert outs == [(0, D.CHILD0), (0, D.CHILD1), (1, D.KEEP), (1, D.CLONE_COPY),
                    (2, D.CHILD0), (2, D.CHILD1), (3, D.KEEP), (3, D.CLONE_COPY), (4, D.KEEP),
                    (5, D.KEEP), (7, D.CHILD0), (7, D.CHILD1)]


def test_opacity_pruning_removes_exactly_the_chosen_splats():
    rng = np.random.default_rng(9)
    P = 50
    log_s = np.log(rng.uniform(0.001, 0.005, (P, 2)))
    chosen = rng.choice(P, 13, replace=False)
    o = rng.uniform(0.01, 0.99, P)
    o[chosen] = rng.uniform(1e-4, 0.0049, 13)
    outs = D.plan(log_s, np.log(o / (1 - o)), np.zeros(P), np.zeros(P), D.DensifyOptions())
    assert [k for k, _ in outs] == sorted(set(range(P)) - set(chosen.tolist()))
    assert all(kind == D.KEEP for _, kind in outs)


def test_optimiser_rows_of_new_splats_start_at_zero():
    means, quats, log_s, logits, tex = _raw(3, 2)
    m = np.random.default_rng(2).standard_normal((3, 4))
    outs = [(0, D.KEEP), (0, D.CLONE_COPY), (1, D.CHILD0), (1, D.CHILD1), (2, D.KEEP)]
    new = D.apply(outs, means, quats, log_s, logits, tex, np.zeros((3, 2, 2)),
                  D.DensifyOptions(), states=[m])
    np.testing.assert_array_equal(new["states"][0], np.stack([m[0], 0 * m[0], 0 * m[0],
                                                              0 * m[0], m[2]]))
    # clone copies are identical to their parent
    for key in ("means", "quats", "log_scales", "textures"):
        np.testing.assert_array_equal(new[key][0], new[key][1])


def test_statistic_accumulates_norms_over_visible_views():
    g1 = np.array([[3.0, 4.0], [1.0, 0.0], [0.0, 0.0]])
    g2 = np.array([[0.0, 2.0], [6.0, 8.0], [1.0, 1.0]])
    acc, cnt = D.accumulate(np.zeros(3), np.zeros(3), [g1, g2],
                            [np.array([True, True, False]), np.array([True, False, True])])
    np.testing.assert_allclose(acc, [7.0, 1.0, math.sqrt(2)])
    np.testing.assert_allclose(cnt, [2.0, 1.0, 1.0])
