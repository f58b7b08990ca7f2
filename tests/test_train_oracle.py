"""Pins of the training-glue oracle (CPU): closed forms, invariants, finite differences and
hand-worked values, so that a dropped term, a wrong sign or a transposed index fails here."""
import math

import numpy as np
import pytest

from oracle import train_oracle as T

rng = np.random.default_rng(5)


def test_rotation_about_z_is_the_closed_form():
    for th in (0.3, -1.2, 2.9):
        q = np.array([math.cos(th / 2), 0.0, 0.0, math.sin(th / 2)])
        t_u, t_v, _, _ = T.activate(q[None], np.zeros((1, 2)), np.zeros(1))
        np.testing.assert_allclose(t_u[0], [math.cos(th), math.sin(th), 0.0], atol=1e-15)
        np.testing.assert_allclose(t_v[0], [-math.sin(th), math.cos(th), 0.0], atol=1e-15)


def test_rotation_about_x_is_the_closed_form():
    th = 0.7
    q = np.array([math.cos(th / 2), math.sin(th / 2), 0.0, 0.0])
    R = T.rotation(q)
    np.testing.assert_allclose(R, [[1, 0, 0], [0, math.cos(th), -math.sin(th)],
                                   [0, math.sin(th), math.cos(th)]], atol=1e-15)


def test_rotations_are_proper_orthonormal_and_scale_invariant():
    q = rng.standard_normal((50, 4))
    R = T.rotation(q)
    np.testing.assert_allclose(np.einsum("nij,nkj->nik", R, R), np.broadcast_to(np.eye(3), R.shape),
                               atol=1e-13)
    np.testing.assert_allclose(np.linalg.det(R), 1.0, atol=1e-13)
    np.testing.assert_allclose(T.rotation(-3.7 * q), R, atol=1e-13)  # q and c q, any c != 0


def test_identity_quaternion_and_scalar_activations():
    t_u, t_v, s, o = T.activate(np.array([[2.0, 0, 0, 0]]), np.array([[0.0, math.log(3.0)]]),
                                np.array([0.0]))
    np.testing.assert_allclose(t_u[0], [1, 0, 0])
    np.testing.assert_allclose(t_v[0], [0, 1, 0])
    np.testing.assert_allclose(s[0], [1.0, 3.0])
    assert o[0] == 0.5


def test_activate_backward_matches_central_differences():
    P = 4
    q, ls, ol = rng.standard_normal((P, 4)), rng.standard_normal((P, 2)), rng.standard_normal(P)
    gu, gv, gs, go = (rng.standard_normal(s) for s in ((P, 3), (P, 3), (P, 2), (P,)))
    dq, dls, dol = T.activate_backward(q, ls, ol, gu, gv, gs, go)

    def L(q_, ls_, ol_):
        a, b, c, d = T.activate(q_, ls_, ol_)
        return (a * gu).sum() + (b * gv).sum() + (c * gs).sum() + (d * go).sum()

    h = 1e-6
    for arr, grad in ((q, dq), (ls, dls), (ol, dol)):
        for idx in np.ndindex(arr.shape):
            e = np.zeros_like(arr)
            e[idx] = h
            args_p = [q, ls, ol]
            args_m = [q, ls, ol]
            k = [q is arr, ls is arr, ol is arr].index(True)
            args_p = [a + e if i == k else a for i, a in enumerate(args_p)]
            args_m = [a - e if i == k else a for i, a in enumerate(args_m)]
            fd = (L(*args_p) - L(*args_m)) / (2 * h)
            assert abs(fd - grad[idx]) <= 1e-7 * max(1.0, abs(fd)), (k, idx, fd, grad[idx])


def test_quaternion_gradient_is_orthogonal_to_the_quaternion():
    q = rng.standard_normal((20, 4))
    dq, _, _ = T.activate_backward(q, np.zeros((20, 2)), np.zeros(20), rng.standard_normal((20, 3)),
                                   rng.standard_normal((20, 3)), np.zeros((20, 2)), np.zeros(20))
    np.testing.assert_allclose((dq * q).sum(1), 0.0, atol=1e-12)


def test_l1_loss_hand_example():
    loss, g = T.l1_loss([0.5, 0.2, 0.9, 0.4], [0.1, 0.2, 1.0, 0.0], 0.25)
    assert loss == pytest.approx(0.25 * (0.4 + 0.0 + 0.1 + 0.4))
    np.testing.assert_array_equal(g, [0.25, 0.0, -0.25, 0.25])


def test_adam_first_step_moves_by_lr_against_the_gradient_sign():
    theta = rng.standard_normal(100)
    g = rng.standard_normal(100)
    new, m, v = T.adam_step(theta, g, np.zeros(100), np.zeros(100), 1, 0.01)
    np.testing.assert_allclose(new, theta - 0.01 * np.sign(g), rtol=0, atol=1e-12)
    np.testing.assert_allclose(m, 0.1 * g)
    np.testing.assert_allclose(v, 0.001 * g * g)


def test_adam_constant_gradient_closed_form():
    # with a constant gradient the bias-corrected moments equal g and g^2 at every step
    theta, g = np.array([1.0, -2.0, 0.5]), np.array([0.3, -4.0, 1e-3])
    m = v = np.zeros(3)
    th = theta
    for t in range(1, 8):
        th, m, v = T.adam_step(th, g, m, v, t, 0.05)
        np.testing.assert_allclose(m, g * (1 - 0.9 ** t), rtol=1e-12)
        np.testing.assert_allclose(v, g * g * (1 - 0.999 ** t), rtol=1e-12)
    np.testing.assert_allclose(th, theta - 7 * 0.05 * np.sign(g), atol=1e-9)


def test_adam_zero_gradient_keeps_the_parameter_at_zero_moments():
    th, m, v = T.adam_step(np.array([3.0]), np.array([0.0]), np.zeros(1), np.zeros(1), 1, 1.0)
    assert th[0] == 3.0 and m[0] == 0.0 and v[0] == 0.0


@pytest.mark.parametrize("x,bits", [
    (1.0, 0x3F80), (-2.0, 0xC000), (0.0, 0x0000),
    (1.0 + 2 ** -8, 0x3F80),          # exactly half way between 1.0 and 1.0078125: even stays
    (1.0 + 3 * 2 ** -8, 0x3F82),      # half way between 0x3F81 and 0x3F82: to the even 0x3F82
    (1.0 + 2 ** -8 + 2 ** -20, 0x3F81),  # just above half way: up
    (1.0 + 2 ** -9, 0x3F80),          # below half way: down
    (3.0e38, 0x7F62),
])
def test_bf16_round_to_nearest_even(x, bits):
    assert int(T.bf16_round(np.array([x], dtype=np.float32))[0]) == bits


# --- single-image fitting set-up (Sec. 4): MSE loss, box-filtered grids, rotation about z ---
def test_mse_loss_hand_example():
    loss, d = T.mse_loss([1.0, 2.0, 3.0], [0.0, 4.0, 3.0], 0.5)
    assert loss == pytest.approx(0.5 * (1.0 + 4.0 + 0.0))
    np.testing.assert_allclose(d, [1.0, -2.0, 0.0])


def test_mse_gradient_matches_central_differences():
    rng = np.random.default_rng(4)
    a, b = rng.uniform(0, 1, 12), rng.uniform(0, 1, 12)
    _, d = T.mse_loss(a, b, 0.25)
    h = 1e-6
    for i in range(12):
        e = np.zeros(12)
        e[i] = h
        fd = (T.mse_loss(a + e, b, 0.25)[0] - T.mse_loss(a - e, b, 0.25)[0]) / (2 * h)
        assert fd == pytest.approx(d[i], rel=1e-6, abs=1e-9)


def test_box_filter_hand_example_and_special_cases():
    t = np.arange(4 * 4 * 3, dtype=np.float64).reshape(1, 4, 4, 3)
    out = T.box_filter(t, 2)
    # top-left 2 x 2 block of channel 0 holds 0, 3, 12, 15
    assert out[0, 0, 0, 0] == pytest.approx((0 + 3 + 12 + 15) / 4)
    # bottom-right block of channel 2 holds 32, 35, 44, 47
    assert out[0, 1, 1, 2] == pytest.approx((32 + 35 + 44 + 47) / 4)
    np.testing.assert_array_equal(T.box_filter(t, 4), t)  # M = N: identity
    np.testing.assert_allclose(T.box_filter(t, 1)[0, 0, 0], t[0].mean(axis=(0, 1)))
    const = np.broadcast_to(np.array([0.2, 0.5, 0.9]), (3, 8, 8, 3))
    np.testing.assert_allclose(T.box_filter(const, 2), np.broadcast_to([0.2, 0.5, 0.9],
                                                                       (3, 2, 2, 3)))
    rng = np.random.default_rng(2)
    r = rng.uniform(0, 1, (5, 8, 8, 3))
    # the mean colour of every grid is kept, and filtering in steps equals filtering at once
    np.testing.assert_allclose(T.box_filter(r, 2).mean(axis=(1, 2)), r.mean(axis=(1, 2)))
    np.testing.assert_allclose(T.box_filter(T.box_filter(r, 4), 2), T.box_filter(r, 2))
    with pytest.raises(ValueError):
        T.box_filter(r, 3)


def test_rotz_only_keeps_quaternions_about_z_and_tangents_in_plane():
    rng = np.random.default_rng(6)
    P = 40
    a = rng.uniform(0, 2 * np.pi, P)
    q = np.stack([np.cos(a / 2), np.zeros(P), np.zeros(P), np.sin(a / 2)], axis=1)
    m, v = np.zeros_like(q), np.zeros_like(q)
    for step in range(1, 6):
        g = T.rotz_only(rng.standard_normal((P, 4)))
        assert np.all(g[:, 1:3] == 0.0)
        q, m, v = T.adam_step(q, g, m, v, step, 1e-2)
    assert np.all(q[:, 1:3] == 0.0)
    t_u, t_v, _, _ = T.activate(q, np.zeros((P, 2)), np.zeros(P))
    # a rotation about z by angle b = 2 atan2(z, w): t_u = (cos b, sin b, 0), t_v = (-sin b, cos b, 0)
    b = 2.0 * np.arctan2(q[:, 3], q[:, 0])
    np.testing.assert_allclose(t_u, np.stack([np.cos(b), np.sin(b), np.zeros(P)], 1), atol=1e-12)
    np.testing.assert_allclose(t_v, np.stack([-np.sin(b), np.cos(b), np.zeros(P)], 1), atol=1e-12)
