"""The oracle's hand-derived backward against torch float64 autograd (CPU only).

The forward below is an independent torch transcription of the per-pixel definition (Eq. 2-5,
Alg. 1-2 with the readings of the oracle): pinhole camera, ray-plane solve through the
homogeneous cross product, falloff with the screen-space low-pass, opacity clamp, skip and
stop thresholds, border-clamped bilinear colour lookup, front-to-back compositing. Only the
depth order (a discrete input) is taken from the oracle. Autograd of this forward must equal
the oracle's analytic gradient to ~1e-10 relative.
"""
import numpy as np
import pytest

import scenegen as sg
from oracle import gb_oracle as O

torch = pytest.importorskip("torch")


def torch_render(params, view, opts, order, W, H):
    means, tan_u, tan_v, scales, opacity, tex = params
    dt = torch.float64
    R = torch.tensor(np.asarray(view.R, dtype=np.float64), dtype=dt)
    t = torch.tensor(np.asarray(view.t, dtype=np.float64), dtype=dt)
    fx, fy, cx, cy = (float(np.float32(c)) for c in (view.fx, view.fy, view.cx, view.cy))
    Kc = torch.tensor([[fx, 0.0, cx], [0.0, fy, cy], [0.0, 0.0, 1.0]], dtype=dt)
    jj, ii = torch.meshgrid(torch.arange(H, dtype=dt), torch.arange(W, dtype=dt), indexing="ij")
    x = ii.reshape(-1) + 0.5
    y = jj.reshape(-1) + 0.5
    n = x.shape[0]
    T = torch.ones(n, dtype=dt)
    acc = torch.zeros(n, 3, dtype=dt)
    done = torch.zeros(n, dtype=torch.bool)
    N = tex.shape[1]
    sig = opts.sigma
    for k in order:
        a = R @ (scales[k, 0] * tan_u[k])
        b = R @ (scales[k, 1] * tan_v[k])
        pc = R @ means[k] + t
        M = Kc @ torch.stack([a, b, pc], dim=1)
        hx = x[:, None] * M[2][None, :] - M[0][None, :]
        hy = y[:, None] * M[2][None, :] - M[1][None, :]
        rho = torch.linalg.cross(hx, hy, dim=1)
        u = rho[:, 0] / rho[:, 2]
        v = rho[:, 1] / rho[:, 2]
        c2x, c2y = M[0, 2] / M[2, 2], M[1, 2] / M[2, 2]
        q_uv = 0.5 * (u * u + v * v)
        q_lp = ((x - c2x) ** 2 + (y - c2y) ** 2) / (2.0 * opts.lowpass_var)
        q = torch.where(q_uv <= q_lp, q_uv, q_lp)
        alpha = torch.clamp(opacity[k] * torch.exp(-q), max=opts.alpha_max)
        contrib = (~done) & (alpha.detach() >= opts.alpha_min)
        Tn = T * (1.0 - alpha)
        stop = contrib & (Tn.detach() < opts.t_min)
        blend = contrib & ~stop
        # bilinear lookup, corner-aligned grid over [-sigma, sigma], coordinates clamped
        if N == 1:
            col = tex[k, 0, 0][None, :].expand(n, 3)
        else:
            def coord(w):
                wp = torch.clamp((N - 1) * (w + sig) / (2.0 * sig), 0.0, N - 1)
                i = torch.clamp(torch.floor(wp.detach()), max=N - 2).long()
                return i, wp - i
            iu, fu = coord(u)
            iv, fv = coord(v)
            fu, fv = fu[:, None], fv[:, None]
            C = tex[k]
            col = (C[iu, iv] * (1 - fu) * (1 - fv) + C[iu + 1, iv] * fu * (1 - fv)
                   + C[iu, iv + 1] * (1 - fu) * fv + C[iu + 1, iv + 1] * fu * fv)
        wgt = torch.where(blend, alpha * T, torch.zeros_like(T))
        acc = acc + wgt[:, None] * col
        T = torch.where(blend, Tn, T)
        done = done | stop
    bg = torch.tensor(opts.bg, dtype=dt)
    return acc + T[:, None] * bg[None, :]


@pytest.mark.parametrize("case", ["default", "off", "n1", "lowpass"])
def test_oracle_backward_equals_torch_autograd(case):
    rng = np.random.default_rng({"default": 1, "off": 2, "n1": 3, "lowpass": 4}[case])
    N = 1 if case == "n1" else 3
    s_lo, s_hi = (0.002, 0.01) if case == "lowpass" else (0.08, 0.35)
    scene = sg.make_scene(40 + len(case), 5, -0.3, 0.3, s_lo, s_hi, N)
    W, H = 22, 18
    view = sg.look_at_view((0.15, -0.1, -2.0), W, H)
    if case == "off":
        opts = O.Options(alpha_min=0.0, t_min=0.0, alpha_max=1.0, bg=(0.3, 0.1, 0.2))
    else:
        opts = O.Options(bg=tuple(rng.uniform(0, 1, 3)), lowpass_var=1.0 if case == "lowpass"
                         else 0.5)
    g = rng.standard_normal((W * H, 3))
    r = O.render(scene, view, opts, keep_saved=True)
    # pixels next to a decision or kink have no unique gradient: zero their adjoint
    g = np.where(O.grad_flags(r).reshape(-1, 1), 0.0, g)
    ana = O.render_backward(scene, view, opts, r, g)
    order = [int(k) for k in O.depth_order(O.key_stage(scene, view, opts))]
    params = [torch.tensor(a.astype(np.float64), requires_grad=True) for a in
              (scene.means, scene.tan_u, scene.tan_v, scene.scales, scene.opacity, scene.textures)]
    rgb = torch_render(params, view, opts, order, W, H)
    np.testing.assert_allclose(rgb.detach().numpy().reshape(H, W, 3), r.rgb, rtol=0, atol=1e-12)
    (rgb * torch.tensor(g)).sum().backward()
    for name, p in zip(("means", "tan_u", "tan_v", "scales", "opacity", "textures"), params):
        want = p.grad.numpy()
        got = getattr(ana, name)
        scale = max(np.abs(want).max(), 1e-30)
        np.testing.assert_allclose(got, want, rtol=1e-9, atol=1e-10 * scale, err_msg=name)
