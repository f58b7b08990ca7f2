"""The differentiable entry point (the torch.autograd.Function over the C ABI) and GPU
gradients against central finite differences of the FP64 oracle's forward."""
import numpy as np
import pytest

import scenegen as sg
from oracle import gb_oracle as O

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gb():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2412_12734_amd as gb
    gb.load()
    return gb


def leaf(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda().requires_grad_(True)


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30))


def test_autograd_function_matches_oracle(gb):
    """render() + loss.backward() gives the oracle's analytic gradients (1e-3 relative L2) and
    the raw backward's gradients, and its image matches the oracle."""
    scene, views = sg.config("C1", P=400)
    view = views[0]
    opts = O.Options()
    rast = gb.Rasterizer([view])
    params = [leaf(a) for a in (scene.means, scene.tan_u, scene.tan_v, scene.scales,
                                scene.opacity, scene.textures)]
    rgb, T = gb.render(rast, *params)
    ref = O.render(scene, view, opts, keep_saved=True)
    ok = ~O.grad_flags(ref).reshape(-1)
    g = sg.make_dl_drgb(9, [view])
    g = np.where(ok[:, None], g, 0.0).astype(np.float32)
    loss = (rgb * torch.from_numpy(g).cuda()).sum()
    loss.backward()
    img = rgb.detach().cpu().numpy().reshape(ref.rgb.shape)
    assert np.abs(img - ref.rgb)[~O.image_flags(ref)].max() <= 1e-5
    want = O.render_backward(scene, view, opts, ref, g.astype(np.float64))
    for name, p in zip(("means", "tan_u", "tan_v", "scales", "opacity", "textures"), params):
        err = rel_l2(p.grad.cpu().numpy().astype(np.float64), getattr(want, name))
        print(name, f"{err:.2e}")
        assert err <= 1e-3, (name, err)
    # the same gradients as the raw Rasterizer.backward on the same forward
    sp = gb.Splats.from_numpy(scene)
    rgb2, T2 = rast.forward(sp)
    raw = rast.backward(sp, T2, torch.from_numpy(g).cuda())
    for name, p in zip(("means", "tan_u", "tan_v", "scales", "opacity", "textures"), params):
        assert rel_l2(p.grad.cpu().numpy().astype(np.float64),
                      raw[name].cpu().numpy().astype(np.float64)) <= 1e-5, name


def test_autograd_function_rejects_a_stale_workspace(gb):
    """Two renders on one Rasterizer before the first backward: the first render's backward
    would read the second's pair lists, so it raises; the second still differentiates."""
    scene, views = sg.config("C1", P=200)
    rast = gb.Rasterizer(views)
    p1 = [leaf(a) for a in (scene.means, scene.tan_u, scene.tan_v, scene.scales,
                            scene.opacity, scene.textures)]
    p2 = [leaf(a) for a in (scene.means, scene.tan_u, scene.tan_v, scene.scales,
                            scene.opacity, scene.textures)]
    rgb1, _ = gb.render(rast, *p1)
    rgb2, _ = gb.render(rast, *p2)
    with pytest.raises(RuntimeError, match="another forward"):
        rgb1.sum().backward()
    rgb2.sum().backward()
    assert p2[5].grad is not None and float(p2[5].grad.abs().sum()) > 0.0


def test_autograd_function_bf16_textures(gb):
    """BF16 textures through the autograd function: the texture gradient comes back in the
    parameter's dtype, the geometry gradients in float32."""
    scene, views = sg.config("C1", P=300)
    rast = gb.Rasterizer(views)
    params = [leaf(a) for a in (scene.means, scene.tan_u, scene.tan_v, scene.scales,
                                scene.opacity)]
    tex = torch.from_numpy(scene.textures).cuda().to(torch.bfloat16).requires_grad_(True)
    rgb, T = gb.render(rast, *params, tex)
    rgb.sum().backward()
    assert tex.grad.dtype == torch.bfloat16 and params[0].grad.dtype == torch.float32
    assert float(tex.grad.float().abs().sum()) > 0.0


@pytest.mark.parametrize("seed", [0, 1])
def test_gpu_gradients_match_central_differences(gb, seed):
    """GPU gradients (float32, hand-written backward) against central differences of the FP64
    oracle forward, on a tiny scene with the thresholds switched off (no skip, no stop, no
    clamp, so the image is smooth in every parameter). Per tensor, 12 sampled elements; the
    relative L2 error of the sampled gradient vector must be <= 1e-3."""
    rng = np.random.default_rng(70 + seed)
    N = [4, 2][seed]
    scene = sg.make_scene(80 + seed, 6, -0.35, 0.35, 0.06, 0.3, N)
    W, H = 28, 22
    view = sg.look_at_view(np.array([0.2, -0.1, -2.2]) + 0.2 * rng.standard_normal(3), W, H)
    opts = O.Options(alpha_min=0.0, t_min=0.0, alpha_max=1.0, bg=(0.2, 0.4, 0.1))
    g = sg.make_dl_drgb(seed, [view]).astype(np.float64)
    gpu_opts = gb.Options(alpha_min=0.0, t_min=0.0, alpha_max=1.0, bg=(0.2, 0.4, 0.1))
    sp = gb.Splats.from_numpy(scene)
    rast = gb.Rasterizer([view], gpu_opts)
    rgb, T = rast.forward(sp)
    grads = rast.backward(sp, T, torch.from_numpy(g.astype(np.float32)).cuda())
    torch.cuda.synchronize()

    def loss(sc):
        return float(np.sum(O.render(sc, view, opts).rgb.reshape(-1, 3) * g))

    base = [a.astype(np.float64) for a in (scene.means, scene.tan_u, scene.tan_v, scene.scales,
                                           scene.opacity, scene.textures)]
    for fi, name in enumerate(("means", "tan_u", "tan_v", "scales", "opacity", "textures")):
        arr = base[fi]
        got = grads[name].cpu().numpy().astype(np.float64)
        picks = rng.choice(arr.size, size=min(12, arr.size), replace=False)
        fd, an = [], []
        for flat in picks:
            idx = np.unravel_index(flat, arr.shape)
            h = 1e-6 * max(1.0, abs(float(arr[idx])))
            vals = []
            for sgn in (1.0, -1.0):
                parts = [a.copy() for a in base]
                parts[fi][idx] = arr[idx] + sgn * h
                vals.append(loss(sg.Scene(*parts)))
            fd.append((vals[0] - vals[1]) / (2.0 * h))
            an.append(got[idx])
        err = rel_l2(np.array(an), np.array(fd))
        print(name, f"{err:.2e}")
        assert err <= 1e-3, (name, err, an, fd)
