"""FP64 reference for the training glue around the rasterizer (test infrastructure only).

Only tests, the package's smoke check and the benchmark's CPU baseline use this module; the
product path never imports it. It shares no code with the HIP kernels.

The paper trains textured splats with an image loss and Adam (Sec. 3.3); its parameters are
activated as in 2D Gaussian splatting: a quaternion gives the rotation whose first two columns
are the tangents t_u and t_v, log-scales give s = exp, logits give o = sigmoid. The functions
below are those definitions written out:

* ``activate``: (w, x, y, z) / |q| -> R(q) by the standard rotation-matrix formula -> columns;
  exp; logistic sigmoid.
* ``activate_backward``: the chain rule of ``activate`` by PyTorch CPU autograd in float64 over
  the same definition (no hand-derived Jacobian).
* ``l1_loss``: scale * sum |I - I*| and its gradient scale * sign(I - I*).
* ``adam_step``: the Adam update with bias correction, as published (Kingma and Ba, Alg. 1).
* ``bf16_round``: float32 -> nearest bfloat16, ties to even, from the bit pattern.
* ``mse_loss``, ``box_filter``, ``rotz_only``: the single-image fitting set-up of Sec. 4
  (MSE loss; colour grids box-filtered to fewer texels; rotation about Z only).
"""
from __future__ import annotations

import numpy as np


def rotation(q):
    """Rotation matrices (..., 3, 3) of quaternions (..., 4) = (w, x, y, z), normalised first.
    Works on numpy arrays and on torch tensors."""
    n = (q * q).sum(-1, keepdims=True) ** 0.5 if isinstance(q, np.ndarray) else \
        (q * q).sum(-1, keepdim=True).sqrt()
    q = q / n
    w, x, y, z = q[..., 0], q[..., 1], q[..., 2], q[..., 3]
    rows = [
        [1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
        [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
        [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)],
    ]
    if isinstance(q, np.ndarray):
        return np.stack([np.stack(r, -1) for r in rows], -2)
    import torch
    return torch.stack([torch.stack(r, -1) for r in rows], -2)


def activate(quats, log_scales, opacity_logits):
    """Raw parameters -> (t_u, t_v, scales, opacity), float64."""
    q = np.asarray(quats, dtype=np.float64)
    R = rotation(q)
    t_u, t_v = R[..., :, 0], R[..., :, 1]
    s = np.exp(np.asarray(log_scales, dtype=np.float64))
    o = 1.0 / (1.0 + np.exp(-np.asarray(opacity_logits, dtype=np.float64)))
    return t_u, t_v, s, o


def activate_backward(quats, log_scales, opacity_logits, d_tan_u, d_tan_v, d_scales, d_opacity):
    """Gradients with respect to the raw parameters, by float64 autograd of the definition."""
    import torch
    q = torch.tensor(np.asarray(quats, dtype=np.float64), requires_grad=True)
    ls = torch.tensor(np.asarray(log_scales, dtype=np.float64), requires_grad=True)
    ol = torch.tensor(np.asarray(opacity_logits, dtype=np.float64), requires_grad=True)
    R = rotation(q)
    t_u, t_v = R[..., :, 0], R[..., :, 1]
    s = torch.exp(ls)
    o = torch.sigmoid(ol)
    f = lambda a: torch.tensor(np.asarray(a, dtype=np.float64))
    L = ((t_u * f(d_tan_u)).sum() + (t_v * f(d_tan_v)).sum() + (s * f(d_scales)).sum()
         + (o * f(d_opacity)).sum())
    L.backward()
    return q.grad.numpy(), ls.grad.numpy(), ol.grad.numpy()


def l1_loss(rgb, target, scale):
    d = np.asarray(rgb, dtype=np.float64) - np.asarray(target, dtype=np.float64)
    return scale * np.abs(d).sum(), scale * np.sign(d)


def mse_loss(rgb, target, scale):
    """Squared-error image loss (Sec. 4 fits single images with an MSE loss): the loss
    scale * sum (rgb - target)^2 and its gradient 2 scale (rgb - target)."""
    d = np.asarray(rgb, dtype=np.float64) - np.asarray(target, dtype=np.float64)
    return scale * (d * d).sum(), 2.0 * scale * d


def box_filter(textures, M):
    """Box filter of colour grids to M x M (Sec. 4 renders fitted grids downsampled to 2 x 2
    and to one colour): each output texel is the mean of the (N / M)^2 texels it covers.
    textures [P][N][N][3] -> [P][M][M][3], float64."""
    t = np.asarray(textures, dtype=np.float64)
    P, N = t.shape[0], t.shape[1]
    if N % M:
        raise ValueError("M must divide N")
    k = N // M
    out = np.zeros((P, M, M, 3))
    for i in range(M):
        for j in range(M):
            out[:, i, j, :] = t[:, i * k:(i + 1) * k, j * k:(j + 1) * k, :].mean(axis=(1, 2))
    return out


def rotz_only(d_quats):
    """Rotation about the Z axis only (Sec. 4, single-image fitting): the x and y components
    of the quaternion gradient are dropped, so quaternions (w, 0, 0, z) keep that form."""
    d = np.array(d_quats, dtype=np.float64, copy=True)
    d[:, 1:3] = 0.0
    return d


def adam_step(theta, g, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-15):
    """One Adam step (float64): returns the new (theta, m, v)."""
    theta, g, m, v = (np.asarray(a, dtype=np.float64) for a in (theta, g, m, v))
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    m_hat = m / (1.0 - beta1 ** step)
    v_hat = v / (1.0 - beta2 ** step)
    return theta - lr * m_hat / (np.sqrt(v_hat) + eps), m, v


def bf16_round(x):
    """float32 values -> the bit patterns (uint16) of the nearest bfloat16, ties to even.
    Finite inputs only."""
    bits = np.asarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    keep = bits >> np.uint64(16)
    rest = bits & np.uint64(0xFFFF)
    up = (rest > 0x8000) | ((rest == 0x8000) & ((keep & np.uint64(1)) == 1))
    return (keep + up.astype(np.uint64)).astype(np.uint16)
