"""FP64 reference of the droplet-shape surrogate network (TEST INFRASTRUCTURE).

The surrogate maps a window of the velocity-gradient history that drives a
droplet box (the A(t) of Sec. 3, sampled every 50 steps, 64 samples of 9
entries) to the droplet's three inertia-tensor semi-axes (the shape whose
deformation D of Sec. 2 Eq. 4 the paper follows).  The paper has no such
network; its definition here is a plain multilayer perceptron:

    z_1 = x W_1^T + b_1,   h_l = max(z_l, 0),   z_{l+1} = h_l W_{l+1}^T + b_{l+1},
    y = h_L W_out^T + b_out,

trained on the mean squared error  L = (1 / (3 n)) sum_m sum_j (y_mj - t_mj)^2
with Adam (bias-corrected first and second moments).  Weights are stored
[out][in]; the flat parameter vector lists W_1, b_1, W_2, b_2, ..., W_out,
b_out in that order.  Inputs and targets are affinely normalised:
x = (window - in_shift) * in_scale,  t = (semi_axes - out_shift) * out_scale.

Everything is float64 numpy; no blocking, fusion or reordering.
"""
from __future__ import annotations

import numpy as np

WIDTHS = (576, 512, 512, 512, 3)   # 64 samples x 9 entries -> three hidden layers -> 3 semi-axes


def param_shapes(widths=WIDTHS):
    shapes = []
    for i in range(len(widths) - 1):
        shapes.append((widths[i + 1], widths[i]))
        shapes.append((widths[i + 1],))
    return shapes


def param_count(widths=WIDTHS) -> int:
    return int(sum(int(np.prod(s)) for s in param_shapes(widths)))


def unflatten(flat, widths=WIDTHS):
    """Views of the flat vector as [W_1, b_1, ..., W_out, b_out]."""
    flat = np.asarray(flat)
    out, off = [], 0
    for s in param_shapes(widths):
        n = int(np.prod(s))
        out.append(flat[off:off + n].reshape(s))
        off += n
    assert off == flat.size
    return out


def flatten(tensors) -> np.ndarray:
    return np.concatenate([np.asarray(t, dtype=np.float64).ravel() for t in tensors])


def init_params(seed: int, widths=WIDTHS) -> np.ndarray:
    """He-normal weights (std sqrt(2 / fan_in)) and zero biases, float64."""
    rng = np.random.default_rng(seed)
    ts = []
    for s in param_shapes(widths):
        if len(s) == 2:
            ts.append(rng.standard_normal(s) * np.sqrt(2.0 / s[1]))
        else:
            ts.append(np.zeros(s))
    return flatten(ts)


def forward(flat, x, widths=WIDTHS, round_hidden=None):
    """Returns (y, [h_0 = x, h_1, ..., h_L]).  `round_hidden`, if given, is applied
    to every hidden activation after the ReLU (a storage format of the
    activations, e.g. rounding to bfloat16)."""
    ps = unflatten(flat, widths)
    h = np.asarray(x, dtype=np.float64)
    hs = [h]
    nl = len(widths) - 1
    for l in range(nl):
        W, b = ps[2 * l], ps[2 * l + 1]
        z = h @ W.T + b
        if l < nl - 1:
            h = np.maximum(z, 0.0)
            if round_hidden is not None:
                h = round_hidden(h)
            hs.append(h)
        else:
            return z, hs


def mse(y, t) -> float:
    d = np.asarray(y, dtype=np.float64) - np.asarray(t, dtype=np.float64)
    return float(np.mean(d * d))


def backward(flat, x, t, widths=WIDTHS, round_hidden=None, round_grad=None):
    """Loss and gradient of the mean squared error with respect to the flat
    parameter vector (chain rule, layer by layer from the output).
    `round_hidden` as in forward; `round_grad`, if given, is applied to the
    gradient of every hidden pre-activation (a storage format, as above)."""
    y, hs = forward(flat, x, widths, round_hidden)
    ps = unflatten(flat, widths)
    n, nout = y.shape
    dz = 2.0 * (y - t) / (n * nout)
    grads = [None] * len(ps)
    nl = len(widths) - 1
    for l in range(nl - 1, -1, -1):
        h = hs[l]
        grads[2 * l] = dz.T @ h
        grads[2 * l + 1] = dz.sum(axis=0)
        if l > 0:
            dh = dz @ ps[2 * l]
            dz = dh * (h > 0.0)
            if round_grad is not None:
                dz = round_grad(dz)
    return mse(y, t), flatten(grads)


def adam_step(p, g, m, v, step: int, lr: float, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8):
    """One Adam update (in place on p, m, v); `step` counts from 1."""
    m *= beta1
    m += (1.0 - beta1) * g
    v *= beta2
    v += (1.0 - beta2) * g * g
    mhat = m / (1.0 - beta1 ** step)
    vhat = v / (1.0 - beta2 ** step)
    p -= lr * mhat / (np.sqrt(vhat) + eps)
    return p, m, v


def normalize_inputs(windows, in_shift, in_scale):
    w = np.asarray(windows, dtype=np.float64).reshape(len(windows), -1)
    return (w - np.asarray(in_shift)) * np.asarray(in_scale)


def denormalize_outputs(y, out_shift, out_scale):
    return np.asarray(y) / np.asarray(out_scale) + np.asarray(out_shift)


def deformation(semi_axes) -> np.ndarray:
    """D = (L - B) / (L + B) from the largest and smallest semi-axes (Sec. 2 Eq. 4)."""
    a = np.sort(np.asarray(semi_axes, dtype=np.float64), axis=-1)
    return (a[..., 2] - a[..., 0]) / (a[..., 2] + a[..., 0])


def cubic_symmetry(s: int) -> np.ndarray:
    """Signed permutation matrix number s of the 48 symmetries of the cube:
    P[i][perm(i)] = sign(i), perm = the (s // 8)-th permutation of (0, 1, 2) in
    lexicographic order, sign(i) = -1 where bit i of s % 8 is set."""
    import itertools
    perm = list(itertools.permutations(range(3)))[s // 8]
    P = np.zeros((3, 3))
    for i in range(3):
        P[i, perm[i]] = -1.0 if (s % 8) >> i & 1 else 1.0
    return P


def transform_window(window, s: int) -> np.ndarray:
    """Every 3x3 sample A of a flattened window becomes P A P^T (P = cubic_symmetry(s))."""
    P = cubic_symmetry(s)
    A = np.asarray(window, dtype=np.float64).reshape(-1, 3, 3)
    return np.matmul(np.matmul(P, A), P.T).reshape(np.shape(window))


def round_bf16(x) -> np.ndarray:
    """Round float64 values to the nearest bfloat16 (ties to even) through float32:
    the float32 value first (round to nearest), then its 16 high bits with the
    low 16 rounded to nearest even."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    u = (u + 0x7FFF + lsb) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)
