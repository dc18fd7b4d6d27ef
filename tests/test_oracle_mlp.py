"""Pins of the FP64 surrogate-network reference (oracle/mlp.py) against facts
that do not come from the reference itself: central finite differences of the
loss, a network built by hand to compute a known function, Adam's closed-form
first two steps, and the bfloat16 format's definition."""
import numpy as np
import pytest

from oracle import mlp

TINY = (7, 5, 6, 4, 3)


def test_param_layout():
    assert mlp.param_count() == 576 * 512 + 512 + 2 * (512 * 512 + 512) + 3 * 512 + 3
    ps = mlp.unflatten(np.arange(mlp.param_count(TINY), dtype=np.float64), TINY)
    assert [p.shape for p in ps] == [(5, 7), (5,), (6, 5), (6,), (4, 6), (4,), (3, 4), (3,)]
    assert ps[1][0] == 35 and ps[2][0, 0] == 40


def test_forward_computes_hand_built_function():
    """A net whose first layer holds [I; -I] and whose later layers add the two
    halves computes y_j = sum_i |x_i| + j for every output j: relu(x) + relu(-x) = |x|."""
    d = 4
    widths = (d, 2 * d, 2 * d, 2 * d, 3)
    W1 = np.vstack([np.eye(d), -np.eye(d)])
    W2 = np.eye(2 * d)
    W3 = np.eye(2 * d)
    W4 = np.ones((3, 2 * d))
    b4 = np.array([0.0, 1.0, 2.0])
    flat = mlp.flatten([W1, np.zeros(2 * d), W2, np.zeros(2 * d), W3, np.zeros(2 * d), W4, b4])
    x = np.random.default_rng(0).standard_normal((10, d))
    y, hs = mlp.forward(flat, x, widths)
    expect = np.abs(x).sum(1)[:, None] + b4[None]
    assert np.allclose(y, expect, rtol=0, atol=1e-14)
    assert np.all(hs[1] >= 0) and len(hs) == 4
    # a bias that shifts the first layer is visible after the ReLU
    flat2 = mlp.flatten([W1, np.full(2 * d, 10.0), W2, np.zeros(2 * d), W3, np.zeros(2 * d), W4, b4])
    y2, _ = mlp.forward(flat2, x, widths)
    assert np.allclose(y2, np.full((10, 1), 20.0 * d) + b4[None], atol=1e-12)


def test_gradient_matches_central_differences():
    rng = np.random.default_rng(1)
    flat = mlp.init_params(3, TINY) + 0.05 * rng.standard_normal(mlp.param_count(TINY))
    x = rng.standard_normal((9, TINY[0]))
    t = rng.standard_normal((9, 3))
    loss, g = mlp.backward(flat, x, t, TINY)
    assert loss == pytest.approx(mlp.mse(mlp.forward(flat, x, TINY)[0], t), rel=1e-15)
    h = 1e-6
    num = np.empty_like(flat)
    for i in range(flat.size):
        e = np.zeros_like(flat)
        e[i] = h
        num[i] = (mlp.mse(mlp.forward(flat + e, x, TINY)[0], t) - mlp.mse(mlp.forward(flat - e, x, TINY)[0], t)) / (2 * h)
    assert np.max(np.abs(num - g)) <= 1e-8 * max(1.0, np.max(np.abs(g)))
    # every tensor's gradient is exercised (no dead layer in this draw)
    for gt in mlp.unflatten(g, TINY):
        assert np.any(gt != 0)


def test_adam_first_two_steps_closed_form():
    lr, b1, b2, eps = 1e-2, 0.9, 0.999, 1e-8
    g1 = np.array([0.3, -2.0, 1e-3, 0.0])
    g2 = np.array([-0.1, -1.0, 2e-3, 5.0])
    p = np.zeros(4)
    m = np.zeros(4)
    v = np.zeros(4)
    mlp.adam_step(p, g1, m, v, 1, lr, b1, b2, eps)
    # step 1: mhat = g, vhat = g^2 -> p = -lr g / (|g| + eps)
    assert np.allclose(p, -lr * g1 / (np.abs(g1) + eps), rtol=1e-12, atol=0)
    p1 = p.copy()
    mlp.adam_step(p, g2, m, v, 2, lr, b1, b2, eps)
    mhat = (b1 * (1 - b1) * g1 + (1 - b1) * g2) / (1 - b1 ** 2)
    vhat = (b2 * (1 - b2) * g1 ** 2 + (1 - b2) * g2 ** 2) / (1 - b2 ** 2)
    assert np.allclose(p, p1 - lr * mhat / (np.sqrt(vhat) + eps), rtol=1e-12, atol=1e-18)


def test_training_fits_a_linear_teacher():
    """Adam on the MSE drives a tiny net to fit y = x B (a function it can represent
    through paired ReLUs) to a small residual."""
    rng = np.random.default_rng(5)
    widths = (4, 16, 16, 16, 3)
    B = rng.standard_normal((4, 3))
    x = rng.standard_normal((256, 4))
    t = x @ B
    p = mlp.init_params(6, widths)
    m = np.zeros_like(p)
    v = np.zeros_like(p)
    loss0 = mlp.mse(mlp.forward(p, x, widths)[0], t)
    for k in range(1, 1501):
        loss, g = mlp.backward(p, x, t, widths)
        mlp.adam_step(p, g, m, v, k, 3e-3)
    assert loss < 1e-2 * loss0


def test_round_bf16_definition():
    # exactly representable values stay; halfway cases go to even; 8 significant bits
    assert mlp.round_bf16(1.0) == 1.0 and mlp.round_bf16(-3.0) == -3.0
    assert mlp.round_bf16(1.0 + 2.0 ** -8) == 1.0                       # tie, even mantissa below
    assert mlp.round_bf16(1.0 + 3 * 2.0 ** -8) == 1.0 + 2.0 ** -6      # tie, rounds up to even
    assert mlp.round_bf16(1.0 + 2.0 ** -8 + 2.0 ** -12) == 1.0 + 2.0 ** -7
    x = np.random.default_rng(2).standard_normal(1000) * 100
    r = mlp.round_bf16(x)
    assert np.all(np.abs(r - x) <= np.abs(x) * 2.0 ** -8)


def test_deformation_of_semi_axes():
    assert mlp.deformation([3.0, 2.0, 1.0]) == pytest.approx(0.5)
    assert mlp.deformation([[1.0, 1.0, 1.0]])[0] == 0.0


def test_cubic_symmetries_form_the_octahedral_group():
    Ps = [mlp.cubic_symmetry(s) for s in range(48)]
    assert np.array_equal(Ps[0], np.eye(3))
    keys = {P.tobytes() for P in Ps}
    assert len(keys) == 48
    for P in Ps:
        assert np.array_equal(P @ P.T, np.eye(3)) and np.all(np.abs(P).sum(0) == 1)
    for P in Ps[::5]:
        for Q in Ps[::7]:
            assert (P @ Q).tobytes() in keys
    # the conjugation keeps the eigenvalues of the strain (the shape-relevant invariants)
    A = np.random.default_rng(0).standard_normal(9)
    w = mlp.transform_window(A, 29).reshape(3, 3)
    S, S2 = 0.5 * (A.reshape(3, 3) + A.reshape(3, 3).T), 0.5 * (w + w.T)
    assert np.allclose(np.linalg.eigvalsh(S), np.linalg.eigvalsh(S2), atol=1e-14)
