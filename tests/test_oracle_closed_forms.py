"""Pins of the oracle's building blocks against closed forms (no GPU).

* D3Q19 stencil moments: sum w = 1, sum w c_a c_b = delta_ab / 3, fourth moments
  1/3 and 1/9 (the isotropy that makes c_s^2 = 1/3 consistent with the 3, 9/2, 3/2
  coefficients of Sec. 2 Eq. 8).
* Equilibrium of Sec. 2 Eq. 8: zeroth, first and second moments equal rho,
  rho u and rho c_s^2 I + rho u u exactly.
* The force of Sec. 2 Eq. 7 on a quadratic density field equals
  -G rho_s c_s^2 grad rho_s' exactly (the stencil's odd moments vanish and its
  second moment is c_s^2 I), and the total force on a periodic box vanishes.
* The numpy transcription (oracle/tiny_ref.py) and the C oracle agree on tiny
  boxes in both boundary modes.
"""
import numpy as np
import pytest

import oracle
from oracle import tiny_ref


def test_stencil_moments():
    c, w = oracle.stencil()
    assert c.shape == (19, 3)
    assert len({tuple(v) for v in c}) == 19
    assert np.all(np.sum(c * c, axis=1) <= 2)
    assert abs(w.sum() - 1.0) < 1e-15
    second = np.einsum("i,ia,ib->ab", w, c, c)
    assert np.allclose(second, np.eye(3) / 3.0, atol=1e-15, rtol=0)
    assert np.allclose(np.einsum("i,ia->a", w, c), 0.0, atol=1e-16)
    assert abs(np.sum(w * c[:, 0] ** 4) - 1.0 / 3.0) < 1e-15
    assert abs(np.sum(w * c[:, 0] ** 2 * c[:, 1] ** 2) - 1.0 / 9.0) < 1e-15
    third = np.einsum("i,ia,ib,ic->abc", w, c, c, c)
    assert np.abs(third).max() < 1e-16


@pytest.mark.parametrize("rho,u", [(1.0, (0.0, 0.0, 0.0)), (0.04, (0.05, -0.02, 0.03)),
                                   (1.3, (-0.1, 0.07, 0.02))])
def test_equilibrium_moments(rho, u):
    c, w = oracle.stencil()
    u = np.array(u)
    g = oracle.equilibrium(rho, u)
    assert abs(g.sum() - rho) < 1e-15 * max(1, rho) * 4
    assert np.allclose(g @ c, rho * u, atol=1e-15, rtol=0)
    P = np.einsum("i,ia,ib->ab", g, c, c)
    assert np.allclose(P, rho * np.eye(3) / 3.0 + rho * np.outer(u, u), atol=2e-15, rtol=0)
    # the weights: g at u = 0 is w rho
    g0 = oracle.equilibrium(rho, np.zeros(3))
    assert np.allclose(g0, w * rho, atol=1e-16, rtol=0)


def test_force_quadratic_field_closed_form():
    """Eq. 7 on rho_B quadratic in x: F_A = -G rho_A c_s^2 grad rho_B exactly."""
    n = 8
    G = 1.7
    o = oracle.Oracle(n, n, n, periodic=False, tau=(1.0, 1.0), g=G, rho_b=(0.5, 0.5))
    z, y, x = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    ra = 0.3 + 0.01 * x + 0.02 * y * y / n
    rb = 0.4 + 0.015 * z + 0.01 * x * y / n - 0.005 * z * z / n
    o.init_fields(ra, rb)
    fa, fb, u, F = o.fields(with_force=True)
    assert np.allclose(fa, ra, atol=1e-15) and np.allclose(fb, rb, atol=1e-15)
    grad_b = np.stack([0.01 * y / n, 0.01 * x / n, 0.015 - 0.01 * z / n])
    grad_a = np.stack([0.01 + 0 * x, 0.04 * y / n, 0 * z])
    inner = (slice(1, n - 1),) * 3  # away from the ghost layer
    FA = -G * ra * grad_b / 3.0
    FB = -G * rb * grad_a / 3.0
    assert np.abs(F[0][(slice(None),) + inner] - FA[(slice(None),) + inner]).max() < 1e-15
    assert np.abs(F[1][(slice(None),) + inner] - FB[(slice(None),) + inner]).max() < 1e-15


def test_force_sums_to_zero_periodic():
    rng = np.random.default_rng(5)
    n = 6
    o = oracle.Oracle(n, n + 1, n + 2, periodic=True, tau=(1.0, 1.0), g=1.64, rho_b=(0.04, 1.0))
    ra = rng.uniform(0.04, 1.0, size=o.shape)
    rb = rng.uniform(0.04, 1.0, size=o.shape)
    o.init_fields(ra, rb)
    _, _, _, F = o.fields(with_force=True)
    tot = F.sum(axis=(2, 3, 4)).sum(axis=0)
    scale = np.abs(F).sum()
    assert np.all(np.abs(tot) < 1e-15 * scale + 1e-16)
    # the pair form: component forces are not separately zero
    assert np.abs(F[0].sum(axis=(1, 2, 3))).max() > 1e-6


@pytest.mark.parametrize("periodic", [True, False])
def test_numpy_transcription_agrees(periodic):
    rng = np.random.default_rng(11 if periodic else 12)
    shape = (5, 6, 7)  # (z, y, x)
    G = 1.64
    tau = (1.0, 0.8)
    rho_b = (0.04, 1.0)
    o = oracle.Oracle(shape[2], shape[1], shape[0], periodic=periodic, tau=tau, g=G, rho_b=rho_b)
    t = tiny_ref.TinyLBM(shape, periodic, tau, G, rho_b)
    ra = rng.uniform(0.04, 1.0, size=shape)
    rb = 1.04 - ra
    u = rng.uniform(-0.03, 0.03, size=(3,) + shape)
    o.init_fields(ra, rb, u)
    t.init(ra, rb, u)
    A = np.array([[0.001, 0.0, 0.004], [0.0, -0.002, 0.0], [0.0015, 0.0, 0.001]])
    for _ in range(10):
        o.step(A)
        t.step(A)
    a1, b1, u1 = o.fields()
    a2, b2, u2 = t.fields()
    assert np.abs(a1 - a2).max() < 1e-13
    assert np.abs(b1 - b2).max() < 1e-13
    assert np.abs(u1 - u2).max() < 1e-13


def test_velocity_error_closed_forms():
    n = 8
    A = np.array([[0, 0, 0.01], [0, 0, 0], [0, 0, 0]], float)
    xc = np.array([(n - 1) / 2] * 3)
    z, y, x = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    d = np.stack([x - xc[0], y - xc[1], z - xc[2]])
    u_exact = np.einsum("ab,bzyx->azyx", A, d)
    assert oracle.velocity_error(u_exact, A, xc) == 0.0
    assert abs(oracle.velocity_error(np.zeros_like(u_exact), A, xc) - 1.0) < 1e-15
    assert abs(oracle.velocity_error(2 * u_exact, A, xc) - 1.0) < 1e-15
