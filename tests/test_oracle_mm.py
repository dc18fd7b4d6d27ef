"""Pins of the FP64 Maffettone-Minale reference (oracle/mm.py), Sec. 2 Eqs. 1, 2, 5.

* Small-Ca steady simple shear reproduces Taylor's D = (35/32) Ca at chi = 1
  (the linearised steady state is D = f2 Ca / (2 f1) and f2/(2 f1) = 35/32).
* The volume det M = 1 is conserved (the strain term is traceless, the
  rotation term commutes out, the relaxation term is built to keep it).
* A pure rotation leaves the sphere a sphere, and a rotated ellipsoid keeps
  its semi-axes.
* The coefficients of Eq. 5 at chi = 1: f1 = 16/35, f2(Ca = 0) = 1.
* The sense of rotation: under a pure rotation M(t) = e^{Wt} M0 e^{Wt}^T entry by
  entry, and the steady simple-shear droplet points into the extensional
  quadrant at theta = atan(f1/Ca)/2 from the flow direction.  Both fail when the
  vorticity term's sign is flipped or A is taken transposed.
"""
import numpy as np
import pytest

from oracle import mm


def test_coefficients():
    assert abs(mm.f1(1.0) - 16.0 / 35.0) < 1e-15
    assert mm.f2(1.0, 0.0) == 1.0
    assert abs(mm.f2(1.0, 1e6) - 1.5) < 1e-9


def test_small_ca_steady_shear_is_taylor():
    tau_d = 50.0
    for ca in (0.002, 0.005):
        gamma = ca / tau_d
        A = np.zeros((3, 3))
        A[0, 2] = gamma
        rows = np.tile(A, (2001, 1, 1))
        Ms = mm.integrate(rows, tau_d, 1.0, substeps=1, record_every=2000)
        D = mm.deformation(Ms[-1])
        assert abs(D / ca - 35.0 / 32.0) < 0.01, D / ca


def test_moderate_ca_steady_shear():
    """Full MM steady state at Ca = 0.1, chi = 1: D = 0.1097 (numerically converged)."""
    tau_d = 40.0
    A = np.zeros((3, 3))
    A[0, 2] = 0.1 / tau_d
    Ms = mm.integrate(np.tile(A, (3001, 1, 1)), tau_d, 1.0, record_every=1000)
    D = mm.deformation(Ms[-1])
    assert abs(D - 0.1097) < 5e-4
    assert abs(mm.deformation(Ms[-2]) - D) < 1e-6  # steady


def test_volume_conserved_and_rotation_invariance():
    # smooth traceless drive: det M = 1 is an invariant of the ODE, so its drift is
    # pure RK4 truncation error and falls ~16x when the step is halved
    t = np.arange(801)[:, None, None]
    rng = np.random.default_rng(4)
    amp, ph = rng.normal(size=(3, 3)) * 0.01, rng.uniform(0, 6.28, size=(3, 3))
    rows = amp * np.sin(2 * np.pi * t / 300.0 + ph)
    rows -= np.trace(rows, axis1=1, axis2=2)[:, None, None] * np.eye(3) / 3.0
    errs = []
    for sub in (1, 2):
        Ms = mm.integrate(rows, 30.0, 1.0, substeps=sub)
        errs.append(max(abs(np.linalg.det(M) - 1.0) for M in Ms))
    assert errs[1] < errs[0] / 8 and errs[1] < 1e-8, errs
    # pure rotation: sphere stays a sphere
    W = np.array([[0, -0.01, 0.003], [0.01, 0, -0.002], [-0.003, 0.002, 0]])
    Ms = mm.integrate(np.tile(W, (500, 1, 1)), 30.0, 1.0)
    assert np.abs(Ms[-1] - np.eye(3)).max() < 1e-12
    # rotating a deformed droplet keeps its semi-axes (relaxation off: large tau_d)
    M0 = np.diag([1.2, 1.0, 1.0 / 1.2])
    Ms = mm.integrate(np.tile(W, (300, 1, 1)), 1e12, 1.0, M0=M0)
    assert np.allclose(np.sort(np.linalg.eigvalsh(Ms[-1])), np.sort(np.diag(M0)), atol=1e-9)


def test_pure_rotation_rotates_the_tensor():
    """With relaxation off (tau_d -> infinity) and A = W antisymmetric, Eq. 1 reduces
    to dM/dt = W M - M W, whose solution is M(t) = e^{W t} M0 e^{W t}^T: entry by
    entry, not only in the eigenvalues, so the sense of rotation is fixed (a
    sign error in the vorticity term, or A taken transposed, rotates the other
    way)."""
    from scipy.linalg import expm
    W = np.array([[0.0, -0.012, 0.004], [0.012, 0.0, -0.003], [-0.004, 0.003, 0.0]])
    M0 = np.array([[1.3, 0.1, 0.0], [0.1, 0.9, 0.05], [0.0, 0.05, 1.0 / (1.3 * 0.9)]])
    t = 300
    Ms = mm.integrate(np.tile(W, (t + 1, 1, 1)), 1e12, 1.0, M0=M0)
    R = expm(W * t)
    exact = R @ M0 @ R.T
    assert np.abs(Ms[-1] - exact).max() < 1e-8
    wrong = R.T @ M0 @ R
    assert np.abs(Ms[-1] - wrong).max() > 0.05


@pytest.mark.parametrize("ca", [0.005, 0.02, 0.1, 0.3])
def test_steady_shear_orientation(ca):
    """Simple shear u = (gamma z, 0, 0): linearising Eq. 1 about the sphere gives a
    steady M - I in the x-z plane whose major axis makes the angle
    theta = atan(f1 / Ca) / 2 with the flow direction x, towards +z (the
    extensional quadrant): 45 degrees as Ca -> 0, turning towards x as Ca grows.
    The full model keeps this angle to round-off at every Ca tested (the
    relaxation term and the Ca-dependence of f2 do not turn the axes).  Reversed
    vorticity, or A taken transposed, puts the axis at 90 degrees - theta."""
    tau_d = 40.0
    A = np.zeros((3, 3))
    A[0, 2] = ca / tau_d
    Ms = mm.integrate(np.tile(A, (4001, 1, 1)), tau_d, 1.0, record_every=4000)
    lam, vec = np.linalg.eigh(Ms[-1])
    v = vec[:, -1]
    assert abs(v[1]) < 1e-9
    assert v[0] * v[2] > 0
    theta = np.degrees(np.arctan2(abs(v[2]), abs(v[0])))
    pred = np.degrees(0.5 * np.arctan(mm.f1(1.0) / ca))
    assert abs(theta - pred) < 1e-6, (theta, pred)
    assert theta < 45.0
