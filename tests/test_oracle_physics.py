"""Physics pins of the oracle (no GPU): invariants and laws that the model of
Sec. 2 must satisfy whatever the implementation.

* Stationarity: a uniform state outside the spinodal stays put (periodic box at
  rest and in uniform motion, ghost box with A = 0).
* Conservation: in a periodic box each component's mass and the total momentum
  are constant (the pair form of Sec. 2 Eq. 7 makes the total force vanish).
* Symmetry: the centred droplet in a linear flow is symmetric under x -> (L-1) - x,
  its centre of mass stays at the box centre (Sec. 3), and at rest the lattice's
  cubic symmetry leaves it undeformed.
* Viscosity: a decaying shear wave decays at nu k^2 with nu = (tau - 1/2)/3
  (Sec. 2 Eq. 10).
* Flat interface: in the regime where the velocity-shift forcing error is small
  (tau = 3) the coexisting densities satisfy the mean-field condition
  ln(a/b) = G (a - b) of the psi = rho model.
* Laplace law: the pressure jump across static droplets is linear in 1/R with
  vanishing intercept.
* Boundary: a single-phase box driven only by its ghost nodes relaxes to the
  imposed linear flow with global error E0 < 0.1 (Sec. 4 Eq. 16 and the acceptance
  level the paper uses there).
* Taylor law: in steady simple shear at viscosity ratio 1 the droplet deforms as
  D = (35/32) Ca for small Ca.
* Ellipsoid moments: the sharp indicator of an ellipsoid returns its semi-axes.
"""
import numpy as np
import pytest

import oracle


def uniform_state(o, ra, rb, u):
    o.init_fields(np.full(o.shape, ra), np.full(o.shape, rb), np.asarray(u, float))


@pytest.mark.parametrize("periodic,u", [(True, (0.0, 0.0, 0.0)), (True, (0.05, -0.02, 0.03)),
                                        (False, (0.0, 0.0, 0.0))])
def test_uniform_state_is_stationary(calibration, periodic, u):
    G = calibration["g_ab"]
    o = oracle.Oracle(8, 7, 6, periodic=periodic, tau=(1.0, 1.0), g=G, rho_b=(0.04, 1.0))
    uniform_state(o, 0.04, 1.0, u)
    f0 = o.get_f()
    o.run(500, np.zeros((500, 9)))
    assert np.abs(o.get_f() - f0).max() <= 1e-14


def test_periodic_droplet_conserves_mass_and_momentum(calibration):
    G = calibration["g_ab"]
    n = 20
    o = oracle.Oracle(n, n, n, periodic=True, tau=(1.0, 1.0), g=G, rho_b=(0.04, 1.0))
    o.init_droplet([(n - 1) / 2.0] * 3, 5.0, 2.0, 1.0, 0.04, None)
    m0, p0 = o.totals()
    for _ in range(4):
        o.run(250)
        m, p = o.totals()
        assert np.all(np.abs(m - m0) / m0 <= 1e-13)
        assert np.abs(p).max() / m0.sum() <= 1e-13
    # the droplet has not dissolved: it is still a droplet
    ra, rb, _ = o.fields()
    assert ra.max() > 0.9 and ra.min() < 0.08


def test_moving_droplet_conserves_momentum(calibration):
    """A periodic droplet in uniform motion keeps its total momentum."""
    G = calibration["g_ab"]
    n = 16
    o = oracle.Oracle(n, n, n, periodic=True, tau=(1.0, 1.0), g=G, rho_b=(0.04, 1.0))
    ctr = [(n - 1) / 2.0] * 3
    z, y, x = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    r = np.sqrt((x - ctr[0]) ** 2 + (y - ctr[1]) ** 2 + (z - ctr[2]) ** 2)
    ra = 0.52 - 0.48 * np.tanh((r - 4.0) / 2.0)
    o.init_fields(ra, 1.04 - ra, np.array([0.02, -0.01, 0.005]))
    m0, p0 = o.totals()
    o.run(300)
    m, p = o.totals()
    assert np.all(np.abs(m - m0) / m0 <= 1e-13)
    assert np.abs(p - p0).max() / m0.sum() <= 1e-13


def test_point_symmetry_under_linear_flow(calibration):
    G = calibration["g_ab"]
    sigma = calibration["sigma"]
    n, R = 24, 5.0
    eta = 1.04 * (1.0 - 0.5) / 3.0
    gamma = 0.1 * sigma / (eta * R)
    A = np.zeros(9)
    A[2] = gamma  # u = (gamma z, 0, 0)
    o = oracle.Oracle(n, n, n, periodic=False, tau=(1.0, 1.0), g=G, rho_b=(0.04, 1.0))
    o.init_droplet(o.xc, R, 2.0, 1.0, 0.04, A)
    o.run(300, np.tile(A, (300, 1)))
    ra, rb, u = o.fields()
    inv = lambda a: a[::-1, ::-1, ::-1]
    assert np.abs(ra - inv(ra)).max() < 1e-12
    assert np.abs(rb - inv(rb)).max() < 1e-12
    assert np.abs(u + u[:, ::-1, ::-1, ::-1]).max() < 1e-12  # velocity is odd
    st = oracle.droplet_stats(ra, rb, o.xc)
    assert np.abs(st["com"] - o.xc).max() < 1e-12
    # mirror y -> (L-1) - y leaves simple shear in the xz plane invariant
    assert np.abs(ra - ra[:, ::-1, :]).max() < 1e-12
    # the shear deforms it
    assert st["deformation"] > 1e-3


def cubic_map_field(F_zyx, P):
    """The scalar field F(x) carried along by d -> P d about the box centre
    (d = x - x_c; F indexed [z][y][x]; P a signed permutation)."""
    F = np.transpose(F_zyx, (2, 1, 0))                       # [x][y][z]
    perm = [int(np.nonzero(P[i])[0][0]) for i in range(3)]
    T = np.transpose(F, perm)
    for i in range(3):
        if P[i, perm[i]] < 0:
            T = np.flip(T, axis=i)
    return np.transpose(T, (2, 1, 0))


@pytest.mark.parametrize("s", [13, 29, 46])
def test_box_is_invariant_under_cubic_symmetries(calibration, s):
    """Driving the box with P A P^T (P a signed permutation of the axes, about the
    centre) gives the density field carried along by P, and the same semi-axes:
    the cube, the D3Q19 velocity set, the centred droplet and the ghost velocity
    A (x - x_c) all map onto themselves.  (This is what makes the 48 maps exact
    augmentations of the surrogate's training windows.)"""
    from oracle import mlp
    G = calibration["g_ab"]
    n, R, steps = 14, 3.5, 30
    A = np.array([0.004, -0.002, 0.003, 0.001, -0.003, 0.0025, -0.0015, 0.002, -0.001])
    P = mlp.cubic_symmetry(s)
    A2 = mlp.transform_window(A, s)
    out = []
    for a in (A, A2):
        o = oracle.Oracle(n, n, n, periodic=False, tau=(1.0, 1.0), g=G, rho_b=(0.05, 1.0))
        o.init_droplet(o.xc, R, 2.0, 1.0, 0.04, a)
        o.run(steps, np.tile(a, (steps, 1)))
        out.append(o.fields())
    (ra, rb, _), (ra2, rb2, _) = out
    assert np.abs(cubic_map_field(ra, P) - ra2).max() < 1e-13
    assert np.abs(cubic_map_field(rb, P) - rb2).max() < 1e-13
    xc = np.full(3, (n - 1) / 2.0)
    a1 = oracle.droplet_stats(ra, rb, xc)["semi_axes"]
    a2 = oracle.droplet_stats(ra2, rb2, xc)["semi_axes"]
    assert np.allclose(a1, a2, rtol=1e-12)
    assert np.abs(ra - ra2).max() > 1e-6          # the map is not trivial for this drive


def test_droplet_at_rest_stays_spherical(calibration):
    G = calibration["g_ab"]
    n = 20
    o = oracle.Oracle(n, n, n, periodic=True, tau=(1.0, 1.0), g=G, rho_b=(0.04, 1.0))
    o.init_droplet(o.xc, 5.0, 2.0, 1.0, 0.04, None)
    o.run(200)
    ra, rb, _ = o.fields()
    st = oracle.droplet_stats(ra, rb, o.xc)
    assert st["deformation"] <= 1e-12
    # the three diagonal second moments are equal by the lattice's cubic symmetry
    d = np.diag(st["cov"])
    assert np.abs(d - d.mean()).max() < 1e-11


@pytest.mark.parametrize("tau", [0.8, 1.0, 1.7])
def test_shear_wave_decay_gives_viscosity(tau):
    """u_x(z, t) = U sin(k z) exp(-nu k^2 t) with nu = (tau - 1/2)/3, Sec. 2 Eq. 10."""
    L = 64
    o = oracle.Oracle(1, 1, L, periodic=True, tau=(tau, tau), g=0.0, rho_b=(0.5, 0.5))
    k = 2 * np.pi / L
    z = np.arange(L)
    U = 1e-4
    u = np.zeros((3, L, 1, 1))
    u[0, :, 0, 0] = U * np.sin(k * z)
    o.init_fields(np.full(o.shape, 0.5), np.full(o.shape, 0.5), u)
    t0 = 50  # let the initial non-equilibrium part settle
    o.run(t0)
    a0 = np.dot(o.fields()[2][0, :, 0, 0], np.sin(k * z))
    nu = (tau - 0.5) / 3.0
    T = int(0.7 / (nu * k * k))
    o.run(T)
    a1 = np.dot(o.fields()[2][0, :, 0, 0], np.sin(k * z))
    nu_measured = -np.log(a1 / a0) / (k * k * T)
    nu = (tau - 0.5) / 3.0
    assert abs(nu_measured - nu) / nu < 5e-3


def test_flat_interface_mean_field_coexistence():
    """tau = 3, G = 2.4: ln(a/b) = G (a - b) within 3 %."""
    import importlib.util, os
    spec = importlib.util.spec_from_file_location(
        "calib", os.path.join(os.path.dirname(__file__), "golden", "calibrate.py"))
    cal = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(cal)
    G = 2.4
    a, b, umax = cal.slab_coexistence(G, tau=3.0, steps=40000)
    g_mf = np.log(a / b) / (a - b)
    assert abs(g_mf - G) / G < 0.03
    assert umax < 1e-10


def test_calibrated_coupling_gives_target_ratio(calibration):
    import importlib.util, os
    spec = importlib.util.spec_from_file_location(
        "calib", os.path.join(os.path.dirname(__file__), "golden", "calibrate.py"))
    cal = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(cal)
    a, b, umax = cal.slab_coexistence(calibration["g_ab"])
    assert abs(b / a - 0.04) < 1e-3
    assert umax < 1e-10


def test_laplace_law(calibration):
    G = calibration["g_ab"]
    L, steps = 28, 2000
    pts = []
    for R in (5.0, 6.0, 7.0, 8.0):
        o = oracle.Oracle(L, L, L, periodic=True, tau=(1.0, 1.0), g=G, rho_b=(0.04, 1.0))
        o.init_droplet(o.xc, R, 2.0, 1.0, 0.04, None)
        o.run(steps)
        ra, rb, _ = o.fields()
        st = oracle.droplet_stats(ra, rb, o.xc)
        c = L // 2
        dp = oracle.bulk_pressure(ra[c, c, c], rb[c, c, c], G) - oracle.bulk_pressure(ra[0, 0, 0], rb[0, 0, 0], G)
        pts.append((1.0 / st["r_eq"], dp))
    x, y = np.array(pts).T
    slope, icpt = np.polyfit(x, y, 1)
    r2 = 1 - np.sum((y - (slope * x + icpt)) ** 2) / np.sum((y - y.mean()) ** 2)
    assert r2 > 0.99
    assert abs(icpt) < 0.1 * y.min()
    assert abs(slope / 2.0 - calibration["sigma"]) / calibration["sigma"] < 0.1


def test_ghost_boundary_relaxes_to_linear_flow():
    """Single phase (G = 0), fluid at rest, simple shear imposed only through the
    ghost nodes of a box of the paper's validation size L_s = 48 at tau = 1 with
    the velocity scale u_LBM = L_s ||G||_inf = 0.1 (Table 1, Sec. 4 Eq. 15): the
    global error E0 of Sec. 4 Eq. 16 falls below the paper's acceptance level 0.1
    within 500 steps and keeps falling (below 0.01 at 1000 steps; the linear
    profile with equilibrium ghosts is a steady state of the scheme)."""
    L = 48
    gamma = 0.1 / L
    A = np.zeros(9)
    A[2] = gamma
    o = oracle.Oracle(L, L, L, periodic=False, tau=(1.0, 1.0), g=0.0, rho_b=(0.5, 0.5))
    o.init_fields(np.full(o.shape, 0.5), np.full(o.shape, 0.5))
    errs = [oracle.velocity_error(o.fields()[2], A, o.xc)]
    for _ in range(2):
        o.run(500, np.tile(A, (500, 1)))
        errs.append(oracle.velocity_error(o.fields()[2], A, o.xc))
    assert errs[0] > 0.99  # at rest: E0 = 1
    assert errs[1] < 0.1
    assert errs[2] < 0.01
    # a wrong-signed boundary would drive the opposite flow: E0 near 2
    assert oracle.velocity_error(-o.fields()[2], A, o.xc) > 1.5


def far_field(calibration, R):
    a = calibration["far_field_a"]
    b = calibration["far_field_b"]
    return (a[0] / R + a[1], b[0] / R + b[1])


def test_taylor_deformation(calibration):
    """Steady simple shear at viscosity ratio 1, Ca = 0.025, 0.05, 0.1: D = (35/32) Ca
    for an unbounded droplet, raised by the confinement of the driven boundary.
    The closed form of Shapira and Haber for a droplet midway between two plates a
    distance h from its centre, D = (35/32) Ca [1 + C_s (1 + 5 chi / 2)/(1 + chi)
    (R/h)^3] with C_s = 5.6996, is first order in Ca: the slope of D against Ca
    over the two smaller Ca (least squares through the origin) matches it within
    10 %, every Ca within 20 %, and at Ca = 0.1 D lies above the linear law (the
    second-order growth of the deformation)."""
    G = calibration["g_ab"]
    sigma = calibration["sigma"]
    L, R = 48, 8.0
    eta = 1.04 * (1.0 - 0.5) / 3.0
    h, chi = L / 2.0, 1.0
    cas, Ds, preds = (0.025, 0.05, 0.1), [], []
    for Ca in cas:
        gamma = Ca * sigma / (eta * R)
        A = np.zeros(9)
        A[2] = gamma
        o = oracle.Oracle(L, L, L, periodic=False, tau=(1.0, 1.0), g=G, rho_b=far_field(calibration, R))
        o.init_droplet(o.xc, R, 2.0, 1.0, 0.04, A)
        D = []
        for steps in (750, 250):
            o.run(steps, np.tile(A, (steps, 1)))
            ra, rb, _ = o.fields()
            st = oracle.droplet_stats(ra, rb, o.xc)
            D.append(st["deformation"])
        assert abs(D[1] - D[0]) < 0.05 * D[1], (Ca, D)  # steady
        Ds.append(D[1])
        preds.append(35.0 / 32.0 * Ca * (1.0 + 5.6996 * (1 + 2.5 * chi) / (1 + chi) * (st["r_eq"] / h) ** 3))
    cas, Ds, preds = np.array(cas), np.array(Ds), np.array(preds)
    slope = np.dot(cas[:2], Ds[:2]) / np.dot(cas[:2], cas[:2])
    slope_pred = np.mean(preds[:2] / cas[:2])
    print("D", Ds, "D/Ca", Ds / cas, "slope %.4f against %.4f" % (slope, slope_pred))
    assert abs(slope / slope_pred - 1.0) < 0.10
    assert np.all(np.abs(Ds / preds - 1.0) < 0.20)
    assert Ds[2] > slope * cas[2]
    # well above the unbounded value for this confined box
    assert np.all(Ds > 35.0 / 32.0 * cas)


@pytest.mark.parametrize("axes,rot", [((10.0, 8.0, 6.0), False), ((9.0, 7.0, 5.0), True)])
def test_sharp_ellipsoid_semi_axes(axes, rot):
    n = 40
    c = np.array([(n - 1) / 2.0] * 3)
    z, y, x = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    d = np.stack([x - c[0], y - c[1], z - c[2]]).reshape(3, -1)
    if rot:
        th = np.pi / 5
        Rm = np.array([[np.cos(th), -np.sin(th), 0], [np.sin(th), np.cos(th), 0], [0, 0, 1]])
        d = Rm.T @ d
    inside = (d[0] / axes[0]) ** 2 + (d[1] / axes[1]) ** 2 + (d[2] / axes[2]) ** 2 < 1.0
    ra = np.where(inside, 1.0, 0.04).reshape(n, n, n)
    rb = 1.04 - ra
    st = oracle.droplet_stats(ra, rb, c)
    assert np.allclose(st["semi_axes"], axes, rtol=0.015)
    vol = 4 / 3 * np.pi * np.prod(axes)
    assert abs(st["volume"] - vol) / vol < 0.02
    D = (axes[0] - axes[2]) / (axes[0] + axes[2])
    assert abs(st["deformation"] - D) < 0.01
