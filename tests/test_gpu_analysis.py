"""GPU parity of the droplet analysis calls against the FP64 oracle: the surface
area / enclosed volume behind D_LBM (Sec. 5 Eq. 17), the droplet mass and the
mass reinjection (Sec. 2), through the C ABI."""
import numpy as np
import pytest

import oracle
from paper_2112_09972_amd import workloads as wl

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sc():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2112_09972_amd as sc
    sc.load()
    return sc


def pair(sc, n, R, A, steps, prec="f64", nxyz=None):
    nx, ny, nz = nxyz or (n, n, n)
    rho_b = wl.ghost_densities(R)
    lat = sc.Lattice(nx, ny, nz, bc="ghost", prec=prec, table_len=max(steps, 1), g_ab=wl.G_AB, rho_b=rho_b)
    o = oracle.Oracle(nx, ny, nz, periodic=False, g=wl.G_AB, rho_b=rho_b)
    lat.init_droplet(lat.xc, R, wl.WIDTH, wl.RHO_HI, wl.RHO_LO, A)
    o.init_droplet(o.xc, R, wl.WIDTH, wl.RHO_HI, wl.RHO_LO, A)
    if steps:
        tab = np.tile(A, (steps, 1))
        lat.set_gradient_table(tab, 0)
        lat.step(steps)
        o.run(steps, tab)
    return lat, o


def test_surface_of_linear_field_is_exact(sc):
    """rho_A - rho_B linear (a tilted plane): the GPU area and volume are exact,
    on a box whose x and y sizes are ragged against the 16-cell tiles."""
    nx, ny, nz = 37, 21, 14
    a, b, z0 = 0.15, -0.1, 6.5          # the plane stays inside 0 < z < nz - 1
    cx, cy = (nx - 1) / 2, (ny - 1) / 2
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    phi = z0 + a * (x - cx) + b * (y - cy) - z
    lat = sc.Lattice(nx, ny, nz, bc="periodic", prec="f64", g_ab=0.0, rho_b=(1.0, 1.0))
    lat.init_fields(1.0 + 0.01 * phi, np.ones(lat.shape))
    assert phi.max() < z0 + 4 and phi[-1].max() < 0 and phi[0].min() > 0
    area, vol, _ = lat.droplet_surface()
    assert area == pytest.approx((nx - 1) * (ny - 1) * np.sqrt(1 + a * a + b * b), rel=1e-12)
    assert vol == pytest.approx((nx - 1) * (ny - 1) * z0, rel=1e-12)


@pytest.mark.parametrize("nxyz", [(32, 32, 32), (45, 19, 23)])
def test_surface_and_mass_match_oracle(sc, nxyz):
    A = wl.simple_shear(wl.shear_rate_for_ca(0.1, 6.0))
    lat, o = pair(sc, None, 6.0, A, 300, nxyz=nxyz)
    area, vol, d = lat.droplet_surface()
    ra, rb, _ = o.fields()
    ao, vo = oracle.droplet_surface(ra, rb)
    print("area %.10g vs %.10g, volume %.10g vs %.10g, D_LBM %.5f" % (area, ao, vol, vo, d))
    assert area == pytest.approx(ao, rel=1e-10)
    assert vol == pytest.approx(vo, rel=1e-10)
    assert d == pytest.approx(oracle.deformation_lbm(ao, vo), abs=1e-8)
    assert lat.droplet_mass()[0] == pytest.approx(o.droplet_mass(), rel=1e-12)


def test_reinjection_matches_oracle(sc):
    A = wl.simple_shear(wl.shear_rate_for_ca(0.1, 6.0))
    lat, o = pair(sc, 28, 6.0, A, 200)
    target = 1.03 * o.droplet_mass()
    lat.reinject([target])
    o.reinject(target)
    assert lat.droplet_mass()[0] == pytest.approx(target, rel=1e-12)
    tab = np.tile(A, (100, 1))
    lat.set_gradient_table(tab, 200)
    lat.step(100)
    o.run(100, tab)
    ra, rb, _ = (t.cpu().numpy() for t in lat.fields())
    oa, ob, _ = o.fields()
    err = max(np.max(np.abs(ra - oa) / oa), np.max(np.abs(rb - ob) / ob))
    print("after reinjection + 100 steps: max rel density error %.2e" % err)
    assert err <= 1e-11


@pytest.mark.parametrize("prec,tol", [("f32", 1e-6), ("f16dev", 2e-3), ("bf16dev", 2e-3)])
def test_reinjection_per_box_all_formats(sc, prec, tol):
    """Three boxes, one target each; every format reaches its target within its
    storage rounding (FP16 reference densities for the deviation formats)."""
    n, R, steps = 24, 5.0, 100
    tabs = [wl.ou_gradient_table(40 + b, n, steps, mach=0.1) for b in range(3)]
    lat = sc.Lattice(n, n, n, nbox=3, bc="ghost", prec=prec, table_len=steps, g_ab=wl.G_AB,
                     rho_b=wl.ghost_densities(R))
    for b in range(3):
        lat.init_droplet(lat.xc, R, wl.WIDTH, wl.RHO_HI, wl.RHO_LO, tabs[b][0], box=b)
        lat.set_gradient_table(tabs[b], 0, box=b)
    lat.step(steps)
    m0 = lat.droplet_mass()
    target = m0 * np.array([1.02, 1.04, 1.01])
    lat.reinject(target)
    m1 = lat.droplet_mass()
    print(prec, "mass", m0, "->", m1, "target", target)
    assert np.all(np.abs(m1 / target - 1) <= tol)
    # one box alone
    lat.reinject([1.01 * m1[1]], box=1)
    m2 = lat.droplet_mass()
    assert m2[1] == pytest.approx(1.01 * m1[1], rel=tol)
    assert m2[0] == m1[0] and m2[2] == m1[2]


def test_analysis_errors(sc):
    lat, _ = pair(sc, 16, 4.0, None, 0)
    with pytest.raises(sc.SclbmError):
        lat.reinject([-1.0])
    with pytest.raises(sc.SclbmError):
        lat.reinject([1.0], box=3)
    with pytest.raises(sc.SclbmError):
        sc.sclbm_deformation_lbm(0.0, 1.0)
