"""GPU checks of the boundary calls that set up and guard a run: a constant
velocity gradient, a uniform initial state and the health check of the step
calls (through the C ABI)."""
import numpy as np
import pytest

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


def lattice(sc, n=20, nbox=1, steps=30, prec="f64", bc="ghost"):
    return sc.Lattice(n, n, n, nbox=nbox, bc=bc, prec=prec, table_len=steps, g_ab=wl.G_AB,
                      rho_b=wl.ghost_densities(5.0), mach_max=0.2)


def test_constant_gradient_equals_table(sc):
    """sclbm_set_gradient(A) gives the same bits as the table of A repeated, from
    the current time on, for one box and for every box at once."""
    A = wl.simple_shear(wl.shear_rate_for_ca(0.05, 5.0))
    out = []
    for how in ("table", "one", "all"):
        lat = lattice(sc, nbox=2)
        lat.init_droplet(lat.xc, 5.0, wl.WIDTH, wl.RHO_HI, wl.RHO_LO, A)
        if how == "table":
            for b in range(2):
                lat.set_gradient_table(np.tile(A, (30, 1)), 0, box=b)
        elif how == "one":
            lat.set_gradient(A, box=0)
            lat.set_gradient(A, box=1)
        else:
            lat.set_gradient(A)
        lat.step(20)
        if how != "table":
            lat.set_gradient(A)  # refilled from time 20: 30 more steps allowed
            lat.step(10)
        else:
            lat.step(10)
        out.append(lat.save())
        lat.close()
    assert np.array_equal(out[0][64:], out[1][64:]) and np.array_equal(out[0][64:], out[2][64:])
    lat = lattice(sc)
    with pytest.raises(sc.SclbmError) as ei:
        lat.set_gradient(wl.simple_shear(0.05))  # ghost speed above 0.2 c_s
    assert ei.value.status == sc.SCLBM_EINVAL
    lat.close()
    per = lattice(sc, bc="periodic")
    with pytest.raises(sc.SclbmError) as ei:
        per.set_gradient(A)
    assert ei.value.status == sc.SCLBM_ESTATE
    per.close()


@pytest.mark.parametrize("prec", ["f64", "f32", "f16dev"])
def test_uniform_init_equals_uniform_fields(sc, prec):
    """sclbm_init_uniform gives the same populations as sclbm_init_fields of
    uniform fields, and the state is stationary (periodic, moving)."""
    rho = wl.ghost_densities(6.0)
    u0 = np.array([0.04, -0.01, 0.02])
    a = lattice(sc, prec=prec, bc="periodic")
    a.init_uniform(rho[0], rho[1], u0)
    b = lattice(sc, prec=prec, bc="periodic")
    b.init_fields(np.full(b.shape, rho[0]), np.full(b.shape, rho[1]), u0)
    sa, sb = a.save(), b.save()
    assert np.array_equal(sa[64:], sb[64:])
    a.step(50)
    ra, rb, u = (t.cpu().numpy() for t in a.fields())
    # FP16 deviations: this moving state's relative deviations reach 3 |c.u| ~ 0.15,
    # stored with FP16's relative half-ulp 2^-11, i.e. 7e-5 of a population
    tol = {"f64": 1e-13, "f32": 1e-5, "f16dev": 2e-4}[prec]
    assert np.abs(ra / rho[0] - 1).max() <= tol and np.abs(rb / rho[1] - 1).max() <= tol
    assert np.abs(u - u0[:, None, None, None]).max() <= tol
    with pytest.raises(sc.SclbmError) as ei:
        a.init_uniform(-1.0, rho[1])
    assert ei.value.status == sc.SCLBM_EINVAL
    a.close()
    b.close()


@pytest.mark.parametrize("graph", [False, True])
def test_health_check_reports_unstable_state(sc, graph):
    """With the health check on, a state holding one NaN density stops the step
    call with EUNSTABLE at the first checked time; a healthy box passes, and with
    the check off the same bad state steps without complaint."""
    n = 16
    A = wl.simple_shear(wl.shear_rate_for_ca(0.05, 4.0))
    good = lattice(sc, n=n, nbox=2, steps=40)
    good.init_droplet(good.xc, 4.0, wl.WIDTH, wl.RHO_HI, wl.RHO_LO, A)
    good.set_gradient(A)
    good.set_health_check(4)
    if graph:
        good.step_graph(8)
    else:
        good.step(10)  # checked at times 4 and 8
    good.close()

    bad = lattice(sc, n=n, nbox=2, steps=40)
    ra = np.full(bad.shape, 0.05)
    rb = np.full(bad.shape, 1.0)
    ra[3, 5, 7] = np.nan
    bad.init_uniform(0.05, 1.0)
    bad.init_fields(ra, rb, box=1)
    bad.set_gradient(A)
    bad.step(2)  # check off: no error
    bad.set_health_check(3)
    with pytest.raises(sc.SclbmError) as ei:
        if graph:
            bad.step_graph(2)
        else:
            bad.step(5)
    assert ei.value.status == sc.SCLBM_EUNSTABLE
    assert "box 1" in str(ei.value)
    assert bad.step_count == (4 if graph else 3)
    with pytest.raises(sc.SclbmError):
        bad.set_health_check(-1)
    bad.close()
