"""The allocation-free droplet moments (sclbm_droplet_moments_all_static, whose
reduction lives in the library's static device array) against
sclbm_droplet_moments_all (the workspace's reduction area), through the C ABI:
bit for bit on two calls in a row, the second on a smaller ensemble that finds
the first call's values still in the array; a context too large for the array
is refused."""
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


def ensemble(sc, nbox, n, prec, steps):
    """nbox boxes of n^3, droplets of different radii and drives, `steps` steps."""
    lat = sc.Lattice(n, n, n, nbox=nbox, bc="ghost", prec=prec, table_len=steps, g_ab=wl.G_AB,
                     rho_b=wl.ghost_densities(0.25 * n))
    rng = np.random.default_rng(nbox * 1000 + n)
    for b in range(nbox):
        A = 2e-3 * rng.standard_normal(9)
        A[8] = -A[0] - A[4]
        lat.init_droplet(lat.xc + rng.uniform(-1.5, 1.5, 3), 0.2 * n + b % 3, wl.WIDTH, wl.RHO_HI, wl.RHO_LO, A,
                         box=b)
        lat.set_gradient_table(np.tile(A, (steps, 1)), 0, box=b)
    lat.step(steps)
    return lat


def both(sc, lat):
    import torch
    ref = torch.zeros((lat.nbox, 10), dtype=torch.float64, device=lat.device)
    out = torch.full((lat.nbox, 10), float("nan"), dtype=torch.float64, device=lat.device)
    lat._sync_torch()  # the output tensors were filled on torch's stream
    sc.sclbm_droplet_moments_all(lat.ctx, ref.data_ptr())
    sc.sclbm_droplet_moments_all_static(lat.ctx, out.data_ptr())
    lat.synchronize()
    return ref.cpu().numpy(), out.cpu().numpy()


def test_static_moments_match_workspace_moments(sc):
    big = ensemble(sc, 12, 40, "f32", 30)
    ref, out = both(sc, big)
    assert np.all(ref[:, 0] > 0)              # every box holds a droplet
    assert np.array_equal(ref, out)
    big.close()
    # second call: a smaller ensemble (fewer boxes, fewer blocks per box) in another format
    small = ensemble(sc, 3, 24, "f64", 20)
    ref2, out2 = both(sc, small)
    assert np.all(ref2[:, 0] > 0)
    assert np.array_equal(ref2, out2)
    # the same context again, after the smaller one: still identical
    ref3, out3 = both(sc, small)
    assert np.array_equal(ref3, ref2) and np.array_equal(out3, out2)
    small.close()


def test_static_moments_refuse_too_many_boxes(sc):
    # 20000 boxes of 4^3: one block per box, 20000 * 2 * 16 doubles > 2 MiB
    lat = sc.Lattice(4, 4, 4, nbox=20000, bc="periodic", prec="f32", g_ab=wl.G_AB, rho_b=(0.05, 1.0))
    import torch
    out = torch.zeros((lat.nbox, 10), dtype=torch.float64, device=lat.device)
    lat._sync_torch()
    with pytest.raises(sc.SclbmError) as ei:
        sc.sclbm_droplet_moments_all_static(lat.ctx, out.data_ptr())
    assert ei.value.status == sc.SCLBM_ESIZE
    assert "static scratch" in str(ei.value)
    lat.close()
