"""GPU checks of the batched ensemble: several independent boxes in one launch
per step, the hipGraph-captured step loop, and the autotuner (through the C ABI).
"""
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


def ou_tables(n, nbox, steps, seed0=1000):
    return [wl.ou_gradient_table(seed0 + b, n, steps, mach=0.1 + 0.05 * b) for b in range(nbox)]


@pytest.mark.parametrize("launch", [None, (4, 6, 1), (4, 7, 2)])
def test_ensemble_equals_independent_boxes(sc, launch):
    """Every box of a 3-box ensemble is bit-identical to the same box run alone,
    and box 1 matches the oracle; also with four z-chunks per box grouped in the
    tile order (chunks of 6, and of 7 with a ragged last chunk on 128-wide
    tiles), marching in alternating directions, where a run of tiles on one
    XCD spans chunks of several boxes."""
    n, nbox, steps, R = 24, 3, 40, 5.0
    tabs = ou_tables(n, nbox, steps)
    ens = sc.Lattice(n, n, n, nbox=nbox, bc="ghost", prec="f64", table_len=steps, g_ab=wl.G_AB,
                     rho_b=wl.ghost_densities(R))
    if launch:
        ens.set_launch(*launch)
    for b in range(nbox):
        ens.init_droplet(ens.xc, R, wl.WIDTH, wl.RHO_HI, wl.RHO_LO, tabs[b][0], box=b)
        ens.set_gradient_table(tabs[b], 0, box=b)
    ens.step(steps)
    state = ens.save()[64:]
    per_box = state.size // nbox
    for b in range(nbox):
        one = sc.Lattice(n, n, n, bc="ghost", prec="f64", table_len=steps, g_ab=wl.G_AB, rho_b=wl.ghost_densities(R))
        one.init_droplet(one.xc, R, wl.WIDTH, wl.RHO_HI, wl.RHO_LO, tabs[b][0])
        one.set_gradient_table(tabs[b], 0)
        one.step(steps)
        assert np.array_equal(one.save()[64:], state[b * per_box:(b + 1) * per_box]), b
    o = oracle.Oracle(n, n, n, periodic=False, g=wl.G_AB, rho_b=wl.ghost_densities(R))
    o.init_droplet(o.xc, R, wl.WIDTH, wl.RHO_HI, wl.RHO_LO, tabs[1][0])
    o.run(steps, tabs[1])
    ra, rb, _ = (t.cpu().numpy() for t in ens.fields(box=1))
    oa, ob, _ = o.fields()
    assert max(np.max(np.abs(ra - oa) / oa), np.max(np.abs(rb - ob) / ob)) <= 1e-11


@pytest.mark.parametrize("prec,tol", [("f64", 1e-11), ("f32", 1e-5)])
def test_ensemble_tau3_boxes_and_totals_match_oracle(sc, prec, tol):
    """A 3-box ensemble at tau = 3 for both phases (Table 2; coupling and interface
    densities of wl.TAU3), each box with its own drive: every box's densities and
    FP64 totals (mass per component, momentum) against the oracle's after 40 steps."""
    n, nbox, steps, R = 24, 3, 40, 5.0
    T3 = wl.TAU3
    rho_b = (T3["rho_lo"], T3["rho_hi"])
    tabs = ou_tables(n, nbox, steps)
    ens = sc.Lattice(n, n, n, nbox=nbox, bc="ghost", prec=prec, table_len=steps, tau=(3.0, 3.0), g_ab=T3["g_ab"],
                     rho_b=rho_b)
    for b in range(nbox):
        ens.init_droplet(ens.xc + 0.7 * b, R, wl.WIDTH, T3["rho_hi"], T3["rho_lo"], tabs[b][0], box=b)
        ens.set_gradient_table(tabs[b], 0, box=b)
    ens.step(steps)
    for b in range(nbox):
        o = oracle.Oracle(n, n, n, periodic=False, tau=(3.0, 3.0), g=T3["g_ab"], rho_b=rho_b)
        o.init_droplet(o.xc + 0.7 * b, R, wl.WIDTH, T3["rho_hi"], T3["rho_lo"], tabs[b][0])
        o.run(steps, tabs[b])
        ra, rb, _ = (t.cpu().numpy() for t in ens.fields(box=b))
        oa, ob, _ = o.fields()
        err = max(np.max(np.abs(ra - oa) / oa), np.max(np.abs(rb - ob) / ob))
        print("%s box %d: max rel density error %.3e" % (prec, b, err))
        assert err <= tol, b
        m, p = ens.totals(box=b)
        om, op = o.totals()
        assert np.all(np.abs(m - om) / om <= 10 * tol), b
        assert np.abs(p - op).max() <= 10 * tol * om.sum() * 0.05, b
    ens.close()


@pytest.mark.parametrize("prec,wide", [("f16dev", 2), ("bf16dev", 2), ("f16dev", 1), ("bf16dev", 4)])
def test_deviation_ensemble_tiles(sc, prec, wide):
    """16-bit formats on 128 x 4, 64 x 4 or 256 x 4 tiles: every box of a 3-box ensemble of
    70 x 10 x 9 boxes (three z-chunks per box) gives the same fields, bit for bit,
    as the box run alone on the same tiles and as the box run alone on 64 x 4
    tiles."""
    nxyz, nbox, steps, R = (70, 10, 9), 3, 20, 3.0
    tabs = [wl.ou_gradient_table(2000 + b, 70, steps, mach=0.1 + 0.05 * b) for b in range(nbox)]

    def lattice(nb, launch):
        lat = sc.Lattice(*nxyz, nbox=nb, bc="ghost", prec=prec, table_len=steps, g_ab=wl.G_AB,
                         rho_b=wl.ghost_densities(R))
        lat.set_launch(*launch)
        return lat

    ens = lattice(nbox, (4, 3, wide))
    for b in range(nbox):
        ens.init_droplet(ens.xc, R, wl.WIDTH, wl.RHO_HI, wl.RHO_LO, tabs[b][0], box=b)
        ens.set_gradient_table(tabs[b], 0, box=b)
    ens.step(steps)
    for b in range(nbox):
        got = [t.cpu().numpy() for t in ens.fields(box=b)]
        for launch in ((4, 3, wide), (4, 3, 1)):
            one = lattice(1, launch)
            one.init_droplet(one.xc, R, wl.WIDTH, wl.RHO_HI, wl.RHO_LO, tabs[b][0])
            one.set_gradient_table(tabs[b], 0)
            one.step(steps)
            ref = [t.cpu().numpy() for t in one.fields()]
            assert all(np.array_equal(g, r) for g, r in zip(got, ref)), (b, launch)
            one.close()
    ens.close()


@pytest.mark.parametrize("prec,nx,launch", [("f32", 20, None), ("f16dev", 150, (4, 3, 4)), ("bf16dev", 100, (8, 3, 1))])
def test_graph_replays_match_eager(sc, prec, nx, launch):
    """A captured 10-step loop replayed five times, with eager work and
    synchronisations between replays, equals eager stepping after every replay
    (also for the 16-bit formats)."""
    n, nbox, steps, R = 20, 2, 60, 4.0
    tabs = ou_tables(nx, nbox, steps, seed0=77)

    def make():
        lat = sc.Lattice(nx, n, n, nbox=nbox, bc="ghost", prec=prec, table_len=steps, g_ab=wl.G_AB,
                         rho_b=wl.ghost_densities(R))
        if launch:
            lat.set_launch(*launch)
        for b in range(nbox):
            lat.init_droplet(lat.xc, R, wl.WIDTH, wl.RHO_HI, wl.RHO_LO, tabs[b][0], box=b)
            lat.set_gradient_table(tabs[b], 0, box=b)
        return lat

    g, e = make(), make()
    for rep in range(5):
        g.step_graph(10)
        e.step(10)
        # eager work on the graph's context between replays
        g.totals()
        g.synchronize()
        assert g.step_count == e.step_count == 10 * (rep + 1)
        assert np.array_equal(g.save(), e.save()), rep
    # odd eager step flips the buffer parity: the graph is recaptured, still exact
    g.step(1)
    e.step(1)
    g.step_graph(2)
    e.step(2)
    assert np.array_equal(g.save(), e.save())


@pytest.mark.parametrize("prec,nxyz,shapes", [
    ("f32", (40, 40, 40), ((4, 1), (8, 1))),                        # nx <= 64: one column of 64 nodes
    ("f16dev", (150, 12, 10), ((4, 1), (8, 1), (4, 2), (4, 4))),   # 16-bit, nx > 128: 256-wide tiles too
])
def test_autotune_keeps_results(sc, prec, nxyz, shapes):
    """The autotuner sets a valid shape of those it may try, restores the time, and
    the tuned context gives the same bits as one at the default launch."""
    n, steps, R = nxyz[0], 30, 5.0
    A = wl.simple_shear(0.0006)
    lat = sc.Lattice(*nxyz, bc="ghost", prec=prec, table_len=steps, g_ab=wl.G_AB, rho_b=wl.ghost_densities(R))
    lat.set_gradient_table(np.tile(A, (steps, 1)), 0)
    ty, zc, wx, ms = sc.sclbm_autotune(lat.ctx, 3)
    assert (ty, wx) in shapes and 1 <= zc <= nxyz[2] and ms > 0
    assert lat.get_launch() == (ty, zc, wx)
    assert lat.step_count == 0
    lat.init_droplet(lat.xc, R, wl.WIDTH, wl.RHO_HI, wl.RHO_LO, A)
    lat.step(steps)
    ref = sc.Lattice(*nxyz, bc="ghost", prec=prec, table_len=steps, g_ab=wl.G_AB, rho_b=wl.ghost_densities(R))
    ref.set_gradient_table(np.tile(A, (steps, 1)), 0)
    ref.init_droplet(ref.xc, R, wl.WIDTH, wl.RHO_HI, wl.RHO_LO, A)
    ref.step(steps)
    assert np.array_equal(lat.save(), ref.save())


def test_moments_of_all_boxes_in_one_pass(sc):
    import torch
    n, nbox, steps, R = 24, 4, 20, 5.0
    tabs = ou_tables(n, nbox, steps, seed0=300)
    lat = sc.Lattice(n, n, n, nbox=nbox, bc="ghost", prec="f32", table_len=steps, g_ab=wl.G_AB,
                     rho_b=wl.ghost_densities(R))
    for b in range(nbox):
        lat.init_droplet(lat.xc, R + 0.5 * b, wl.WIDTH, wl.RHO_HI, wl.RHO_LO, tabs[b][0], box=b)
        lat.set_gradient_table(tabs[b], 0, box=b)
    lat.step(steps)
    allm = torch.zeros((nbox, 10), dtype=torch.float64, device=lat.device)
    lat.droplet_moments_all(allm)
    one = torch.zeros(10, dtype=torch.float64, device=lat.device)
    for b in range(nbox):
        lat.droplet_moments(one, box=b)
        lat.synchronize()
        assert torch.equal(allm[b], one), b
        ra, rb, _ = (t.cpu().numpy() for t in lat.fields(box=b))
        ref = oracle.droplet_moments(ra, rb, lat.xc)
        assert np.allclose(allm[b].cpu().numpy(), ref, rtol=1e-12, atol=1e-9)
