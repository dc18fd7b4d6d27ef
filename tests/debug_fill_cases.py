"""Runs a set of small boxes (every step kernel, tile shape and storage format,
ragged and whole-row tiles, both boundary modes) and prints one JSON line of
state hashes.  Run as a script with SCLBM_LIBRARY pointing at the library build
to use; tests/test_gpu_debug_fill.py compares the regular and the LDS NaN-fill
builds."""
import hashlib
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

CASES = [
    ("f32", "ghost", (128, 10, 9), (4, 3, 2)), ("f32", "periodic", (128, 10, 9), (4, 3, 2)),
    ("f32", "ghost", (64, 13, 11), (8, 5, 1)), ("f32", "periodic", (70, 13, 11), (4, 3, 1)),
    ("f32", "ghost", (150, 13, 11), (4, 5, 2)), ("f32", "periodic", (45, 13, 11), (4, 5, 2)),
    ("f64", "ghost", (100, 10, 9), (4, 3, 2)), ("f64", "periodic", (100, 10, 9), (8, 4, 1)),
    ("f32d", "ghost", (40, 12, 9), (8, 4, 1)),
    ("f16dev", "ghost", (150, 13, 11), (4, 5, 2)), ("f16dev", "periodic", (300, 6, 5), (8, 2, 1)),
    ("f16dev", "ghost", (70, 9, 7), (4, 3, 1)), ("bf16dev", "ghost", (270, 6, 5), (4, 3, 2)),
    ("bf16dev", "ghost", (45, 13, 11), (4, 5, 2)), ("f16dev", "ghost", (300, 6, 5), (4, 2, 4)),
    ("bf16dev", "periodic", (257, 6, 5), (4, 3, 4)),
    ("bf16dev", "periodic", (46, 6, 5), (4, 3, 2)),
    # boxes thin in y and z: both y faces in one tile, tiles with rows beyond the box
    ("f32", "ghost", (70, 3, 5), (4, 2, 1)), ("f64", "ghost", (45, 6, 7), (4, 5, 2)),
    ("f16dev", "ghost", (130, 4, 3), (4, 3, 4)), ("bf16dev", "ghost", (150, 9, 4), (8, 3, 1)),
]


def main():
    import paper_2112_09972_amd as sc
    from paper_2112_09972_amd import workloads as wl
    A = np.array([0.0004, 0.0, 0.002, 0.0, -0.0007, 0.0, 0.0011, 0.0, 0.0003])
    steps = 10
    out = {}
    for prec, bc, nxyz, launch in CASES:
        lat = sc.Lattice(*nxyz, bc=bc, prec=prec, table_len=steps, g_ab=wl.G_AB, rho_b=wl.ghost_densities(4.0))
        lat.set_launch(*launch)
        lat.init_droplet(lat.xc, 4.0, wl.WIDTH, wl.RHO_HI, wl.RHO_LO, A if bc == "ghost" else None)
        if bc == "ghost":
            lat.set_gradient_table(np.tile(A, (steps, 1)), 0)
        lat.step(steps)
        st = lat.save()
        key = "%s %s %s %s" % (prec, bc, "x".join(map(str, nxyz)), ",".join(map(str, launch)))
        f = st[64:]
        out[key] = {"sha": hashlib.sha256(f.tobytes()).hexdigest()[:16], "finite": bool(lat.totals(check=False)[0].sum() > 0)}
        lat.close()
    print(json.dumps({"library": sc.LIB_PATH, "cases": out}))


if __name__ == "__main__":
    main()
