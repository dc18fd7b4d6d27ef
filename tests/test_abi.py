"""C-ABI checks that need no GPU: the library loads, exports every call that
include/*.h declares, validates configurations, and its host-only droplet
analysis (closed-form 3x3 eigenvalues) matches the oracle's on known moments."""
import os
import re

import numpy as np
import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    names = set()
    for h in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if not h.endswith(".h"):
            continue
        with open(os.path.join(ROOT, "include", h)) as fh:
            text = fh.read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        names |= set(re.findall(r"\b(scl(?:bm|mlp)_[a-z0-9_]+)\s*\(", text))
    return sorted(names)


def test_library_exports_every_declared_call():
    import paper_2112_09972_amd as sc
    lib = sc.load()                     # the package's loader (one HIP runtime per process)
    names = header_functions()
    assert len(names) >= 38
    for name in names:
        assert hasattr(lib, name), name
    assert sorted(sc.EXPORTS) == names


def test_library_shares_torch_hip_runtime():
    """Loading the library makes it bind to PyTorch's HIP runtime: the process
    then maps a single HIP runtime, whatever was imported first (two runtimes in
    one process leave the library without a device)."""
    import subprocess
    import sys
    code = ("import paper_2112_09972_amd as sc; sc.load(); "
            "maps = open('/proc/self/maps').read(); "
            "print(len({l.split()[-1] for l in maps.splitlines() if 'libamdhip64' in l}))")
    out = subprocess.run([sys.executable, "-c", code], cwd=ROOT, capture_output=True, text=True, timeout=300)
    assert out.returncode == 0, out.stderr
    assert out.stdout.strip().splitlines()[-1] == "1"


def cfg(**kw):
    import paper_2112_09972_amd as sc
    base = dict(nx=32, ny=32, nz=32, nbox=1, bc=1, prec=0, table_len=10, g_ab=1.64, mach_max=0.0)
    base.update(kw)
    tau = base.pop("tau", (1.0, 1.0))
    rho_b = base.pop("rho_b", (0.04, 1.0))
    import ctypes
    return sc.sclbm_config(tau=(ctypes.c_double * 2)(*tau), rho_b=(ctypes.c_double * 2)(*rho_b), **base)


def test_workspace_size():
    import paper_2112_09972_amd as sc
    b64 = sc.sclbm_workspace_bytes(cfg())
    b32 = sc.sclbm_workspace_bytes(cfg(prec=1))
    pop64 = 2 * 19 * 32 ** 3 * 8
    assert b64 >= 2 * pop64
    assert b64 - b32 == 2 * (pop64 // 2)
    b16 = sc.sclbm_workspace_bytes(cfg(prec=2, nbox=3))
    assert b16 >= 2 * 3 * 2 * 19 * 32 ** 3 * 2


@pytest.mark.parametrize("bad", [dict(nx=2), dict(nbox=0), dict(bc=7), dict(prec=9), dict(tau=(0.5, 1.0)),
                                 dict(rho_b=(0.0, 1.0)), dict(table_len=0), dict(mach_max=-1.0),
                                 dict(g_ab=float("nan"))])
def test_invalid_configs_rejected(bad):
    import paper_2112_09972_amd as sc
    with pytest.raises(sc.SclbmError) as ei:
        sc.sclbm_workspace_bytes(cfg(**bad))
    assert ei.value.status == sc.SCLBM_EINVAL
    assert "invalid config" in sc.sclbm_last_error()


@pytest.mark.parametrize("axes,th", [((10.0, 8.0, 6.0), 0.0), ((9.0, 7.0, 5.0), 0.6), ((6.0, 6.0, 6.0), 0.0),
                                     ((7.0, 7.0, 4.0), 1.1)])
def test_host_droplet_analysis_matches_oracle(axes, th):
    import paper_2112_09972_amd as sc
    n = 36
    c = np.array([(n - 1) / 2.0] * 3)
    z, y, x = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    d = np.stack([x - c[0] - 0.3, y - c[1] + 0.2, z - c[2]]).reshape(3, -1)
    Rm = np.array([[np.cos(th), -np.sin(th), 0], [np.sin(th), np.cos(th), 0], [0, 0, 1]])
    d = Rm.T @ d
    inside = (d[0] / axes[0]) ** 2 + (d[1] / axes[1]) ** 2 + (d[2] / axes[2]) ** 2 < 1.0
    ra = np.where(inside, 1.0, 0.04).reshape(n, n, n)
    rb = 1.04 - ra
    mom = oracle.droplet_moments(ra, rb, c)
    ref = oracle.droplet_stats_from_moments(mom, c)
    got = sc.sclbm_droplet_from_moments(mom, c, 7)
    assert got["step"] == 7
    assert np.allclose(got["semi_axes"], ref["semi_axes"], rtol=1e-10, atol=1e-12)
    assert abs(got["deformation"] - ref["deformation"]) < 1e-10
    assert np.allclose(got["com"], ref["com"], rtol=0, atol=1e-12)
    assert abs(got["r_eq"] - ref["r_eq"]) < 1e-12


def test_empty_droplet():
    import paper_2112_09972_amd as sc
    got = sc.sclbm_droplet_from_moments(np.zeros(10), [1.0, 2.0, 3.0])
    assert got["volume"] == 0.0 and np.all(got["semi_axes"] == 0.0)
    assert np.allclose(got["com"], [1, 2, 3])


@pytest.mark.parametrize("n,nbox,prec,expect", [
    (128, 1, 1, (4, 16, 2)),   # benchmark box: whole 128-wide rows, 256 workgroups in one round
    (256, 1, 1, (4, 128, 2)),  # two tiles per row, two chunks: one round
    (64, 64, 1, (8, 64, 1)),   # ensemble of 64^3 boxes: whole-box chunks, two rounds
    (160, 1, 1, (8, 40, 1)),   # last 128-wide tile a quarter full: 64 x 8 tiles
    (192, 1, 1, (8, 28, 1)),   # last 128-wide tile half full: 64 x 8 tiles; two rounds of 30
    (96, 1, 1, (4, 10, 2)),    # 240 workgroups, not 264 (a second, nearly empty round)
    (200, 1, 1, (4, 40, 2)),
    (32, 1, 0, (8, 2, 1)),
    (256, 1, 2, (4, 64, 4)),   # 16-bit formats: 256-wide tiles, four waves per SIMD, chunks <= 64 planes
    (200, 1, 3, (4, 40, 4)),   # last 256-wide tile more than 160 nodes
    (192, 1, 2, (4, 39, 4)),   # a 256-wide tile holds the row: four rows, even where the 128-wide rules take 64 x 8
    (64, 64, 2, (8, 64, 1)),   # 16-bit ensemble of 64^3 boxes: whole-box chunks
    (160, 1, 2, (8, 20, 1)),   # not: 128-wide rules
    (150, 1, 2, (8, 19, 1)),
    (128, 1, 2, (4, 8, 2)),
    (45, 1, 2, (8, 3, 1)),
])
def test_default_launch_rules(n, nbox, prec, expect):
    """The default launch shape (tile rows, z-chunk, 64-node columns) a context
    starts with, computed on the host: fill of the last tile, then the chunk
    count that minimises rounds of resident workgroups times planes per chunk
    (16-bit formats: 256-wide tiles where the last one of a row is more than
    160 nodes long, twice the resident waves, chunks of at most 64 planes)."""
    import paper_2112_09972_amd as sc
    assert sc.sclbm_default_launch(cfg(nx=n, ny=n, nz=n, nbox=nbox, prec=prec)) == expect


def test_default_launch_rejects_invalid_config():
    import paper_2112_09972_amd as sc
    with pytest.raises(sc.SclbmError) as ei:
        sc.sclbm_default_launch(cfg(nx=2))
    assert ei.value.status == sc.SCLBM_EINVAL


def test_mm_semi_axes_host_call():
    """sclbm_mm_semi_axes (host only): square roots of the eigenvalues of the
    symmetric part, descending, against numpy's symmetric eigen-solver on
    ellipsoids R diag(a^2) R^T with random rotations, plus the sphere and a
    repeated axis (the trigonometric solution's degenerate branches)."""
    import paper_2112_09972_amd as sc
    rng = np.random.default_rng(7)
    Ms = []
    for _ in range(200):
        q, _ = np.linalg.qr(rng.standard_normal((3, 3)))
        a = np.sort(rng.uniform(0.3, 3.0, 3))[::-1]
        M = q @ np.diag(a * a) @ q.T
        M += 1e-14 * rng.standard_normal((3, 3))  # not exactly symmetric, as an integrator leaves it
        Ms.append(M)
    Ms.append(np.eye(3))
    Ms.append(np.diag([2.0, 0.5, 0.5]))
    Ms = np.array(Ms)
    got = sc.sclbm_mm_semi_axes(Ms.reshape(2, -1, 3, 3)).reshape(-1, 3)
    ref = np.sqrt(np.linalg.eigvalsh(0.5 * (Ms + Ms.transpose(0, 2, 1)))[:, ::-1])
    assert np.allclose(got, ref, rtol=1e-10, atol=1e-12)
    assert np.all(np.diff(got, axis=1) <= 0)
