"""FP64 CPU oracle for the two-component Shan-Chen lattice Boltzmann droplet model
of arXiv 2112.09972 (Sec. 2 Eqs. 6-10, Sec. 3 Eq. 14, Sec. 4 Eq. 16, Sec. 2 Eq. 4).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the CPU-baseline leg
of the benchmark are the only callers.  The product library never imports it, and
it imports nothing from the product.

The arithmetic of a time step lives in ``sclbm_oracle.c`` (plain C, FP64,
no FMA contraction), loaded with ctypes.  The host-side analysis of the droplet
(inertia tensor -> semi-axes -> deformation, Sec. 2 Eq. 4) and the global
velocity error (Sec. 4 Eq. 16) are written here in numpy.

Parity status: every function here is pinned by the non-GPU tests (closed forms,
conservation, stationarity, symmetry, Laplace law, Taylor deformation, shear-wave
decay, ellipsoid moments); see the test files for the pin of each.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sclbm_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

Q = 19


def build(force: bool = False) -> str:
    """Compile the C oracle into ``oracle/liboracle.so`` with gcc (OpenMP over z)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O3", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared",
               "-std=c11", "-Wall", "-Wextra", "-o", tmp, _SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        D = ctypes.c_double
        I = ctypes.c_int
        I64 = ctypes.c_int64
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        lib.orc_create.restype = P
        lib.orc_create.argtypes = [I, I, I, I, D, D, D, D, D]
        lib.orc_destroy.argtypes = [P]
        lib.orc_get_step.restype = I64
        lib.orc_get_step.argtypes = [P]
        lib.orc_set_step.argtypes = [P, I64]
        lib.orc_get_f.argtypes = [P, dp]
        lib.orc_set_f.argtypes = [P, dp]
        lib.orc_init_fields.argtypes = [P, dp, dp, dp]
        lib.orc_init_droplet.argtypes = [P, dp, D, D, D, D, dp]
        lib.orc_step.argtypes = [P, dp]
        lib.orc_run.argtypes = [P, dp, I64]
        lib.orc_fields.argtypes = [P, dp, dp, dp, dp]
        lib.orc_totals.argtypes = [P, dp, dp]
        lib.orc_droplet_moments.argtypes = [I, I, I, dp, dp, dp, dp]
        lib.orc_droplet_surface.argtypes = [I, I, I, dp, dp, dp]
        lib.orc_droplet_mass.restype = D
        lib.orc_droplet_mass.argtypes = [P]
        lib.orc_reinject.restype = D
        lib.orc_reinject.argtypes = [P, D]
        lib.orc_stencil.argtypes = [ip, dp]
        lib.orc_equilibrium.argtypes = [D, dp, dp]
        lib.orc_num_threads.restype = I
        lib.orc_set_num_threads.argtypes = [I]
        _lib = lib
    return _lib


def _dp(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def stencil():
    """D3Q19 velocities (19,3) int and weights (19,) as the oracle builds them."""
    lib = _load()
    c = np.zeros((Q, 3), dtype=np.int32)
    w = np.zeros(Q, dtype=np.float64)
    lib.orc_stencil(c.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), _dp(w))
    return c.astype(np.int64), w


def num_threads() -> int:
    """OpenMP threads the oracle's loops run on."""
    return int(_load().orc_num_threads())


def set_num_threads(n: int) -> None:
    """Threads of the oracle's following loops (n >= 1)."""
    _load().orc_set_num_threads(int(n))


def equilibrium(rho: float, u) -> np.ndarray:
    """g_eq_i(rho, u), Sec. 2 Eq. 8, in the oracle's velocity order."""
    lib = _load()
    uu = np.ascontiguousarray(u, dtype=np.float64)
    out = np.zeros(Q)
    lib.orc_equilibrium(float(rho), _dp(uu), _dp(out))
    return out


class Oracle:
    """One box of the two-component model; state = post-streaming populations f(n).

    ``periodic`` selects the periodic box; otherwise the faces carry ghost nodes
    with density ``rho_b`` and the linear velocity A (x - x_c) (Sec. 3, Fig. 1,
    Eq. 14), x_c = ((nx-1)/2, (ny-1)/2, (nz-1)/2).
    """

    def __init__(self, nx, ny, nz, *, periodic, tau=(1.0, 1.0), g=0.0, rho_b=(0.04, 1.0)):
        self.lib = _load()
        self.shape = (nz, ny, nx)
        self.nx, self.ny, self.nz = nx, ny, nz
        self.n = nx * ny * nz
        self.periodic = bool(periodic)
        self.tau = tuple(float(t) for t in tau)
        self.g = float(g)
        self.rho_b = tuple(float(r) for r in rho_b)
        self.xc = np.array([(nx - 1) / 2.0, (ny - 1) / 2.0, (nz - 1) / 2.0])
        self.h = self.lib.orc_create(nx, ny, nz, 1 if periodic else 0, self.tau[0], self.tau[1],
                                     self.g, self.rho_b[0], self.rho_b[1])
        if not self.h:
            raise MemoryError("oracle allocation failed")

    def __del__(self):
        h = getattr(self, "h", None)
        if h:
            self.lib.orc_destroy(h)
            self.h = None

    @property
    def step_count(self) -> int:
        return int(self.lib.orc_get_step(self.h))

    # --- state ------------------------------------------------------------
    def init_droplet(self, center, radius, width, rho_in, rho_out, A0=None):
        ctr = np.ascontiguousarray(center, dtype=np.float64)
        A = np.zeros(9) if A0 is None else np.ascontiguousarray(np.asarray(A0, dtype=np.float64).reshape(9))
        self.lib.orc_init_droplet(self.h, _dp(ctr), float(radius), float(width), float(rho_in),
                                  float(rho_out), _dp(A))

    def init_fields(self, rho_a, rho_b, u=None):
        ra = np.ascontiguousarray(np.broadcast_to(rho_a, self.shape), dtype=np.float64)
        rb = np.ascontiguousarray(np.broadcast_to(rho_b, self.shape), dtype=np.float64)
        if u is None:
            u = np.zeros(3)
        u = np.asarray(u, dtype=np.float64)
        if u.shape == (3,):
            u = u.reshape(3, 1, 1, 1)
        uu = np.ascontiguousarray(np.broadcast_to(u, (3,) + self.shape), dtype=np.float64)
        self.lib.orc_init_fields(self.h, _dp(ra), _dp(rb), _dp(uu))

    def get_f(self) -> np.ndarray:
        out = np.zeros((2, Q) + self.shape)
        self.lib.orc_get_f(self.h, _dp(out))
        return out

    def set_f(self, f: np.ndarray):
        f = np.ascontiguousarray(f, dtype=np.float64)
        assert f.shape == (2, Q) + self.shape
        self.lib.orc_set_f(self.h, _dp(f))

    # --- time stepping ------------------------------------------------------
    def step(self, A=None):
        if A is None:
            self.lib.orc_step(self.h, None)
        else:
            a = np.ascontiguousarray(np.asarray(A, dtype=np.float64).reshape(9))
            self.lib.orc_step(self.h, _dp(a))

    def run(self, nsteps: int, Atab=None):
        """Advance nsteps; Atab[t] (t = 0..nsteps-1, each 9 doubles) drives step t."""
        if Atab is None:
            self.lib.orc_run(self.h, None, int(nsteps))
        else:
            a = np.ascontiguousarray(np.asarray(Atab, dtype=np.float64).reshape(-1, 9))
            assert a.shape[0] >= nsteps
            self.lib.orc_run(self.h, _dp(a), int(nsteps))

    # --- observables ----------------------------------------------------------
    def fields(self, with_force: bool = False):
        ra = np.zeros(self.shape)
        rb = np.zeros(self.shape)
        u = np.zeros((3,) + self.shape)
        F = np.zeros((2, 3) + self.shape) if with_force else None
        self.lib.orc_fields(self.h, _dp(ra), _dp(rb), _dp(u), _dp(F) if with_force else None)
        if with_force:
            return ra, rb, u, F
        return ra, rb, u

    def totals(self):
        m = np.zeros(2)
        p = np.zeros(3)
        self.lib.orc_totals(self.h, _dp(m), _dp(p))
        return m, p

    def droplet_mass(self) -> float:
        """Sum of rho_A over the nodes with rho_A > rho_B."""
        return float(self.lib.orc_droplet_mass(self.h))

    def reinject(self, target: float) -> float:
        """Scale the A populations of the droplet nodes so that the droplet mass
        becomes ``target``; returns the mass before."""
        return float(self.lib.orc_reinject(self.h, float(target)))


def droplet_moments(rho_a: np.ndarray, rho_b: np.ndarray, center) -> np.ndarray:
    """{S0, S1(3), S2(xx,xy,xz,yy,yz,zz)} of phi = [rho_A > rho_B] about ``center``."""
    lib = _load()
    ra = np.ascontiguousarray(rho_a, dtype=np.float64)
    rb = np.ascontiguousarray(rho_b, dtype=np.float64)
    nz, ny, nx = ra.shape
    ctr = np.ascontiguousarray(center, dtype=np.float64)
    out = np.zeros(10)
    lib.orc_droplet_moments(nx, ny, nz, _dp(ra), _dp(rb), _dp(ctr), _dp(out))
    return out


def droplet_surface(rho_a: np.ndarray, rho_b: np.ndarray):
    """(area, volume) of the level set rho_A = rho_B and of the region rho_A > rho_B,
    phi = rho_A - rho_B linear inside the six diagonal tetrahedra of every cell."""
    lib = _load()
    ra = np.ascontiguousarray(rho_a, dtype=np.float64)
    rb = np.ascontiguousarray(rho_b, dtype=np.float64)
    nz, ny, nx = ra.shape
    out = np.zeros(2)
    lib.orc_droplet_surface(nx, ny, nz, _dp(ra), _dp(rb), _dp(out))
    return float(out[0]), float(out[1])


def deformation_lbm(area: float, volume: float) -> float:
    """D_LBM = sqrt(1 - Omega_0 / Omega) (Sec. 5 Eq. 17), Omega_0 = (36 pi V^2)^(1/3)
    the area of the sphere of volume V."""
    omega0 = (36.0 * np.pi * volume * volume) ** (1.0 / 3.0)
    return float(np.sqrt(max(0.0, 1.0 - omega0 / area)))


def droplet_stats_from_moments(mom: np.ndarray, center) -> dict:
    """Semi-axes and deformation from the indicator moments.

    The second moment of a uniform solid ellipsoid with semi-axes a_k about its
    centre is diag(a_k^2)/5, so a_k = sqrt(5 lambda_k) for the eigenvalues
    lambda_k of the covariance; D = (L - W)/(L + W) with L, W the major and minor
    semi-axes (Sec. 2 Eq. 4); R_eq = (3 V / 4 pi)^(1/3).
    """
    S0 = mom[0]
    if S0 <= 0:
        return dict(volume=0.0, com=np.array(center, float), semi_axes=np.zeros(3), deformation=0.0,
                    r_eq=0.0, cov=np.zeros((3, 3)))
    S1 = mom[1:4] / S0
    xx, xy, xz, yy, yz, zz = mom[4:10] / S0
    M = np.array([[xx, xy, xz], [xy, yy, yz], [xz, yz, zz]]) - np.outer(S1, S1)
    lam = np.linalg.eigvalsh(M)[::-1]
    axes = np.sqrt(5.0 * np.clip(lam, 0.0, None))
    D = (axes[0] - axes[2]) / (axes[0] + axes[2]) if axes[0] + axes[2] > 0 else 0.0
    return dict(volume=S0, com=np.asarray(center, float) + S1, semi_axes=axes, deformation=D,
                r_eq=(3.0 * S0 / (4.0 * np.pi)) ** (1.0 / 3.0), cov=M)


def droplet_stats(rho_a: np.ndarray, rho_b: np.ndarray, center) -> dict:
    return droplet_stats_from_moments(droplet_moments(rho_a, rho_b, center), center)


def velocity_error(u: np.ndarray, A, xc) -> float:
    """Global L2 velocity error E0 of Sec. 4 Eq. 16: the rms of |u - A x| over the
    box divided by the rms of |A x|, x measured from x_c (Sec. 3 Eq. 14)."""
    A = np.asarray(A, dtype=np.float64).reshape(3, 3)
    nz, ny, nx = u.shape[1:]
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    d = np.stack([x - xc[0], y - xc[1], z - xc[2]]).astype(np.float64)
    v0 = np.einsum("ij,jzyx->izyx", A, d)
    num = np.mean(np.sum((u - v0) ** 2, axis=0))
    den = np.mean(np.sum(v0 ** 2, axis=0))
    return float(np.sqrt(num) / np.sqrt(den))


def bulk_pressure(rho_a, rho_b, g):
    """Bulk equation of state of the two-component model with psi = rho:
    p = c_s^2 (rho_A + rho_B) + c_s^2 G rho_A rho_B, c_s^2 = 1/3."""
    return (rho_a + rho_b) / 3.0 + g * rho_a * rho_b / 3.0
