"""Second, independent transcription of the oracle's time step in numpy, for tiny
boxes only (TEST INFRASTRUCTURE).

It is written from the same passages as ``sclbm_oracle.c`` (Sec. 2 Eqs. 6-9 and the
ghost equilibria of Sec. 2 Eq. 8 / Sec. 3 Eq. 14) but with whole-array operations,
a hand-listed velocity order that differs from the C oracle's, and no shared
helper.  Agreement of the two on 4^3..8^3 boxes catches indexing and sign slips
that a single implementation could hide.
"""
from __future__ import annotations

import numpy as np

# hand-listed D3Q19 (rest, 6 axis, 12 face diagonals)
VEL = np.array([
    (0, 0, 0),
    (1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1),
    (1, 1, 0), (-1, -1, 0), (1, -1, 0), (-1, 1, 0),
    (1, 0, 1), (-1, 0, -1), (1, 0, -1), (-1, 0, 1),
    (0, 1, 1), (0, -1, -1), (0, 1, -1), (0, -1, 1),
], dtype=np.int64)
WGT = np.array([1 / 3] + [1 / 18] * 6 + [1 / 36] * 12)


def equilibrium(rho, u):
    """rho: (...), u: (3, ...) -> (19, ...)."""
    cu = np.tensordot(VEL.astype(np.float64), u, axes=(1, 0))
    uu = np.sum(u * u, axis=0)
    return WGT.reshape((19,) + (1,) * rho.ndim) * rho * (1 + 3 * cu + 4.5 * cu ** 2 - 1.5 * uu)


def _neighbour(field, c, periodic, ghost_value):
    """field(x + c) on a (nz, ny, nx) array."""
    if periodic:
        return np.roll(field, shift=(-c[2], -c[1], -c[0]), axis=(0, 1, 2))
    padded = np.pad(field, 1, mode="constant", constant_values=ghost_value)
    nz, ny, nx = field.shape
    return padded[1 + c[2]:1 + c[2] + nz, 1 + c[1]:1 + c[1] + ny, 1 + c[0]:1 + c[0] + nx]


class TinyLBM:
    def __init__(self, shape_zyx, periodic, tau, g, rho_b):
        self.shape = tuple(shape_zyx)
        self.periodic = periodic
        self.tau = tau
        self.g = g
        self.rho_b = rho_b
        nz, ny, nx = self.shape
        self.xc = np.array([(nx - 1) / 2, (ny - 1) / 2, (nz - 1) / 2])
        self.f = np.zeros((2, 19) + self.shape)

    def init(self, rho_a, rho_b, u):
        self.f[0] = equilibrium(rho_a, u)
        self.f[1] = equilibrium(rho_b, u)

    def moments(self):
        rho = self.f.sum(axis=1)                                   # (2, z, y, x)
        j = np.einsum("sizyx,ia->sazyx", self.f, VEL.astype(np.float64))
        return rho, j

    def force(self, rho):
        F = np.zeros((2, 3) + self.shape)
        for s in range(2):
            o = 1 - s
            acc = np.zeros((3,) + self.shape)
            for i in range(1, 19):
                nb = _neighbour(rho[o], VEL[i], self.periodic, self.rho_b[o])
                acc += WGT[i] * nb[None] * VEL[i].reshape(3, 1, 1, 1)
            F[s] = -self.g * rho[s][None] * acc
        return F

    def step(self, A=None):
        A = np.zeros((3, 3)) if A is None else np.asarray(A, float).reshape(3, 3)
        rho, j = self.moments()
        F = self.force(rho)
        up = (j[0] / self.tau[0] + j[1] / self.tau[1]) / (rho[0] / self.tau[0] + rho[1] / self.tau[1])
        post = np.empty_like(self.f)
        for s in range(2):
            ueq = up + self.tau[s] * F[s] / rho[s][None]
            post[s] = self.f[s] - (self.f[s] - equilibrium(rho[s], ueq)) / self.tau[s]
        nz, ny, nx = self.shape
        new = np.empty_like(self.f)
        for i in range(19):
            c = VEL[i]
            if self.periodic:
                new[:, i] = np.roll(post[:, i], shift=(c[2], c[1], c[0]), axis=(1, 2, 3))
                continue
            # source position x - c for each destination x
            z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
            sx, sy, sz = x - c[0], y - c[1], z - c[2]
            inside = (sx >= 0) & (sx < nx) & (sy >= 0) & (sy < ny) & (sz >= 0) & (sz < nz)
            out = np.empty((2,) + self.shape)
            out[:, inside] = post[:, i][:, sz[inside], sy[inside], sx[inside]]
            d = np.stack([sx - self.xc[0], sy - self.xc[1], sz - self.xc[2]]).astype(np.float64)
            ug = np.einsum("ab,bzyx->azyx", A, d)
            for s in range(2):
                geq = equilibrium(np.full(self.shape, self.rho_b[s]), ug)[i]
                out[s][~inside] = geq[~inside]
            new[:, i] = out
        self.f = new

    def fields(self):
        rho, j = self.moments()
        F = self.force(rho)
        u = (j[0] + j[1] + 0.5 * (F[0] + F[1])) / (rho[0] + rho[1])[None]
        return rho[0], rho[1], u
