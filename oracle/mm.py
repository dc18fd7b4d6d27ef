"""Maffettone-Minale (MM) droplet model, FP64 reference (TEST INFRASTRUCTURE).

The ellipsoidal droplet of Sec. 2 is the morphology tensor M (M = I for the
undeformed sphere of radius R; the eigenvalues of M are the squared semi-axes
over R^2).  Its evolution, Sec. 2 Eq. 1, with the strain and vorticity of the
velocity gradient, Sec. 2 Eq. 2, and the coefficients of Sec. 2 Eq. 5:

    dM/dt* = Ca [ f2 (S M + M S) + Omega M - M Omega ] - f1 (M - 3 III_M / II_M I)

with t* in units of the droplet time tau_d = eta_s R / sigma and S, Omega
normalised by the shear rate G(t) = ||A(t)||_inf (so that Ca = tau_d G).  In the
lattice units of the driving table this reads

    dM/dt = f2(Ca) (S M + M S) + Omega M - M Omega - (f1 / tau_d) (M - 3 III_M / II_M I),

S and Omega the symmetric and antisymmetric parts of A(t), Ca(t) = tau_d ||A(t)||_inf,
f1(chi) = 40 (chi + 1) / ((3 + 2 chi)(16 + 19 chi)),
f2(chi, Ca) = 5 / (3 + 2 chi) + 3 Ca^2 / (2 + 6 Ca^2),
III_M = det M, II_M = (tr(M)^2 - M:M) / 2.

Integration (a reading: the paper does not say how it integrates): classical RK4
with `substeps` equal steps per table row, A(t) linear between consecutive rows
(row n at time n).
"""
from __future__ import annotations

import numpy as np


def f1(chi: float) -> float:
    return 40.0 * (chi + 1.0) / ((3.0 + 2.0 * chi) * (16.0 + 19.0 * chi))


def f2(chi: float, ca: float) -> float:
    return 5.0 / (3.0 + 2.0 * chi) + 3.0 * ca * ca / (2.0 + 6.0 * ca * ca)


def rhs(M: np.ndarray, A: np.ndarray, tau_d: float, chi: float) -> np.ndarray:
    S = 0.5 * (A + A.T)
    W = 0.5 * (A - A.T)
    ca = tau_d * np.max(np.abs(A))
    II = 0.5 * (np.trace(M) ** 2 - np.sum(M * M))
    III = np.linalg.det(M)
    return (f2(chi, ca) * (S @ M + M @ S) + W @ M - M @ W
            - (f1(chi) / tau_d) * (M - 3.0 * III / II * np.eye(3)))


def integrate(A_rows: np.ndarray, tau_d: float, chi: float = 1.0, substeps: int = 1, M0=None,
              record_every: int = 1) -> np.ndarray:
    """Integrate from M0 (default I) over the table rows; returns M at times
    0, record_every, 2 record_every, ... (shape (k, 3, 3))."""
    A_rows = np.asarray(A_rows, dtype=np.float64).reshape(-1, 3, 3)
    M = np.eye(3) if M0 is None else np.array(M0, dtype=np.float64)
    h = 1.0 / substeps
    out = [M.copy()]
    nsteps = A_rows.shape[0] - 1
    for n in range(nsteps):
        A0, A1 = A_rows[n], A_rows[n + 1]
        for s in range(substeps):
            t0 = s * h
            Aa = A0 + (A1 - A0) * t0
            Am = A0 + (A1 - A0) * (t0 + 0.5 * h)
            Ab = A0 + (A1 - A0) * (t0 + h)
            k1 = rhs(M, Aa, tau_d, chi)
            k2 = rhs(M + 0.5 * h * k1, Am, tau_d, chi)
            k3 = rhs(M + 0.5 * h * k2, Am, tau_d, chi)
            k4 = rhs(M + h * k3, Ab, tau_d, chi)
            M = M + (h / 6.0) * (k1 + 2.0 * k2 + 2.0 * k3 + k4)
        if (n + 1) % record_every == 0:
            out.append(M.copy())
    return np.array(out)


def semi_axes(M: np.ndarray, radius: float) -> np.ndarray:
    """Semi-axes R sqrt(eig M), descending."""
    lam = np.linalg.eigvalsh(0.5 * (M + M.T))[::-1]
    return radius * np.sqrt(np.clip(lam, 0.0, None))


def deformation(M: np.ndarray) -> float:
    """D = (L - W)/(L + W), Sec. 2 Eq. 4, from the largest and smallest semi-axes."""
    a = semi_axes(M, 1.0)
    return float((a[0] - a[2]) / (a[0] + a[2]))
