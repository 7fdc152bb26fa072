"""A separately written one-dimensional PPM + central-upwind + SSP-RK2 scheme
(vectorised numpy) for the planar-reduction and Sod-convergence pins.

For data that varies only along x, every one of the nine points of an x-face
sees the same one-dimensional profile, so the three-dimensional step must
reduce to this scheme.  Fields are the same seven conserved ones; the
boundaries are zero-gradient outflow at both ends.
"""
from __future__ import annotations

import numpy as np


def _slope(qm, q0, qp):
    dl, dr = q0 - qm, qp - q0
    c = 0.5 * (qp - qm)
    m = np.minimum(np.minimum(np.abs(c), 2.0 * np.abs(dl)), 2.0 * np.abs(dr))
    return np.where(dl * dr > 0.0, np.copysign(m, c), 0.0)


def ppm_faces(q):
    """q has 3 ghost cells per side (n + 6 values); returns the (L, R) edge
    values of padded cells 2..n+3, i.e. the interior plus one ghost each side."""
    s = _slope(q[:-2], q[1:-1], q[2:])           # slopes of cells 1..-2
    q0 = q[2:-2]                                  # cells 2..-3 (need slopes each side)
    sm, s0, sp = s[:-2], s[1:-1], s[2:]
    qm, qp = q[1:-3], q[3:-1]
    six = 1.0 / 6.0
    R = q0 + 0.5 * (qp - q0) - (sp - s0) * six
    L = qm + 0.5 * (q0 - qm) - (s0 - sm) * six
    flat = (R - q0) * (q0 - L) <= 0.0
    D = R - L
    M6 = 6.0 * (q0 - 0.5 * (L + R))
    L2 = np.where(D * M6 > D * D, 3.0 * q0 - 2.0 * R, L)
    R2 = np.where((D * M6 <= D * D) & (D * M6 < -(D * D)), 3.0 * q0 - 2.0 * L, R)
    L = np.where(flat, q0, L2)
    R = np.where(flat, q0, R2)
    return L, R


def euler_flux(U, gamma, eta1):
    rho, sx, sy, sz, E, tau, X = U
    rinv = 1.0 / rho
    vx = sx * rinv
    ek = 0.5 * (sx * sx + sy * sy + sz * sz) * rinv
    e = E - ek
    e = np.where(e < eta1 * E, tau ** gamma, e)
    p = (gamma - 1.0) * e
    c = np.sqrt(gamma * p * rinv)
    F = np.array([rho * vx, sx * vx + p, sy * vx, sz * vx, E * vx + p * vx, tau * vx, X * vx])
    return F, np.abs(vx) + c


def rhs(U, dx, gamma, eta1):
    """L(U) for interior cells of U [7][n] (outflow boundaries)."""
    n = U.shape[1]
    Up = np.concatenate([np.repeat(U[:, :1], 3, axis=1), U, np.repeat(U[:, -1:], 3, axis=1)], axis=1)
    L, R = _faces_all(Up)
    # cell c of the padded array has edges L[c], R[c]; face between padded
    # cells c-1 and c uses R[c-1] (left state) and L[c] (right state)
    UL = R[:, :-1]
    UR = L[:, 1:]
    FL, sL = euler_flux(UL, gamma, eta1)
    FR, sR = euler_flux(UR, gamma, eta1)
    a = np.maximum(sL, sR)
    F = 0.5 * (FL + FR) - 0.5 * a * (UR - UL)     # n+1 faces
    assert F.shape[1] == n + 1
    return -(F[:, 1:] - F[:, :-1]) * (1.0 / dx), float(a.max())


def _faces_all(Up):
    Ls, Rs = [], []
    for f in range(Up.shape[0]):
        L, R = ppm_faces(Up[f])
        Ls.append(L)
        Rs.append(R)
    return np.array(Ls), np.array(Rs)


def step(U, dx, dt, gamma, eta1=1e-3, eta2=1e-1):
    d1, a1 = rhs(U, dx, gamma, eta1)
    U1 = U + dt * d1
    d2, a2 = rhs(U1, dx, gamma, eta1)
    U2 = 0.5 * (U + (U1 + dt * d2))
    rho, sx, sy, sz, E = U2[:5]
    e = E - 0.5 * (sx * sx + sy * sy + sz * sz) * (1.0 / rho)
    U2[5] = np.where(e > eta2 * E, np.abs(e) ** (1.0 / gamma), U2[5])
    return U2, max(a1, a2)


def signal_speed(U, dx, gamma, eta1=1e-3):
    return rhs(U, dx, gamma, eta1)[1]
