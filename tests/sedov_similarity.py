"""Sedov-Taylor self-similar point blast in a uniform gas (spherical).

With R(t) = xi0 (E t^2 / rho0)^(1/5), lambda = r/R and dR/dt = 2R/(5t), write
u = Rdot U(lambda), rho = rho0 G(lambda), p = rho0 Rdot^2 P(lambda).  Mass,
momentum and entropy conservation then give three ODEs in lambda:

    (U - l) G' = -G (U' + 2U/l)
    (U - l) U' = 3U/2 - P'/G
    (U - l) (P'/P - gamma G'/G) = 3

integrated inward from the strong-shock values U = 2/(g+1), G = (g+1)/(g-1),
P = 2/(g+1) at lambda = 1.  The blast energy
    E = (16 pi / 25) rho0 R^5 / t^2 * I,  I = int_0^1 (G U^2/2 + P/(g-1)) l^2 dl
fixes xi0 = (25 / (16 pi I))^(1/5).  Used only to pin the CPU oracle.
"""
from __future__ import annotations

import numpy as np
from scipy.integrate import solve_ivp


def _rhs(lam, y, g):
    U, G, P = y
    W = U - lam
    num = 1.5 * U - 3.0 * P / (G * W) + 2.0 * g * P * U / (lam * G * W)
    den = W - g * P / (G * W)
    dU = num / den
    dG = -G * (dU + 2.0 * U / lam) / W
    dP = P * (3.0 / W + g * dG / G)
    return [dU, dG, dP]


def solve(gamma: float, lam_min: float = 1e-5):
    y0 = [2.0 / (gamma + 1.0), (gamma + 1.0) / (gamma - 1.0), 2.0 / (gamma + 1.0)]
    lam = np.concatenate([np.linspace(1.0, 0.1, 2000), np.geomspace(0.1, lam_min, 2000)[1:]])
    sol = solve_ivp(_rhs, (1.0, lam_min), y0, t_eval=lam, args=(gamma,), rtol=1e-11,
                    atol=1e-14, method="DOP853")
    if not sol.success:
        raise RuntimeError(sol.message)
    return sol.t, sol.y


def xi0(gamma: float) -> float:
    lam, (U, G, P) = solve(gamma)
    f = (0.5 * G * U * U + P / (gamma - 1.0)) * lam * lam
    order = np.argsort(lam)
    I = np.trapezoid(f[order], lam[order])
    return float((25.0 / (16.0 * np.pi * I)) ** 0.2)


def shock_radius(t: float, E: float = 1.0, rho0: float = 1.0, gamma: float = 5.0 / 3.0) -> float:
    return xi0(gamma) * (E * t * t / rho0) ** 0.2
