"""Exact solution of the Riemann problem for the 1D Euler equations of an
ideal gas (Toro, "Riemann Solvers and Numerical Methods for Fluid Dynamics",
chapter 4): Newton iteration for the star-region pressure, then sampling of
the wave pattern.  Used only to pin the CPU oracle on the Sod shock tube."""
from __future__ import annotations

import numpy as np


def _fk(p, rk, pk, ck, g):
    if p > pk:  # shock
        A = 2.0 / ((g + 1.0) * rk)
        B = (g - 1.0) / (g + 1.0) * pk
        f = (p - pk) * np.sqrt(A / (p + B))
        df = np.sqrt(A / (B + p)) * (1.0 - 0.5 * (p - pk) / (B + p))
    else:       # rarefaction
        f = 2.0 * ck / (g - 1.0) * ((p / pk) ** ((g - 1.0) / (2.0 * g)) - 1.0)
        df = 1.0 / (rk * ck) * (p / pk) ** (-(g + 1.0) / (2.0 * g))
    return f, df


def star_state(rl, ul, pl, rr, ur, pr, g):
    cl, cr = np.sqrt(g * pl / rl), np.sqrt(g * pr / rr)
    p = max(1e-12, 0.5 * (pl + pr) - 0.125 * (ur - ul) * (rl + rr) * (cl + cr))
    for _ in range(200):
        fl, dfl = _fk(p, rl, pl, cl, g)
        fr, dfr = _fk(p, rr, pr, cr, g)
        dp = (fl + fr + ur - ul) / (dfl + dfr)
        pn = max(1e-14, p - dp)
        if abs(pn - p) < 1e-15 * (pn + p):
            p = pn
            break
        p = pn
    fl, _ = _fk(p, rl, pl, cl, g)
    fr, _ = _fk(p, rr, pr, cr, g)
    u = 0.5 * (ul + ur) + 0.5 * (fr - fl)
    return p, u


def sample(xi, rl, ul, pl, rr, ur, pr, g):
    """(rho, u, p) at similarity coordinate xi = x/t."""
    ps, us = star_state(rl, ul, pl, rr, ur, pr, g)
    cl, cr = np.sqrt(g * pl / rl), np.sqrt(g * pr / rr)
    if xi <= us:  # left of contact
        if ps > pl:
            sl = ul - cl * np.sqrt((g + 1) / (2 * g) * ps / pl + (g - 1) / (2 * g))
            if xi <= sl:
                return rl, ul, pl
            r = rl * (ps / pl + (g - 1) / (g + 1)) / ((g - 1) / (g + 1) * ps / pl + 1)
            return r, us, ps
        csl = cl * (ps / pl) ** ((g - 1) / (2 * g))
        shl, stl = ul - cl, us - csl
        if xi <= shl:
            return rl, ul, pl
        if xi >= stl:
            return rl * (ps / pl) ** (1 / g), us, ps
        c = 2 / (g + 1) * (cl + (g - 1) / 2 * (ul - xi))
        u = 2 / (g + 1) * (cl + (g - 1) / 2 * ul + xi)
        r = rl * (c / cl) ** (2 / (g - 1))
        return r, u, pl * (c / cl) ** (2 * g / (g - 1))
    if ps > pr:
        sr = ur + cr * np.sqrt((g + 1) / (2 * g) * ps / pr + (g - 1) / (2 * g))
        if xi >= sr:
            return rr, ur, pr
        r = rr * (ps / pr + (g - 1) / (g + 1)) / ((g - 1) / (g + 1) * ps / pr + 1)
        return r, us, ps
    csr = cr * (ps / pr) ** ((g - 1) / (2 * g))
    shr, str_ = ur + cr, us + csr
    if xi >= shr:
        return rr, ur, pr
    if xi <= str_:
        return rr * (ps / pr) ** (1 / g), us, ps
    c = 2 / (g + 1) * (cr - (g - 1) / 2 * (ur - xi))
    u = 2 / (g + 1) * (-cr + (g - 1) / 2 * ur + xi)
    r = rr * (c / cr) ** (2 / (g - 1))
    return r, u, pr * (c / cr) ** (2 * g / (g - 1))


def profile(x, t, x0, left, right, g):
    """Exact density, velocity and pressure at points x and time t."""
    out = np.array([sample((xx - x0) / t, *left, *right, g) for xx in np.asarray(x)])
    return out[:, 0], out[:, 1], out[:, 2]


def cell_average(xl, xr, t, x0, left, right, g, sub=64):
    """Cell averages of the exact density over cells [xl, xr] (midpoint rule
    with ``sub`` points per cell)."""
    xl, xr = np.asarray(xl), np.asarray(xr)
    s = (np.arange(sub) + 0.5) / sub
    pts = xl[:, None] + (xr - xl)[:, None] * s[None, :]
    r, _, _ = profile(pts.ravel(), t, x0, left, right, g)
    return r.reshape(pts.shape).mean(axis=1)
