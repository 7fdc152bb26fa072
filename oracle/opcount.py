"""Algorithmic FP64 operation count of one cell-update, from the counting
build of the oracle (opcount.cpp).  TEST INFRASTRUCTURE.

The count covers the work the method needs per interior cell and stage:
  * PPM on 19.75 lines per cell and field: a leaf reconstructs 13 lines at
    each of its 512 cells and 9 lines at each of the 384 ghost cells that
    share a face with it, (512*13 + 384*9)/512 = 19.75;
  * 30.375 face-point fluxes per cell: 3 axes x 9 faces x 64 x 9 points / 512;
  * Simpson accumulation, point positions, flux divergence and source;
  * the stage combine and, in the second stage, the tracer resync.
The oracle reconstructs a few more cells than needed (every cell -1..8 per
axis); those lines are subtracted.  Flops are adds, subtracts, multiplies,
divides, square roots and powers; comparisons are reported apart.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "opcount.cpp")
LIB = os.path.join(HERE, "_build", "libopcount.so")

LINES_PER_CELL = (512 * 13 + 384 * 9) / 512          # 19.75
POINTS_PER_CELL = 3 * 9 * 64 * 9 / 512               # 30.375
ORACLE_RECON_CELLS = 10 ** 3                         # cells -1..8 per axis
NEEDED_RECON_LINES = 512 * 13 + 384 * 9


def build(force: bool = False) -> str:
    os.makedirs(os.path.dirname(LIB), exist_ok=True)
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < max(
            os.path.getmtime(SRC), os.path.getmtime(os.path.join(HERE, "hydro_oracle.c"))):
        subprocess.check_call(["g++", "-O1", "-ffp-contract=off", "-std=c++17", "-fPIC", "-shared",
                               "-o", LIB + ".tmp", SRC])
        os.replace(LIB + ".tmp", LIB)
    return LIB


def _lib():
    L = C.CDLL(build())
    dp = C.POINTER(C.c_double)
    L.opcount_reset.argtypes = []
    L.opcount_read.argtypes = [C.POINTER(C.c_uint64), C.POINTER(C.c_uint64)]
    L.opcount_ppm.argtypes = [dp, dp]
    L.opcount_point_flux.argtypes = [C.c_int, dp, dp, dp, C.c_double, C.c_double, C.c_double, dp]
    L.opcount_point_flux.restype = C.c_double
    L.opcount_leaf_rhs.argtypes = [dp, C.c_double, dp, C.c_double, C.c_double, C.c_double, C.c_int, dp]
    return L


def _p(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _read(L):
    f, c = C.c_uint64(), C.c_uint64()
    L.opcount_read(C.byref(f), C.byref(c))
    return f.value, c.value


def smooth_block(seed=0, gamma=5.0 / 3.0):
    """A smooth, non-degenerate padded state (no limiter clipping, no tracer
    pressure): the common path of every step of the method."""
    rng = np.random.default_rng(seed)
    r = np.arange(-3, 11, dtype=float) / 14.0
    k, j, i = np.meshgrid(r, r, r, indexing="ij")
    a = rng.uniform(0.2, 0.4, size=(7, 3))
    rho = 1.0 + a[0, 0] * i + a[0, 1] * j + a[0, 2] * k
    v = [0.1 + a[f, 0] * i + a[f, 1] * j + a[f, 2] * k for f in (1, 2, 3)]
    p = 1.0 + a[4, 0] * i + a[4, 1] * j + a[4, 2] * k
    P = np.empty((7, 14, 14, 14))
    P[0] = rho
    for d in range(3):
        P[1 + d] = rho * v[d]
    e = p / (gamma - 1.0)
    P[4] = e + 0.5 * rho * (v[0] ** 2 + v[1] ** 2 + v[2] ** 2)
    P[5] = e ** (1.0 / gamma)
    P[6] = rho * (0.5 + a[6, 0] * i)
    return np.ascontiguousarray(P)


def counts(gamma=5.0 / 3.0, omega=0.1):
    """Per-step counts {name: (flops, comparisons)} and the total flops per
    interior cell-update of one stage (mean of the two stages)."""
    L = _lib()
    P = smooth_block(gamma=gamma)
    # one PPM line (both ends)
    L.opcount_reset()
    q = np.ascontiguousarray(P[0, 3, 3, 3:8])
    lr = np.zeros(2)
    L.opcount_ppm(_p(q), _p(lr))
    ppm = _read(L)
    # one face-point flux
    UL = np.ascontiguousarray(P[:, 6, 6, 6])
    UR = np.ascontiguousarray(P[:, 6, 6, 7])
    x = np.array([0.1, 0.2, 0.3])
    F = np.zeros(7)
    L.opcount_reset()
    L.opcount_point_flux(0, _p(UL), _p(UR), _p(x), gamma, omega, 1e-3, _p(F))
    flux = _read(L)
    # whole L(U) of a leaf as the oracle computes it
    dU = np.zeros((7, 512))
    L.opcount_reset()
    L.opcount_leaf_rhs(_p(P), 1.0 / 64, _p(np.zeros(3)), gamma, omega, 1e-3, 0, _p(dU))
    rhs = _read(L)
    oracle_lines = ORACLE_RECON_CELLS * 13 * 7
    needed_lines = NEEDED_RECON_LINES * 7
    rhs_needed = rhs[0] - (oracle_lines - needed_lines) * ppm[0]
    # stage combine: stage 1 u + dt L (2 per field); stage 2 (Un + (u + dt L))/2
    # (4 per field) plus the resync (1/rho, kinetic energy 7, e, eta2 E: 10)
    combine = (2 * 7 + (4 * 7 + 10)) / 2.0
    per_cell = rhs_needed / 512.0 + combine
    parts = {"ppm_line": ppm, "point_flux": flux, "leaf_rhs_oracle": rhs,
             "leaf_rhs_needed_flops": rhs_needed, "combine_mean": combine}
    return parts, per_cell


# the old face-centre scheme: the axis line of every interior cell in each
# direction and, at each face-adjacent ghost cell, the axis line normal to its
# slab; one flux point per face
OLD_NEEDED_RECON_LINES = 512 * 3 + 384 * 1         # 3.75 per cell
OLD_POINTS_PER_LEAF = 3 * 9 * 64


def counts_old(gamma=5.0 / 3.0, omega=0.1):
    """Flops per interior cell-update of one stage (mean of the two stages)
    of the old scheme: the oracle's L(U) with one point per face, less the
    lines it reconstructs beyond the 3.75 per cell and field the scheme needs
    and less the multiplications by the unit face weight."""
    L = _lib()
    P = smooth_block(gamma=gamma)
    q = np.ascontiguousarray(P[0, 3, 3, 3:8])
    lr = np.zeros(2)
    L.opcount_reset()
    L.opcount_ppm(_p(q), _p(lr))
    ppm = _read(L)
    dU = np.zeros((7, 512))
    L.opcount_reset()
    L.opcount_leaf_rhs(_p(P), 1.0 / 64, _p(np.zeros(3)), gamma, omega, 1e-3, 1, _p(dU))
    rhs = _read(L)
    surplus = (ORACLE_RECON_CELLS * 13 - OLD_NEEDED_RECON_LINES) * 7
    rhs_needed = rhs[0] - surplus * ppm[0] - OLD_POINTS_PER_LEAF * 7
    combine = (2 * 7 + (4 * 7 + 10)) / 2.0
    return rhs_needed / 512.0 + combine


if __name__ == "__main__":
    parts, per_cell = counts()
    for k, v in parts.items():
        print(k, v)
    print("flops per cell-update", per_cell)
    print("old scheme: flops per cell-update", counts_old())
