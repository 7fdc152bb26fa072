"""Seeded synthetic initial states for the hydro workloads.

Each setup returns a :class:`Workload`: an octree leaf layout plus the conserved
state ``U[n][7][8][8][8]`` (float64, field order rho, sx, sy, sz, E, tau, X;
cells indexed [k][j][i] with i fastest), the rotation rate and gamma.  The
workloads stand in for the paper's Sedov-Taylor blast (section V-A) and
rotating-star (section V-B) inputs, which are not available; they take the
paper's shapes: 8^3 leaves with three ghost layers.

Converting the initial pressure to a total energy and an entropy tracer is
input preparation shared by both implementations; no step of the hydro
update is computed here.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from .tree import (NX, OUTFLOW, PERIODIC, LeafSet, Tree, box_distance, morton_of,
                   uniform_tree)

NF = 7
RHO, SX, SY, SZ, EGAS, TAU, SPC = range(NF)
FIELD_NAMES = ("rho", "sx", "sy", "sz", "egas", "tau", "spc")
GAMMA = 5.0 / 3.0


@dataclass
class Workload:
    name: str
    tree: Tree
    U: np.ndarray
    omega: float
    gamma: float = GAMMA
    cfl: float = 0.4
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return self.tree.n

    @property
    def cells(self) -> int:
        return self.tree.n * self.tree.leaf_edge ** 3


def conserved_from_primitive(rho, vx, vy, vz, p, spc, gamma):
    """Stack (rho, s, E, tau, X) with E = p/(gamma-1) + rho|v|^2/2 and
    tau = (p/(gamma-1))**(1/gamma)."""
    rho = np.asarray(rho, dtype=np.float64)
    U = np.empty((rho.shape[0], 7) + rho.shape[1:], dtype=np.float64)
    eint = p / (gamma - 1.0)
    U[:, 0] = rho
    np.multiply(rho, vx, out=U[:, 1])
    np.multiply(rho, vy, out=U[:, 2])
    np.multiply(rho, vz, out=U[:, 3])
    U[:, 4] = eint + 0.5 * rho * (vx * vx + vy * vy + vz * vz)
    np.power(eint, 1.0 / gamma, out=U[:, 5])
    U[:, 6] = spc
    return U


# --------------------------------------------------------------------------
# small blast in one periodic leaf
# --------------------------------------------------------------------------
def blast_single_leaf(seed: int = 0, gamma: float = GAMMA) -> Workload:
    """One periodic 8^3 leaf on [0,1]^3, dx = 1/8.

    rho = 1 + 1e-6 * U(-1,1) noise drawn from ``default_rng(seed)`` in [k][j][i]
    order, zero velocity, p = 1e-5, plus a total energy of 1 spread evenly over
    the 2^3 central cells (i, j, k in {3, 4}).  X = rho.
    """
    tree = uniform_tree((1, 1, 1), (PERIODIC,) * 3, (0.0, 0.0, 0.0), 1.0 / NX)
    xi = np.random.default_rng(seed).uniform(-1.0, 1.0, (NX, NX, NX))
    rho = (1.0 + 1e-6 * xi)[None]
    z = np.zeros_like(rho)
    p = np.full_like(rho, 1e-5)
    U = conserved_from_primitive(rho, z, z, z, p, rho.copy(), gamma)
    dx = 1.0 / NX
    boost = 1.0 / (8.0 * dx ** 3)
    U[0, EGAS, 3:5, 3:5, 3:5] += boost
    U[0, TAU] = (U[0, EGAS]) ** (1.0 / gamma)
    return Workload("blast-1leaf", tree, np.ascontiguousarray(U), 0.0, gamma)


# --------------------------------------------------------------------------
# Sedov-Taylor blast on a uniform grid of leaves
# --------------------------------------------------------------------------
def sedov_uniform(leaves_per_axis: int = 8, gamma: float = GAMMA, e_blast: float = 1.0,
                  p_amb: float = 1e-5, rho_amb: float = 1.0, leaf_edge: int = NX) -> Workload:
    """Uniform (E m)^3 grid on [-1/2, 1/2]^3 as m^3 leaves of E^3 cells
    (E = leaf_edge, 8 or 16) with outflow faces.

    rho = 1, v = 0, p = 1e-5, and an energy ``e_blast`` deposited uniformly in
    the 2^3 cells around the box centre.  X = rho.
    """
    m = int(leaves_per_axis)
    E = int(leaf_edge)
    ncell = E * m
    tree = uniform_tree((m, m, m), (OUTFLOW,) * 3, (-0.5, -0.5, -0.5), 1.0 / ncell, leaf_edge=E)
    n = tree.n
    rho = np.full((n, E, E, E), rho_amb)
    z = np.zeros_like(rho)
    p = np.full_like(rho, p_amb)
    U = conserved_from_primitive(rho, z, z, z, p, rho.copy(), gamma)
    dx = 1.0 / ncell
    c = ncell // 2
    g = tree.coord[:, :, None] * E + np.arange(E)[None, None, :]        # [n, 3, E] global index
    inx = (g[:, 0] == c - 1) | (g[:, 0] == c)
    iny = (g[:, 1] == c - 1) | (g[:, 1] == c)
    inz = (g[:, 2] == c - 1) | (g[:, 2] == c)
    mask = inz[:, :, None, None] & iny[:, None, :, None] & inx[:, None, None, :]
    U[:, EGAS][mask] += e_blast / (8.0 * dx ** 3)
    eint = U[:, EGAS]
    U[:, TAU] = eint ** (1.0 / gamma)
    return Workload(f"sedov-{ncell}^3", tree, np.ascontiguousarray(U), 0.0, gamma,
                    meta=dict(e_blast=e_blast, rho_amb=rho_amb))


# --------------------------------------------------------------------------
# Lane-Emden polytropes
# --------------------------------------------------------------------------
def lane_emden(n: float = 1.5, h: float = 1e-4):
    """theta(xi) for the Lane-Emden equation of index n by classical RK4.

    Returns (xi, theta, xi1) where xi1 is the first zero, found by linear
    interpolation of the last step.
    """
    def rhs(x, y):
        th, dth = y
        t = max(th, 0.0)
        return np.array([dth, -t ** n - 2.0 * dth / x])

    x = 1e-6
    y = np.array([1.0 - x * x / 6.0, -x / 3.0])
    xs, ts = [0.0, x], [1.0, y[0]]
    while y[0] > 0.0:
        k1 = rhs(x, y)
        k2 = rhs(x + h / 2, y + h / 2 * k1)
        k3 = rhs(x + h / 2, y + h / 2 * k2)
        k4 = rhs(x + h, y + h * k3)
        y = y + h / 6 * (k1 + 2 * k2 + 2 * k3 + k4)
        x += h
        xs.append(x)
        ts.append(y[0])
    xs, ts = np.array(xs), np.array(ts)
    x1 = xs[-2] + (xs[-1] - xs[-2]) * ts[-2] / (ts[-2] - ts[-1])
    return xs, ts, float(x1)


_LE_CACHE: dict = {}


def _le():
    if "t" not in _LE_CACHE:
        _LE_CACHE["t"] = lane_emden()
    return _LE_CACHE["t"]


def polytrope_density(r, R, rho_c):
    xs, ts, x1 = _le()
    xi = np.asarray(r) / R * x1
    th = np.interp(xi, xs, np.maximum(ts, 0.0), right=0.0)
    return rho_c * th ** 1.5


def polytrope_K(R, rho_c, G=1.0, n=1.5):
    _, _, x1 = _le()
    return 4.0 * np.pi * G * R * R * rho_c ** (1.0 / 3.0) / ((n + 1.0) * x1 * x1)


def polytrope_mass(R, rho_c, nr: int = 20000):
    r = np.linspace(0.0, R, nr + 1)
    f = 4.0 * np.pi * r * r * polytrope_density(r, R, rho_c)
    return float(np.sum(0.5 * (f[1:] + f[:-1]) * np.diff(r)))


# --------------------------------------------------------------------------
# AMR trees with exact leaf counts
# --------------------------------------------------------------------------
def _dist_key(centres):
    def key(ls: LeafSet, lf):
        lo, hi = ls.node_box(lf[0], lf[1:])
        mid = 0.5 * (lo + hi)
        d = min(np.linalg.norm(mid - np.asarray(c)) / rr for (c, rr) in centres)
        return (round(d, 12), morton_of(ls, lf))
    return key


def _intersects(centres):
    def sel(ls: LeafSet, lf):
        lo, hi = ls.node_box(lf[0], lf[1:])
        return any(box_distance(lo, hi, np.asarray(c)) <= rr for (c, rr) in centres)
    return sel


def polytrope_tree(radius: float = 0.3, target_leaves: int = 4096) -> Tree:
    """Three-level octree with exactly ``target_leaves`` leaves.

    Root grid of 8^3 leaves on [-1/2,1/2]^3 (outflow).  Level 0: split every
    leaf touching the ball r <= radius.  Level 1: split leaves closest to the
    origin first (ties by Morton key), skipping any split that would break 2:1
    balance, until the leaf count is reached.
    """
    ls = LeafSet((8, 8, 8), (OUTFLOW,) * 3, (-0.5,) * 3, 1.0 / 64,
                 [(0, i, j, k) for i in range(8) for j in range(8) for k in range(8)])
    centres = [((0.0, 0.0, 0.0), radius)]
    m = ls.refine_level(0, _dist_key(centres), select=_intersects(centres))
    need = (target_leaves - len(ls.leaves)) // 7
    if (target_leaves - len(ls.leaves)) % 7:
        raise ValueError("leaf count not reachable")
    got = ls.refine_level(1, _dist_key(centres), count=need)
    if got != need:
        raise RuntimeError(f"only {got} of {need} level-1 splits keep 2:1 balance")
    assert len(ls.leaves) == target_leaves and ls.check_balance()
    return ls.tree(dict(level0_splits=m, level1_splits=got))


def rotating_polytrope(omega: float = 0.1, radius: float = 0.3, rho_c: float = 1.0,
                       rho_atm: float = 1e-10, gamma: float = GAMMA,
                       target_leaves: int = 4096) -> Workload:
    """n = 1.5 polytrope of radius 0.3 centred at the origin on a 3-level AMR
    octree, co-rotating (s = rho * Omega x r) in a frame rotating at ``omega``
    about the z axis.  p = K rho^(5/3); atmosphere rho = 1e-10.  X = rho."""
    tree = polytrope_tree(radius, target_leaves)
    xc = tree.cell_centres()
    r = np.sqrt(np.sum(xc * xc, axis=1))
    rho = np.maximum(polytrope_density(r, radius, rho_c), rho_atm)
    K = polytrope_K(radius, rho_c)
    p = K * rho ** gamma
    vx = -omega * xc[:, 1]
    vy = omega * xc[:, 0]
    vz = np.zeros_like(rho)
    U = conserved_from_primitive(rho, vx, vy, vz, p, rho.copy(), gamma)
    return Workload("polytrope-4096", tree, np.ascontiguousarray(U), omega, gamma,
                    meta=dict(K=K, radius=radius))


def binary_tree(stars, target_leaves: int = 32768) -> Tree:
    """Four-level octree over a 16^3 root grid with exactly ``target_leaves``.

    Levels 0 and 1: split every leaf touching either star.  Level 2: split the
    leaves closest to a star (distance over that star's radius) first, skipping
    splits that would break 2:1 balance, until the leaf count is reached.
    """
    ls = LeafSet((16, 16, 16), (OUTFLOW,) * 3, (-0.5,) * 3, 1.0 / 128,
                 [(0, i, j, k) for i in range(16) for j in range(16) for k in range(16)])
    key, sel = _dist_key(stars), _intersects(stars)
    ls.refine_level(0, key, select=sel)
    ls.refine_level(1, key, select=sel)
    rest = target_leaves - len(ls.leaves)
    if rest < 0 or rest % 7:
        raise ValueError("leaf count not reachable")
    got = ls.refine_level(2, key, count=rest // 7)
    if got != rest // 7:
        raise RuntimeError("not enough balanced level-2 splits")
    assert len(ls.leaves) == target_leaves and ls.check_balance()
    return ls.tree()


def binary_star(mass_ratio: float = 0.5, separation: float = 0.5, r1: float = 0.12,
                rho_c1: float = 1.0, rho_atm: float = 1e-10, gamma: float = GAMMA,
                target_leaves: int = 32768) -> Workload:
    """Two n = 1.5 polytropes with the same K, mass ratio 0.5 and separation
    0.5, on the x axis about their centre of mass, co-rotating at the Keplerian
    rate Omega = sqrt(G (M1+M2) / a^3).  X = rho inside star 1, 0 elsewhere."""
    r2 = r1 * mass_ratio ** (-1.0 / 3.0)
    rho_c2 = rho_c1 * mass_ratio ** 2
    m1, m2 = polytrope_mass(r1, rho_c1), polytrope_mass(r2, rho_c2)
    x1 = -separation * m2 / (m1 + m2)
    x2 = separation * m1 / (m1 + m2)
    omega = float(np.sqrt((m1 + m2) / separation ** 3))
    stars = [((x1, 0.0, 0.0), r1), ((x2, 0.0, 0.0), r2)]
    tree = binary_tree(stars, target_leaves)
    xc = tree.cell_centres()
    d1 = np.sqrt((xc[:, 0] - x1) ** 2 + xc[:, 1] ** 2 + xc[:, 2] ** 2)
    d2 = np.sqrt((xc[:, 0] - x2) ** 2 + xc[:, 1] ** 2 + xc[:, 2] ** 2)
    rho1 = polytrope_density(d1, r1, rho_c1)
    rho2 = polytrope_density(d2, r2, rho_c2)
    rho = np.maximum(rho1 + rho2, rho_atm)
    K = polytrope_K(r1, rho_c1)
    p = K * rho ** gamma
    vx = -omega * xc[:, 1]
    vy = omega * xc[:, 0]
    spc = np.where(rho1 > 0.0, rho, 0.0)
    U = conserved_from_primitive(rho, vx, vy, np.zeros_like(rho), p, spc, gamma)
    return Workload("binary-32768", tree, np.ascontiguousarray(U), omega, gamma,
                    meta=dict(m1=m1, m2=m2, stars=stars))


# --------------------------------------------------------------------------
# uneven batches
# --------------------------------------------------------------------------
def uneven_batches(n_leaves: int, seed: int = 2107, max_size: int = 4096) -> np.ndarray:
    """Partition leaves 0..n-1 (Morton order) into consecutive batches whose
    sizes are floor(exp(U(0, ln(max_size+1)))) drawn from ``default_rng(seed)``;
    the last batch is truncated.  Returns offsets [n_batches + 1]."""
    rng = np.random.default_rng(seed)
    offs = [0]
    while offs[-1] < n_leaves:
        s = int(np.floor(np.exp(rng.uniform(0.0, np.log(max_size + 1)))))
        s = max(1, min(s, max_size))
        offs.append(min(n_leaves, offs[-1] + s))
    return np.asarray(offs, dtype=np.int32)
