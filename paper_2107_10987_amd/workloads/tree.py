"""Octree leaf layouts for the hydro workloads.

The mesh is an adaptive octree whose every node is either a leaf or split
into eight children at twice the resolution; the evolved fields live on the
leaves, each an 8^3 block of cells (paper section IV-B).  A layout here is a
set of leaves over a root grid of ``nb`` level-0 leaves per axis, each leaf
named by its level and its integer coordinates at that level.

This module only describes geometry.  It holds none of the hydro method's
arithmetic: ghost filling, reconstruction and fluxes live in the library and,
independently, in the CPU oracle.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Callable, Iterable

import numpy as np

NX = 8            # interior cells per leaf and axis
GHOST = 3         # ghost layers (five-point stencil, section IV-B)
PERIODIC = 0
OUTFLOW = 1


def morton3(ix: np.ndarray, iy: np.ndarray, iz: np.ndarray, bits: int = 21) -> np.ndarray:
    """Interleave the bits of three non-negative integer arrays (x lowest)."""
    ix = np.asarray(ix, dtype=np.uint64)
    iy = np.asarray(iy, dtype=np.uint64)
    iz = np.asarray(iz, dtype=np.uint64)
    key = np.zeros(np.broadcast(ix, iy, iz).shape, dtype=np.uint64)
    for b in range(bits):
        one = np.uint64(1)
        key |= ((ix >> np.uint64(b)) & one) << np.uint64(3 * b)
        key |= ((iy >> np.uint64(b)) & one) << np.uint64(3 * b + 1)
        key |= ((iz >> np.uint64(b)) & one) << np.uint64(3 * b + 2)
    return key


@dataclass
class Tree:
    """Leaves of an octree over a box of ``nb`` root leaves per axis.

    ``level[n]`` and ``coord[n, 3]`` name each leaf; at level ``l`` there are
    ``nb * 2**l`` leaf slots per axis and the cell size is ``dx0 / 2**l``.
    ``bc[a]`` is PERIODIC or OUTFLOW for axis ``a``.  Leaves are kept in Morton
    order of their lower corner at the finest level present.
    """
    nb: np.ndarray
    bc: np.ndarray
    x0: np.ndarray
    dx0: float
    level: np.ndarray
    coord: np.ndarray
    meta: dict = field(default_factory=dict)
    leaf_edge: int = NX      # cells per leaf edge: 8, or 16 (eight 8^3 tiles per leaf)

    @property
    def n(self) -> int:
        return int(self.level.shape[0])

    @property
    def max_level(self) -> int:
        return int(self.level.max()) if self.n else 0

    @property
    def dx(self) -> np.ndarray:
        return self.dx0 / (2.0 ** self.level.astype(np.float64))

    @property
    def origin(self) -> np.ndarray:
        """Centre of cell (0,0,0) of every leaf, shape [n, 3]."""
        dx = self.dx[:, None]
        return self.x0[None, :] + (self.leaf_edge * self.coord.astype(np.float64) + 0.5) * dx

    def cell_centres(self) -> np.ndarray:
        """Centres of all interior cells, shape [n, 3, E, E, E] as (x, y, z)[k][j][i],
        E = leaf_edge."""
        o = self.origin
        dx = self.dx
        E = self.leaf_edge
        r = np.arange(E, dtype=np.float64)
        out = np.empty((self.n, 3, E, E, E))
        out[:, 0] = o[:, 0, None, None, None] + r[None, None, None, :] * dx[:, None, None, None]
        out[:, 1] = o[:, 1, None, None, None] + r[None, None, :, None] * dx[:, None, None, None]
        out[:, 2] = o[:, 2, None, None, None] + r[None, :, None, None] * dx[:, None, None, None]
        return out

    def arrays(self) -> dict:
        """Contiguous typed arrays as passed across the C boundary."""
        return dict(
            nb=np.ascontiguousarray(self.nb, dtype=np.int32),
            bc=np.ascontiguousarray(self.bc, dtype=np.int32),
            level=np.ascontiguousarray(self.level, dtype=np.int32),
            coord=np.ascontiguousarray(self.coord, dtype=np.int32),
            dx=np.ascontiguousarray(self.dx, dtype=np.float64),
            origin=np.ascontiguousarray(self.origin, dtype=np.float64),
            leaf_edge=int(self.leaf_edge),
        )


def _sorted_tree(nb, bc, x0, dx0, leaves: Iterable[tuple], meta=None, leaf_edge: int = NX) -> Tree:
    leaves = sorted(leaves)
    if not leaves:
        raise ValueError("empty tree")
    lv = np.array([l for (l, _, _, _) in leaves], dtype=np.int32)
    co = np.array([[x, y, z] for (_, x, y, z) in leaves], dtype=np.int32)
    lmax = int(lv.max())
    sh = (lmax - lv).astype(np.uint64)
    fine = co.astype(np.uint64) << sh[:, None]
    key = morton3(fine[:, 0], fine[:, 1], fine[:, 2])
    order = np.lexsort((lv, key))
    return Tree(np.asarray(nb, np.int32), np.asarray(bc, np.int32),
                np.asarray(x0, np.float64), float(dx0), lv[order], co[order],
                dict(meta or {}), int(leaf_edge))


def uniform_tree(nb=(1, 1, 1), bc=(PERIODIC,) * 3, x0=(0.0, 0.0, 0.0), dx0=1.0 / NX,
                 leaf_edge: int = NX) -> Tree:
    """All leaves at level 0: a uniform grid of nb[0]*nb[1]*nb[2] leaves."""
    nb = tuple(int(v) for v in nb)
    leaves = [(0, i, j, k) for k in range(nb[2]) for j in range(nb[1]) for i in range(nb[0])]
    return _sorted_tree(nb, bc, x0, dx0, leaves, leaf_edge=leaf_edge)


def split_octets(tree: Tree) -> Tree:
    """The same mesh as leaves of 8^3 cells: leaf L of a 16^3-leaf tree becomes
    the eight 8^3 leaves 8L + t, t = ti + 2 tj + 4 tk for the tile at cell
    offset 8 (ti, tj, tk) (same levels, doubled root grid).  Cells, levels and
    neighbour relations are unchanged, so every ghost cell has the same source."""
    if tree.leaf_edge == NX:
        return tree
    assert tree.leaf_edge == 2 * NX
    t = np.arange(8)
    off = np.stack([t & 1, (t >> 1) & 1, t >> 2], axis=1)                # [8, 3]
    coord = (2 * tree.coord[:, None, :] + off[None]).reshape(-1, 3)
    level = np.repeat(tree.level, 8)
    return Tree(2 * np.asarray(tree.nb, np.int32), np.asarray(tree.bc, np.int32),
                np.asarray(tree.x0, np.float64), float(tree.dx0), level.astype(np.int32),
                coord.astype(np.int32), dict(tree.meta), NX)


def to_tiles8(U: np.ndarray) -> np.ndarray:
    """[n, F, 16, 16, 16] -> [8 n, F, 8, 8, 8] in the leaf order of split_octets."""
    n, F = U.shape[:2]
    V = U.reshape(n, F, 2, NX, 2, NX, 2, NX)                 # (tk, k, tj, j, ti, i)
    return np.ascontiguousarray(V.transpose(0, 2, 4, 6, 1, 3, 5, 7).reshape(8 * n, F, NX, NX, NX))


def from_tiles8(V: np.ndarray) -> np.ndarray:
    """Inverse of to_tiles8."""
    m, F = V.shape[:2]
    n = m // 8
    W = V.reshape(n, 2, 2, 2, F, NX, NX, NX)                 # (tk, tj, ti, f, k, j, i)
    return np.ascontiguousarray(W.transpose(0, 4, 1, 5, 2, 6, 3, 7).reshape(n, F, 2 * NX, 2 * NX, 2 * NX))


class LeafSet:
    """Mutable leaf set used while refining; checks 2:1 balance on every split."""

    def __init__(self, nb, bc, x0, dx0, leaves, leaf_edge: int = NX):
        self.nb = np.asarray(nb, np.int64)
        self.bc = np.asarray(bc, np.int64)
        self.x0 = np.asarray(x0, np.float64)
        self.dx0 = float(dx0)
        self.leaves = set(leaves)
        self.leaf_edge = int(leaf_edge)

    def slots(self, l: int) -> np.ndarray:
        return self.nb << l

    def covered_by_coarser(self, l: int, c) -> bool:
        """Whether the level-l node c lies inside a leaf of level < l."""
        for lc in range(l - 1, -1, -1):
            sh = l - lc
            if (lc, c[0] >> sh, c[1] >> sh, c[2] >> sh) in self.leaves:
                return True
        return False

    def neighbours(self, l: int, c):
        n = self.slots(l)
        for dz in (-1, 0, 1):
            for dy in (-1, 0, 1):
                for dx in (-1, 0, 1):
                    if dx == dy == dz == 0:
                        continue
                    q = [c[0] + dx, c[1] + dy, c[2] + dz]
                    ok = True
                    for a in range(3):
                        if q[a] < 0 or q[a] >= n[a]:
                            if self.bc[a] == PERIODIC:
                                q[a] %= int(n[a])
                            else:
                                ok = False
                    if ok:
                        yield tuple(int(v) for v in q)

    def can_refine(self, l: int, c) -> bool:
        """Splitting leaf (l, c) keeps 2:1 balance iff no face/edge/corner
        neighbour region is covered by a leaf coarser than l."""
        return all(not self.covered_by_coarser(l, q) for q in self.neighbours(l, c))

    def refine(self, l: int, c) -> None:
        self.leaves.remove((l,) + tuple(c))
        for oz in (0, 1):
            for oy in (0, 1):
                for ox in (0, 1):
                    self.leaves.add((l + 1, 2 * c[0] + ox, 2 * c[1] + oy, 2 * c[2] + oz))

    def node_box(self, l: int, c):
        size = self.leaf_edge * self.dx0 / (1 << l)
        lo = self.x0 + np.asarray(c, np.float64) * size
        return lo, lo + size

    def refine_level(self, l: int, key: Callable, count: int | None = None,
                     select: Callable | None = None) -> int:
        """Split level-l leaves in ascending ``key`` order.

        Only leaves for which ``select`` holds are considered; at most ``count``
        are split (all eligible ones if None).  A leaf whose split would break
        2:1 balance is skipped.  Returns the number split.
        """
        cand = [lf for lf in self.leaves if lf[0] == l]
        if select is not None:
            cand = [lf for lf in cand if select(self, lf)]
        cand.sort(key=lambda lf: key(self, lf))
        done = 0
        for lf in cand:
            if count is not None and done >= count:
                break
            c = lf[1:]
            if self.can_refine(l, c):
                self.refine(l, c)
                done += 1
        return done

    def check_balance(self) -> bool:
        """2:1 balance: no leaf touches (by face, edge or corner) a leaf more
        than one level coarser.  Checking the finer side of every pair covers
        both directions."""
        for lf in self.leaves:
            l, c = lf[0], lf[1:]
            if l < 2:
                continue
            for q in self.neighbours(l, c):
                if self.covered_by_coarser(l - 1, (q[0] >> 1, q[1] >> 1, q[2] >> 1)):
                    return False
        return True

    def tree(self, meta=None) -> Tree:
        return _sorted_tree(tuple(self.nb), tuple(self.bc), tuple(self.x0), self.dx0,
                            self.leaves, meta, self.leaf_edge)


def box_distance(lo, hi, p) -> float:
    """Euclidean distance from point p to the axis-aligned box [lo, hi]."""
    d = np.maximum(np.maximum(lo - p, 0.0), p - hi)
    return float(np.sqrt(np.sum(d * d)))


def morton_of(ls: LeafSet, lf) -> int:
    l, x, y, z = lf
    return int(morton3(np.array([x]), np.array([y]), np.array([z]))[0])
