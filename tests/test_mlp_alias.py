"""Host checks of the learned reconstruction's shared-row table
(hydro_mlp_alias_map), no GPU needed.  A face-adjacent ghost cell of one
block may take its network row from the cell it copies in another block only
if the two 3x3x3 neighbourhoods hold the same values in every state: checked
here against the oracle's own ghost fill (an independent implementation) on
random states, with the expected sharing on uniform meshes: every ghost slab
shared on a periodic mesh, none at an outflow boundary (a zero-gradient ghost
copies the boundary cell, whose neighbourhood differs)."""
import os

import numpy as np
import pytest

from paper_2107_10987_amd import hydro
from paper_2107_10987_amd.build import LIB
from paper_2107_10987_amd.workloads import (OUTFLOW, PERIODIC, LeafSet, rotating_polytrope, sedov_uniform,
                                            uniform_tree)

pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="libhydro.so not built")


def _ghost_cell(s):
    """(i, j, k) of ghost-slab slot 512 + s (slab x-, x+, y-, y+, z-, z+)."""
    slab, u, v = s // 64, s % 8, (s // 8) % 8
    e = 8 if slab & 1 else -1
    if slab < 2:
        return e, u, v
    if slab < 4:
        return u, e, v
    return u, v, e


def _nbhd(P, i, j, k):
    """The 3x3x3 neighbourhood (7 fields) of cell (i, j, k) of a padded block
    [7][14][14][14] (index 0 is cell -3)."""
    return P[:, k + 2:k + 5, j + 2:j + 5, i + 2:i + 5]


def _amr(bc):
    ls = LeafSet((2, 2, 2), bc, (0, 0, 0), 1 / 16,
                 [(0, i, j, k) for i in range(2) for j in range(2) for k in range(2)])
    ls.refine(0, (0, 0, 0))
    if ls.can_refine(1, (0, 0, 0)):
        ls.refine(1, (0, 0, 0))
    return ls.tree()


@pytest.mark.parametrize("make", ["amr_out", "amr_per", "polytrope"])
def test_shared_rows_have_equal_neighbourhoods(oracle_mod, make):
    if make == "polytrope":
        tree = rotating_polytrope().tree
    else:
        tree = _amr((OUTFLOW,) * 3 if make == "amr_out" else (PERIODIC, OUTFLOW, PERIODIC))
    al = hydro.mlp_alias_map(tree, hydro.ghost_map(tree))
    assert al.shape == (tree.n, 384)
    o = oracle_mod.Oracle(tree)
    n = min(tree.n, 400)
    U = np.random.default_rng(5).uniform(0.5, 2.0, (tree.n, 7, 8, 8, 8))
    P = o.padded(U)
    shared = 0
    for b in range(n):
        for s in np.nonzero(al[b] >= 0)[0]:
            b2, s2 = divmod(int(al[b, s]), 896)
            assert s2 < 512                                    # an interior cell of b2
            ci, cj, ck = s2 % 8, (s2 // 8) % 8, s2 // 64
            i, j, k = _ghost_cell(int(s))
            assert np.array_equal(_nbhd(P[b], i, j, k), _nbhd(P[b2], ci, cj, ck)), (b, s, b2, s2)
            shared += 1
    assert shared > 0


def test_uniform_periodic_mesh_shares_every_slab():
    tree = uniform_tree((4, 4, 4), (PERIODIC,) * 3)
    al = hydro.mlp_alias_map(tree, hydro.ghost_map(tree))
    assert np.all(al >= 0)


def test_outflow_boundary_slabs_are_not_shared():
    w = sedov_uniform(4)                     # 4^3 leaves of 8^3, outflow on every side
    al = hydro.mlp_alias_map(w.tree, hydro.ghost_map(w.tree))
    coord = w.tree.arrays()["coord"].reshape(-1, 3)
    for b in range(w.tree.n):
        for slab in range(6):
            a, side = slab // 2, slab & 1
            at_boundary = coord[b, a] == (3 if side else 0)
            rows = al[b, 64 * slab:64 * slab + 64]
            assert np.all(rows < 0) if at_boundary else np.all(rows >= 0), (b, slab)
