"""The full-size workloads against the configurations the paper prints
(tests/golden/sedov_table.txt: section V-A1, the table of Sedov-Taylor blast
wave details): a uniform octree refined `level` times from one root sub-grid
holds `count` sub-grids and 16,777,216 cells, and the uniform grids built
here for 8^3 and 16^3 leaves have those sizes."""
import os

import numpy as np

from paper_2107_10987_amd.workloads import LeafSet, OUTFLOW, split_octets, uniform_tree

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "sedov_table.txt")


def _rows():
    rows = []
    for line in open(GOLDEN):
        line = line.strip()
        if line and not line.startswith("#"):
            rows.append(tuple(int(v) for v in line.split()))
    return rows


def test_table_is_self_consistent():
    rows = _rows()
    assert [r[0] for r in rows] == [8, 16, 32]
    for edge, count, level in rows:
        assert count * edge ** 3 == 16_777_216
        assert count == 8 ** level          # a uniform octree refined `level` times


def test_uniform_grids_match_table():
    for edge, count, level in _rows():
        if edge == 32:
            continue   # leaves of 8^3 and 16^3 cells are built here
        m = 2 ** level
        t = uniform_tree((m, m, m), (OUTFLOW,) * 3, leaf_edge=edge)
        assert t.n == count and t.n * edge ** 3 == 16_777_216
        if edge == 16:   # the 16^3 mesh is cell for cell the 8^3 one
            t8 = split_octets(t)
            assert t8.n == [c for e, c, _ in _rows() if e == 8][0]


def test_refined_root_equals_uniform_grid():
    # one root sub-grid refined uniformly twice is the 4^3 uniform grid: same
    # leaves (as cells of the finest level), same cell size
    ls = LeafSet((1, 1, 1), (OUTFLOW,) * 3, (0.0, 0.0, 0.0), 1.0 / 8, [(0, 0, 0, 0)])
    ls.refine(0, (0, 0, 0))
    for i in range(2):
        for j in range(2):
            for k in range(2):
                ls.refine(1, (i, j, k))
    t = ls.tree()
    u = uniform_tree((4, 4, 4), (OUTFLOW,) * 3, dx0=1.0 / 32)
    assert t.n == u.n == 64
    assert np.allclose(np.sort(t.dx), np.sort(u.dx))
    key = lambda tr: sorted(map(tuple, (tr.coord * (2 ** (2 - tr.level))[:, None]).tolist()))
    assert key(t) == sorted(map(tuple, u.coord.tolist()))
