"""Sedov-Taylor pin of the oracle: a point blast of energy E in gas of density
rho0 has its shock at R = xi0 (E t^2 / rho0)^(1/5), with xi0(gamma) from the
self-similar solution (computed in sedov_similarity.py, not assumed); the
density jump cannot exceed the strong-shock limit (gamma+1)/(gamma-1) = 4; and
the total energy is conserved while the shock is inside the box."""
import numpy as np

import sedov_similarity as ss
from paper_2107_10987_amd.workloads import sedov_uniform


def _radial_profile(w, U):
    xc = w.tree.cell_centres()
    r = np.sqrt((xc ** 2).sum(axis=1)).ravel()
    rho = U[:, 0].ravel()
    dx = w.tree.dx0
    edges = np.arange(0.0, 0.5, dx)
    idx = np.digitize(r, edges)
    prof = np.array([rho[idx == i].mean() for i in range(1, len(edges))])
    return 0.5 * (edges[1:] + edges[:-1]), prof, rho


def test_similarity_constant_matches_classic_value():
    # Sedov's classic constant for gamma = 7/5 is 1.033
    assert abs(ss.xi0(1.4) - 1.033) < 1e-3


def test_sedov_shock_radius_32cubed(oracle_mod):
    w = sedov_uniform(4)                       # 32^3 cells, outflow, E = 1
    o = oracle_mod.Oracle(w.tree, w.gamma, 0.0)
    xi = ss.xi0(w.gamma)
    E0 = w.U[:, 4].sum() * w.tree.dx0 ** 3
    U, t = w.U, 0.0
    radii = []
    for R_target in (0.2, 0.3):
        t_end = (R_target / xi) ** 2.5
        while t < t_end - 1e-14:
            dt = min(o.dt(U), t_end - t)
            U, _ = o.step(dt, U)
            t += dt
        rc, prof, rho = _radial_profile(w, U)
        r_peak = rc[np.argmax(prof)]
        assert abs(r_peak - R_target) <= 0.05 * R_target, (r_peak, R_target)
        assert rho.max() <= (w.gamma + 1) / (w.gamma - 1)
        E = U[:, 4].sum() * w.tree.dx0 ** 3
        assert abs(E - E0) <= 1e-13 * E0
        radii.append(r_peak)
    # R grows as t^(2/5)
    assert radii[1] > radii[0]
