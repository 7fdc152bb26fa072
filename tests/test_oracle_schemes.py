"""Accuracy of the paper's old face-centre scheme against the new 26-point
scheme (section IV-B), both run by the CPU oracle on the 32^3 Sedov blast to
a shock radius of 0.3 and compared with the self-similar solution
(sedov_similarity.py): the density-profile L1 error, the shock radius, and
the anisotropy of the shock (its radius along a body diagonal against its
radius along a coordinate axis; a grid-aligned error shows there).  Both
schemes conserve mass and energy to round-off; the comparison is printed and
kept in the design notes."""
import pytest

import sedov_metrics as sm
from paper_2107_10987_amd.workloads import sedov_uniform


def _run(oracle_mod, centre_only, R_target=0.3):
    w = sedov_uniform(4)
    o = oracle_mod.Oracle(w.tree, w.gamma, 0.0, centre_only=centre_only)
    t_end = sm.end_time(R_target, w.gamma)
    U, t, steps = w.U, 0.0, 0
    M0 = U[:, 0].sum()
    E0 = U[:, 4].sum()
    while t < t_end - 1e-14:
        dt = min(o.dt(U), t_end - t)
        U, _ = o.step(dt, U)
        t += dt
        steps += 1
    assert abs(U[:, 0].sum() - M0) <= 1e-13 * M0
    assert abs(U[:, 4].sum() - E0) <= 1e-13 * E0
    d = sm.metrics(w.tree, U, R_target, w.gamma)
    d["steps"] = steps
    return d


@pytest.mark.slow
def test_old_and_new_scheme_accuracy_on_sedov(oracle_mod):
    new = _run(oracle_mod, False)
    old = _run(oracle_mod, True)
    for name, d in (("new (9 points per face)", new), ("old (face centre)", old)):
        print(sm.describe(name, d, d["steps"]), flush=True)
    for d in (new, old):
        assert abs(d["r_peak"] - d["R"]) <= 0.05 * d["R"]
        assert d["rho_max"] <= 4.0
        assert d["l1"] < 0.5
