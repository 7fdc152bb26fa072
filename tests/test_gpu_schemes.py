"""The paper's old face-centre scheme against the new 26-point scheme
(section IV-B) on the GPU at the 64^3 Sedov blast of the benchmark, run to a
shock radius of 0.3 and compared with the self-similar solution
(sedov_metrics.py): the accuracy half of the A/B whose throughput half is the
benchmark's old-scheme leg.  The oracle makes the same comparison at 32^3
(test_oracle_schemes.py).  Both schemes must put the shock within a cell of
the exact radius and conserve mass and energy to round-off; the new scheme's
edge and corner points must make the shock more isotropic (the density peak
along a body diagonal closer to the one along an axis, less angular scatter
in the shells around the shock)."""
import numpy as np
import pytest

import sedov_metrics as sm
from paper_2107_10987_amd.workloads import sedov_uniform

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _run(torch, centre_only, R=0.3):
    from paper_2107_10987_amd.hydro import Hydro
    w = sedov_uniform(8)
    hy = Hydro(max_leaves=w.n, schedule="column", centre_only=centre_only)
    try:
        g = hy.grid(w.tree, torch.tensor(w.U, device="cuda"), w.omega, w.gamma)
        t_end = sm.end_time(R, w.gamma)
        t, steps = 0.0, 0
        M0, E0 = w.U[:, 0].sum(), w.U[:, 4].sum()
        while t < t_end - 1e-14:
            a = hy.signal_speed(g).cpu().numpy()
            dt = min(float(w.cfl * np.min(w.tree.dx / a)), t_end - t)
            hy.step(g, dt)
            t += dt
            steps += 1
        U = g.U.cpu().numpy()
    finally:
        hy.close()
    assert abs(U[:, 0].sum() - M0) <= 1e-12 * M0
    assert abs(U[:, 4].sum() - E0) <= 1e-12 * E0
    d = sm.metrics(w.tree, U, R, w.gamma)
    d["steps"] = steps
    d["dx"] = w.tree.dx0
    return d


def test_old_and_new_scheme_accuracy_on_sedov_64(torch):
    print("case: Sedov 64^3 to R = 0.3, new and old scheme", flush=True)
    new = _run(torch, False)
    old = _run(torch, True)
    for name, d in (("new (9 points per face)", new), ("old (face centre)", old)):
        print(sm.describe(name, d, d["steps"]), flush=True)
    for d in (new, old):
        assert abs(d["r_peak"] - d["R"]) <= d["dx"] + 1e-12
        assert d["l1"] < 0.5
    aniso_new = abs(new["rho_diag"] / new["rho_axis"] - 1.0)
    aniso_old = abs(old["rho_diag"] / old["rho_axis"] - 1.0)
    print(f"diagonal/axis peak density - 1: new {aniso_new:.4f}, old {aniso_old:.4f}", flush=True)
    assert aniso_new < aniso_old
    assert new["scatter"] < old["scatter"]
