"""GPU parity of linear-limited prolongation of ghost cells from coarser
leaves against the CPU oracle with the same option: every schedule, with and
without the coarse/fine flux correction (whose conservation it keeps), 16^3
leaves, the 4096-leaf polytrope in uneven launches, and the learned path's
fallback.  Tolerance (FP64): per field, max |gpu - oracle| / max |oracle_f|
<= 1e-12."""
import numpy as np
import pytest

from paper_2107_10987_amd.workloads import (PERIODIC, LeafSet, conserved_from_primitive,
                                            rotating_polytrope, split_octets, to_tiles8,
                                            uneven_batches)

pytestmark = pytest.mark.gpu
TOL = 1e-12
G = 5.0 / 3.0


@pytest.fixture(scope="module")
def torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _amr_tree(E=8):
    ls = LeafSet((2, 2, 2), (PERIODIC,) * 3, (0.0, 0.0, 0.0), 1.0 / (2 * E),
                 [(0, i, j, k) for i in range(2) for j in range(2) for k in range(2)], leaf_edge=E)
    ls.refine(0, (0, 0, 0))
    ls.refine(0, (1, 1, 1))
    return ls.tree()


def _state(tree, seed=5):
    rng = np.random.default_rng(seed)
    x = tree.cell_centres()
    ph = rng.uniform(0, 2 * np.pi, size=6)
    r2 = ((x[:, 0] - 0.45) ** 2 + (x[:, 1] - 0.5) ** 2 + (x[:, 2] - 0.55) ** 2)
    rho = 1.0 + 2.0 * np.exp(-r2 / 0.02) + 0.2 * np.sin(2 * np.pi * x[:, 1] + ph[0])
    vx = 0.5 + 0.3 * np.sin(2 * np.pi * (x[:, 1] + x[:, 2]) + ph[1])
    vy = -0.4 + 0.2 * np.sin(2 * np.pi * (x[:, 0] + x[:, 2]) + ph[2])
    vz = 0.3 * np.sin(2 * np.pi * (x[:, 0] + x[:, 1]) + ph[3])
    p = 1.0 + 0.5 * np.exp(-r2 / 0.03) + 0.1 * np.sin(2 * np.pi * x[:, 0] + ph[4])
    spc = rho * (0.5 + 0.4 * np.sin(2 * np.pi * x[:, 2] + ph[5]))
    return np.ascontiguousarray(conserved_from_primitive(rho, vx, vy, vz, p, spc, G))


from parity import check, field_err  # noqa: E402


@pytest.mark.parametrize("schedule,reflux", [("column", False), ("face", False), ("persistent", True),
                                             ("tiled", True), ("column", True)])
def test_prolongation_steps_match_oracle(torch, schedule, reflux):
    import oracle
    from paper_2107_10987_amd.hydro import Hydro
    print(f"case: prolongation, periodic AMR, schedule {schedule}, reflux {reflux}", flush=True)
    t = _amr_tree()
    U = _state(t)
    o = oracle.Oracle(t, G, 0.1, reflux=reflux, prolong=True)
    hy = Hydro(max_leaves=t.n, schedule=schedule, reflux=reflux, prolong=True)
    try:
        g = hy.grid(t, torch.tensor(U, device="cuda"), 0.1, G)
        assert g.ptable is not None and g.ptable.shape[0] > 0
        a = hy.signal_speed(g).cpu().numpy()
        ao = o.signal_speed(U)
        assert np.abs(a - ao).max() <= TOL * ao.max()
        dt = float(0.4 * np.min(t.dx / a))
        Uo = U
        for s in range(3):
            am = hy.step(g, dt)
            Uprev = Uo
            Uo, amo = o.step(dt, Uo)
            check(g.U.cpu().numpy(), Uo, o, Uprev, size=7, label=f"prolongation step {s}")
            dt = float(0.4 * np.min(t.dx / amo))
    finally:
        hy.close()


def test_prolongation_with_reflux_conserves(torch):
    from paper_2107_10987_amd.hydro import Hydro
    print("case: prolongation + reflux conservation, periodic AMR, 5 steps", flush=True)
    t = _amr_tree()
    U = _state(t, seed=9)
    vol = t.dx ** 3
    tot0 = np.einsum("n,nfc->f", vol, U.reshape(t.n, 7, -1))
    scale = np.einsum("n,nfc->f", vol, np.abs(U).reshape(t.n, 7, -1))
    hy = Hydro(max_leaves=t.n, reflux=True, prolong=True)
    try:
        g = hy.grid(t, torch.tensor(U, device="cuda"), 0.0, G)
        dt = float(0.4 * np.min(t.dx / hy.signal_speed(g).cpu().numpy()))
        for _ in range(5):
            am = hy.step(g, dt)
            dt = float(0.4 * np.min(t.dx / am))
        Ue = g.U.cpu().numpy()
    finally:
        hy.close()
    err = np.abs(np.einsum("n,nfc->f", vol, Ue.reshape(t.n, 7, -1)) - tot0) / scale
    print("relative total change", err, flush=True)
    assert np.all(err[[0, 1, 2, 3, 4, 6]] <= 1e-14), err


def test_prolongation_16cubed_leaves(torch):
    import oracle
    from paper_2107_10987_amd.hydro import Hydro
    print("case: prolongation with 16^3 leaves vs oracle on the split tree, 2 steps", flush=True)
    t16 = _amr_tree(16)
    U16 = _state(t16, seed=3)
    o = oracle.Oracle(split_octets(t16), G, 0.0, prolong=True)
    hy = Hydro(max_leaves=t16.n, leaf_edge=16, prolong=True)
    try:
        g = hy.grid(t16, torch.tensor(U16, device="cuda"), 0.0, G)
        U8 = to_tiles8(U16)
        dt = o.dt(U8)
        for s in range(2):
            hy.step(g, dt)
            U8, _ = o.step(dt, U8)
            err = field_err(to_tiles8(g.U.cpu().numpy()), U8)
            print(f"step {s} err", err, flush=True)
            assert np.all(err <= TOL), err
    finally:
        hy.close()


def test_prolongation_polytrope_uneven_launches(torch):
    import oracle
    from paper_2107_10987_amd.hydro import Hydro
    print("case: prolongation, rotating polytrope 4096 leaves, uneven launches", flush=True)
    w = rotating_polytrope()
    off = uneven_batches(w.n)
    o = oracle.Oracle(w.tree, w.gamma, w.omega, prolong=True)
    hy = Hydro(max_leaves=w.n, schedule="auto", prolong=True)
    try:
        g = hy.grid(w.tree, torch.tensor(w.U, device="cuda"), w.omega, w.gamma, launch_off=off)
        print("prolongation rows:", g.ptable.shape[0], flush=True)
        dt = float(w.cfl * np.min(w.tree.dx / o.signal_speed(w.U)))
        hy.step(g, dt)
        Uo, _ = o.step(dt, w.U)
        check(g.U.cpu().numpy(), Uo, o, w.U, size=7, label="polytrope prolongation")
    finally:
        hy.close()


def test_prolongation_learned_nan_network_is_the_plain_step(torch):
    from paper_2107_10987_amd.hydro import Hydro
    print("case: prolongation + learned with a NaN network == plain", flush=True)
    t = _amr_tree()
    U = _state(t, seed=13)
    p = (np.random.default_rng(7).normal(size=8090) * 0.3).astype(np.float32)
    p[8064:] = np.nan
    plain = Hydro(max_leaves=t.n, schedule="column", prolong=True)
    lrn = Hydro(max_leaves=t.n, schedule="column", prolong=True, learned=True)
    try:
        lrn.mlp_load(p)
        ga = plain.grid(t, torch.tensor(U, device="cuda"), 0.0, G)
        gb = lrn.grid(t, torch.tensor(U, device="cuda"), 0.0, G)
        dt = float(0.4 * np.min(t.dx / plain.signal_speed(ga).cpu().numpy()))
        plain.step(ga, dt)
        lrn.step(gb, dt)
        assert torch.equal(ga.U, gb.U)
    finally:
        plain.close()
        lrn.close()


def test_prolongation_reflux_graph_replay_uneven(torch):
    # prolongation and flux correction over four concurrent uneven launches,
    # captured in a HIP graph with the device time step: every replay equals
    # the eager steps bit for bit
    from paper_2107_10987_amd.hydro import Hydro
    print("case: prolongation + reflux, 4 uneven launches, graph replay vs eager", flush=True)
    t = _amr_tree()
    U = _state(t, seed=21)
    off = np.array([0, 2, 3, 11, t.n], np.int32)
    he = Hydro(max_leaves=t.n, schedule="auto", reflux=True, prolong=True)
    hg = Hydro(max_leaves=t.n, schedule="auto", reflux=True, prolong=True)
    try:
        s = torch.cuda.Stream()
        ge = he.grid(t, torch.tensor(U, device="cuda"), 0.1, G, launch_off=off)
        gg = hg.grid(t, torch.tensor(U, device="cuda"), 0.1, G, launch_off=off, stream=s)
        dte = torch.zeros(1, dtype=torch.float64, device="cuda")
        dtg = torch.zeros(1, dtype=torch.float64, device="cuda")
        torch.cuda.synchronize()
        he.dt(ge, 0.4, dte)
        hg.dt(gg, 0.4, dtg)
        torch.cuda.synchronize()
        hg.graph_capture(gg, 0.4, dtg, 2)
        torch.cuda.synchronize()
        for replay in range(3):
            for _ in range(2):
                he.step_dev(ge, 0.4, dte)
            hg.graph_launch(s)
            torch.cuda.synchronize()
            _ = (ge.U.sum() + 1.0).item()        # unrelated eager work between replays
            assert torch.equal(ge.U, gg.U), replay
            assert dte.item() == dtg.item()
    finally:
        he.close()
        hg.close()
