"""GPU tests of the batching layer: device-driven time steps, HIP-graph
replay of whole steps, persistent and tiled launches over uneven batches, and
the schedule autotuner."""
import json
import os

import numpy as np
import pytest

from paper_2107_10987_amd.workloads import rotating_polytrope, sedov_uniform, uneven_batches

pytestmark = pytest.mark.gpu
TOL = 1e-12


@pytest.fixture(scope="module")
def torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _err(a, b):
    a = a.reshape(a.shape[0], 7, -1)
    b = b.reshape(b.shape[0], 7, -1)
    return np.array([np.abs(a[:, f] - b[:, f]).max() / max(np.abs(b[:, f]).max(), 1e-300)
                     for f in range(7)])


def test_device_dt_step_matches_host_dt(torch):
    from paper_2107_10987_amd.hydro import Hydro
    print("case: device-driven dt vs host dt, sedov-32^3", flush=True)
    w = sedov_uniform(4)
    hy = Hydro(max_leaves=w.n)
    try:
        ga = hy.grid(w.tree, torch.tensor(w.U, device="cuda"), w.omega, w.gamma)
        gb = hy.grid(w.tree, torch.tensor(w.U, device="cuda"), w.omega, w.gamma)
        a = hy.signal_speed(ga).cpu().numpy()
        dt = float(w.cfl * np.min(w.tree.dx / a))
        dt_dev = torch.zeros(1, dtype=torch.float64, device="cuda")
        hy.dt(gb, w.cfl, dt_dev)
        assert dt_dev.item() == dt
        for _ in range(5):
            am = hy.step(ga, dt)
            dt = float(w.cfl * np.min(w.tree.dx / am))
            hy.step_dev(gb, w.cfl, dt_dev)
            assert dt_dev.item() == dt
        assert torch.equal(ga.U, gb.U)
    finally:
        hy.close()


@pytest.mark.parametrize("rk", [2, 3])
def test_device_dt_one_and_two_launches(torch, rk):
    # the same grid as one column launch per stage and as two concurrent
    # launches gives the same device time steps and states bit for bit,
    # eagerly and replayed from a graph
    from paper_2107_10987_amd.hydro import Hydro
    print(f"case: device dt, one vs two launches per stage, sedov-32^3, RK{rk}", flush=True)
    w = sedov_uniform(4)
    one = Hydro(max_leaves=w.n, schedule="column", rk_order=rk)
    two = Hydro(max_leaves=w.n, schedule="column", rk_order=rk)
    gr = Hydro(max_leaves=w.n, schedule="column", rk_order=rk)
    try:
        s = torch.cuda.Stream()
        U0 = torch.tensor(w.U, device="cuda")
        ga = one.grid(w.tree, U0.clone(), w.omega, w.gamma)
        gb = two.grid(w.tree, U0.clone(), w.omega, w.gamma,
                      launch_off=np.array([0, w.n // 2, w.n], np.int32))
        gg = gr.grid(w.tree, U0.clone(), w.omega, w.gamma, stream=s)
        da, db, dg = (torch.zeros(1, dtype=torch.float64, device="cuda") for _ in range(3))
        torch.cuda.synchronize()
        one.dt(ga, w.cfl, da)
        two.dt(gb, w.cfl, db)
        gr.dt(gg, w.cfl, dg)
        torch.cuda.synchronize()
        gr.graph_capture(gg, w.cfl, dg, 3)
        torch.cuda.synchronize()
        for replay in range(2):
            for _ in range(3):
                one.step_dev(ga, w.cfl, da)
                two.step_dev(gb, w.cfl, db)
            gr.graph_launch(s)
            torch.cuda.synchronize()
            assert da.item() == db.item() == dg.item(), (replay, da.item(), db.item(), dg.item())
            assert torch.equal(ga.U, gb.U) and torch.equal(ga.U, gg.U), replay
    finally:
        one.close()
        two.close()
        gr.close()


def test_timing_counts_the_stage_launches_of_steps(torch):
    from paper_2107_10987_amd.hydro import Hydro
    print("case: stage timing, 3 device-dt steps of sedov-32^3 (RK2 and RK3)", flush=True)
    w = sedov_uniform(4)
    for rk in (2, 3):
        hy = Hydro(max_leaves=w.n, rk_order=rk)
        try:
            g = hy.grid(w.tree, torch.tensor(w.U, device="cuda"), w.omega, w.gamma)
            dt_dev = torch.zeros(1, dtype=torch.float64, device="cuda")
            hy.timing(True)
            hy.dt(g, w.cfl, dt_dev)          # pre-pass: not recorded
            hy.signal_speed(g)               # not recorded either
            for _ in range(3):
                hy.step_dev(g, w.cfl, dt_dev)
            ms, n = hy.timing(False)
            assert n == 3 * rk and ms > 0.0
            assert hy.timing(False) == (0.0, 0)   # cleared by the report
        finally:
            hy.close()


@pytest.mark.parametrize("schedule", ["column", "tiled", "auto"])
def test_graph_replay_matches_eager(torch, schedule):
    from paper_2107_10987_amd.hydro import Hydro
    print(f"case: graph replay, schedule {schedule}", flush=True)
    w = sedov_uniform(4)
    off = np.array([0, 3, 4, 20, 64], np.int32)
    # separate handles: each owns its workspace, and the two streams are not ordered
    he = Hydro(max_leaves=w.n, schedule=schedule)
    hg = Hydro(max_leaves=w.n, schedule=schedule)
    try:
        s = torch.cuda.Stream()
        U0 = torch.tensor(w.U, device="cuda")
        torch.cuda.synchronize()
        ge = he.grid(w.tree, U0.clone(), w.omega, w.gamma, launch_off=off)
        gg = hg.grid(w.tree, U0.clone(), w.omega, w.gamma, launch_off=off, stream=s)
        dte = torch.zeros(1, dtype=torch.float64, device="cuda")
        dtg = torch.zeros(1, dtype=torch.float64, device="cuda")
        torch.cuda.synchronize()
        he.dt(ge, w.cfl, dte)
        hg.dt(gg, w.cfl, dtg)
        torch.cuda.synchronize()
        hg.graph_capture(gg, w.cfl, dtg, 3)
        torch.cuda.synchronize()
        for replay in range(3):
            for _ in range(3):
                he.step_dev(ge, w.cfl, dte)
            hg.graph_launch(s)
            torch.cuda.synchronize()
            _ = (ge.U.sum() + 1.0).item()        # unrelated eager work between replays
            assert torch.equal(ge.U, gg.U), replay
            assert dte.item() == dtg.item()
    finally:
        he.close()
        hg.close()


def test_uneven_batches_all_schedules_bitwise(torch):
    # the column-walk schedules (direct, persistent, tiled) run the same
    # arithmetic per leaf and must agree bit for bit on the uneven batches
    from paper_2107_10987_amd.hydro import Hydro
    print("case: polytrope uneven batches, column/persistent/tiled", flush=True)
    w = rotating_polytrope()
    off = uneven_batches(w.n)
    outs = []
    for sched in ("column", "persistent", "tiled"):
        hy = Hydro(max_leaves=w.n, schedule=sched)
        try:
            g = hy.grid(w.tree, torch.tensor(w.U, device="cuda"), w.omega, w.gamma, launch_off=off)
            dt = float(w.cfl * np.min(w.tree.dx / hy.signal_speed(g).cpu().numpy()))
            am = hy.step(g, dt)
            am2 = hy.step(g, float(w.cfl * np.min(w.tree.dx / am)))
            outs.append((g.U.cpu().numpy(), am, am2))
        finally:
            hy.close()
    for U, am, am2 in outs[1:]:
        assert np.array_equal(U, outs[0][0])
        assert np.array_equal(am, outs[0][1]) and np.array_equal(am2, outs[0][2])


def test_autotune_table_and_cache(torch, tmp_path):
    from paper_2107_10987_amd.hydro import Hydro
    print("case: autotune on sedov-64^3", flush=True)
    w = sedov_uniform(8)
    hy = Hydro(max_leaves=w.n, schedule="auto")
    path = os.path.join(tmp_path, "tune.json")
    try:
        g = hy.grid(w.tree, torch.tensor(w.U, device="cuda"), w.omega, w.gamma)
        U_before = g.U.clone()
        table = hy.autotune(g, path)
        print("autotuned schedules per size bucket:", table, flush=True)
        assert len(table) == 16 and set(table) <= {"face", "column", "persistent", "tiled"}
        assert torch.equal(g.U, U_before)          # the tuner does not touch U
        doc = json.load(open(path))
        assert len(doc["schedule"]) == 16
    finally:
        hy.close()
    hy2 = Hydro(max_leaves=w.n, schedule="auto", tune_cache=path)
    ref = Hydro(max_leaves=w.n, schedule="face")
    try:
        ga = hy2.grid(w.tree, torch.tensor(w.U, device="cuda"), w.omega, w.gamma)
        gb = ref.grid(w.tree, torch.tensor(w.U, device="cuda"), w.omega, w.gamma)
        dt = float(w.cfl * np.min(w.tree.dx / ref.signal_speed(gb).cpu().numpy()))
        hy2.step(ga, dt)
        ref.step(gb, dt)
        assert np.all(_err(ga.U.cpu().numpy(), gb.U.cpu().numpy()) <= TOL)
    finally:
        hy2.close()
        ref.close()


def test_bench_configuration_matches_oracle(torch):
    # the timed configuration of the benchmark: 64^3 Sedov as 512 leaves,
    # column walk, dt0 from the signal-speed pre-pass, then 20 SSP-RK2 steps
    # with the time step on the device, replayed from one HIP graph on a
    # non-default stream; the oracle runs the same 20 steps with its own dt
    import oracle
    from paper_2107_10987_amd.hydro import Hydro
    print("case: sedov-64^3, 20 graph-replayed device-dt steps vs oracle", flush=True)
    w = sedov_uniform(8)
    o = oracle.Oracle(w.tree, w.gamma, w.omega)
    hy = Hydro(max_leaves=w.n, schedule="column")
    try:
        s = torch.cuda.Stream()
        g = hy.grid(w.tree, torch.tensor(w.U, device="cuda"), w.omega, w.gamma, stream=s)
        dt_dev = torch.zeros(1, dtype=torch.float64, device="cuda")
        hy.graph_capture(g, w.cfl, dt_dev, 20)
        hy.dt(g, w.cfl, dt_dev)
        hy.graph_launch(s)
        s.synchronize()
        hy.check()
        U, dt = w.U.copy(), o.dt(w.U)
        for _ in range(20):
            U, am = o.step(dt, U)
            dt = float(w.cfl * np.min(w.tree.dx / am))
        got = g.U.cpu().numpy().reshape(w.n, 7, -1)
        want = U.reshape(w.n, 7, -1)
        err = np.array([np.abs(got[:, f] - want[:, f]).max() / np.abs(want[:, f]).max() for f in range(7)])
        print("max rel err per field", err, "dt", dt_dev.item(), dt, flush=True)
        assert np.all(err <= 1e-12), err
        assert abs(dt_dev.item() - dt) <= 1e-12 * dt
    finally:
        hy.close()


def test_autotune_concurrent_partition(torch, tmp_path):
    # with several launches per stage the tuner also times whole stages of the
    # grid's own partition and may pick one schedule for all of them; the
    # choice is cached, and steps stay within the parity bound of the column walk
    from paper_2107_10987_amd.hydro import Hydro
    print("case: autotune on the polytrope's uneven partition", flush=True)
    w = rotating_polytrope()
    off = uneven_batches(w.n)
    path = os.path.join(tmp_path, "tune.json")
    hy = Hydro(max_leaves=w.n, schedule="auto")
    try:
        g = hy.grid(w.tree, torch.tensor(w.U, device="cuda"), w.omega, w.gamma, launch_off=off)
        U_before = g.U.clone()
        hy.autotune(g, path)
        assert torch.equal(g.U, U_before)
        doc = json.load(open(path))
        print("concurrent schedule:", doc["concurrent"], flush=True)
        assert doc["concurrent"] in (-1, 2, 3, 4, 5)  # table; column, persistent, tiled; one launch
    finally:
        hy.close()
    tuned = Hydro(max_leaves=w.n, schedule="auto", tune_cache=path)
    col = Hydro(max_leaves=w.n, schedule="column")
    try:
        ga = tuned.grid(w.tree, torch.tensor(w.U, device="cuda"), w.omega, w.gamma, launch_off=off)
        gb = col.grid(w.tree, torch.tensor(w.U, device="cuda"), w.omega, w.gamma)
        dt = float(w.cfl * np.min(w.tree.dx / col.signal_speed(gb).cpu().numpy()))
        tuned.step(ga, dt)
        col.step(gb, dt)
        assert np.all(_err(ga.U.cpu().numpy(), gb.U.cpu().numpy()) <= TOL)
    finally:
        tuned.close()
        col.close()


def test_aggregated_launch_is_bitwise_the_partitioned_step(torch, tmp_path):
    # a tune cache whose choice for stages of several launches is one launch
    # over the whole partition (the tuner's aggregation): each stage is then a
    # single launch, and the step is bit for bit the step of the six
    # concurrent launches
    from paper_2107_10987_amd.hydro import Hydro
    print("case: the polytrope's uneven partition as one launch per stage", flush=True)
    w = rotating_polytrope()
    off = uneven_batches(w.n)
    path = os.path.join(tmp_path, "merge.json")
    with open(path, "w") as f:
        json.dump({"schedule": [2] * 16, "concurrent": 5}, f)
    merged = Hydro(max_leaves=w.n, schedule="auto", tune_cache=path)
    col = Hydro(max_leaves=w.n, schedule="column")
    try:
        ga = merged.grid(w.tree, torch.tensor(w.U, device="cuda"), w.omega, w.gamma, launch_off=off)
        gb = col.grid(w.tree, torch.tensor(w.U, device="cuda"), w.omega, w.gamma, launch_off=off)
        dt = float(w.cfl * np.min(w.tree.dx / col.signal_speed(gb).cpu().numpy()))
        merged.timing(True)
        merged.step(ga, dt)
        _, merged_launches = merged.timing(False)
        col.timing(True)
        col.step(gb, dt)
        _, col_launches = col.timing(False)
        assert merged_launches == 2 and col_launches == 2 * (len(off) - 1)
        assert torch.equal(ga.U, gb.U)
    finally:
        merged.close()
        col.close()
