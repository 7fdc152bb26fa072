"""GPU parity: the HIP path through the C ABI against the CPU FP64 oracle on
identical seeded inputs.

Tolerance (FP64): per field f, max |gpu - oracle| / max(max |oracle_f|, 1e-300)
<= 1e-12, the parity bound for FP64 results; and per element, |gpu - oracle|
<= 1e-12 times the largest magnitude of that field among the values the
cell's update is formed from (tests/parity.py), so small values of a field
(an atmosphere, a cold tracer) are checked at their own scale."""
import numpy as np
import pytest

from parity import TOL, check
from paper_2107_10987_amd.workloads import (PERIODIC, blast_single_leaf, rotating_polytrope,
                                            sedov_uniform, uneven_batches, uniform_tree)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.fixture(scope="module", params=["column", "face", "persistent", "tiled"])
def hy(torch, request):
    from paper_2107_10987_amd.hydro import Hydro
    print(f"schedule: {request.param}", flush=True)
    h = Hydro(max_leaves=4096, schedule=request.param)
    yield h
    h.close()


from parity import field_err  # noqa: E402


def _oracle(w, threads=None):
    import oracle
    return oracle.Oracle(w.tree, w.gamma, w.omega, threads=threads)


def _grid(hy, torch, w, U=None, launch_off=None):
    U = w.U if U is None else U
    return hy.grid(w.tree, torch.tensor(U, device="cuda"), w.omega, w.gamma, launch_off=launch_off)


def _cold_flow(seed=7):
    """A cold supersonic flow on 2^3 leaves of 8^3 cells: internal energy
    about 1e-6 of the total, so the dual-energy switch takes tau^gamma at
    every face point; on the odd leaves the internal energy is below the
    rounding of E - e_kin and tau lies near 1e-124, under the 2^-330 where
    the fast power gives way to pow."""
    w = sedov_uniform(2)
    rng = np.random.default_rng(seed)
    n, m = w.n, 512
    rho = 1.0 + 0.2 * rng.random((n, m))
    v = np.array([3.0, 1.0, -2.0])[None, :, None] + 0.3 * rng.standard_normal((n, 3, m))
    s = rho[:, None] * v
    eint = 1e-6 * (1.0 + rng.random((n, m))) * np.where(np.arange(n) % 2 == 0, 1.0, 1e-200)[:, None]
    U = np.empty((n, 7, m))
    U[:, 0] = rho
    U[:, 1:4] = s
    U[:, 4] = 0.5 * (s ** 2).sum(1) / rho + eint
    U[:, 5] = eint ** (1.0 / w.gamma) * (1.0 + 0.05 * rng.random((n, m)))
    U[:, 6] = rho
    return w, np.ascontiguousarray(U.reshape(w.U.shape))


def test_dual_energy_switch_cold_flow(hy, torch):
    print("case: cold supersonic flow, dual-energy switch at every face point", flush=True)
    w, U = _cold_flow()
    o = _oracle(w)
    g = _grid(hy, torch, w, U=U)
    dt = o.dt(U)
    U1_ora, a1 = o.stage(1, dt, U)
    U2_ora, a2 = o.stage(2, dt, U1_ora, U)
    Uin = torch.tensor(U, device="cuda")
    U1 = torch.empty_like(Uin)
    am = torch.zeros(w.n, dtype=torch.float64, device="cuda")
    hy.stage(g, 1, dt, Uin, None, U1, am)
    assert np.abs(am.cpu().numpy() - a1).max() <= TOL * a1.max()
    U2 = torch.empty_like(Uin)
    hy.stage(g, 2, dt, torch.tensor(U1_ora, device="cuda"), Uin, U2, am)
    check(U1.cpu().numpy(), U1_ora, o, U, label="cold flow stage 1")
    check(U2.cpu().numpy(), U2_ora, o, U1_ora, extra=(U,), label="cold flow stage 2")
    for got, want in ((U1.cpu().numpy(), U1_ora), (U2.cpu().numpy(), U2_ora)):
        # the two tracer scales separately, so the tiny one is seen
        for sel in (slice(0, None, 2), slice(1, None, 2)):
            err = field_err(got[sel], want[sel])
            assert np.all(err <= TOL), err
    assert np.isfinite(U2.cpu().numpy()).all()


def _cold_transverse_flow(tau_scale):
    """Uniform density and a uniform velocity along z, cold (internal energy
    1e-6 of E or below the rounding of E - e_kin), with the tracer varying
    along x: every x-face point takes the dual-energy pressure (gamma - 1)
    tau^gamma, and sx, zero initially with no x-velocity, changes by the
    pressure's face-flux differences alone.  So the x-momentum update is the
    switch's pressure, checked at its own scale (tau ~ tau_scale; below
    2^-330 the kernels' fast power gives way to pow)."""
    t = uniform_tree((2, 2, 1), (PERIODIC,) * 3, (0.0, 0.0, 0.0), 1.0 / 16)
    x = t.cell_centres()
    rho = np.full(x.shape[:1] + x.shape[2:], 1.3)
    vz = 2.0
    tau = tau_scale * (1.0 + 0.4 * np.sin(2 * np.pi * x[:, 0] + 0.3)
                       + 0.2 * np.cos(4 * np.pi * x[:, 0]))
    U = np.zeros((t.n, 7) + rho.shape[1:])
    U[:, 0] = rho
    U[:, 3] = rho * vz
    U[:, 4] = 0.5 * rho * vz * vz * (1.0 + 1e-6)
    U[:, 5] = tau
    U[:, 6] = rho
    return t, np.ascontiguousarray(U)


@pytest.mark.parametrize("tau_scale", [1e-3, 1e-124])
def test_dual_energy_pressure_pinned(hy, torch, tau_scale):
    import oracle
    print(f"case: cold transverse flow, tau ~ {tau_scale}", flush=True)
    t, U = _cold_transverse_flow(tau_scale)
    o = oracle.Oracle(t, 5.0 / 3.0, 0.0)
    g = hy.grid(t, torch.tensor(U, device="cuda"), 0.0, 5.0 / 3.0)
    dt = o.dt(U)
    U1o, _ = o.stage(1, dt, U)
    sx = U1o[:, 1]
    assert np.abs(sx).max() > 0.0 and np.abs(sx).max() < 1e3 * tau_scale ** (5.0 / 3.0)
    Uin = torch.tensor(U, device="cuda")
    U1 = torch.empty_like(Uin)
    hy.stage(g, 1, dt, Uin, None, U1, None)
    # sx is the pressure term alone: its per-field bound is at the scale of
    # the switch's pressure
    err = field_err(U1.cpu().numpy(), U1o)
    print(f"cold transverse tau~{tau_scale} per-field", err, flush=True)
    assert np.all(err <= TOL), err


def test_nonphysical_face_state_matches_oracle(hy, torch):
    # a cell of negative density next to a cell of positive density: the
    # face states on its faces have no real sound speed; both sides give
    # NaN in exactly the cells whose fluxes touch such a state
    print("case: negative density cell, NaN pattern", flush=True)
    from paper_2107_10987_amd import hydro as H
    w = blast_single_leaf()
    U = w.U.copy()
    U[0, 0, 3, 4, 2] = -0.5
    o = _oracle(w)
    U1o, _ = o.stage(1, 1e-3, U)
    g = _grid(hy, torch, w, U)
    Uin = torch.tensor(U, device="cuda")
    U1 = torch.empty_like(Uin)
    with pytest.raises(H.HydroError) as e:
        hy.stage(g, 1, 1e-3, Uin, None, U1, None)
        hy.check()
    assert e.value.code == H.ENONPHYS
    got = U1.cpu().numpy()
    bad = ~np.isfinite(U1o)
    assert bad.any()
    assert np.array_equal(~np.isfinite(got), bad)
    fin = ~bad
    assert np.abs(got[fin] - U1o[fin]).max() <= TOL * np.abs(U1o[fin]).max()


def test_signal_speed_and_one_step_blast(hy, torch):
    print("case: blast-1leaf one step", flush=True)
    w = blast_single_leaf()
    o = _oracle(w)
    g = _grid(hy, torch, w)
    a_gpu = hy.signal_speed(g).cpu().numpy()
    a_ora = o.signal_speed(w.U)
    assert np.abs(a_gpu - a_ora).max() <= TOL * a_ora.max()
    dt = float(0.4 * w.tree.dx[0] / a_ora[0])
    amax = hy.step(g, dt)
    U_ora, am_ora = o.step(dt, w.U)
    err = field_err(g.U.cpu().numpy(), U_ora)
    print("blast max rel err per field", err, flush=True)
    assert np.all(err <= TOL), err
    assert np.abs(amax - am_ora).max() <= TOL * am_ora.max()


def test_stage_parity_sedov64(hy, torch):
    print("case: sedov-64^3 stages", flush=True)
    w = sedov_uniform(8)
    o = _oracle(w)
    g = _grid(hy, torch, w)
    dt = o.dt(w.U)
    U1_ora, a1 = o.stage(1, dt, w.U)
    U2_ora, a2 = o.stage(2, dt, U1_ora, w.U)
    Uin = torch.tensor(w.U, device="cuda")
    U1 = torch.empty_like(Uin)
    am = torch.zeros(w.n, dtype=torch.float64, device="cuda")
    hy.stage(g, 1, dt, Uin, None, U1, am)
    check(U1.cpu().numpy(), U1_ora, o, w.U, label="sedov stage 1")
    assert np.abs(am.cpu().numpy() - a1).max() <= TOL * a1.max()
    # stage 2 from the oracle's stage-1 state: identical inputs
    U1o = torch.tensor(U1_ora, device="cuda")
    U2 = torch.empty_like(Uin)
    hy.stage(g, 2, dt, U1o, Uin, U2, am)
    check(U2.cpu().numpy(), U2_ora, o, U1_ora, extra=(w.U,), label="sedov stage 2")


def test_trajectory_sedov64_20_steps(hy, torch):
    # the benchmarked workload: 64^3 Sedov as 512 leaves, 20 SSP-RK2 steps at
    # CFL 0.4; both sides take the same dt sequence (from the oracle)
    print("case: sedov-64^3 20-step trajectory", flush=True)
    w = sedov_uniform(8)
    o = _oracle(w)
    g = _grid(hy, torch, w)
    U = w.U.copy()
    dt = o.dt(U)
    worst = np.zeros(7)
    for s in range(20):
        amax_gpu = hy.step(g, dt)
        Uprev = U
        U, am = o.step(dt, U)
        err, _ = check(g.U.cpu().numpy(), U, o, Uprev, size=7, label=f"sedov step {s}")
        worst = np.maximum(worst, err)
        assert np.abs(amax_gpu - am).max() <= TOL * am.max()
        dt = float(w.cfl * np.min(w.tree.dx / am))
    print("sedov 20-step worst rel err per field", worst, flush=True)


def test_reconstruct_parity(hy, torch):
    print("case: reconstruction blast + sedov-32^3", flush=True)
    for w in (blast_single_leaf(), sedov_uniform(4)):
        o = _oracle(w)
        U = w.U.copy()
        if w.n > 1:   # move the blast a little so the limiter is exercised everywhere
            U, _ = o.step(o.dt(U), U)
            U, _ = o.step(o.dt(U), U)
        g = _grid(hy, torch, w, U)
        r_gpu = hy.reconstruct(g).cpu().numpy()
        r_ora = o.reconstruct(U)
        for f in range(7):
            scale = max(np.abs(r_ora[:, f]).max(), 1e-300)
            assert np.abs(r_gpu[:, f] - r_ora[:, f]).max() <= TOL * scale, (w.name, f)


def test_polytrope_amr_rotating_step_uneven_launches(hy, torch):
    # 4096-leaf, 3-level octree, Omega = 0.1, launched as seeded uneven batches
    print("case: polytrope-4096 AMR one step, uneven launches", flush=True)
    w = rotating_polytrope()
    off = uneven_batches(w.n)
    o = _oracle(w)
    g = _grid(hy, torch, w, launch_off=off)
    dt = o.dt(w.U)
    amax = hy.step(g, dt)
    U_ora, am = o.step(dt, w.U)
    print("launches", len(off) - 1, flush=True)
    check(g.U.cpu().numpy(), U_ora, o, w.U, size=7, label="polytrope step")
    assert np.abs(amax - am).max() <= TOL * am.max()


def test_launch_partition_is_bitwise_neutral(hy, torch):
    print("case: launch partitions bitwise", flush=True)
    w = sedov_uniform(4)
    dt = 1e-4
    ga = _grid(hy, torch, w)
    gb = _grid(hy, torch, w, launch_off=np.array([0, 1, 2, 7, 30, 31, 64], np.int32))
    hy.step(ga, dt)
    hy.step(gb, dt)
    assert torch.equal(ga.U, gb.U)


def test_schedules_agree(hy, torch):
    # every stage schedule evaluates the same expressions; only the order of
    # the nine-point face sums differs between the face and column walks
    from paper_2107_10987_amd.hydro import Hydro
    other = Hydro(max_leaves=64, schedule="face")
    try:
        w = sedov_uniform(4)
        ga, gb = _grid(hy, torch, w), _grid(other, torch, w)
        for _ in range(3):
            hy.step(ga, 2e-4)
            other.step(gb, 2e-4)
        assert np.all(field_err(ga.U.cpu().numpy(), gb.U.cpu().numpy()) <= TOL)
    finally:
        other.close()


def test_deterministic(hy, torch):
    w = sedov_uniform(4)
    ga, gb = _grid(hy, torch, w), _grid(hy, torch, w)
    for _ in range(3):
        hy.step(ga, 2e-4)
        hy.step(gb, 2e-4)
    assert torch.equal(ga.U, gb.U)


def test_errors(hy, torch):
    from paper_2107_10987_amd import hydro as H
    print("case: error paths", flush=True)
    w = sedov_uniform(4)
    g = _grid(hy, torch, w)
    with pytest.raises(H.HydroError) as e:
        hy.stage(g, 3, 1e-4, g.U, g.U, torch.empty_like(g.U))
    assert e.value.code == H.EINVAL
    with pytest.raises(H.HydroError) as e:
        hy.stage(g, 1, 1e-4, g.U, None, g.U)          # Uout aliases Uin
    assert e.value.code == H.EINVAL
    with pytest.raises(H.HydroError) as e:
        hy.step(g, float("nan"))
    assert e.value.code == H.EINVAL
    bad = _grid(hy, torch, w)
    bad.c.gamma = 1.0
    with pytest.raises(H.HydroError) as e:
        hy.step(bad, 1e-4)
    assert e.value.code == H.EINVAL
    small = H.Hydro(max_leaves=8, schedule=hy.schedule)
    try:
        with pytest.raises(H.HydroError) as e:
            small.step(_grid(small, torch, w), 1e-4)
        assert e.value.code == H.ENOMEM
    finally:
        small.close()


def test_nonphysical_state_reported(hy, torch):
    print("case: non-physical input", flush=True)
    from paper_2107_10987_amd import hydro as H
    w = blast_single_leaf()
    U = w.U.copy()
    U[0, 0, 2, 2, 2] = -1.0
    g = _grid(hy, torch, w, U)
    with pytest.raises(H.HydroError) as e:
        hy.step(g, 1e-3)
    assert e.value.code == H.ENONPHYS
    # the flag is cleared: a good state steps cleanly afterwards
    g2 = _grid(hy, torch, w)
    hy.step(g2, 1e-3)


@pytest.mark.parametrize("schedule", ["column", "tiled"])
def test_rk3_steps_match_oracle(torch, schedule):
    # three-stage SSP-RK (the paper's integrator) on the 32^3 Sedov blast
    from paper_2107_10987_amd.hydro import Hydro
    print(f"case: SSP-RK3, sedov-32^3, {schedule}", flush=True)
    w = sedov_uniform(4)
    o = _oracle(w)
    hy = Hydro(max_leaves=w.n, schedule=schedule, rk_order=3)
    try:
        g = _grid(hy, torch, w)
        U = w.U.copy()
        dt = o.dt(U)
        for s in range(3):
            amax = hy.step(g, dt)
            U, am = o.step(dt, U, order=3)
            err = field_err(g.U.cpu().numpy(), U)
            assert np.all(err <= TOL), (s, err)
            assert np.abs(amax - am).max() <= TOL * am.max()
            dt = float(w.cfl * np.min(w.tree.dx / am))
    finally:
        hy.close()


@pytest.mark.parametrize("schedule", ["column", "face"])
def test_old_scheme_matches_oracle(torch, schedule):
    # the paper's old scheme: same reconstruction, flux at face centres only
    import oracle
    from paper_2107_10987_amd.hydro import Hydro
    print(f"case: face-centre scheme, sedov-32^3, {schedule}", flush=True)
    w = sedov_uniform(4)
    o = oracle.Oracle(w.tree, w.gamma, w.omega, centre_only=True)
    hy = Hydro(max_leaves=w.n, schedule=schedule, centre_only=True)
    try:
        g = _grid(hy, torch, w)
        U = w.U.copy()
        dt = o.dt(U)
        for s in range(3):
            amax = hy.step(g, dt)
            U, am = o.step(dt, U)
            assert np.all(field_err(g.U.cpu().numpy(), U) <= TOL), s
            assert np.abs(amax - am).max() <= TOL * am.max()
            dt = float(w.cfl * np.min(w.tree.dx / am))
    finally:
        hy.close()
