"""Full-size checks on the binary-star workload of 32768 leaves (16,777,216
cells, the paper's problem size) on a 4-level octree in the rotating frame:
one stage in uneven launches (autotuned and tiled schedules) against the
oracle on sampled leaves it computes one by one from the same input, and the
benchmark's headline configuration (one launch per stage, a graph-captured
step with the time step on the device) against a whole oracle step."""
import numpy as np
import pytest

from paper_2107_10987_amd.workloads import binary_star, uneven_batches

pytestmark = pytest.mark.gpu
TOL = 1e-12


@pytest.fixture(scope="module")
def torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.fixture(scope="module")
def binary():
    print("case: building the 32768-leaf binary-star octree", flush=True)
    return binary_star()


@pytest.mark.parametrize("schedule", ["auto", "tiled"])
def test_binary_32768_stage_sampled_parity(torch, binary, schedule):
    import oracle
    from paper_2107_10987_amd.hydro import Hydro
    w = binary
    print(f"case: binary-32768 stage 1, schedule {schedule}", flush=True)
    off = uneven_batches(w.n)
    hy = Hydro(max_leaves=w.n, schedule=schedule)
    try:
        g = hy.grid(w.tree, torch.tensor(w.U, device="cuda"), w.omega, w.gamma, launch_off=off)
        a = hy.signal_speed(g).cpu().numpy()
        dt = float(w.cfl * np.min(w.tree.dx / a))
        U1 = torch.empty_like(g.U)
        am = torch.zeros(w.n, dtype=torch.float64, device="cuda")
        hy.stage(g, 1, dt, g.U, None, U1, am)
        U1 = U1.cpu().numpy()
        am = am.cpu().numpy()
    finally:
        hy.close()
    assert np.isfinite(U1).all() and (U1[:, 0] > 0).all()
    o = oracle.Oracle(w.tree, w.gamma, w.omega)
    rng = np.random.default_rng(11)
    starts = np.sort(rng.choice(w.n - 8, 12, replace=False))
    for l0 in starts:
        Uo, ao = o.stage(1, dt, w.U, l0=int(l0), l1=int(l0) + 8)
        got = U1[l0:l0 + 8].reshape(8, 7, -1)
        ref = Uo.reshape(8, 7, -1)
        for f in range(7):
            scale = max(np.abs(ref[:, f]).max(), 1e-300)
            assert np.abs(got[:, f] - ref[:, f]).max() <= TOL * scale, (l0, f)
        assert np.abs(am[l0:l0 + 8] - ao).max() <= TOL * ao.max()


@pytest.fixture(scope="module")
def sedov256():
    from paper_2107_10987_amd.workloads import sedov_uniform
    print("case: building the 256^3 Sedov blast (32768 leaves)", flush=True)
    return sedov_uniform(32)


@pytest.mark.parametrize("name", ["binary", "sedov256"])
def test_headline_configuration_step_parity(torch, request, name):
    """The configuration bench.py times for its headline (the binary; the
    256^3 Sedov leg runs the same way): every leaf in one
    launch per stage (the schedule the built-in rule picks for 32,768 leaves),
    a whole SSP-RK2 step captured in a HIP graph with the time step read from
    and written to device memory.  Against one oracle step of the whole mesh
    (fed the same dt): every element within the FP64 parity bound per field,
    the element-wise bound on sampled leaf ranges, and the device's next time
    step equal to the oracle's to 1e-12."""
    import oracle
    import parity
    from paper_2107_10987_amd.hydro import Hydro
    w = request.getfixturevalue(name)
    print(f"case: {name} (32768 leaves), one launch per stage, graph step with device dt", flush=True)
    hy = Hydro(max_leaves=w.n, schedule="auto")
    try:
        s = torch.cuda.Stream()
        g = hy.grid(w.tree, torch.tensor(w.U, device="cuda"), w.omega, w.gamma, stream=s)
        dt_dev = torch.zeros(1, dtype=torch.float64, device="cuda")
        hy.graph_capture(g, w.cfl, dt_dev, 1)
        hy.dt(g, w.cfl, dt_dev)
        s.synchronize()
        dt0 = float(dt_dev.item())
        hy.graph_launch(s)
        s.synchronize()
        hy.check(s)
        got = g.U.cpu().numpy()
        dt1 = float(dt_dev.item())
    finally:
        hy.close()
    o = oracle.Oracle(w.tree, w.gamma, w.omega)
    dto = o.dt(w.U, w.cfl)
    assert abs(dt0 - dto) <= 1e-12 * dto
    Uo, am = o.step(dt0, w.U)
    dto1 = float(w.cfl * np.min(w.tree.dx / am))
    assert abs(dt1 - dto1) <= 1e-12 * dto1, (dt1, dto1)
    fe = parity.field_err(got, Uo)
    print(f"{name} step per-field {np.array2string(fe, precision=2)}", flush=True)
    assert np.all(fe <= TOL), fe
    rng = np.random.default_rng(12)
    for l0 in np.sort(rng.choice(w.n - 8, 8, replace=False)):
        l0 = int(l0)
        parity.check(got[l0:l0 + 8], Uo[l0:l0 + 8], o, w.U, size=7, l0=l0, l1=l0 + 8,
                     label=f"{name} leaves [{l0}, {l0 + 8})")


def _constant_network(seed=11, scale=0.6):
    """Output weights zero: the network outputs its biases exactly on both
    sides, so the learned point values are the same arithmetic on the GPU and
    in the oracle (bit for bit)."""
    rng = np.random.default_rng(seed)
    p = (rng.normal(size=8090) * 0.3).astype(np.float32)
    p[6400:8064] = 0.0
    p[8064:] = rng.uniform(-scale, scale, 26).astype(np.float32)
    return p


def test_binary_learned_stage_sampled_parity(torch, binary):
    """The learned configuration at full size: all 32,768 leaves in one
    launch per stage, the inference pre-pass with the shared ghost rows, the
    learned column walk; stage 1 against the oracle's learned stage on
    sampled leaf ranges, per field and per element."""
    import oracle
    import parity
    from paper_2107_10987_amd.hydro import Hydro
    w = binary
    p = _constant_network()
    print("case: binary-32768 learned stage 1, constant-output network, shared ghost rows", flush=True)
    hy = Hydro(max_leaves=w.n, schedule="auto", learned=True)
    try:
        hy.mlp_load(p)
        g = hy.grid(w.tree, torch.tensor(w.U, device="cuda"), w.omega, w.gamma)
        assert g.alias is not None
        a = hy.signal_speed(g).cpu().numpy()
        dt = float(w.cfl * np.min(w.tree.dx / a))
        hy.mlp_stats()
        U1 = torch.empty_like(g.U)
        am = torch.zeros(w.n, dtype=torch.float64, device="cuda")
        hy.stage(g, 1, dt, g.U, None, U1, am)
        cells, fb = hy.mlp_stats()
        U1 = U1.cpu().numpy()
        am = am.cpu().numpy()
    finally:
        hy.close()
    assert cells == w.n * 512 and 0 < fb < cells
    o = oracle.Oracle(w.tree, w.gamma, w.omega)
    rng = np.random.default_rng(13)
    for l0 in np.sort(rng.choice(w.n - 8, 8, replace=False)):
        l0 = int(l0)
        Uo, ao, fbo = o.stage_learned(p, 1, dt, w.U, l0=l0, l1=l0 + 8)
        parity.check(U1[l0:l0 + 8], Uo, o, w.U, size=7, l0=l0, l1=l0 + 8,
                     label=f"binary learned leaves [{l0}, {l0 + 8})")
        assert np.abs(am[l0:l0 + 8] - ao).max() <= TOL * ao.max()
    print(f"binary learned: {fb} of {cells} interior cells fall back", flush=True)
