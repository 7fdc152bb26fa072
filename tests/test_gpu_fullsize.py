"""Full-size check: the binary-star workload of 32768 leaves (16,777,216
cells, the paper's problem size) on a 4-level octree in the rotating frame,
one stage on the GPU in the persistent/tiled launch configuration, compared
with the oracle on sampled leaves that the oracle computes one by one from
the same input, plus properties that hold at any size."""
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
