"""The allocation-free step (hydro_step_noalloc) against hydro_step.

Both run the same column-walk kernels with the same launch shape, so their
results must agree bit for bit: state and per-leaf signal speeds, on two calls
in a row (the second on a smaller grid, after the first left the shared
scratch array full of its own data), with and without waiting for the
stream.  Sizes beyond the scratch array's capacity are refused."""
import numpy as np
import pytest

from paper_2107_10987_amd.workloads import sedov_uniform

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _advanced(torch, w, omega, steps):
    """The workload's state after `steps` ordinary steps (nontrivial flow)."""
    from paper_2107_10987_amd.hydro import Hydro
    hy = Hydro(max_leaves=w.n, schedule="column")
    try:
        g = hy.grid(w.tree, torch.tensor(w.U, device="cuda"), omega, w.gamma)
        for _ in range(steps):
            a = hy.signal_speed(g).cpu().numpy()
            hy.step(g, float(0.4 * np.min(w.tree.dx / a)))
        return g.U.clone()
    finally:
        hy.close()


def _compare(torch, w, omega, U0, sync):
    from paper_2107_10987_amd.hydro import Hydro, step_noalloc
    hy = Hydro(max_leaves=w.n, schedule="column")
    try:
        ref = hy.grid(w.tree, U0.clone(), omega, w.gamma)
        got = hy.grid(w.tree, U0.clone(), omega, w.gamma)
        dt = float(0.4 * np.min(w.tree.dx / hy.signal_speed(ref).cpu().numpy()))
        a_ref = hy.step(ref, dt)
        a_got = torch.full((w.n,), -1.0, dtype=torch.float64, device="cuda")
        step_noalloc(got, dt, amax=a_got, sync=sync)
        torch.cuda.synchronize()
        assert torch.equal(ref.U, got.U)
        assert np.array_equal(a_ref, a_got.cpu().numpy())
        assert not torch.equal(U0, got.U)
    finally:
        hy.close()


def test_noalloc_step_equals_hydro_step_twice(torch):
    print("case: noalloc step, sedov-32^3 (64 leaves, the maximum) rotating, then sedov-16^3 (8 leaves)",
          flush=True)
    big = sedov_uniform(4)
    _compare(torch, big, 0.3, _advanced(torch, big, 0.3, 2), sync=True)
    small = sedov_uniform(2)
    _compare(torch, small, 0.0, _advanced(torch, small, 0.0, 1), sync=False)


def test_noalloc_step_without_amax_output(torch):
    from paper_2107_10987_amd.hydro import Hydro, step_noalloc
    print("case: noalloc step without amax output, sedov-16^3 rotating", flush=True)
    w = sedov_uniform(2)
    U0 = _advanced(torch, w, 0.2, 1)
    hy = Hydro(max_leaves=w.n, schedule="column")
    try:
        ref = hy.grid(w.tree, U0.clone(), 0.2, w.gamma)
        got = hy.grid(w.tree, U0.clone(), 0.2, w.gamma)
        hy.step(ref, 1e-4)
        step_noalloc(got, 1e-4)
        assert torch.equal(ref.U, got.U)
    finally:
        hy.close()


def test_noalloc_refuses_oversized_grid(torch):
    from paper_2107_10987_amd.hydro import Hydro, HydroError, NOALLOC_MAX_LEAVES, step_noalloc
    print("case: noalloc step refuses 512 leaves", flush=True)
    w = sedov_uniform(8)
    assert w.n > NOALLOC_MAX_LEAVES
    hy = Hydro(max_leaves=w.n, schedule="column")
    try:
        g = hy.grid(w.tree, torch.tensor(w.U, device="cuda"), w.omega, w.gamma)
        with pytest.raises(HydroError) as e:
            step_noalloc(g, 1e-5)
        assert e.value.code == -1 and "at most 64" in str(e.value)
        assert torch.equal(g.U, torch.tensor(w.U, device="cuda"))
    finally:
        hy.close()
