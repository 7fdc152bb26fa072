"""Pins of the oracle's dual-energy tracer resync (Bryan et al.'s dual
energy formalism, which section IV-B names for the entropy tracer; read as:
after each full step, tau = e^(1/gamma) wherever e = E - |s|^2/(2 rho) exceeds
eta2 E, and tau keeps its advected value elsewhere).

Both branches are pinned by what the scheme fixes independently of the
resync formula:
* a uniform periodic flow has a bitwise-zero update of rho, s and E, so e
  after the step is e before it; the resync must fire exactly when
  e > eta2 E, for cells a hair above and below the threshold and for a
  threshold other than the default;
* tau and the passive species X have the same flux form (a density carried
  with the grid-relative velocity), so with tau = X initially the two stay
  equal bit for bit in every cell where the resync does not fire, and tau is
  e^(1/gamma) of the updated state in every cell where it does.
An unconditional resync, one that never fires, or a wrong threshold fails."""
import math

import numpy as np
import pytest

from paper_2107_10987_amd.workloads import PERIODIC, conserved_from_primitive, uniform_tree

G = 5.0 / 3.0


def _eint(U):
    # internal energy density of each cell, e = E - |s|^2 / (2 rho)
    rho, sx, sy, sz, E = (U[:, f] for f in range(5))
    return E - 0.5 * ((sx * sx + sy * sy) + sz * sz) * (1.0 / rho)


def _uniform_flow(e_over_E, tau0, v=(0.6, -0.3, 0.2), rho=1.3):
    """One periodic leaf of uniform gas whose internal energy is the given
    fraction of E, with an entropy tracer tau0 unrelated to e."""
    t = uniform_tree((1, 1, 1), (PERIODIC,) * 3, (0, 0, 0), 1.0 / 8)
    ek = 0.5 * rho * (v[0] ** 2 + v[1] ** 2 + v[2] ** 2)
    e = e_over_E * ek / (1.0 - e_over_E)          # e / (e + ek) = e_over_E
    sh = (1, 8, 8, 8)
    U = conserved_from_primitive(np.full(sh, rho), np.full(sh, v[0]), np.full(sh, v[1]),
                                 np.full(sh, v[2]), np.full(sh, (G - 1.0) * e),
                                 np.full(sh, rho), G)
    U[:, 5] = tau0
    return t, np.ascontiguousarray(U)


@pytest.mark.parametrize("eta2", [0.1, 0.3])
@pytest.mark.parametrize("side", [-1, +1])
def test_threshold_of_uniform_flow(oracle_mod, eta2, side):
    # e / E a relative 1e-10 below or above eta2 (far above the rounding of e)
    t, U = _uniform_flow(eta2 * (1.0 + side * 1e-10), tau0=7.25)
    o = oracle_mod.Oracle(t, G, 0.0, eta2=eta2)
    U1, _ = o.step(1e-3, U)
    for f in (0, 1, 2, 3, 4, 6):
        assert np.array_equal(U1[:, f], U[:, f]), f
    e = _eint(U)
    fires = e > eta2 * U[:, 4]
    assert bool(fires.all()) == (side > 0) and bool(fires.any()) == (side > 0)
    if side > 0:
        want = np.array([math.pow(x, 1.0 / G) for x in e.ravel()]).reshape(e.shape)
        assert np.allclose(U1[:, 5], want, rtol=4e-16, atol=0)
        assert abs(want.ravel()[0] - 7.25) > 1.0          # tau0 is far from the resync value
    else:
        assert np.array_equal(U1[:, 5], U[:, 5])          # advected, untouched


def _mixed_flow(tree):
    """Smooth density, a fast jet and gas at rest: e / E runs from 1 down to
    ~0.03, so the resync fires in part of the leaf only."""
    x = tree.cell_centres()
    L = np.asarray(tree.nb) * 8 * tree.dx0
    px, py, pz = (2 * np.pi * x[:, a] / L[a] for a in range(3))
    rho = 1.0 + 0.2 * np.sin(px + 0.3) + 0.1 * np.cos(py)
    vx = 2.0 * (0.5 + 0.5 * np.sin(px))
    vy = 0.3 * np.cos(pz)
    vz = np.zeros_like(vx)
    p = np.full_like(rho, 0.05)
    U = conserved_from_primitive(rho, vx, vy, vz, p, rho.copy(), G)
    U[:, 5] = U[:, 6]                                      # tau = X, unrelated to e
    return np.ascontiguousarray(U)


@pytest.mark.parametrize("eta2", [0.1, 0.25])
def test_tau_tracks_species_where_resync_is_off(oracle_mod, eta2):
    t = uniform_tree((2, 1, 1), (PERIODIC,) * 3, (0, 0, 0), 1.0 / 16)
    U = _mixed_flow(t)
    o = oracle_mod.Oracle(t, G, 0.0, eta2=eta2)
    dt = o.dt(U)
    U1, _ = o.step(dt, U)
    e1 = _eint(U1)
    E1 = U1[:, 4]
    margin = np.abs(e1 - eta2 * E1) > 1e-9 * np.abs(E1)
    fires = (e1 > eta2 * E1) & margin
    quiet = (e1 <= eta2 * E1) & margin
    assert fires.sum() > 50 and quiet.sum() > 50, (fires.sum(), quiet.sum())
    # off: tau has been advected exactly like X
    assert np.array_equal(U1[:, 5][quiet], U1[:, 6][quiet])
    # on: tau = e^(1/gamma) of the updated state, unrelated to X there
    want = np.array([math.pow(v, 1.0 / G) for v in e1[fires]])
    assert np.allclose(U1[:, 5][fires], want, rtol=4e-16, atol=0)
    assert np.max(np.abs(U1[:, 6][fires] - want) / want) > 0.1


def test_resync_skips_stage_one(oracle_mod):
    # the resync follows the last stage only: after stage 1 tau is the
    # advected value everywhere, also where e > eta2 E
    t = uniform_tree((2, 1, 1), (PERIODIC,) * 3, (0, 0, 0), 1.0 / 16)
    U = _mixed_flow(t)
    o = oracle_mod.Oracle(t, G, 0.0)
    U1, _ = o.stage(1, o.dt(U), U)
    assert np.array_equal(U1[:, 5], U1[:, 6])
    assert (_eint(U1) > 0.1 * U1[:, 4]).sum() > 50
