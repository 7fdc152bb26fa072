"""Pins of the oracle's point flux and face quadrature (section IV-B: the
central-upwind scheme of Kurganov et al. at every face point, summed over the
face by Newton-Cotes quadrature).

Facts used: equal states give the physical Euler flux; the local speed is
|u_n| + sqrt(gamma p / rho); mirroring the problem through the face negates the
odd flux components; the dissipation of unequal states at rest is
-a (U_R - U_L)/2; the tracer pressure (gamma-1) tau^gamma takes over where the
kinetic energy dominates; a quadratic transverse profile of a passive scalar
gives the (1,4,1)/6 Simpson face flux of the PPM point values."""
import numpy as np
import pytest

G = 5.0 / 3.0


def state(rho, v, p, X=None, gamma=G):
    v = np.asarray(v, float)
    e = p / (gamma - 1.0)
    E = e + 0.5 * rho * v @ v
    return np.array([rho, *(rho * v), E, e ** (1.0 / gamma), rho if X is None else X])


@pytest.mark.parametrize("n", [0, 1, 2])
def test_equal_states_give_euler_flux(oracle_mod, n):
    rho, v, p = 1.3, np.array([0.4, -0.7, 0.25]), 2.1
    U = state(rho, v, p, X=0.6)
    F, a = oracle_mod.point_flux(n, U, U, [0.1, 0.2, 0.3])
    vn = v[n]
    expect = np.array([rho * vn, *(rho * v * vn), (U[4] + p) * vn, U[5] * vn, 0.6 * vn])
    expect[1 + n] += p
    assert np.allclose(F, expect, rtol=1e-15, atol=1e-15)
    assert a == pytest.approx(abs(vn) + np.sqrt(G * p / rho), rel=1e-15)


@pytest.mark.parametrize("n", [0, 1, 2])
def test_mirror_through_face_negates_odd_components(oracle_mod, n):
    rng = np.random.default_rng(n)
    for _ in range(50):
        UL = state(rng.uniform(0.5, 2), rng.normal(size=3), rng.uniform(0.5, 2))
        UR = state(rng.uniform(0.5, 2), rng.normal(size=3), rng.uniform(0.5, 2))
        F, a = oracle_mod.point_flux(n, UL, UR, [0, 0, 0])
        flip = np.ones(7)
        flip[1 + n] = -1.0
        Fm, am = oracle_mod.point_flux(n, UR * flip, UL * flip, [0, 0, 0])
        # mass, transverse momenta, energy, tracer and species fluxes change
        # sign; the normal momentum flux does not
        sign = -np.ones(7)
        sign[1 + n] = 1.0
        assert np.allclose(Fm, sign * F, rtol=1e-14, atol=1e-14)
        assert am == a


def test_dissipation_of_states_at_rest(oracle_mod):
    UL = state(1.0, [0, 0, 0], 1.0)
    UR = state(0.125, [0, 0, 0], 0.1)
    F, a = oracle_mod.point_flux(0, UL, UR, [0, 0, 0])
    cl, cr = np.sqrt(G * 1.0 / 1.0), np.sqrt(G * 0.1 / 0.125)
    assert a == pytest.approx(max(cl, cr), rel=1e-15)
    assert F[0] == pytest.approx(-0.5 * a * (0.125 - 1.0), rel=1e-15)
    assert F[1] == pytest.approx(0.5 * (1.0 + 0.1), rel=1e-15)


def test_tracer_pressure_where_kinetic_energy_dominates(oracle_mod):
    # internal energy 1e-6 of a total of ~0.5: below eta1 = 1e-3 of E, so the
    # pressure must come from the tracer, p = (gamma-1) tau^gamma
    rho, v = 1.0, np.array([1.0, 0.0, 0.0])
    tau = 0.37
    U = np.array([rho, rho * v[0], 0.0, 0.0, 0.5 + 1e-6, tau, rho])
    F, a = oracle_mod.point_flux(1, U, U, [0, 0, 0])      # y-face: u_n = 0
    assert F[2] == pytest.approx((G - 1.0) * tau ** G, rel=1e-14)
    U2 = U.copy()
    U2[4] = 0.5 + 0.01                                     # above the switch
    F2, _ = oracle_mod.point_flux(1, U2, U2, [0, 0, 0])
    assert F2[2] == pytest.approx((G - 1.0) * 0.01, rel=1e-9)


def test_rotating_frame_advection_velocity(oracle_mod):
    # a fluid at rest in the inertial frame moves with -Omega x r relative to
    # the grid: mass flux rho*(Omega*y) through an x-face at height y
    U = state(2.0, [0, 0, 0], 1.0)
    om = 0.3
    F, _ = oracle_mod.point_flux(0, U, U, [0.2, 0.5, 0.0], omega=om)
    assert F[0] == pytest.approx(2.0 * om * 0.5, rel=1e-15)
    F, _ = oracle_mod.point_flux(1, U, U, [0.2, 0.5, 0.0], omega=om)
    assert F[0] == pytest.approx(-2.0 * om * 0.2, rel=1e-15)


def test_simpson_face_quadrature(oracle_mod):
    # rho = 1, v = (u0,0,0), p = 1 everywhere; the species X(j) = Q(j) varies
    # quadratically in y only (monotone, limiter inactive).  At an x-face the
    # left and right values coincide and equal the PPM value at y = j + a/2,
    # Q(j + a/2) - g/12 for a = +-1 and Q(j) for a = 0, so the face flux of X
    # is u0 * [ (1/6) X(-1) + (4/6) X(0) + (1/6) X(+1) ].
    u0 = 0.7
    c0, c1, c2 = 1.0, 0.3, 0.02
    Q = lambda y: c0 + c1 * y + c2 * y * y                       # noqa: E731
    g = c2
    r = np.arange(-3, 11, dtype=float)
    k, j, i = np.meshgrid(r, r, r, indexing="ij")
    P = np.zeros((7, 14, 14, 14))
    P[0] = 1.0
    P[1] = u0
    P[4] = 1.0 / (G - 1.0) + 0.5 * u0 * u0
    P[5] = (1.0 / (G - 1.0)) ** (1.0 / G)
    P[6] = Q(j)
    Fn, a = oracle_mod.leaf_fluxes(P, 0.125, [0.0, 0.0, 0.0])
    jj = np.arange(8, dtype=float)
    expect = u0 * ((Q(jj - 0.5) - g / 12) / 6 + 4 * Q(jj) / 6 + (Q(jj + 0.5) - g / 12) / 6)
    got = Fn[0, :, :, :, 6]                     # [face i][t1 = j][t2 = k]
    assert np.allclose(got, expect[None, :, None], rtol=1e-14, atol=0)
    # the midpoint rule would give u0*Q(j); make sure the test can tell
    assert np.max(np.abs(u0 * Q(jj) - expect)) > 1e-4


@pytest.mark.parametrize("side", ["left", "right"])
def test_state_without_sound_speed_gives_nan_flux(oracle_mod, side):
    # a point state of negative density has no real sound speed, so the
    # maximum signal speed is undefined on either side; the flux is NaN and
    # the stage's result is reported as non-physical
    good = state(1.0, [0.2, 0.0, 0.0], 1.0)
    bad = good.copy()
    bad[0] = -0.5
    UL, UR = (bad, good) if side == "left" else (good, bad)
    F, a = oracle_mod.point_flux(0, UL, UR, [0, 0, 0])
    assert np.isnan(a) and np.isnan(F).all()
