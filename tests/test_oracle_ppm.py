"""Pins of the oracle's PPM reconstruction (section IV-B: PPM of Colella and
Woodward applied along the 13 lines through each cell centre).

Closed forms: linear data is reproduced exactly; a quadratic with the limiter
inactive gives the PPM interface value Q(c + d/2) - g_d/12, g_d being the
second-order coefficient of Q along the line; hand-derived one-dimensional
limiter cases; the bound that limited values stay between neighbouring
cell values."""
import itertools

import numpy as np
import pytest


def test_linear_data_exact(oracle_mod):
    for a, b in [(2.5, 0.25), (-1.0, -0.125), (3.0, 0.0), (0.5, 4.0)]:
        q = [a + b * m for m in range(-2, 3)]
        L, R = oracle_mod.ppm(q)
        assert L == a - b / 2 and R == a + b / 2


@pytest.mark.parametrize("q,expect", [
    ([1.0, 2.0, 3.0, 2.0, 1.0], (3.0, 3.0)),        # local maximum: flat
    ([0.0, 1.0, -1.0, 1.0, 0.0], (-1.0, -1.0)),     # local minimum: flat
    ([0.0, 0.0, 0.0, 1.0, 1.0], (0.0, 0.0)),        # foot of a step: flat
    ([0.0, 0.0, 0.2, 1.0, 1.0], (1.0 / 30.0, 8.0 / 15.0)),   # overshoot on the right
    ([1.0, 1.0, 0.2, 0.0, 0.0], (8.0 / 15.0, 1.0 / 30.0)),   # overshoot on the left
])
def test_hand_derived_limiter_cases(oracle_mod, q, expect):
    # [0,0,0.2,1,1]: slopes (0, 0.4, 0) with 0.4 = 2|0.2| capping the centred 0.5;
    # R = 0.2+0.4+0.4/6 = 2/3, L = 0.1-0.4/6 = 1/30; D = 19/30, M6 = -0.9,
    # D*M6 < -D^2, so R = 3*0.2 - 2/30 = 8/15.  The mirrored data swaps L and R.
    L, R = oracle_mod.ppm(q)
    assert L == pytest.approx(expect[0], rel=1e-14, abs=1e-15)
    assert R == pytest.approx(expect[1], rel=1e-14, abs=1e-15)


def test_mirror_swaps_left_and_right(oracle_mod):
    rng = np.random.default_rng(5)
    for _ in range(2000):
        q = rng.normal(size=5)
        L, R = oracle_mod.ppm(q)
        Lm, Rm = oracle_mod.ppm(q[::-1].copy())
        s = np.abs(q).max()
        assert abs(Lm - R) <= 1e-14 * s and abs(Rm - L) <= 1e-14 * s


def test_limited_values_between_neighbours(oracle_mod):
    rng = np.random.default_rng(7)
    for trial in range(20000):
        q = rng.normal(size=5) if trial % 2 else np.cumsum(rng.exponential(size=5)) * rng.choice([-1, 1])
        L, R = oracle_mod.ppm(q)
        tol = 8 * np.finfo(float).eps * np.abs(q).max()
        assert min(q[1], q[2]) - tol <= L <= max(q[1], q[2]) + tol
        assert min(q[2], q[3]) - tol <= R <= max(q[2], q[3]) + tol


DIRS = [d for d in itertools.product((-1, 0, 1), repeat=3) if d != (0, 0, 0)]


def _dir26(d):
    k = 9 * (d[2] + 1) + 3 * (d[1] + 1) + (d[0] + 1)
    return k if k < 13 else k - 1


def _block(fn):
    r = np.arange(-3, 11, dtype=float)
    k, j, i = np.meshgrid(r, r, r, indexing="ij")
    P = np.empty((7, 14, 14, 14))
    for f in range(7):
        P[f] = fn(i, j, k, f)
    return P


def test_quadratic_closed_form_all_26_directions(oracle_mod):
    # Q has a dominant linear part so no line through any stencil has an
    # extremum and no limiter branch is taken; any branch would break the
    # closed form.
    # every +-1 combination of each row has magnitude >= 0.09 > max curvature slope
    lin = np.array([[0.5, 0.3, 0.11], [0.11, -0.5, 0.3], [-0.3, 0.11, 0.5]])
    H = 1e-3 * np.array([[2.0, 0.2, 0.0], [0.2, 1.0, 0.1], [0.0, 0.1, 0.6]])

    def Q(x, y, z, f):
        c = lin[f % 3]
        X = np.stack([x, y, z])
        quad = 0.5 * np.einsum("a...,ab,b...->...", X, H, X)
        return 2.0 + f + c[0] * x + c[1] * y + c[2] * z + quad

    P = _block(Q)
    out = oracle_mod.leaf_reconstruct(P)
    r = np.arange(8, dtype=float)
    kk, jj, ii = np.meshgrid(r, r, r, indexing="ij")
    for f in range(7):
        for d in DIRS:
            dv = np.array(d, float)
            g = 0.5 * dv @ H @ dv          # coefficient of m^2 along the line
            exact = Q(ii + dv[0] / 2, jj + dv[1] / 2, kk + dv[2] / 2, f) - g / 12.0
            got = out[f, :, _dir26(d)].reshape(8, 8, 8)
            assert np.max(np.abs(got - exact)) <= 1e-14 * np.abs(exact).max(), (f, d)


def test_linear_field_exact_at_all_points(oracle_mod):
    def Q(x, y, z, f):
        return 1.0 + 0.25 * x - 0.125 * y + 0.0625 * z + f
    out = oracle_mod.leaf_reconstruct(_block(Q))
    r = np.arange(8, dtype=float)
    kk, jj, ii = np.meshgrid(r, r, r, indexing="ij")
    for d in DIRS:
        exact = Q(ii + d[0] / 2, jj + d[1] / 2, kk + d[2] / 2, 3)
        assert np.array_equal(out[3, :, _dir26(d)].reshape(8, 8, 8), exact)
