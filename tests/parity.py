"""Error measures of the GPU-vs-oracle parity tests (FP64).

field_err: per field f, max over cells of |g - o| / max(max |o_f|, 1e-300),
the parity bound's per-field form.

elem_err: per field, max over cells of |g - o| / s_c, with s_c a bound on
the magnitudes the cell's update is formed from.  A cell's update is its
value plus dt times a sum of face fluxes of cells within its stencil box
(5^3 for a stage: the two-cell reach of PPM along the 13 lines; 7^3 for a
two-stage step, as far as three ghost layers reach); under the CFL limit
dt |F| / dx is bounded by the magnitudes of the box's states: q |u| and
a |dq| / 2 by |q| for rho, E, tau and X; for the momenta s u + p by
sqrt(2 rho E), which bounds both |s| and rho times the sound speed.  So s_c
is the maximum over the box of |q| (of sqrt(2 rho |E|) and |s_f| for a
momentum component), the cell's own result, and any extra states given
(the step-start state of a second stage).  Rounding in the cell's update is
relative to that scale, so this bound sees errors in a field's small values
(the polytrope's 1e-10 atmosphere, a tracer near 1e-124) that the
per-field bound scales away against the field's largest value elsewhere.
"""
import numpy as np
from scipy.ndimage import maximum_filter

TOL = 1e-12          # per-field parity bound
ELEM_TOL = 1e-12     # per-element bound against the local scale


def field_err(g, o):
    g = np.asarray(g).reshape(g.shape[0], 7, -1)
    o = np.asarray(o).reshape(o.shape[0], 7, -1)
    return np.array([np.abs(g[:, f] - o[:, f]).max() / max(np.abs(o[:, f]).max(), 1e-300)
                     for f in range(7)])


def _box_scale(ora, U, size, l0=0, l1=None):
    P = np.abs(ora.padded(U, l0, l1))                            # [l1-l0][7][14][14][14]
    S = P.copy()
    mom = np.sqrt(2.0 * P[:, 0] * P[:, 4])
    for f in (1, 2, 3):
        S[:, f] = np.maximum(P[:, f], mom)
    M = maximum_filter(S, size=(1, 1, size, size, size), mode="nearest")[:, :, 3:11, 3:11, 3:11]
    return M.reshape(M.shape[0], 7, -1)


def local_scale(ora, Uin, want, extra=(), size=5, l0=0, l1=None):
    """Per-cell, per-field scale [l1-l0][7][512] of leaves [l0, l1) (see the
    module docstring)."""
    M = _box_scale(ora, Uin, size, l0, l1)
    M = np.maximum(M, np.abs(np.asarray(want)).reshape(M.shape))
    for X in extra:
        M = np.maximum(M, _box_scale(ora, X, size, l0, l1))
    return M


def elem_err(g, o, scale):
    g = np.asarray(g).reshape(scale.shape)
    o = np.asarray(o).reshape(scale.shape)
    r = np.abs(g - o) / np.maximum(scale, 1e-300)
    return r.max(axis=(0, 2))


def check(g, o, ora, Uin, extra=(), size=5, tol=TOL, elem_tol=ELEM_TOL, label="", l0=0, l1=None):
    """Assert both bounds on leaves [l0, l1) (g and o hold just those);
    returns (field_err, elem_err)."""
    fe = field_err(g, o)
    ee = elem_err(g, o, local_scale(ora, Uin, o, extra, size, l0, l1))
    print(f"{label} per-field {np.array2string(fe, precision=2)} "
          f"per-element {np.array2string(ee, precision=2)}", flush=True)
    assert np.all(fe <= tol), (label, fe)
    assert np.all(ee <= elem_tol), (label, ee)
    return fe, ee
