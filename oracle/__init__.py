"""CPU FP64 oracle of the hydro step: TEST INFRASTRUCTURE.

Only the tests, the smoke check and the benchmark's CPU-baseline leg import
this package.  It wraps ``hydro_oracle.c`` (plain scalar C built with FMA
contraction off) through ctypes and splits leaves over host threads; ctypes
releases the GIL during each call, so the threads run the C code in parallel.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from concurrent.futures import ThreadPoolExecutor

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "hydro_oracle.c")
SRCS = [SRC, os.path.join(HERE, "mlp_oracle.c")]
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(BUILD, "libhydro_oracle.so")
CFLAGS = ["-O2", "-ffp-contract=off", "-fno-fast-math", "-std=c11", "-fPIC", "-shared", "-lm"]

NF, NC = 7, 512


def build(force: bool = True) -> str:
    """Compile the oracle library with gcc (contraction off, IEEE FP64)."""
    os.makedirs(BUILD, exist_ok=True)
    newest = max(os.path.getmtime(f) for f in SRCS + [os.path.join(HERE, "hydro_oracle.h")])
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < newest:
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", *CFLAGS[:-3], "-fPIC", "-shared", "-o", tmp, *SRCS, "-lm"])
        os.replace(tmp, LIB)
    return LIB


class Phys(C.Structure):
    _fields_ = [("gamma", C.c_double), ("omega", C.c_double),
                ("eta1", C.c_double), ("eta2", C.c_double), ("centre_only", C.c_int),
                ("reflux", C.c_int)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        build(force=False)
        L = C.CDLL(LIB)
        dp = C.POINTER(C.c_double)
        ip = C.POINTER(C.c_int)
        L.oracle_ppm.argtypes = [dp, dp, dp]
        L.oracle_point_flux.argtypes = [C.c_int, dp, dp, dp, C.POINTER(Phys), dp]
        L.oracle_point_flux.restype = C.c_double
        L.oracle_tree_create.argtypes = [ip, ip, C.c_int, ip, ip]
        L.oracle_tree_create.restype = C.c_void_p
        L.oracle_tree_destroy.argtypes = [C.c_void_p]
        L.oracle_tree_set_prolong.argtypes = [C.c_void_p, C.c_int]
        L.oracle_fill_padded.argtypes = [C.c_void_p, dp, C.c_int, C.c_int, dp]
        L.oracle_leaf_reconstruct.argtypes = [dp, dp]
        L.oracle_leaf_fluxes.argtypes = [dp, C.c_double, dp, C.POINTER(Phys), dp]
        L.oracle_leaf_fluxes.restype = C.c_double
        L.oracle_leaf_rhs.argtypes = [dp, C.c_double, dp, C.POINTER(Phys), dp, dp]
        L.oracle_stage.argtypes = [C.c_void_p, C.c_int, C.c_double, dp, dp, dp, dp,
                                   C.POINTER(Phys), C.c_int, C.c_int, dp, dp]
        L.oracle_stage_rk.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_double, dp, dp, dp, dp,
                                      C.POINTER(Phys), C.c_int, C.c_int, dp, dp]
        L.oracle_signal_speed.argtypes = [C.c_void_p, dp, dp, dp, C.POINTER(Phys),
                                          C.c_int, C.c_int, dp]
        L.oracle_reconstruct.argtypes = [C.c_void_p, dp, C.c_int, C.c_int, dp]
        fp = C.POINTER(C.c_float)
        L.oracle_bf16.argtypes = [C.c_double]
        L.oracle_bf16.restype = C.c_double
        L.oracle_mlp_forward.argtypes = [fp, C.c_int, dp, C.c_int, dp, dp, dp, dp, dp]
        L.oracle_mlp_loss_grad.argtypes = [fp, C.c_int, dp, dp, C.c_int, dp]
        L.oracle_mlp_loss_grad.restype = C.c_double
        L.oracle_adam.argtypes = [fp, dp, dp, dp, C.c_int, C.c_double, C.c_double, C.c_double,
                                  C.c_double, C.c_int]
        L.oracle_mlp_features.argtypes = [dp, C.c_int, C.c_int, C.c_int, C.c_int, dp, dp, dp]
        L.oracle_mlp_row_ok.argtypes = [dp, dp, C.c_int]
        L.oracle_mlp_limit.argtypes = [dp, dp]
        L.oracle_learned_values.argtypes = [dp, fp, dp, ip, ip]
        u8p = C.POINTER(C.c_uint8)
        L.oracle_learned_rows.argtypes = [dp, fp, dp, dp, u8p, u8p]
        L.oracle_reconstruct_values.argtypes = [dp, dp]
        L.oracle_stage_learned.argtypes = [C.c_void_p, fp, C.c_int, C.c_double, dp, dp, dp, dp,
                                           C.POINTER(Phys), C.c_int, C.c_int, dp, dp, ip]
        _lib = L
    return _lib


def _p(a: np.ndarray, t=C.c_double):
    return a.ctypes.data_as(C.POINTER(t))


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def ppm(q) -> tuple[float, float]:
    q = _f64(q)
    L, R = C.c_double(), C.c_double()
    lib().oracle_ppm(_p(q), C.byref(L), C.byref(R))
    return L.value, R.value


def point_flux(n: int, UL, UR, xq, gamma=5 / 3, omega=0.0, eta1=1e-3, eta2=1e-1):
    UL, UR, xq = _f64(UL), _f64(UR), _f64(xq)
    F = np.zeros(7)
    ph = Phys(gamma, omega, eta1, eta2, 0, 0)
    a = lib().oracle_point_flux(int(n), _p(UL), _p(UR), _p(xq), C.byref(ph), _p(F))
    return F, a


def default_threads() -> int:
    return max(1, min(16, os.cpu_count() or 1))


class Oracle:
    """The oracle bound to one octree layout.

    ``stage``/``step`` mirror the library's stage and step on host arrays.
    """

    def __init__(self, tree, gamma=5 / 3, omega=0.0, eta1=1e-3, eta2=1e-1, threads=None,
                 centre_only=False, reflux=False, prolong=False):
        a = tree.arrays()
        self._keep = a
        self.n = tree.n
        self.dx = a["dx"]
        self.origin = a["origin"]
        self.phys = Phys(gamma, omega, eta1, eta2, int(centre_only), int(reflux))
        self.threads = threads or default_threads()
        ip = C.POINTER(C.c_int)
        self._t = lib().oracle_tree_create(_p(a["nb"], C.c_int), _p(a["bc"], C.c_int), self.n,
                                           _p(a["level"], C.c_int), _p(a["coord"], C.c_int))
        if not self._t:
            raise RuntimeError("oracle_tree_create failed")
        lib().oracle_tree_set_prolong(self._t, int(bool(prolong)))
        del ip

    def __del__(self):
        t = getattr(self, "_t", None)
        if t and _lib is not None:
            _lib.oracle_tree_destroy(t)
            self._t = None

    def _ranges(self, l0=0, l1=None):
        l1 = self.n if l1 is None else l1
        k = max(1, min(self.threads, l1 - l0))
        cuts = np.linspace(l0, l1, k + 1).astype(int)
        return [(int(cuts[i]), int(cuts[i + 1])) for i in range(k) if cuts[i + 1] > cuts[i]]

    def _run(self, fn, ranges):
        if len(ranges) == 1:
            rcs = [fn(*ranges[0])]
        else:
            with ThreadPoolExecutor(len(ranges)) as ex:
                rcs = list(ex.map(lambda r: fn(*r), ranges))
        if any(rcs):
            raise RuntimeError(f"oracle call failed: {rcs}")

    def padded(self, U, l0=0, l1=None):
        U = _f64(U)
        l1 = self.n if l1 is None else l1
        P = np.zeros((l1 - l0, NF, 14, 14, 14))
        rc = lib().oracle_fill_padded(self._t, _p(U), l0, l1, _p(P))
        if rc:
            raise RuntimeError("ghost fill failed")
        return P

    def stage(self, stage: int, dt: float, Uin, Un=None, l0=0, l1=None):
        """One stage over leaves [l0, l1); returns (Uout, amax) for those leaves."""
        Uin = _f64(Uin)
        Un = Uin if Un is None else _f64(Un)
        # every value of the returned leaves is written; the rest of the mesh
        # is never touched (no full-mesh memset per call on a leaf range)
        Uout = np.empty_like(Uin)
        amax = np.zeros(self.n)
        L = lib()

        def fn(a, b):
            return L.oracle_stage(self._t, stage, float(dt), _p(Uin), _p(Un), _p(self.dx),
                                  _p(self.origin), C.byref(self.phys), a, b, _p(Uout), _p(amax))
        rng = self._ranges(l0, l1)
        self._run(fn, rng)
        l1 = self.n if l1 is None else l1
        return Uout[l0:l1], amax[l0:l1]

    def step(self, dt: float, U, order: int = 2):
        """Full SSP-RK step of order 2 or 3; returns (U_next, amax per leaf
        over all stages)."""
        if order == 2:
            U1, a1 = self.stage(1, dt, U)
            U2, a2 = self.stage(2, dt, U1, U)
            return U2, np.maximum(a1, a2)
        Un = _f64(U)
        cur, amax = Un, np.zeros(self.n)
        for s in range(1, order + 1):
            cur, a = self.stage_rk(order, s, dt, cur, Un)
            amax = np.maximum(amax, a)
        return cur, amax

    def stage_rk(self, order: int, stage: int, dt: float, Uin, Un):
        Uin, Un = _f64(Uin), _f64(Un)
        Uout = np.zeros_like(Uin)
        amax = np.zeros(self.n)
        L = lib()

        def fn(a, b):
            return L.oracle_stage_rk(self._t, order, stage, float(dt), _p(Uin), _p(Un), _p(self.dx),
                                     _p(self.origin), C.byref(self.phys), a, b, _p(Uout), _p(amax))
        self._run(fn, self._ranges())
        return Uout, amax

    def signal_speed(self, U, l0=0, l1=None):
        U = _f64(U)
        amax = np.zeros(self.n)
        L = lib()

        def fn(a, b):
            return L.oracle_signal_speed(self._t, _p(U), _p(self.dx), _p(self.origin),
                                         C.byref(self.phys), a, b, _p(amax))
        self._run(fn, self._ranges(l0, l1))
        l1 = self.n if l1 is None else l1
        return amax[l0:l1]

    def stage_learned(self, params, stage: int, dt: float, Uin, Un=None, l0=0, l1=None):
        """One stage with the learned reconstruction (plain-PPM fallback per
        cell); returns (Uout, amax, interior cells per leaf that fell back)
        for [l0, l1)."""
        par = np.ascontiguousarray(params, dtype=np.float32)
        Uin = _f64(Uin)
        Un = Uin if Un is None else _f64(Un)
        Uout = np.empty_like(Uin)   # (as in stage)
        amax = np.zeros(self.n)
        fb = np.zeros(self.n, dtype=np.int32)
        L = lib()

        def fn(a, b):
            return L.oracle_stage_learned(self._t, _p(par, C.c_float), stage, float(dt), _p(Uin),
                                          _p(Un), _p(self.dx), _p(self.origin), C.byref(self.phys),
                                          a, b, _p(Uout), _p(amax), _p(fb, C.c_int))
        self._run(fn, self._ranges(l0, l1))
        l1 = self.n if l1 is None else l1
        return Uout[l0:l1], amax[l0:l1], fb[l0:l1]

    def step_learned(self, params, dt: float, U):
        U1, a1, f1 = self.stage_learned(params, 1, dt, U)
        U2, a2, f2 = self.stage_learned(params, 2, dt, U1, U)
        return U2, np.maximum(a1, a2), f1 + f2

    def dt(self, U, cfl=0.4):
        a = self.signal_speed(U)
        return float(cfl * np.min(self.dx / a))

    def reconstruct(self, U, l0=0, l1=None):
        """Reconstructed values [l1-l0][7][512][26] of interior cells."""
        U = _f64(U)
        l1 = self.n if l1 is None else l1
        out = np.zeros((l1 - l0, NF, NC, 26))
        L = lib()

        def fn(a, b):
            return L.oracle_reconstruct(self._t, _p(U), a, b, _p(out[a - l0:]))
        self._run(fn, self._ranges(l0, l1))
        return out


def leaf_rhs(P, dx, origin, gamma=5 / 3, omega=0.0, eta1=1e-3, eta2=1e-1):
    """L(U) [7][512] and max signal speed of one padded block [7][14][14][14]."""
    P = _f64(P)
    dU = np.zeros((NF, NC))
    amax = C.c_double()
    org = _f64(origin)
    ph = Phys(gamma, omega, eta1, eta2, 0, 0)
    lib().oracle_leaf_rhs(_p(P), float(dx), _p(org), C.byref(ph), _p(dU), C.byref(amax))
    return dU, amax.value


def leaf_reconstruct(P):
    """Values at the 26 points of the interior cells of one padded block:
    out[7][512][26] (direction order dir26)."""
    P = _f64(P)
    out = np.zeros((NF, NC, 26))
    lib().oracle_leaf_reconstruct(_p(P), _p(out))
    return out


def leaf_fluxes(P, dx, origin, gamma=5 / 3, omega=0.0, eta1=1e-3, eta2=1e-1):
    """Face fluxes [3][9][8][8][7] and max signal speed of one padded block."""
    P = _f64(P)
    Fn = np.zeros((3, 9, 8, 8, NF))
    org = _f64(origin)
    ph = Phys(gamma, omega, eta1, eta2, 0, 0)
    a = lib().oracle_leaf_fluxes(_p(P), float(dx), _p(org), C.byref(ph), _p(Fn))
    return Fn, a


def dir26(d) -> int:
    k = 9 * (d[2] + 1) + 3 * (d[1] + 1) + (d[0] + 1)
    return k if k < 13 else k - 1


# ---------------------------------------------------------------------------
# learned reconstruction (MLP) oracle
# ---------------------------------------------------------------------------
MLP_NPARAM = 8090
MLP_SLICES = {"W1": (0, (64, 34)), "b1": (2176, (64,)), "W2": (2240, (64, 64)), "b2": (6336, (64,)),
              "W3": (6400, (26, 64)), "b3": (8064, (26,))}


def bf16(v: float) -> float:
    return lib().oracle_bf16(float(v))


def mlp_forward(params, x, emulate=True):
    par = np.ascontiguousarray(params, dtype=np.float32)
    x = _f64(x)
    B = x.shape[0]
    y = np.zeros((B, 26))
    lib().oracle_mlp_forward(_p(par, C.c_float), int(emulate), _p(x), B, _p(y), None, None, None, None)
    return y


def mlp_loss_grad(params, x, t, emulate=True):
    par = np.ascontiguousarray(params, dtype=np.float32)
    x, t = _f64(x), _f64(t)
    g = np.zeros(MLP_NPARAM)
    loss = lib().oracle_mlp_loss_grad(_p(par, C.c_float), int(emulate), _p(x), _p(t), x.shape[0], _p(g))
    return loss, g


def adam(params, grad, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """In-place Adam step on float32 params and float64 moments."""
    n = params.size
    lib().oracle_adam(_p(params, C.c_float), _p(_f64(grad)), _p(m), _p(v), int(t), lr, b1, b2, eps, n)


def mlp_features(P, i, j, k, f):
    """(nb[27], sigma, x[34] or None if flat) of field f at cell (i,j,k)."""
    P = _f64(P)
    nb, s, x = np.zeros(27), C.c_double(), np.zeros(34)
    flat = lib().oracle_mlp_features(_p(P), i, j, k, f, _p(nb), C.byref(s), _p(x))
    return nb, s.value, (None if flat else x)


def mlp_row_ok(nb, vals, f) -> bool:
    return bool(lib().oracle_mlp_row_ok(_p(_f64(nb)), _p(_f64(vals)), int(f)))


def mlp_limit(nb, vals):
    """The plain limiter applied to one row of predicted values (copy)."""
    v = _f64(vals).copy()
    lib().oracle_mlp_limit(_p(_f64(nb)), _p(v))
    return v


def learned_values(P, params):
    """Learned point-value table [1000][26][7] of one padded block, with the
    count of its interior cells and of those that fell back to plain PPM."""
    P = _f64(P)
    par = np.ascontiguousarray(params, dtype=np.float32)
    V = np.zeros((1000, 26, NF))
    nn, nf = C.c_int(), C.c_int()
    lib().oracle_learned_values(_p(P), _p(par, C.c_float), _p(V), C.byref(nn), C.byref(nf))
    return V, nn.value, nf.value


def learned_rows(P, params):
    """The learned reconstruction of one padded block row by row, before any
    fallback, over the cells (k, j, i) in -1..8 (index (k+1)*100 + (j+1)*10 +
    (i+1)): network outputs y [1000][7][26] (NaN on flat rows), limited point
    values val [1000][7][26], the rows' verdicts ok [1000][7] and flat
    [1000][7] (sigma = 0)."""
    P = _f64(P)
    par = np.ascontiguousarray(params, dtype=np.float32)
    y = np.full((1000, NF, 26), np.nan)
    val = np.zeros((1000, NF, 26))
    ok = np.zeros((1000, NF), np.uint8)
    flat = np.zeros((1000, NF), np.uint8)
    u8p = C.POINTER(C.c_uint8)
    lib().oracle_learned_rows(_p(P), _p(par, C.c_float), _p(y), _p(val), ok.ctypes.data_as(u8p),
                              flat.ctypes.data_as(u8p))
    return y, val, ok.astype(bool), flat.astype(bool)


def reconstruct_values(P):
    P = _f64(P)
    V = np.zeros((1000, 26, NF))
    lib().oracle_reconstruct_values(_p(P), _p(V))
    return V
