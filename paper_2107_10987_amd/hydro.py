"""Thin ctypes binding of the gfx950 hydro library (include/hydro.h).

Argument marshalling only: every step of the hydro update runs in the HIP
kernels of ``libhydro.so``.  PyTorch supplies device memory and streams.
There is no CPU fallback: if the built library is missing, loading fails.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "_build", "libhydro.so")

OK, EINVAL, ENOMEM, EHIP, ENONPHYS = 0, -1, -2, -3, -4
NX, NF, NC, NGHOST = 8, 7, 512, 2232
REFLUX_ENTRY = 26

EXPORTS = ("hydro_create", "hydro_destroy", "hydro_ghost_map", "hydro_ghost_map_linear",
           "hydro_reflux_map", "hydro_step",
           "hydro_stage",
           "hydro_signal_speed", "hydro_reconstruct", "hydro_step_dev", "hydro_dt",
           "hydro_graph_capture", "hydro_graph_launch", "hydro_autotune", "hydro_mlp_load",
           "hydro_mlp_save", "hydro_mlp_forward", "hydro_mlp_grad", "hydro_mlp_train_step",
           "hydro_mlp_pairs", "hydro_mlp_stats", "hydro_amax_device",
           "hydro_check", "hydro_timing", "hydro_strerror", "hydro_last_error",
           "hydro_step_noalloc", "hydro_mlp_values", "hydro_mlp_alias_map", "hydro_fp64_probe")
NOALLOC_MAX_LEAVES = 64
SCHEDULES = {"auto": 0, "face": 1, "column": 2, "persistent": 3, "tiled": 4}
NBUCKET = 16


class HydroError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{msg} (code {code})")
        self.code = code


class Params(C.Structure):
    _fields_ = [("max_leaves", C.c_int32), ("device", C.c_int32), ("recon", C.c_int32),
                ("schedule", C.c_int32), ("eta1", C.c_double), ("eta2", C.c_double),
                ("tune_cache", C.c_char_p), ("mlp_batch", C.c_int32), ("rk_order", C.c_int32),
                ("scheme", C.c_int32), ("reflux", C.c_int32), ("leaf_edge", C.c_int32)]


class Grid(C.Structure):
    _fields_ = [("n", C.c_int32), ("n_launch", C.c_int32), ("launch_off", C.POINTER(C.c_int32)),
                ("U", C.c_void_p), ("dx", C.c_void_p), ("origin", C.c_void_p),
                ("ghost_map", C.c_void_p), ("omega", C.c_double), ("gamma", C.c_double),
                ("stream", C.c_void_p), ("face_flags", C.c_void_p), ("reflux", C.c_void_p),
                ("n_reflux", C.c_int32), ("prolong", C.c_void_p), ("n_prolong", C.c_int32),
                ("mlp_alias", C.c_void_p)]


class Tree(C.Structure):
    _fields_ = [("n", C.c_int32), ("nb", C.c_int32 * 3), ("bc", C.c_int32 * 3),
                ("level", C.POINTER(C.c_int32)), ("coord", C.POINTER(C.c_int32)),
                ("leaf_edge", C.c_int32)]


_lib = None


def load(path: str = LIB_PATH) -> C.CDLL:
    """Load libhydro.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"HIP hydro library not built: {path} is missing "
                           "(run paper_2107_10987_amd/build.py)")
    L = C.CDLL(path)
    vp, dp = C.c_void_p, C.POINTER(C.c_double)
    L.hydro_create.argtypes = [C.POINTER(Params), C.POINTER(vp)]
    L.hydro_destroy.argtypes = [vp]
    L.hydro_ghost_map.argtypes = [C.POINTER(Tree), C.POINTER(C.c_int32)]
    ip = C.POINTER(C.c_int32)
    L.hydro_reflux_map.argtypes = [C.POINTER(Tree), ip, ip, ip]
    L.hydro_ghost_map_linear.argtypes = [C.POINTER(Tree), ip, ip, C.c_int32, ip]
    L.hydro_mlp_alias_map.argtypes = [C.POINTER(Tree), ip, ip]
    L.hydro_step.argtypes = [vp, C.POINTER(Grid), C.c_double, dp]
    L.hydro_stage.argtypes = [vp, C.POINTER(Grid), C.c_int, C.c_double, vp, vp, vp, vp]
    L.hydro_signal_speed.argtypes = [vp, C.POINTER(Grid), vp]
    L.hydro_reconstruct.argtypes = [vp, C.POINTER(Grid), vp]
    L.hydro_step_dev.argtypes = [vp, C.POINTER(Grid), C.c_double, vp]
    L.hydro_dt.argtypes = [vp, C.POINTER(Grid), C.c_double, vp]
    L.hydro_graph_capture.argtypes = [vp, C.POINTER(Grid), C.c_double, vp, C.c_int]
    L.hydro_graph_launch.argtypes = [vp, vp]
    L.hydro_autotune.argtypes = [vp, C.POINTER(Grid), C.c_char_p, C.POINTER(C.c_int32)]
    fp = C.POINTER(C.c_float)
    L.hydro_mlp_load.argtypes = [vp, fp]
    L.hydro_mlp_save.argtypes = [vp, fp]
    L.hydro_mlp_forward.argtypes = [vp, vp, C.c_int, vp, vp]
    L.hydro_mlp_grad.argtypes = [vp, vp, vp, C.c_int, vp, vp, vp]
    L.hydro_mlp_train_step.argtypes = [vp, vp, vp, C.c_int, C.c_double, vp, vp]
    L.hydro_mlp_pairs.argtypes = [vp, C.POINTER(Grid), vp, vp, vp]
    L.hydro_mlp_stats.argtypes = [vp, C.POINTER(C.c_int64), C.POINTER(C.c_int64)]
    L.hydro_mlp_values.argtypes = [vp, C.POINTER(Grid), vp, vp, vp]
    L.hydro_amax_device.argtypes = [vp]
    L.hydro_amax_device.restype = vp
    L.hydro_check.argtypes = [vp, vp]
    L.hydro_timing.argtypes = [vp, C.c_int, C.POINTER(C.c_double), C.POINTER(C.c_int64)]
    L.hydro_strerror.argtypes = [C.c_int]
    L.hydro_strerror.restype = C.c_char_p
    L.hydro_last_error.argtypes = [vp]
    L.hydro_last_error.restype = C.c_char_p
    L.hydro_step_noalloc.argtypes = [C.POINTER(Grid), C.c_double, C.c_double, C.c_double, vp, C.c_int]
    L.hydro_fp64_probe.argtypes = [vp, C.c_int32, C.c_int32, C.c_double, C.c_double, vp]
    for name in EXPORTS:
        getattr(L, name).restype = getattr(L, name).restype or C.c_int
    L.hydro_amax_device.restype = vp
    L.hydro_strerror.restype = C.c_char_p
    L.hydro_last_error.restype = C.c_char_p
    _lib = L
    return L


def _tree_struct(tree):
    a = tree.arrays()
    t = Tree(tree.n, (C.c_int32 * 3)(*a["nb"]), (C.c_int32 * 3)(*a["bc"]),
             a["level"].ctypes.data_as(C.POINTER(C.c_int32)),
             a["coord"].ctypes.data_as(C.POINTER(C.c_int32)), int(a["leaf_edge"]))
    return t, a


def ghost_map(tree) -> np.ndarray:
    """Ghost map of a workloads.Tree, built by the library: int32 [n][2232] for
    8^3 leaves, [n][8][2232] (one map per 8^3 tile) for 16^3 leaves."""
    L = load()
    t, _keep = _tree_struct(tree)
    shape = (tree.n, NGHOST) if tree.leaf_edge == NX else (tree.n, 8, NGHOST)
    out = np.empty(shape, dtype=np.int32)
    rc = L.hydro_ghost_map(C.byref(t), out.ctypes.data_as(C.POINTER(C.c_int32)))
    if rc:
        raise HydroError(rc, L.hydro_last_error(None).decode())
    return out


def mlp_alias_map(tree, gmap) -> np.ndarray:
    """Learned-reconstruction rows that blocks share (hydro_mlp_alias_map):
    int32 [n T][384], block * 896 + slot or -1, from the tree and its host
    ghost map."""
    L = load()
    t, _keep = _tree_struct(tree)
    gm = np.ascontiguousarray(gmap, dtype=np.int32)
    T = 1 if tree.leaf_edge == NX else 8
    assert gm.size == tree.n * T * NGHOST
    out = np.empty((tree.n * T, 384), dtype=np.int32)
    ip = C.POINTER(C.c_int32)
    rc = L.hydro_mlp_alias_map(C.byref(t), gm.ctypes.data_as(ip), out.ctypes.data_as(ip))
    if rc:
        raise HydroError(rc, L.hydro_last_error(None).decode())
    return out


def ghost_map_linear(tree):
    """Ghost map with linear-limited prolongation from coarser leaves, and its
    table of prolongation rows int32 [m][8], built by the library."""
    L = load()
    t, _keep = _tree_struct(tree)
    shape = (tree.n, NGHOST) if tree.leaf_edge == NX else (tree.n, 8, NGHOST)
    out = np.empty(shape, dtype=np.int32)
    m = C.c_int32()
    ip = C.POINTER(C.c_int32)
    rc = L.hydro_ghost_map_linear(C.byref(t), out.ctypes.data_as(ip), None, 0, C.byref(m))
    if rc not in (OK, ENOMEM):
        raise HydroError(rc, L.hydro_last_error(None).decode())
    table = np.empty((max(m.value, 1), 8), dtype=np.int32)
    rc = L.hydro_ghost_map_linear(C.byref(t), out.ctypes.data_as(ip), table.ctypes.data_as(ip),
                                  m.value, C.byref(m))
    if rc:
        raise HydroError(rc, L.hydro_last_error(None).decode())
    return out, table[:m.value].copy()


def reflux_map(tree):
    """Coarse/fine face lists of a workloads.Tree, built by the library, per
    8^3 block (a leaf, or one of the eight octants of a 16^3 leaf):
    (face_flags int32 [blocks], entries int32 [m][26])."""
    L = load()
    t, _keep = _tree_struct(tree)
    nblk = tree.n * (tree.leaf_edge // NX) ** 3
    flags = np.empty(nblk, dtype=np.int32)
    ent = np.empty((nblk, REFLUX_ENTRY), dtype=np.int32)
    m = C.c_int32()
    ip = C.POINTER(C.c_int32)
    rc = L.hydro_reflux_map(C.byref(t), flags.ctypes.data_as(ip), ent.ctypes.data_as(ip), C.byref(m))
    if rc:
        raise HydroError(rc, L.hydro_last_error(None).decode())
    return flags, ent[:m.value].copy()


def _ptr(t) -> int:
    return 0 if t is None else int(t.data_ptr())


def fp64_probe(out, blocks: int, iters: int, m: float = 1.0, c: float = 1.0, stream=None):
    """hydro_fp64_probe into the device tensor out (float64, >= blocks*256)."""
    L = load()
    assert out.dtype.is_floating_point and out.element_size() == 8 and out.numel() >= blocks * 256
    s = None if stream is None else int(stream.cuda_stream) or None
    rc = L.hydro_fp64_probe(_ptr(out), int(blocks), int(iters), float(m), float(c), s)
    if rc:
        raise HydroError(rc, L.hydro_last_error(None).decode())


def step_noalloc(g: "DeviceGrid", dt: float, eta1: float = 1e-3, eta2: float = 1e-1, amax=None,
                 sync: bool = True):
    """One SSP-RK2 step of g (8^3 leaves, at most NOALLOC_MAX_LEAVES) through
    the allocation-free entry point: no handle, the library's fixed device
    scratch array; amax (device float64 [n] or None) receives the per-leaf
    signal speeds."""
    L = load()
    rc = L.hydro_step_noalloc(C.byref(g.c), float(dt), float(eta1), float(eta2), _ptr(amax) or None,
                              int(bool(sync)))
    if rc:
        raise HydroError(rc, L.hydro_last_error(None).decode())


def _sptr(stream):
    return None if stream is None else (int(stream.cuda_stream) or None)


class Hydro:
    """A library handle: owns the device workspace for up to ``max_leaves``."""

    def __init__(self, max_leaves: int, device: int = 0, eta1: float = 1e-3, eta2: float = 1e-1,
                 schedule: str = "auto", tune_cache: str | None = None, learned: bool = False,
                 mlp_batch: int = 4096, rk_order: int = 2, centre_only: bool = False,
                 reflux: bool = False, leaf_edge: int = NX, prolong: bool = False):
        import torch
        self.torch = torch
        self.L = load()
        self.device = device
        self.schedule = schedule
        self.learned = learned
        self.reflux = reflux
        self.prolong = prolong          # grids get ghost maps with linear prolongation
        self.leaf_edge = int(leaf_edge)
        self.p = Params(int(max_leaves), int(device), int(bool(learned)), SCHEDULES[schedule],
                        float(eta1), float(eta2), tune_cache.encode() if tune_cache else None,
                        int(mlp_batch), int(rk_order), int(bool(centre_only)), int(bool(reflux)),
                        int(leaf_edge))
        h = C.c_void_p()
        rc = self.L.hydro_create(C.byref(self.p), C.byref(h))
        if rc:
            raise HydroError(rc, self.L.hydro_last_error(None).decode())
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            self.L.hydro_destroy(self.h)
            self.h = None

    def __del__(self):
        self.close()

    def _check(self, rc):
        if rc:
            raise HydroError(rc, self.L.hydro_last_error(self.h).decode())

    # -- grids ---------------------------------------------------------------
    def grid(self, tree, U, omega: float, gamma: float, launch_off=None, stream=None,
             gmap=None, mlp_alias: bool = True) -> "DeviceGrid":
        """mlp_alias: with learned reconstruction, pass the shared-row table
        (hydro_mlp_alias_map) so the pre-pass skips ghost slabs other blocks
        compute."""
        return DeviceGrid(self, tree, U, omega, gamma, launch_off, stream, gmap, mlp_alias)

    # -- calls ---------------------------------------------------------------
    def step(self, g: "DeviceGrid", dt: float, want_amax: bool = True):
        if want_amax:
            out = np.empty(g.n, dtype=np.float64)
            self._check(self.L.hydro_step(self.h, C.byref(g.c), float(dt),
                                          out.ctypes.data_as(C.POINTER(C.c_double))))
            return out
        self._check(self.L.hydro_step(self.h, C.byref(g.c), float(dt), None))
        return None

    def stage(self, g: "DeviceGrid", stage: int, dt: float, Uin, Un, Uout, amax=None):
        self._check(self.L.hydro_stage(self.h, C.byref(g.c), int(stage), float(dt), _ptr(Uin),
                                       _ptr(Un), _ptr(Uout), _ptr(amax)))

    def step_dev(self, g: "DeviceGrid", cfl: float, dt_dev):
        """Step with dt read from / the next dt written to device dt_dev."""
        self._check(self.L.hydro_step_dev(self.h, C.byref(g.c), float(cfl), _ptr(dt_dev)))

    def dt(self, g: "DeviceGrid", cfl: float, dt_dev):
        self._check(self.L.hydro_dt(self.h, C.byref(g.c), float(cfl), _ptr(dt_dev)))

    def graph_capture(self, g: "DeviceGrid", cfl: float, dt_dev, nsteps: int):
        self._check(self.L.hydro_graph_capture(self.h, C.byref(g.c), float(cfl), _ptr(dt_dev),
                                               int(nsteps)))

    def graph_launch(self, stream=None):
        s = None if stream is None else int(stream.cuda_stream) or None
        self._check(self.L.hydro_graph_launch(self.h, s))

    def autotune(self, g: "DeviceGrid", cache_path: str | None = None):
        table = (C.c_int32 * NBUCKET)()
        self._check(self.L.hydro_autotune(self.h, C.byref(g.c),
                                          cache_path.encode() if cache_path else None, table))
        inv = {v: k for k, v in SCHEDULES.items()}
        return [inv[v] for v in table]

    # -- learned reconstruction ---------------------------------------------
    def mlp_load(self, params):
        par = np.ascontiguousarray(params, dtype=np.float32)
        assert par.shape == (8090,)
        self._check(self.L.hydro_mlp_load(self.h, par.ctypes.data_as(C.POINTER(C.c_float))))

    def mlp_save(self):
        par = np.zeros(8090, dtype=np.float32)
        self._check(self.L.hydro_mlp_save(self.h, par.ctypes.data_as(C.POINTER(C.c_float))))
        return par

    def mlp_forward(self, X, stream=None):
        Y = self.torch.empty((X.shape[0], 26), dtype=self.torch.float32, device=X.device)
        self._check(self.L.hydro_mlp_forward(self.h, _ptr(X), X.shape[0], _ptr(Y), _sptr(stream)))
        return Y

    def mlp_grad(self, X, T, stream=None):
        g = self.torch.empty(8090, dtype=self.torch.float32, device=X.device)
        loss = self.torch.empty(1, dtype=self.torch.float32, device=X.device)
        self._check(self.L.hydro_mlp_grad(self.h, _ptr(X), _ptr(T), X.shape[0], _ptr(g), _ptr(loss),
                                          _sptr(stream)))
        return g, loss

    def mlp_train_step(self, X, T, lr: float, loss=None, stream=None):
        self._check(self.L.hydro_mlp_train_step(self.h, _ptr(X), _ptr(T), X.shape[0], float(lr),
                                                _ptr(loss), _sptr(stream)))

    def mlp_pairs(self, g: "DeviceGrid"):
        n = g.n * NC * NF
        t = self.torch
        X = t.empty((n, 34), dtype=t.float32, device=g.U.device)
        T = t.empty((n, 26), dtype=t.float32, device=g.U.device)
        V = t.empty(n, dtype=t.uint8, device=g.U.device)
        self._check(self.L.hydro_mlp_pairs(self.h, C.byref(g.c), _ptr(X), _ptr(T), _ptr(V)))
        return X, T, V

    def mlp_values(self, g: "DeviceGrid", want_y: bool = False, into_handle: bool = False):
        """The inference pre-pass alone: (val [blocks][7][26][896] float64,
        ok [blocks][896] uint8, y [blocks][7][896][26] float32 or None);
        into_handle: into the handle's own workspace, returns nothing."""
        if into_handle:
            self._check(self.L.hydro_mlp_values(self.h, C.byref(g.c), None, None, None))
            return None
        t = self.torch
        nb = g.n * (self.leaf_edge // NX) ** 3
        val = t.empty((nb, NF, 26, 896), dtype=t.float64, device=g.U.device)
        ok = t.empty((nb, 896), dtype=t.uint8, device=g.U.device)
        y = t.full((nb, NF, 896, 26), float("nan"), dtype=t.float32, device=g.U.device) if want_y else None
        self._check(self.L.hydro_mlp_values(self.h, C.byref(g.c), _ptr(val), _ptr(ok), _ptr(y)))
        return val, ok, y

    def mlp_stats(self):
        c, f = C.c_int64(), C.c_int64()
        self._check(self.L.hydro_mlp_stats(self.h, C.byref(c), C.byref(f)))
        return c.value, f.value

    def signal_speed(self, g: "DeviceGrid"):
        a = self.torch.empty(g.n, dtype=self.torch.float64, device=g.U.device)
        self._check(self.L.hydro_signal_speed(self.h, C.byref(g.c), _ptr(a)))
        return a

    def reconstruct(self, g: "DeviceGrid"):
        out = self.torch.empty((g.n, NF, NC, 26), dtype=self.torch.float64, device=g.U.device)
        self._check(self.L.hydro_reconstruct(self.h, C.byref(g.c), _ptr(out)))
        return out

    def check(self, stream=None):
        self._check(self.L.hydro_check(self.h, stream))

    def timing(self, enable: bool = True):
        """Start/stop stage-kernel event timing; returns (ms, launches)
        recorded since the previous call."""
        ms, n = C.c_double(), C.c_int64()
        self._check(self.L.hydro_timing(self.h, int(enable), C.byref(ms), C.byref(n)))
        return ms.value, n.value


class DeviceGrid:
    """Device-resident mesh of one step: U, dx, origin and ghost map as torch
    tensors, plus the C struct that points at them."""

    def __init__(self, hy: Hydro, tree, U, omega, gamma, launch_off=None, stream=None, gmap=None,
                 mlp_alias: bool = True):
        torch = hy.torch
        dev = torch.device("cuda", hy.device)
        a = tree.arrays()
        self.n = tree.n
        self.U = U if isinstance(U, torch.Tensor) else torch.as_tensor(np.ascontiguousarray(U), device=dev)
        E = tree.leaf_edge
        if E != hy.leaf_edge:
            raise ValueError(f"tree has {E}^3 leaves, the handle {hy.leaf_edge}^3")
        assert self.U.dtype == torch.float64 and self.U.is_contiguous()
        assert tuple(self.U.shape) == (tree.n, NF, E, E, E)
        self.dx = torch.as_tensor(a["dx"], device=dev)
        self.origin = torch.as_tensor(a["origin"], device=dev)
        self.ptable, npro = None, 0
        if gmap is not None:
            gm = gmap
        elif hy.prolong:
            gm, tab = ghost_map_linear(tree)
            npro = tab.shape[0]
            if npro:
                self.ptable = torch.as_tensor(tab, device=dev)
        else:
            gm = ghost_map(tree)
        self.gmap = torch.as_tensor(gm, device=dev)
        self.alias = None
        if hy.learned and mlp_alias:
            gh = gm.cpu().numpy() if isinstance(gm, torch.Tensor) else np.asarray(gm)
            self.alias = torch.as_tensor(mlp_alias_map(tree, gh), device=dev)
        self.stream = stream
        if launch_off is not None:
            self._off = np.ascontiguousarray(launch_off, dtype=np.int32)
            nl, offp = len(self._off) - 1, self._off.ctypes.data_as(C.POINTER(C.c_int32))
        else:
            self._off, nl, offp = None, 0, None
        s = 0 if stream is None else int(stream.cuda_stream)
        self.flags = self.reflux = None
        nr = 0
        if hy.reflux:
            fl, ent = reflux_map(tree)
            self.flags = torch.as_tensor(fl, device=dev)
            self.reflux = torch.as_tensor(ent, device=dev)
            nr = ent.shape[0]
        self.n_reflux = nr
        self.c = Grid(tree.n, nl, offp, _ptr(self.U), _ptr(self.dx), _ptr(self.origin),
                      _ptr(self.gmap), float(omega), float(gamma), s or None,
                      _ptr(self.flags) or None, (_ptr(self.reflux) if nr else 0) or None, nr,
                      _ptr(self.ptable) or None, npro, _ptr(self.alias) or None)
