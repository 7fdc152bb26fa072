"""Training driver of the learned reconstruction.

Pairs come from the plain reconstruction (the library's pair kernel) on the
stage inputs of the 1-leaf blast and of the 64^3 Sedov run, augmented by the
48 symmetries of the cube and by a sign flip; the network is trained by the
library's own MFMA forward/backward and Adam kernels.  This module only
orchestrates: it selects, permutes and batches rows (device gathers) and
schedules the learning rate.  Nothing here computes a step of the method.
"""
from __future__ import annotations

import itertools
import math
import time

import numpy as np

from .hydro import Hydro
from .workloads import blast_single_leaf, sedov_uniform

NPARAM = 8090
SHAPES = (("W1", 2176, 34), ("b1", 64, None), ("W2", 4096, 64), ("b2", 64, None),
          ("W3", 1664, 64), ("b3", 26, None))


def init_params(seed: int = 0) -> np.ndarray:
    """He-uniform weights U(-sqrt(6/fan_in), +sqrt(6/fan_in)), zero biases."""
    rng = np.random.default_rng(seed)
    out = []
    for _, size, fan_in in SHAPES:
        if fan_in is None:
            out.append(np.zeros(size))
        else:
            lim = math.sqrt(6.0 / fan_in)
            out.append(rng.uniform(-lim, lim, size))
    return np.concatenate(out).astype(np.float32)


def collect_pairs(torch, sedov_steps: int = 20, leaves_per_axis: int = 8):
    """Valid (non-flat) training rows from every stage input of one blast step
    and of `sedov_steps` Sedov steps; returns device tensors X [N,34], T [N,26]."""
    Xs, Ts = [], []
    for w, nsteps in ((blast_single_leaf(), 1), (sedov_uniform(leaves_per_axis), sedov_steps)):
        hy = Hydro(max_leaves=w.n, schedule="column")
        try:
            g = hy.grid(w.tree, torch.tensor(w.U, device="cuda"), w.omega, w.gamma)
            U1 = torch.empty_like(g.U)
            U2 = torch.empty_like(g.U)
            dt = float(w.cfl * np.min(w.tree.dx / hy.signal_speed(g).cpu().numpy()))
            am = torch.zeros(w.n, dtype=torch.float64, device="cuda")
            for _ in range(nsteps):
                for U in (g.U, None):
                    if U is None:
                        hy.stage(g, 1, dt, g.U, None, U1, am)
                        src = U1
                    else:
                        src = g.U
                    sub = hy.grid(w.tree, src, w.omega, w.gamma, gmap=g.gmap.cpu().numpy())
                    X, T, V = hy.mlp_pairs(sub)
                    idx = torch.nonzero(V, as_tuple=True)[0]
                    Xs.append(X.index_select(0, idx))
                    Ts.append(T.index_select(0, idx))
                a2 = torch.zeros_like(am)
                hy.stage(g, 2, dt, U1, g.U, U2, a2)
                g.U.copy_(U2)
                amax = torch.maximum(am, a2).cpu().numpy()
                dt = float(w.cfl * np.min(w.tree.dx / amax))
        finally:
            hy.close()
    return torch.cat(Xs), torch.cat(Ts)


def sample(torch, X, T, n: int, seed: int = 1):
    """n rows drawn with default_rng(seed), without replacement when possible."""
    N = X.shape[0]
    idx = np.random.default_rng(seed).choice(N, size=n, replace=N < n)
    it = torch.as_tensor(np.sort(idx), device=X.device)
    return X.index_select(0, it), T.index_select(0, it)


def _off27(o: int):
    return (o % 3 - 1, (o // 3) % 3 - 1, o // 9 - 1)


def _idx27(d) -> int:
    return 9 * (d[2] + 1) + 3 * (d[1] + 1) + (d[0] + 1)


def symmetry_tables():
    """The 48 symmetries of the cube as signed axis permutations R, with
    R p = p' where p'[perm[a]] = sign[a] p[a].  Applied to a state (momentum
    transformed as a vector), a training row of cell c and field f becomes the
    row of cell R c and field f' whose inputs and targets are
    x'[o] = e x[R^-1 o], t'[d] = e t[R^-1 d]: the plain reconstruction along
    a line only sees the values on it, so it commutes with R.  Per symmetry:
    gx [27] and gt [26] (the gathers), fmap [7] (f -> f'; the momenta follow
    perm) and fsign [7] (e: the momentum component's sign)."""
    gx, gt, fmap, fsign = [], [], [], []
    for perm in itertools.permutations(range(3)):
        for bits in range(8):
            sg = [-1 if (bits >> a) & 1 else 1 for a in range(3)]
            inv = []
            for o in range(27):
                q = _off27(o)                                   # o' = q
                inv.append(_idx27([sg[a] * q[perm[a]] for a in range(3)]))   # R^-1 q
            gx.append(inv)
            gt.append([(i if i < 13 else i - 1) for o, i in enumerate(inv) if o != 13])
            fm, fs = list(range(7)), [1.0] * 7
            for a in range(3):
                fm[1 + a] = 1 + perm[a]
                fs[1 + a] = float(sg[a])
            fmap.append(fm)
            fsign.append(fs)
    return (np.array(gx, np.int64), np.array(gt, np.int64), np.array(fmap, np.int64),
            np.array(fsign, np.float32))


def sample_augmented(torch, X, T, n: int, seed: int = 1):
    """n rows drawn with default_rng(seed), without replacement, from the
    pool of every row under each of the 48 cube symmetries and both signs
    (PPM is odd in the field values as well); the symmetry and sign of a draw
    are applied by device gathers and sign changes of the FP32 rows."""
    N = X.shape[0]
    pool = N * 96
    idx = np.random.default_rng(seed).choice(pool, size=n, replace=pool < n)
    idx.sort()
    return augment_rows(torch, X, T, idx // 96, (idx % 96) // 2, 1 - 2 * (idx % 2))


def augment_rows(torch, X, T, rows, sym, sign):
    """Rows `rows` of (X, T) under cube symmetries `sym` (indices into
    symmetry_tables) and signs `sign` (+1 / -1), one per output row."""
    row = torch.as_tensor(np.asarray(rows), device=X.device)
    k = torch.as_tensor(np.asarray(sym), device=X.device)
    flip = torch.as_tensor(np.asarray(sign, dtype=np.float32), device=X.device)
    gx, gt, fmap, fsign = (torch.as_tensor(a, device=X.device) for a in symmetry_tables())
    X0, T0 = X.index_select(0, row), T.index_select(0, row)
    f = X0[:, 27:].argmax(dim=1)
    e = (flip * fsign[k, f]).unsqueeze(1)
    Xa = torch.empty_like(X0)
    Xa[:, :27] = torch.gather(X0[:, :27], 1, gx[k]) * e
    Xa[:, 27:] = torch.nn.functional.one_hot(fmap[k, f], 7).to(X0.dtype)
    Ta = torch.gather(T0, 1, gt[k]) * e
    return Xa, Ta


def train(torch, hy: Hydro, X, T, epochs: int = 8, batch: int = 4096, lr0: float = 1e-3,
          lr1: float = 1e-5, holdout: float = 0.05, seed: int = 0, params=None, log=None):
    """Adam with a cosine learning rate from lr0 to lr1; returns (params, history)."""
    N = X.shape[0]
    rng = np.random.default_rng(seed)
    perm = torch.as_tensor(rng.permutation(N), device=X.device)
    n_hold = max(batch, int(holdout * N)) if N > 2 * batch else 0
    hold, tr = perm[:n_hold], perm[n_hold:]
    ntr = tr.shape[0]
    steps_per_epoch = max(1, ntr // batch)
    total = epochs * steps_per_epoch
    hy.mlp_load(init_params(seed) if params is None else params)
    loss = torch.zeros(1, dtype=torch.float32, device=X.device)
    hist = []
    step, t0 = 0, time.perf_counter()
    for ep in range(epochs):
        order = tr[torch.as_tensor(rng.permutation(ntr), device=X.device)]
        run = 0.0
        for b in range(steps_per_epoch):
            idx = order[b * batch:(b + 1) * batch]
            lr = lr1 + 0.5 * (lr0 - lr1) * (1.0 + math.cos(math.pi * step / max(total, 1)))
            hy.mlp_train_step(X.index_select(0, idx), T.index_select(0, idx), lr, loss)
            step += 1
            if b % 64 == 0 or b == steps_per_epoch - 1:
                run = float(loss.item())
        val = held_out_loss(torch, hy, X, T, hold, batch) if n_hold else float("nan")
        hist.append(dict(epoch=ep, train_loss=run, val_loss=val, seconds=time.perf_counter() - t0))
        if log:
            log(hist[-1])
    return hy.mlp_save(), hist


def held_out_loss(torch, hy: Hydro, X, T, hold, batch: int) -> float:
    tot, n = 0.0, 0
    for b in range(0, hold.shape[0], batch):
        idx = hold[b:b + batch]
        _, l = hy.mlp_grad(X.index_select(0, idx), T.index_select(0, idx))
        tot += float(l.item()) * idx.shape[0]
        n += idx.shape[0]
    return tot / max(n, 1)


def train_default(torch, n_pairs: int = 2 ** 22, epochs: int = 8, sedov_steps: int = 20, log=None,
                  augment: bool = True):
    """The configuration of the learned-limiter workload: 2^22 pairs from the
    blast leaf and 20 Sedov steps, augmented by the cube's symmetries and sign
    flips, batch 4096, 8 epochs, lr 1e-3 -> 1e-5.  Returns (params, history,
    {"source_rows", "augmented"})."""
    X, T = collect_pairs(torch, sedov_steps)
    N = int(X.shape[0])
    Xs, Ts = (sample_augmented if augment else sample)(torch, X, T, n_pairs)
    del X, T
    hy = Hydro(max_leaves=1, mlp_batch=4096)
    try:
        params, hist = train(torch, hy, Xs, Ts, epochs=epochs, log=log)
    finally:
        hy.close()
    return params, hist, {"source_rows": N, "augmented": bool(augment)}
