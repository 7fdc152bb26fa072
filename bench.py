"""Benchmark of the hydro hot path on one MI355X.

Workload: the Sedov-Taylor blast on a uniform 64^3 grid held as 512 leaves of
8^3 cells (three ghost layers each), FP64, gamma = 5/3, outflow boundaries;
SSP-RK2 steps at CFL 0.4 of the plain method, one leaf per workgroup.  A
benchmark "step" is one full SSP-RK2 step (two stages: ghost gather, PPM at 26
points, central-upwind fluxes, Simpson quadrature, divergence, sources, stage
combine, dual-energy resync, per-leaf signal speeds) plus the next dt from
the signal speeds, computed on the device.  The timed region starts from the
initial blast state with the fields already resident in HBM, takes dt0 from a
signal-speed pre-pass and runs exactly --steps steps.

Metric: FP64 cell-updates per second per RK stage = interior cells x stages /
wall time.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "FP64 cell-updates/s per RK stage, plain vs batched+learned; % HBM roofline"
# Algorithmic FP64 operations per interior cell-update of one stage (adds,
# subtracts, multiplies, divides, square roots and powers; comparisons not
# counted), from the operation-counting build of the CPU oracle restricted to
# the work the method needs: 19.75 line reconstructions per cell and field,
# 30.375 face-point fluxes per cell, divergence, source and stage combine.
FLOPS_PER_CELL_UPDATE = 10292.0
# Algorithmic HBM bytes per cell-update and stage (mean of the two stages):
# read the stage input once (56 B), write the result once (56 B), and read
# the step-start state in the second stage (+56 B, half of it per stage).
BYTES_PER_CELL_UPDATE = 140.0
PEAK_FP64_TFLOPS = 78.6
PEAK_HBM_GBS = 8000.0


def autotuned(hy, g):
    """Autotune the grid's schedules: the per-size table, and the single
    schedule the tuner keeps for whole stages of the grid's partition
    ("table" when it keeps the table)."""
    import tempfile
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "tune.json")
        table = hy.autotune(g, path)
        with open(path) as f:
            conc = json.load(f).get("concurrent", -1)
    return table, {1: "face", 2: "column", 3: "persistent", 4: "tiled"}.get(conc, "table")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--schedule", default="column", choices=["column", "face", "persistent", "tiled", "auto"])
    ap.add_argument("--no-batched", action="store_true",
                    help="skip the polytrope and binary plain/learned legs (and the network training)")
    ap.add_argument("--no-binary", action="store_true", help="skip the 32768-leaf binary leg")
    ap.add_argument("--train-pairs", type=int, default=2 ** 20)
    ap.add_argument("--train-epochs", type=int, default=2)
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="before the timed steps, one untimed device copy of this many MiB from a "
                         "freshly written buffer (the reference kernel for HBM counter calibration)")
    return ap.parse_args()


# HBM bytes per stage launch of the timed kernel, from rocprofv3 FETCH_SIZE /
# WRITE_SIZE runs calibrated on a plain copy; valid only for the kernel
# sources they were measured on.
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "stage_kernel_col-sedov64-traffic.json")
KERNEL_SOURCES = ("paper_2107_10987_amd/csrc/stage_kernel.hip", "paper_2107_10987_amd/csrc/hydro_common.h")


def kernel_source_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic(schedule: str):
    """Bytes per launch from the committed counter summary, or None when it
    is missing, was taken on another schedule, or the kernel has changed."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("schedule") != schedule or t.get("source_sha256") != kernel_source_hash():
        return None
    return t.get("bytes_per_launch")


def copy_probe(torch, mib: int):
    """src -> dst device copy of `mib` MiB, with 512 MiB written in between
    so that src is no longer in the caches (the 256 MB last-level cache
    included) when the copy reads it."""
    n = mib * 2 ** 20 // 8
    src = torch.arange(n, dtype=torch.float64, device="cuda")
    flush = torch.empty(512 * 2 ** 20 // 8, dtype=torch.float64, device="cuda")
    flush.fill_(1.0)
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst, flush


def cpu_baseline(w, budget_s: float):
    """The CPU oracle on the same workload: whole SSP-RK2 steps over all 512
    leaves from the initial state until about budget_s seconds have passed."""
    import oracle
    threads = oracle.default_threads()
    o = oracle.Oracle(w.tree, w.gamma, w.omega, threads=threads)
    U = w.U.copy()
    dt = o.dt(U)
    steps, t0 = 0, time.perf_counter()
    while True:
        U, am = o.step(dt, U)
        steps += 1
        dt = float(w.cfl * np.min(w.tree.dx / am))
        if time.perf_counter() - t0 >= budget_s:
            break
    el = time.perf_counter() - t0
    # one host thread: stage 1 of the first 256 leaves of the final state
    o1 = oracle.Oracle(w.tree, w.gamma, w.omega, threads=1)
    n1, t1 = 256, time.perf_counter()
    o1.stage(1, dt, U, l0=0, l1=n1)
    el1 = time.perf_counter() - t1
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            model = next((ln.split(":", 1)[1].strip() for ln in f if ln.startswith("model name")), "")
    except OSError:
        pass
    return dict(value=w.cells * 2 * steps / el, unit="cell-updates/s", cores=threads, kind="oracle",
                sample=f"{steps} full SSP-RK2 steps of the same 64^3 Sedov workload from t=0 "
                       f"({w.n} leaves, {threads} host threads, {el:.1f} s)",
                single_thread={"value": n1 * 512 / el1, "unit": "cell-updates/s",
                               "sample": f"stage 1 of {n1} leaves of the final state, 1 thread, {el1:.2f} s"},
                host={"cpu_count": os.cpu_count(), "model": model})


def train_network(torch, args):
    from paper_2107_10987_amd import learned
    t0 = time.perf_counter()
    params, hist = learned.train_default(torch, n_pairs=args.train_pairs, epochs=args.train_epochs)
    info = {"pairs": args.train_pairs, "epochs": args.train_epochs, "seconds": time.perf_counter() - t0,
            "final_train_loss": hist[-1]["train_loss"], "val_loss": hist[-1]["val_loss"]}
    return params, info


def binary_leg(torch, args, params):
    """The 32768-leaf binary star (16,777,216 cells, four levels), launched as
    seeded uneven batches with autotuned schedules; 10 SSP-RK2 steps with the
    time step on the device, captured in one HIP graph and replayed: plain PPM
    and the learned reconstruction with FP64 check and plain-PPM fallback."""
    from paper_2107_10987_amd.hydro import Hydro
    from paper_2107_10987_amd.workloads import binary_star, uneven_batches

    t0 = time.perf_counter()
    w = binary_star()
    build_s = time.perf_counter() - t0
    off = uneven_batches(w.n)
    U0 = torch.tensor(w.U, device="cuda")
    nsteps = 10
    out = {"workload": ("binary-32768: two n=1.5 polytropes (mass ratio 0.5, separation 0.5) on a "
                        f"4-level octree of {w.n} leaves, co-rotating Omega {w.omega:.4f}, "
                        f"{len(off) - 1} seeded uneven launches per stage, autotuned schedules, "
                        f"{nsteps} steps in one HIP graph with the time step on the device"),
           "host_build_seconds": build_s}
    results = {}
    for name, on in (("plain", False), ("learned", True)):
        hy = Hydro(max_leaves=w.n, schedule="auto", learned=on)
        try:
            s = torch.cuda.Stream()
            g = hy.grid(w.tree, U0.clone(), w.omega, w.gamma, launch_off=off, stream=s)
            if on:
                hy.mlp_load(params)
            torch.cuda.synchronize()
            _, conc = autotuned(hy, g)
            dt_dev = torch.zeros(1, dtype=torch.float64, device="cuda")
            hy.dt(g, w.cfl, dt_dev)
            hy.graph_capture(g, w.cfl, dt_dev, nsteps)
            hy.graph_launch(s)            # untimed: the first 10 steps
            s.synchronize()
            if on:
                hy.mlp_stats()            # reset the fallback counters
            t1 = time.perf_counter()
            hy.graph_launch(s)            # timed: steps 11..20
            s.synchronize()
            el = time.perf_counter() - t1
            hy.check(s)
            results[name] = g.U.cpu().numpy()
            out[name] = {"value": w.cells * 2 * nsteps / el, "unit": "cell-updates/s",
                         "ms_per_step": el / nsteps * 1e3, "launches_per_stage": len(off) - 1,
                         "dt_after": float(dt_dev.item()), "autotune_concurrent": conc}
            if on:
                cells, fb = hy.mlp_stats()
                out[name]["fallback_fraction"] = fb / max(cells, 1)
        finally:
            hy.close()
    d = np.abs(results["learned"] - results["plain"])
    out["learned"]["l1_rel_dev_vs_plain"] = float(d.sum() / np.abs(results["plain"]).sum())
    out["learned"]["gain_vs_plain"] = out["learned"]["value"] / out["plain"]["value"]
    return out


def batched_legs(torch, args, params):
    """The 4096-leaf rotating polytrope on a 3-level octree, launched as seeded
    uneven batches with autotuned schedules: one SSP-RK2 step (two stages) at
    the plain path's CFL time step, timed ten times after one untimed (median), plain PPM and the learned
    reconstruction with FP64 check and plain-PPM fallback."""
    from paper_2107_10987_amd.hydro import Hydro
    from paper_2107_10987_amd.workloads import rotating_polytrope, uneven_batches

    w = rotating_polytrope()
    off = uneven_batches(w.n)
    U0 = torch.tensor(w.U, device="cuda")
    out = {}
    table = None
    results = {}
    for name, on in (("plain", False), ("learned", True)):
        hy = Hydro(max_leaves=w.n, schedule="auto", learned=on)
        try:
            g = hy.grid(w.tree, U0.clone(), w.omega, w.gamma, launch_off=off)
            if on:
                hy.mlp_load(params)
            t_, conc = autotuned(hy, g)
            table = t_ if table is None else table
            if not on:   # both paths step with the plain path's CFL time step
                dt = float(w.cfl * np.min(w.tree.dx / hy.signal_speed(g).cpu().numpy()))
            else:
                hy.mlp_stats()   # count the fallbacks of the timed steps only
            times = []
            for r in range(11):
                g.U.copy_(U0)
                torch.cuda.synchronize()
                t1 = time.perf_counter()
                hy.step(g, dt)
                torch.cuda.synchronize()
                times.append(time.perf_counter() - t1)
            med = float(np.median(times[1:]))
            cells, fb = hy.mlp_stats() if on else (0, 0)
            results[name] = g.U.cpu().numpy()
            out[name] = {"value": w.cells * 2 / med, "unit": "cell-updates/s", "ms_per_step": med * 1e3,
                         "launches_per_stage": len(off) - 1, "autotune_concurrent": conc}
            if on:
                out[name]["fallback_fraction"] = fb / max(cells, 1)
        finally:
            hy.close()
    d = np.abs(results["learned"] - results["plain"])
    out["learned"]["l1_rel_dev_vs_plain"] = float(d.sum() / np.abs(results["plain"]).sum())
    out["learned"]["linf_rel_dev_vs_plain"] = float(d.max() / np.abs(results["plain"]).max())
    out["learned"]["gain_vs_plain"] = out["learned"]["value"] / out["plain"]["value"]
    out["workload"] = ("polytrope-4096: rotating n=1.5 polytrope, 3-level octree of 4096 leaves, "
                       f"Omega 0.1, {len(off) - 1} seeded uneven batches, autotuned schedules, dt at CFL 0.4")
    out["autotune_table"] = table
    return out


def timed_sedov(torch, hy, w, args):
    """--warmup untimed device-dt steps, then two passes of exactly --steps
    steps from the same initial state on one stream: eager launches with HIP
    events around every stage launch (kernel-only time), and the whole job --
    the signal-speed pre-pass for dt0, then the steps replayed from one HIP
    graph -- between device synchronisations (end-to-end time).  Returns
    (end-to-end seconds, event milliseconds, stage launches)."""
    s = torch.cuda.Stream()
    U0 = torch.tensor(w.U, device="cuda")
    g = hy.grid(w.tree, U0.clone(), w.omega, w.gamma, stream=s)
    dt_dev = torch.zeros(1, dtype=torch.float64, device="cuda")

    def reset():   # the initial state back in place (not part of the job)
        with torch.cuda.stream(s):
            g.U.copy_(U0)
        s.synchronize()

    def eager(nsteps):
        reset()
        hy.dt(g, w.cfl, dt_dev)   # dt0 from the signal-speed pre-pass, on the device
        for _ in range(nsteps):
            hy.step_dev(g, w.cfl, dt_dev)
        s.synchronize()

    eager(args.warmup)
    hy.timing(True)
    eager(args.steps)
    kms, launches = hy.timing(False)
    hy.check()   # deferred non-physical-state check
    hy.graph_capture(g, w.cfl, dt_dev, args.steps)   # records the steps, runs nothing
    reset()
    hy.dt(g, w.cfl, dt_dev)
    hy.graph_launch(s)                                # one untimed replay
    reset()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    hy.dt(g, w.cfl, dt_dev)
    hy.graph_launch(s)
    s.synchronize()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    hy.check()
    return el, kms, launches


def leaf16_leg(torch, args):
    """The same 64^3 Sedov workload held as 64 leaves of 16^3 cells (the
    paper's production leaf size; each leaf is eight 8^3 tiles, one workgroup
    each), timed like the 8^3 leaves."""
    from paper_2107_10987_amd.hydro import Hydro
    from paper_2107_10987_amd.workloads import sedov_uniform

    w = sedov_uniform(4, leaf_edge=16)
    hy = Hydro(max_leaves=w.n, schedule=args.schedule, leaf_edge=16)
    try:
        el, kms, launches = timed_sedov(torch, hy, w, args)
        avg = kms / 1e3 / max(launches, 1)
        return {"workload": "sedov-64^3 as 64 leaves of 16^3 cells (512 tiles of 8^3)",
                "value": w.cells * 2 * args.steps / el, "unit": "cell-updates/s",
                "ms_per_step": el / args.steps * 1e3, "avg_launch_us": avg * 1e6,
                "kernel_cell_updates_per_s": w.cells / avg}
    finally:
        hy.close()


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the hydro path runs on one GPU; it is not sharded across GPUs)", file=sys.stderr)
        sys.exit(2)
    import torch

    from paper_2107_10987_amd.hydro import Hydro
    from paper_2107_10987_amd.workloads import sedov_uniform

    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    w = sedov_uniform(8)
    hy = Hydro(max_leaves=w.n, schedule=args.schedule)
    if args.copy_probe_mib > 0:
        copy_probe(torch, args.copy_probe_mib)
    elapsed, kms, launches = timed_sedov(torch, hy, w, args)
    stages = 2 * args.steps
    value = w.cells * stages / elapsed
    avg_launch_s = kms / 1e3 / max(launches, 1)
    cells_per_launch = w.cells
    achieved_tflops = FLOPS_PER_CELL_UPDATE * cells_per_launch / avg_launch_s / 1e12
    achieved_gbs = BYTES_PER_CELL_UPDATE * cells_per_launch / avg_launch_s / 1e9

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "sedov-64^3: 512 leaves of 8^3 cells + 3 ghost layers, FP64, gamma 5/3, "
                               "outflow, SSP-RK2 at CFL 0.4, plain PPM, one leaf per workgroup",
                   "leaves": w.n, "cells": w.cells, "stages_per_step": 2, "path": "plain"},
        "kernel": {"name": "stage_kernel_col" if args.schedule == "column" else "stage_kernel",
                   "schedule": args.schedule, "avg_launch_us": avg_launch_s * 1e6, "launches": launches,
                   "kernel_cell_updates_per_s": cells_per_launch / avg_launch_s},
        "roofline": {"bound": "alu", "achieved": achieved_tflops, "peak": PEAK_FP64_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved_tflops / PEAK_FP64_TFLOPS,
                     "traffic": measured_traffic(args.schedule)},
        "hbm": {"achieved": achieved_gbs, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": achieved_gbs / PEAK_HBM_GBS},
    }
    hy.close()
    out["leaf16"] = leaf16_leg(torch, args)
    if not args.no_batched:
        params, info = train_network(torch, args)
        out["batched"] = batched_legs(torch, args, params)
        out["batched"]["training"] = info
        if not args.no_binary:
            out["binary"] = binary_leg(torch, args, params)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
