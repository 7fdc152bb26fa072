"""Benchmark of the hydro hot path on one MI355X.

Headline workload: the binary-star setup on 32,768 leaves of 8^3 cells
(16,777,216 cells, the paper's problem size, four AMR levels), FP64,
gamma = 5/3, co-rotating frame, plain PPM; one launch per Runge-Kutta stage
over all leaves (every leaf batched into one kernel), the SSP-RK2 steps with
the time step on the device captured in one HIP graph and replayed.  A
benchmark "step" is one full SSP-RK2 step (two stages: ghost gather, PPM at 26
points, central-upwind fluxes, Simpson quadrature, divergence, sources, stage
combine, dual-energy resync, per-leaf signal speeds) plus the next dt,
computed on the device.  The timed region starts from the initial state with
the fields already resident in HBM, takes dt0 from a signal-speed pre-pass and
runs exactly --steps steps after --warmup untimed ones.  Its working set
(0.94 GB of fields, 3.8 GB of workspace) is far beyond the 256 MB last-level
cache.

The same line reports the other workloads: the same binary with the learned
reconstruction, the 64^3 Sedov blast (512 leaves; the oracle trajectory
parity case), the same blast as 16^3 leaves, the Sedov blast at the paper's
problem size (256^3 as 32,768 leaves), the 4096-leaf rotating
polytrope in seeded uneven launches (plain and learned), the old face-centre
scheme on the Sedov blast, each with its own roofline, and the CPU oracle.

Metric: FP64 cell-updates per second per RK stage = interior cells x stages /
wall time.  Prints one JSON line.

--profile NAME runs one workload's kernels only (for rocprofv3 counter runs);
--reduce-counters turns two such runs' CSV output into the traffic summary
the roofline's "traffic" field reads.
"""
from __future__ import annotations

import argparse
import glob
import hashlib
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
# The old face-centre scheme, counted the same way: 3.75 line reconstructions
# (the axis lines) per cell and field and 3.375 face-centre fluxes per cell.
FLOPS_PER_CELL_UPDATE_OLD = 1692.0
# Algorithmic HBM bytes per cell-update and stage (mean of the two stages):
# read the stage input once (56 B), write the result once (56 B), and read
# the step-start state in the second stage (+56 B, half of it per stage).
BYTES_PER_CELL_UPDATE = 140.0
# The learned reconstruction's network: 2 (34*64 + 64*64 + 64*26) flops per
# row, 7 rows per cell; an 8^3 block needs the rows of 896 cells, 512 of its
# own and 384 face-adjacent ghost cells (evaluated unless another block's
# pre-pass holds them).
MLP_FLOPS_PER_ROW = 2.0 * (34 * 64 + 64 * 64 + 64 * 26)
PEAK_FP64_TFLOPS = 78.6
PEAK_BF16_TFLOPS = 2500.0
PEAK_HBM_GBS = 8000.0

KERNEL_SOURCES = ("paper_2107_10987_amd/csrc/stage_kernel.hip", "paper_2107_10987_amd/csrc/hydro_common.h",
                  "paper_2107_10987_amd/csrc/mlp_kernels.hip", "paper_2107_10987_amd/csrc/mlp_common.h")
PROFILES = os.path.join(ROOT, "profiles")
KERNEL_OF = {"column": "stage_kernel_col", "face": "stage_kernel", "persistent": "stage_kernel_col_persistent",
             "tiled": "stage_kernel_col_persistent"}


def parse(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=10.0,
                    help="CPU oracle budget of the headline baseline (the others take a few seconds each)")
    ap.add_argument("--schedule", default="auto", choices=["column", "face", "persistent", "tiled", "auto"],
                    help="stage-kernel schedule of the single-launch legs (auto: the autotuner's table)")
    ap.add_argument("--no-learned", action="store_true", help="skip the learned legs (and the training)")
    ap.add_argument("--no-extra", action="store_true",
                    help="headline only: skip the Sedov, 16^3, polytrope and old-scheme legs")
    ap.add_argument("--train-pairs", type=int, default=2 ** 22)
    ap.add_argument("--train-epochs", type=int, default=8)
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="before anything else, one untimed device copy of this many MiB from a freshly "
                         "written buffer (the reference kernel for HBM counter calibration)")
    ap.add_argument("--profile", default=None,
                    choices=["binary-plain", "binary-learned", "sedov64", "sedov256", "sedov64-leaf16",
                             "sedov64-old", "polytrope-plain", "polytrope-learned"],
                    help="run only this workload's kernels, a few eager steps (for counter runs)")
    ap.add_argument("--reduce-trace", metavar="TRACE_DIR",
                    help="per-kernel, per-grid-size dispatch counts and mean durations of a rocprofv3 "
                         "--kernel-trace run, as a markdown table")
    ap.add_argument("--reduce-counters", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="turn the CSV output of a FETCH_SIZE run and a WRITE_SIZE run of --profile NAME "
                         "into profiles/<NAME>-traffic.json (needs --profile NAME for the name)")
    return ap.parse_args(argv)


# ---------------------------------------------------------------------------
# rooflines and counter summaries
# ---------------------------------------------------------------------------

def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def traffic_file(name: str) -> str:
    return os.path.join(PROFILES, f"{name}-traffic.json")


def measured_traffic(name: str, kernel: str):
    """Calibrated HBM bytes per launch of `kernel` in the committed counter
    summary of workload `name`, or None when it is missing or the kernel
    sources have changed since the counters were taken."""
    try:
        with open(traffic_file(name)) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("source_sha256") != kernel_source_hash():
        return None
    k = t.get("kernels", {}).get(kernel)
    return None if k is None else k.get("bytes_per_launch")


def fp64_roofline(kernel: str, cells: int, seconds: float, traffic=None, flops=FLOPS_PER_CELL_UPDATE):
    ach = flops * cells / seconds / 1e12
    return {"kernel": kernel, "bound": "alu", "achieved": ach, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
            "frac": ach / PEAK_FP64_TFLOPS, "traffic": traffic}


def prepass_cells(g) -> int:
    """Cells whose rows one pre-pass over all of g's blocks evaluates: every
    block's 512 interior cells and the 64 of each ghost slab not wholly shared
    with other blocks (hydro_mlp_alias_map; every block is in the one launch)."""
    blocks = g.gmap.numel() // 2232
    if g.alias is None:
        return blocks * 896
    shared = (g.alias.reshape(blocks, 6, 64) >= 0).all(dim=2)
    return int(blocks * 896 - 64 * int(shared.sum()))


def mfma_roofline(cells: int, seconds: float, traffic=None):
    """bf16-MFMA fraction of the pre-pass: the network's flops over the rows
    it evaluates (7 per cell)."""
    ach = MLP_FLOPS_PER_ROW * 7 * cells / seconds / 1e12
    return {"kernel": "mlp_infer_kernel", "bound": "mfma", "achieved": ach, "peak": PEAK_BF16_TFLOPS,
            "unit": "TFLOP/s", "frac": ach / PEAK_BF16_TFLOPS, "traffic": traffic,
            "rows_per_launch": 7 * cells}


def learned_table_bytes(g) -> int:
    """Bytes of the learned values a stage over all of g's blocks needs, each
    once: the 13 lines x 7 fields of every interior cell as stored (two
    binary32 offsets, 8 B), and for every face-adjacent ghost cell whose row
    no block of the launch holds as its own, the 9 lines crossing that face at
    the one end the face uses (4 B); a shared ghost row is the owner's
    interior row, counted there."""
    blocks = g.gmap.numel() // 2232
    own = blocks * 384 if g.alias is None else int((g.alias < 0).sum())
    return blocks * 512 * 13 * 7 * 8 + own * 9 * 7 * 4


def hbm_roofline(kernel: str, alg_bytes: float, seconds: float, traffic=None):
    """HBM fraction of a launch from its algorithmic bytes, with the
    counter-measured bytes beside it."""
    ach = alg_bytes / seconds / 1e9
    return {"kernel": kernel, "bound": "hbm", "achieved": ach, "peak": PEAK_HBM_GBS, "unit": "GB/s",
            "frac": ach / PEAK_HBM_GBS, "traffic": traffic,
            "algorithmic_bytes_per_launch": alg_bytes,
            "counter_frac": None if not traffic else traffic / seconds / 1e9 / PEAK_HBM_GBS}


def hbm_figures(cells: int, seconds: float, traffic=None):
    """Algorithmic HBM rate (140 B per cell-update) and, when the counter
    summary is current, the counter-measured one, against the 8 TB/s peak."""
    alg = BYTES_PER_CELL_UPDATE * cells / seconds / 1e9
    out = {"algorithmic_gbs": alg, "algorithmic_frac": alg / PEAK_HBM_GBS, "peak": PEAK_HBM_GBS,
           "unit": "GB/s", "counter_gbs": None, "counter_frac": None,
           "algorithmic_bytes_per_launch": BYTES_PER_CELL_UPDATE * cells, "counter_bytes_per_launch": traffic}
    if traffic:
        out["counter_gbs"] = traffic / seconds / 1e9
        out["counter_frac"] = out["counter_gbs"] / PEAK_HBM_GBS
    return out


def _csv_rows(d: str):
    import csv
    files = sorted(glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True))
    if not files:
        raise SystemExit(f"no counter_collection.csv under {d}")
    rows = []
    for fn in files:
        with open(fn) as f:
            rows += list(csv.DictReader(f))
    return rows


def _per_dispatch(rows, counter: str):
    """{dispatch id: (kernel name, grid size, summed counter value)} in
    dispatch order."""
    out = {}
    for r in rows:
        if r.get("Counter_Name") != counter:
            continue
        did = int(r["Dispatch_Id"])
        name = r.get("Kernel_Name", "")
        v = float(r["Counter_Value"])
        k, gsz, acc = out.get(did, (name, int(r.get("Grid_Size", 0) or 0), 0.0))
        out[did] = (k, gsz, acc + v)
    return dict(sorted(out.items()))


def _short(name: str, template: bool = False):
    """This library's kernel name in a rocprofv3 kernel name (with its
    template arguments if `template`), or None."""
    import re
    m = re.search(r"\b(stage_kernel\w*|mlp_infer_kernel)(<[^>(]*>)?\(", name)
    if not m:
        return None
    return m.group(1) + (m.group(2) or "") if template else m.group(1)


def reduce_trace(d: str) -> str:
    """Markdown table of a kernel trace: for each of this library's kernels
    and grid size, the dispatches and their mean and median durations."""
    import csv
    files = sorted(glob.glob(os.path.join(d, "**", "*kernel_trace.csv"), recursive=True))
    if not files:
        raise SystemExit(f"no kernel_trace.csv under {d}")
    groups = {}
    for fn in files:
        with open(fn) as f:
            for r in csv.DictReader(f):
                k = _short(r["Kernel_Name"], template=True) or r["Kernel_Name"].split("(")[0]
                if not (k.startswith("stage_kernel") or k.startswith("mlp_") or k.startswith("dt_kernel")
                        or k.startswith("reflux")):
                    continue
                wg = int(r.get("Workgroup_Size_X", 1) or 1)
                grid = int(r.get("Grid_Size_X", 0) or 0) // max(wg, 1)
                dur = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3
                groups.setdefault((k, grid), []).append(dur)
    lines = ["| kernel | workgroups | dispatches | mean us | median us | min us | max us |",
             "|---|---|---|---|---|---|---|"]
    for (k, grid), v in sorted(groups.items()):
        a = np.array(v)
        lines.append(f"| {k} | {grid} | {len(a)} | {a.mean():.1f} | {np.median(a):.1f} | {a.min():.1f} | "
                     f"{a.max():.1f} |")
    return "\n".join(lines)


def reduce_counters(name: str, fetch_dir: str, write_dir: str, cmd_fetch: str, cmd_write: str):
    """profiles/<name>-traffic.json from a FETCH_SIZE and a WRITE_SIZE run of
    --profile <name> --copy-probe-mib 1024: per kernel, the mean calibrated
    bytes per dispatch (FETCH_SIZE scaled so the copy probe reads what it
    copies, WRITE_SIZE likewise)."""
    fetch = _per_dispatch(_csv_rows(fetch_dir), "FETCH_SIZE")
    write = _per_dispatch(_csv_rows(write_dir), "WRITE_SIZE")
    probe_bytes = 1024 * 2 ** 20

    def probe_value(d):
        # the copy probe: the largest dispatch of a device copy kernel
        return max(v for (k, _, v) in d.values() if "copy" in k.lower())

    pf, pw = probe_value(fetch), probe_value(write)
    ff, wf = probe_bytes / 1024 / pf, probe_bytes / 1024 / pw
    kernels = {}
    for label, d in (("fetch", fetch), ("write", write)):
        # the workload's own dispatches are the largest grids of each kernel
        # (the training run's stage launches on smaller grids are left out);
        # a stage kernel's first such dispatch is the signal-speed pass
        big = {}
        for did, (k, gsz, v) in d.items():
            short = _short(k)
            if short is not None:
                big[short] = max(big.get(short, 0), gsz)
        seen = {}
        for did, (k, gsz, v) in d.items():
            short = _short(k)
            if short is None or gsz != big[short]:
                continue
            seen[short] = seen.get(short, 0) + 1
            if short.startswith("stage_kernel") and seen[short] == 1:
                continue
            kernels.setdefault(short, {"fetch_kib": [], "write_kib": []})[label + "_kib"].append(v)
    for short, e in kernels.items():
        fb = float(np.mean(e["fetch_kib"])) * 1024 * ff if e["fetch_kib"] else 0.0
        wb = float(np.mean(e["write_kib"])) * 1024 * wf if e["write_kib"] else 0.0
        e.update(dispatches=len(e["fetch_kib"]), fetch_bytes=fb, write_bytes=wb, bytes_per_launch=fb + wb)
        if short.startswith("stage_kernel"):
            # alternate stages 1 and 2 of the steps
            for st in (1, 2):
                fk, wk = e["fetch_kib"][st - 1::2], e["write_kib"][st - 1::2]
                if fk and wk:
                    e[f"bytes_per_launch_stage{st}"] = float(np.mean(fk)) * 1024 * ff + float(np.mean(wk)) * 1024 * wf
    out = {"workload": name, "source_sha256": kernel_source_hash(),
           "calibration": {"probe": "device copy of 1024 MiB from a buffer evicted by a 512 MiB write",
                           "probe_fetch_kib": pf, "probe_write_kib": pw, "fetch_factor": ff,
                           "write_factor": wf},
           "kernels": kernels, "commands": {"fetch": cmd_fetch, "write": cmd_write}}
    with open(traffic_file(name), "w") as f:
        json.dump(out, f, indent=1)
    return out


# ---------------------------------------------------------------------------
# helpers
# ---------------------------------------------------------------------------

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


def attainable(torch, fp64_iters: int = 4096, copy_mib: int = 1024, reps: int = 3):
    """What this device attains on the two ceilings of the rooflines, measured
    in this run: the FP64 vector rate of a pure fused-multiply-add kernel
    (hydro_fp64_probe: 2048 workgroups of 256 threads, eight independent
    chains per thread) and the HBM rate of a device copy of copy_mib MiB from
    an evicted buffer (bytes read plus written); the best of reps timed runs
    after one untimed one, HIP events on the current stream."""
    from paper_2107_10987_amd import hydro
    blocks = 2048
    out = torch.empty(blocks * 256, dtype=torch.float64, device="cuda")
    flops = 2.0 * 8 * fp64_iters * blocks * 256
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    s = torch.cuda.current_stream()
    best = float("inf")
    for r in range(reps + 1):
        e0.record(s)
        hydro.fp64_probe(out, blocks, fp64_iters, 1.0, 1.0, s)
        e1.record(s)
        e1.synchronize()
        if r:
            best = min(best, e0.elapsed_time(e1) / 1e3)
    n = copy_mib * 2 ** 20 // 8
    src = torch.arange(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    flush = torch.empty(512 * 2 ** 20 // 8, dtype=torch.float64, device="cuda")
    bestc = float("inf")
    for r in range(reps + 1):
        flush.fill_(1.0)
        e0.record(s)
        dst.copy_(src)
        e1.record(s)
        e1.synchronize()
        if r:
            bestc = min(bestc, e0.elapsed_time(e1) / 1e3)
    del src, dst, flush, out
    return {"fp64_tflops": flops / best / 1e12, "hbm_gbs": 2.0 * n * 8 / bestc / 1e9,
            "method": "hydro_fp64_probe (2048 x 256 threads, 8 FMA chains, 4096 iterations); "
                      "1 GiB device copy from an evicted buffer, read + written bytes; best of 3"}


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
    return table, {1: "face", 2: "column", 3: "persistent", 4: "tiled", 5: "one launch"}.get(conc, "table")


def bucket_of(n: int) -> int:
    b = 0
    while (2 << b) <= n and b < 15:
        b += 1
    return b


def timed_steps(torch, hy, w, args, s):
    """--warmup untimed device-dt steps, then two passes of exactly --steps
    steps from the same initial state on stream s: eager launches with HIP
    events around every stage launch (kernel-only time), and the whole job --
    the signal-speed pre-pass for dt0, then the steps replayed from one HIP
    graph -- between device synchronisations (end-to-end time).  Returns
    (end-to-end seconds, event milliseconds, stage launches, grid)."""
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
    hy.check(s)   # deferred non-physical-state check
    hy.graph_capture(g, w.cfl, dt_dev, args.steps)   # records the steps, runs nothing
    reset()
    hy.dt(g, w.cfl, dt_dev)
    hy.graph_launch(s)                                # one untimed replay
    reset()
    if hy.learned:
        hy.mlp_stats()                                # count the timed replay only
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    hy.dt(g, w.cfl, dt_dev)
    hy.graph_launch(s)
    s.synchronize()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    hy.check(s)
    return el, kms, launches, g, float(dt_dev.item())


def time_prepass(torch, hy, g, s, reps: int = 3) -> float:
    """Seconds of one inference pre-pass over every block of g (one launch,
    HIP events on the grid's stream; the first of reps + 1 untimed)."""
    hy.mlp_values(g, into_handle=True)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(reps):
        hy.mlp_values(g, into_handle=True)
    e1.record(s)
    e1.synchronize()
    return e0.elapsed_time(e1) / 1e3 / reps


def train_network(torch, args):
    from paper_2107_10987_amd import learned
    t0 = time.perf_counter()
    params, hist, meta = learned.train_default(torch, n_pairs=args.train_pairs, epochs=args.train_epochs)
    info = {"pairs": args.train_pairs, "epochs": args.train_epochs, "seconds": time.perf_counter() - t0,
            "final_train_loss": hist[-1]["train_loss"], "val_loss": hist[-1]["val_loss"], **meta}
    return params, info


# ---------------------------------------------------------------------------
# legs
# ---------------------------------------------------------------------------

def single_launch_leg(torch, args, w, name, params=None, schedule=None, centre_only=False,
                      flops=FLOPS_PER_CELL_UPDATE, traffic_name=None):
    """One workload with every leaf in one launch per stage, timed by
    timed_steps; plain PPM, or the learned reconstruction when params is
    given.  Returns the leg's dict (value, kernel-only rate, rooflines)."""
    from paper_2107_10987_amd.hydro import Hydro
    sched = schedule or args.schedule
    hy = Hydro(max_leaves=w.n, schedule=sched, learned=params is not None, centre_only=centre_only,
               leaf_edge=w.tree.leaf_edge)
    try:
        s = torch.cuda.Stream()
        table = None
        if params is not None:
            hy.mlp_load(params)
        if sched == "auto":
            gt = hy.grid(w.tree, torch.tensor(w.U, device="cuda"), w.omega, w.gamma, stream=s)
            table, _ = autotuned(hy, gt)
            del gt
            used = table[bucket_of(w.n * (w.tree.leaf_edge // 8) ** 3)]
        else:
            used = sched
        el, kms, launches, g, dt_after = timed_steps(torch, hy, w, args, s)
        avg = kms / 1e3 / max(launches, 1)
        kernel = KERNEL_OF[used]
        tname = traffic_name or name
        traffic = measured_traffic(tname, kernel)
        out = {"workload": w.name, "value": w.cells * 2 * args.steps / el, "unit": "cell-updates/s",
               "ms_per_step": el / args.steps * 1e3, "schedule": used, "autotune_table": table,
               "kernel": {"name": kernel, "avg_launch_us": avg * 1e6, "launches": launches,
                          "kernel_cell_updates_per_s": w.cells / avg},
               "roofline": fp64_roofline(kernel, w.cells, avg, traffic, flops),
               "hbm": hbm_figures(w.cells, avg, traffic), "dt_after": dt_after}
        if params is not None:
            # the learned stage is bound by its reads of the learned values
            out["roofline_fp64"] = out["roofline"]
            out["roofline"] = hbm_roofline(kernel, BYTES_PER_CELL_UPDATE * w.cells + learned_table_bytes(g),
                                           avg, traffic)
            cells, fb = hy.mlp_stats()
            out["fallback_fraction"] = fb / max(cells, 1)
            tp = time_prepass(torch, hy, g, s)
            blocks = w.n * (w.tree.leaf_edge // 8) ** 3
            ptraffic = measured_traffic(tname, "mlp_infer_kernel")
            out["prepass"] = {"seconds": tp, "us_per_block": tp / blocks * 1e6,
                              "roofline": mfma_roofline(prepass_cells(g), tp, ptraffic),
                              "hbm_bytes_per_cell_update": (None if ptraffic is None else ptraffic / w.cells)}
        out["U"] = g.U.cpu().numpy()
        return out
    finally:
        hy.close()


def binary_legs(torch, args, params):
    """Headline: the binary star with plain PPM; then the same with the
    learned reconstruction (FP64 check, plain-PPM fallback)."""
    from paper_2107_10987_amd.workloads import binary_star
    t0 = time.perf_counter()
    w = binary_star()
    build_s = time.perf_counter() - t0
    w.name = (f"binary-32768: two n=1.5 polytropes (mass ratio 0.5, separation 0.5) on a 4-level octree of "
              f"{w.n} leaves of 8^3 cells (16,777,216 cells), co-rotating Omega {w.omega:.4f}, one launch "
              f"per stage over all leaves, SSP-RK2 steps with the device time step in one HIP graph")
    plain = single_launch_leg(torch, args, w, "binary-plain")
    plain["host_build_seconds"] = build_s
    learned = None
    if params is not None:
        learned = single_launch_leg(torch, args, w, "binary-learned", params=params)
        d = np.abs(learned["U"] - plain["U"])
        learned["l1_rel_dev_vs_plain"] = float(d.sum() / np.abs(plain["U"]).sum())
        learned["linf_rel_dev_vs_plain"] = float(d.max() / np.abs(plain["U"]).max())
        learned["gain_vs_plain"] = learned["value"] / plain["value"]
    return w, plain, learned


def polytrope_legs(torch, args, params):
    """The 4096-leaf rotating polytrope on a 3-level octree, launched as
    seeded uneven batches that run concurrently, with autotuned schedules;
    plain PPM and, with params, the learned reconstruction.  `value`: the
    whole job of --steps device-dt steps replayed from one HIP graph (best of
    two after one untimed), as in the binary legs; `ms_per_step_host_call`:
    one step per host call at the plain path's CFL time step (median of ten
    after one untimed), whose end states give the learned path's deviation
    from the plain one.  The stage roofline takes half the step (two stages,
    every launch of a stage); the pre-pass is timed alone."""
    from paper_2107_10987_amd.hydro import Hydro
    from paper_2107_10987_amd.workloads import rotating_polytrope, uneven_batches

    w = rotating_polytrope()
    off = uneven_batches(w.n)
    U0 = torch.tensor(w.U, device="cuda")
    out, results, table = {}, {}, None
    legs = (("plain", False), ("learned", True)) if params is not None else (("plain", False),)
    dt = None
    for name, on in legs:
        hy = Hydro(max_leaves=w.n, schedule="auto", learned=on)
        try:
            g = hy.grid(w.tree, U0.clone(), w.omega, w.gamma, launch_off=off)
            if on:
                hy.mlp_load(params)
            t_, conc = autotuned(hy, g)
            table = t_ if table is None else table
            if dt is None:   # both paths step with the plain path's CFL time step
                dt = float(w.cfl * np.min(w.tree.dx / hy.signal_speed(g).cpu().numpy()))
            if on:
                hy.mlp_stats()
            times = []
            for r in range(11):
                g.U.copy_(U0)
                torch.cuda.synchronize()
                t1 = time.perf_counter()
                hy.step(g, dt)
                torch.cuda.synchronize()
                times.append(time.perf_counter() - t1)
            host_med = float(np.median(times[1:]))
            results[name] = g.U.cpu().numpy()
            # the whole job as in the binary legs: the same uneven launches,
            # --steps device-dt steps replayed from one HIP graph after the
            # signal-speed pre-pass for dt0, between device synchronisations
            gs = torch.cuda.Stream()
            g2 = hy.grid(w.tree, U0.clone(), w.omega, w.gamma, launch_off=off, stream=gs)
            dt_dev = torch.zeros(1, dtype=torch.float64, device="cuda")
            hy.graph_capture(g2, w.cfl, dt_dev, args.steps)
            els = []
            for r in range(3):
                with torch.cuda.stream(gs):
                    g2.U.copy_(U0)
                gs.synchronize()
                torch.cuda.synchronize()
                t1 = time.perf_counter()
                hy.dt(g2, w.cfl, dt_dev)
                hy.graph_launch(gs)
                gs.synchronize()
                torch.cuda.synchronize()
                els.append(time.perf_counter() - t1)
            hy.check(gs)
            med = float(np.min(els[1:])) / args.steps
            tname = f"polytrope-{name}"
            merged = conc == "one launch"
            if merged:   # the tuner replaced the partition by one launch over the mesh
                kernel = KERNEL_OF[t_[bucket_of(w.n)]]
                label = kernel + " (whole stage, one launch over the six batches)"
            else:
                kernel = KERNEL_OF["column"] if conc in ("column", "table") else KERNEL_OF[conc]
                label = kernel + " (whole stage, concurrent launches)"
            traffic = measured_traffic(tname, kernel)
            out[name] = {"value": w.cells * 2 / med, "unit": "cell-updates/s", "ms_per_step": med * 1e3,
                         "ms_per_step_host_call": host_med * 1e3,
                         "launches_per_stage": 1 if merged else len(off) - 1, "batches": len(off) - 1,
                         "autotune_concurrent": conc,
                         "roofline": fp64_roofline(label, w.cells, med / 2, traffic),
                         "hbm": hbm_figures(w.cells, med / 2, traffic)}
            if on:
                out[name]["roofline_fp64"] = out[name]["roofline"]
                out[name]["roofline"] = hbm_roofline(
                    label,
                    BYTES_PER_CELL_UPDATE * w.cells + learned_table_bytes(g), med / 2, traffic)
                cells, fb = hy.mlp_stats()
                out[name]["fallback_fraction"] = fb / max(cells, 1)
                g.U.copy_(U0)
                tp = time_prepass(torch, hy, g, torch.cuda.current_stream())
                ptraffic = measured_traffic(tname, "mlp_infer_kernel")
                out[name]["prepass"] = {"seconds": tp, "us_per_block": tp / w.n * 1e6,
                                        "roofline": mfma_roofline(prepass_cells(g), tp, ptraffic),
                                        "hbm_bytes_per_cell_update": (None if ptraffic is None
                                                                      else ptraffic / w.cells)}
        finally:
            hy.close()
    if params is not None:
        d = np.abs(results["learned"] - results["plain"])
        out["learned"]["l1_rel_dev_vs_plain"] = float(d.sum() / np.abs(results["plain"]).sum())
        out["learned"]["linf_rel_dev_vs_plain"] = float(d.max() / np.abs(results["plain"]).max())
        out["learned"]["gain_vs_plain"] = out["learned"]["value"] / out["plain"]["value"]
    out["workload"] = ("polytrope-4096: rotating n=1.5 polytrope, 3-level octree of 4096 leaves, "
                       f"Omega 0.1, {len(off) - 1} seeded uneven batches launched concurrently, autotuned "
                       "schedules, SSP-RK2 steps with the device time step at CFL 0.4 in one HIP graph")
    out["autotune_table"] = table
    return out


def sedov_legs(torch, args):
    """The 64^3 Sedov blast as 512 leaves of 8^3 (the trajectory the GPU
    parity tests follow), the same blast as 64 leaves of 16^3, at the paper's
    problem size (256^3, 32,768 leaves) and with the paper's old face-centre
    scheme."""
    from paper_2107_10987_amd.workloads import sedov_uniform
    out = {}
    w = sedov_uniform(8)
    w.name = ("sedov-64^3: 512 leaves of 8^3 cells + 3 ghost layers, FP64, gamma 5/3, outflow, SSP-RK2 at "
              "CFL 0.4, plain PPM, one leaf per workgroup")
    r = single_launch_leg(torch, args, w, "sedov64", schedule="column")
    r.pop("U")
    out["sedov64"] = r
    w16 = sedov_uniform(4, leaf_edge=16)
    w16.name = "sedov-64^3 as 64 leaves of 16^3 cells (512 tiles of 8^3)"
    r = single_launch_leg(torch, args, w16, "sedov64-leaf16", schedule="column")
    r.pop("U")
    out["leaf16"] = r
    w256 = sedov_uniform(32)
    w256.name = ("sedov-256^3: the paper's Sedov problem size, 16,777,216 cells as 32,768 leaves of 8^3, "
                 "outflow, plain PPM, one launch per stage over all leaves")
    r = single_launch_leg(torch, args, w256, "sedov256", schedule="column")
    r.pop("U")
    # the paper's own figure for this problem (section V-A2: 286 ms per
    # three-stage step on 128 Summit nodes, 768 V100s, with 8^3 leaves);
    # another machine's whole-code number, quoted for scale only
    paper = 3 * 16777216 / 0.286
    r["paper_context"] = {"value": paper, "unit": "cell-updates/s", "hardware": "128 Summit nodes (768 V100)",
                          "ratio": r["value"] / paper}
    out["sedov256"] = r
    del w256
    wo = sedov_uniform(8)
    wo.name = "sedov-64^3 with the old scheme: one flux point per face (the face centre), weight 1"
    r = single_launch_leg(torch, args, wo, "sedov64-old", schedule="column", centre_only=True,
                          flops=FLOPS_PER_CELL_UPDATE_OLD)
    r.pop("U")
    out["old_scheme"] = r
    return out


# ---------------------------------------------------------------------------
# CPU oracle baselines
# ---------------------------------------------------------------------------

def _host():
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            model = next((ln.split(":", 1)[1].strip() for ln in f if ln.startswith("model name")), "")
    except OSError:
        pass
    return {"cpu_count": os.cpu_count(), "model": model}


def cpu_baselines(budget_s: float, w_binary=None):
    """The CPU oracle, as it stands, on the host cores:
    - headline (binary, 32768 leaves): stage 1 of a seeded 1/64 sample, 8
      Morton ranges of 64 leaves of the initial state, repeated for about
      budget_s seconds with all threads; per-stage rate, extrapolated (stage 2
      does the same arithmetic plus the combine); one thread on one range;
    - polytrope (4096 leaves): one full SSP-RK2 step over all leaves;
    - sedov-64^3 (512 leaves): whole steps from t = 0 for a few seconds."""
    import oracle
    from paper_2107_10987_amd.workloads import binary_star, rotating_polytrope, sedov_uniform
    threads = oracle.default_threads()
    out = {}
    w = w_binary or binary_star()
    o = oracle.Oracle(w.tree, w.gamma, w.omega, threads=threads)
    rng = np.random.default_rng(2107)
    starts = np.sort(rng.choice(w.n // 64, 8, replace=False)) * 64
    dt = 6.7e-7   # about the CFL step of the initial state; the cost does not depend on it
    reps, t0 = 0, time.perf_counter()
    while True:
        for s0 in starts:
            o.stage(1, dt, w.U, l0=int(s0), l1=int(s0) + 64)
        reps += 1
        if time.perf_counter() - t0 >= budget_s:
            break
    el = time.perf_counter() - t0
    o1 = oracle.Oracle(w.tree, w.gamma, w.omega, threads=1)
    t1 = time.perf_counter()
    o1.stage(1, dt, w.U, l0=int(starts[0]), l1=int(starts[0]) + 64)
    el1 = time.perf_counter() - t1
    out["binary"] = {"value": 512 * 512 * reps / el, "unit": "cell-updates/s", "cores": threads, "kind": "oracle",
                     "sample": (f"stage 1 of a seeded 1/64 sample of the binary's 32768 leaves (8 Morton ranges "
                                f"of 64 leaves, initial state), {reps} repetitions, {threads} host threads, "
                                f"{el:.1f} s; extrapolated to the whole workload's per-stage rate"),
                     "single_thread": {"value": 64 * 512 / el1, "unit": "cell-updates/s",
                                       "sample": f"stage 1 of one 64-leaf range, 1 thread, {el1:.2f} s"}}
    wp = rotating_polytrope()
    op = oracle.Oracle(wp.tree, wp.gamma, wp.omega, threads=threads)
    dtp = op.dt(wp.U)
    t2 = time.perf_counter()
    op.step(dtp, wp.U)
    el2 = time.perf_counter() - t2
    out["polytrope"] = {"value": wp.cells * 2 / el2, "unit": "cell-updates/s", "cores": threads,
                        "kind": "oracle",
                        "sample": f"one full SSP-RK2 step of all 4096 leaves, {threads} threads, {el2:.1f} s"}
    ws = sedov_uniform(8)
    os_ = oracle.Oracle(ws.tree, ws.gamma, ws.omega, threads=threads)
    U = ws.U.copy()
    dts = os_.dt(U)
    steps, t3 = 0, time.perf_counter()
    while True:
        U, am = os_.step(dts, U)
        steps += 1
        dts = float(ws.cfl * np.min(ws.tree.dx / am))
        if time.perf_counter() - t3 >= min(5.0, budget_s):
            break
    el3 = time.perf_counter() - t3
    out["sedov64"] = {"value": ws.cells * 2 * steps / el3, "unit": "cell-updates/s", "cores": threads,
                      "kind": "oracle",
                      "sample": f"{steps} full SSP-RK2 steps of the 64^3 Sedov blast from t=0, {threads} threads, "
                                f"{el3:.1f} s"}
    head = dict(out["binary"])
    head["host"] = _host()
    head["configs"] = {"polytrope": out["polytrope"], "sedov64": out["sedov64"]}
    return head


# ---------------------------------------------------------------------------
# counter-run mode
# ---------------------------------------------------------------------------

def profile_mode(torch, args):
    """A few eager steps of one workload (single launch per stage), plus the
    pre-pass alone for the learned ones: the dispatches a counter run
    reduces.  Prints what ran."""
    from paper_2107_10987_amd.hydro import Hydro
    from paper_2107_10987_amd.workloads import binary_star, rotating_polytrope, sedov_uniform
    name = args.profile
    params = None
    if name.endswith("learned"):
        from paper_2107_10987_amd import learned
        params, _, _ = learned.train_default(torch, n_pairs=2 ** 18, epochs=2, sedov_steps=6)
    # one launch per stage over all leaves, so that a dispatch is a whole stage
    if name.startswith("binary"):
        w = binary_star()
    elif name.startswith("polytrope"):
        w = rotating_polytrope()
    elif name == "sedov256":
        w = sedov_uniform(32)
    elif name == "sedov64-leaf16":
        w = sedov_uniform(4, leaf_edge=16)
    else:
        w = sedov_uniform(8)
    if args.copy_probe_mib > 0:
        copy_probe(torch, args.copy_probe_mib)
    # the learned stage runs with both schedules its autotuner chooses from
    # for a whole-mesh launch, so that either one's dispatches are counted
    schedules = ("column", "persistent") if params is not None else ("column",)
    for sched in schedules:
        hy = Hydro(max_leaves=w.n, schedule=sched, learned=params is not None,
                   centre_only=name == "sedov64-old", leaf_edge=w.tree.leaf_edge)
        try:
            if params is not None:
                hy.mlp_load(params)
            s = torch.cuda.Stream()
            g = hy.grid(w.tree, torch.tensor(w.U, device="cuda"), w.omega, w.gamma, stream=s)
            dt_dev = torch.zeros(1, dtype=torch.float64, device="cuda")
            hy.dt(g, w.cfl, dt_dev)
            for _ in range(args.steps):
                hy.step_dev(g, w.cfl, dt_dev)
            if params is not None and sched == schedules[0]:
                hy.mlp_values(g, into_handle=True)
            s.synchronize()
            hy.check(s)
        finally:
            hy.close()
    print(json.dumps({"profile": name, "steps": args.steps, "leaves": w.n, "schedules": schedules}),
          flush=True)


# ---------------------------------------------------------------------------

def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the hydro path runs on one GPU; it is not sharded across GPUs)", file=sys.stderr)
        sys.exit(2)
    if args.reduce_trace:
        print(reduce_trace(args.reduce_trace))
        return
    if args.reduce_counters:
        if not args.profile:
            print("--reduce-counters needs --profile NAME", file=sys.stderr)
            sys.exit(2)
        base = (f"rocprofv3 --pmc {{c}} -d {{d}} --output-format csv -- python3 ./bench.py --profile "
                f"{args.profile} --steps {args.steps} --copy-probe-mib 1024")
        r = reduce_counters(args.profile, *args.reduce_counters,
                            base.format(c="FETCH_SIZE", d=args.reduce_counters[0]),
                            base.format(c="WRITE_SIZE", d=args.reduce_counters[1]))
        print(json.dumps({k: v["bytes_per_launch"] for k, v in r["kernels"].items()}))
        return
    import torch
    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    if args.profile:
        profile_mode(torch, args)
        return
    if args.copy_probe_mib > 0:
        copy_probe(torch, args.copy_probe_mib)

    params, info = (None, None)
    if not args.no_learned:
        params, info = train_network(torch, args)
    w, plain, learned = binary_legs(torch, args, params)
    plain.pop("U")
    if learned is not None:
        learned.pop("U")
    out = {
        "metric": METRIC,
        "value": plain["value"],
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": plain["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": w.name, "leaves": w.n, "cells": w.cells, "stages_per_step": 2, "path": "plain",
                   "schedule": plain["schedule"]},
        "kernel": plain["kernel"],
        "roofline": plain["roofline"],
        "hbm": plain["hbm"],
        "learned": learned,
    }
    if info is not None:
        out["training"] = info
    att = attainable(torch)
    out["attainable"] = att
    out["roofline"]["frac_of_attainable"] = out["roofline"]["achieved"] / att["fp64_tflops"]
    if not args.no_extra:
        out.update(sedov_legs(torch, args))
        out["batched"] = polytrope_legs(torch, args, params)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baselines(args.cpu_seconds, w)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
