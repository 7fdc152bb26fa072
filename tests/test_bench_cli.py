"""The benchmark's command line on the host: it measures one GPU, and asking
for several exits with status 2 and says so before touching a device."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_refuses_several_gpus():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


def _bench():
    import importlib.util
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    m = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(m)
    return m


def test_learned_table_bytes_counts_each_needed_value_once():
    """Two blocks: every interior cell's 13 lines x 7 fields (8 B each), and
    for each ghost row no block owns (alias < 0) the 9 lines crossing its face
    at one end (4 B); shared rows count nothing extra; no alias table means
    every ghost row is the block's own."""
    import types
    import torch
    b = _bench()
    alias = torch.full((2, 384), -1, dtype=torch.int32)
    alias[0, :100] = 5
    g = types.SimpleNamespace(gmap=torch.zeros(2 * 2232, dtype=torch.int32), alias=alias)
    interior = 2 * 512 * 13 * 7 * 8
    assert b.learned_table_bytes(g) == interior + (2 * 384 - 100) * 9 * 7 * 4
    g.alias = None
    assert b.learned_table_bytes(g) == interior + 2 * 384 * 9 * 7 * 4


def test_hbm_roofline_fields():
    b = _bench()
    r = b.hbm_roofline("k", 8e9, 2e-3, traffic=16e9)
    assert r["bound"] == "hbm" and r["unit"] == "GB/s"
    assert abs(r["achieved"] - 4000.0) < 1e-9 and abs(r["frac"] - 0.5) < 1e-12
    assert abs(r["counter_frac"] - 1.0) < 1e-12
    assert b.hbm_roofline("k", 8e9, 2e-3)["counter_frac"] is None
