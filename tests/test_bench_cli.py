"""CPU checks of the benchmark script's host paths (no GPU work):
  - more than one GPU is refused with a message, before anything touches a GPU;
  - the oracle leg of the scaling study prints one JSON line per case, with a
    whole fill up to the full-fill size and one timed sweep beyond it.
"""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def run(*args, timeout=300):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], cwd=ROOT, capture_output=True,
                          text=True, timeout=timeout)


def test_more_than_one_gpu_is_refused():
    r = run("--gpus", "2")
    assert r.returncode == 2
    assert "one GPU only" in r.stderr
    assert r.stdout == ""


def test_cpu_scaling_leg_prints_a_line_per_case():
    sys.path.insert(0, ROOT)
    import bench
    from contextlib import redirect_stdout
    from io import StringIO
    buf = StringIO()
    with redirect_stdout(buf):
        bench.cpu_baseline_scaling([16, 24], fractions=(0.5,), full_fill_max=16)
    rows = [json.loads(line) for line in buf.getvalue().splitlines()]
    assert [(r["L"], r["p_removed"]) for r in rows] == [(16, 0.5), (24, 0.5)]
    full, one = rows
    assert full["kind"] == "oracle" and full["cores"] == 1 and full["gap_sites"] == 128
    assert full["fill_s"] > 0 and full["sweeps"] == full["relax_sweeps"] + 101
    assert full["site_updates_per_s"] > 0
    assert one["fill_s"] is None and one["sweep_s"] > 0 and one["gap_sites"] == 288
