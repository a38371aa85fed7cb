"""CPU checks of the benchmark script's host paths (no GPU work):
  - more than one GPU is refused with a message, before anything touches a GPU;
  - the help lists the extra legs and the sweep shapes;
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


def test_cpu_scaling_gap_fraction_sweep_and_join(tmp_path):
    """The gap-fraction cases come after the size grid, without repeats, and
    the join gives the oracle's fill time (measured, or its sweep time times
    the GPU fill's sweep count) and the speed-ups."""
    sys.path.insert(0, ROOT)
    import bench
    from contextlib import redirect_stdout
    from io import StringIO
    buf = StringIO()
    with redirect_stdout(buf):
        bench.cpu_baseline_scaling([16], fractions=(0.5,), full_fill_max=16, extra=((24, 0.2), (16, 0.5), (24, 0.8)))
    rows = [json.loads(line) for line in buf.getvalue().splitlines()]
    assert [(r["L"], r["p_removed"]) for r in rows] == [(16, 0.5), (24, 0.2), (24, 0.8)]
    cpu = tmp_path / "cpu.jsonl"
    cpu.write_text(buf.getvalue())
    gpu = tmp_path / "gpu.jsonl"
    g = [{"L": 16, "p_removed": 0.5, "relax_sweeps": 30, "K": 100, "time_to_fill_s": 0.01, "site_updates_per_s": 1e9},
         {"L": 24, "p_removed": 0.8, "relax_sweeps": 40, "K": 100, "time_to_fill_s": 0.02, "site_updates_per_s": 2e9},
         {"L": 32, "p_removed": 0.5, "relax_sweeps": 40, "K": 100, "time_to_fill_s": 0.02, "site_updates_per_s": 2e9}]
    gpu.write_text("\n".join(json.dumps(r) for r in g) + "\n| table |\n")
    out = bench.combine_scaling(str(gpu), str(cpu))["rows"]
    assert len(out) == 3
    a, b, c = out
    assert a["oracle_time_to_fill_s"] == rows[0]["fill_s"]
    assert a["speedup_time_to_fill"] == rows[0]["fill_s"] / 0.01
    assert b["oracle_time_to_fill_s"] == rows[2]["sweep_s"] * 141
    assert b["speedup_site_updates"] == 2e9 / rows[2]["site_updates_per_s"]
    assert "oracle_time_to_fill_s" not in c


def test_cpu_baseline_all_cores_runs_independent_chains():
    """The all-cores oracle leg runs one oracle process per chain and adds
    their site-updates over the wall time."""
    sys.path.insert(0, ROOT)
    import bench
    import synth
    im = synth.workload_table2(24, 0.5, 0)
    out = bench.cpu_baseline_all_cores(im, 0.09, 2, 5, 2)
    assert out["cores"] == 2 and out["kind"] == "oracle" and out["value"] > 0
    assert "2 independent chains" in out["sample"]


def test_help_lists_the_extra_legs_and_shapes():
    """The benchmark's extra legs (cloud mask, small fill) can be switched off
    and the sweep shapes named, the persistent ones included."""
    r = run("--help", timeout=120)
    assert r.returncode == 0
    for opt in ("--cloud-steps", "--small-steps", "--tile", "--cnn-only", "--copy-probe"):
        assert opt in r.stdout, opt
    assert "32p" in r.stdout and "48f" in r.stdout
