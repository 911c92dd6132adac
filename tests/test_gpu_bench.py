"""bench.py end to end on the GPU with short legs: one JSON line with the
contract's fields, every optional leg present and none of them refused."""

import json
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_line_with_every_leg():
    args = [sys.executable, "-u", os.path.join(ROOT, "bench.py"), "--steps", "10", "--warmup", "2", "--no-cpu",
            "--forcing-steps", "8", "--heun-steps", "8", "--adjoint-steps", "4", "--ensemble-steps", "8",
            "--circle-steps", "8", "--no-circle-long-run", "--no-long-run"]
    print("bench case: every leg, short", flush=True)
    res = subprocess.run(args, capture_output=True, text=True, timeout=300, cwd=ROOT)
    assert res.returncode == 0, res.stderr[-2000:]
    lines = [l for l in res.stdout.splitlines() if l.startswith("{")]
    assert len(lines) == 1, res.stdout[-2000:]
    d = json.loads(lines[0])
    for key in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better",
                "scaling", "vs_baseline", "dtype", "data", "config", "roofline", "cpu_baseline"):
        assert key in d, key
    assert d["n_gpus"] == 1 and d["steps"] == 10 and d["warmup"] == 2 and d["value"] > 0
    assert d["config"]["workload"] == "flame2048x4096" and d["config"]["timed_region"]["steps"] == 10
    r = d["roofline"]
    assert r["bound"] == "hbm" and r["kernel"] == "col_kernel" and 0 < r["frac"] < 1
    assert d["roofline_row"]["bound"] == "alu" and 0 < d["roofline_row"]["frac"] < 1
    for leg in ("forced", "heun", "adjoint", "ensemble", "circles"):
        assert leg in d and "error" not in d[leg], (leg, d.get(leg))
    for mode in ("graph", "direct", "graph_persistent_config", "persistent", "persistent_graph"):
        assert d["ensemble"][mode]["ms_per_step"] > 0, mode
    assert d["copy_bandwidth"]["GB_s"] > 0 and d["copy_bandwidth"]["resident_GB_s"] > 0
