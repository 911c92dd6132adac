"""Host-side logic of bench.py (no GPU): the byte model, the power-law fit,
the traffic-record lookup and the one-GPU restriction."""

import json
import os
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_algorithmic_bytes_match_the_closed_form():
    # 14 bytes per point-step on the N1-row grid: 117.39 MB at 2048 x 4096
    b = bench.algorithmic_bytes(2048, 4096)
    assert b["row"] + b["col"] == 117_391_360
    k1, k2 = 511, 1023
    assert b["row"] == 8 * 2048 * ((2 * k2 + 1) + (k2 + 1))
    assert b["col"] == 8 * (2048 * (k2 + 1) + 2 * (2 * k1 + 1) * (k2 + 1) + 2048 * (2 * k2 + 1))
    # the product grid moves 3/4 of the intermediates: 92.23 MB
    p = bench.algorithmic_bytes(2048, 4096, 1536)
    assert p["row"] + p["col"] == 92_233_728
    # a forced step also reads the forcing spectrum once
    f = bench.algorithmic_bytes(2048, 4096, 1536, forcing=True)
    assert f["col"] - p["col"] == 8 * (2 * k1 + 1) * (k2 + 1) and f["row"] == p["row"]


def test_power_law_fit_recovers_exponent_and_origin():
    ts = np.arange(1500.0, 2600.0, 5.0)
    v = 0.002 * (ts + 300.0) ** 0.75
    fit = bench.power_law_fit(ts, v, 1500.0)
    assert abs(fit["alpha"] - 0.75) < 1e-6 and abs(fit["t_star"] + 300.0) < 1e-6
    assert fit["rms_log_residual"] < 1e-9 and fit["window"] == [1500.0, 2595.0]
    # with t* pinned at 0 the exponent is the log-log slope
    fixed = bench.power_law_fit(ts, ts ** 1.5, 1500.0, t_star_lo=0.0, step=1500.0)
    assert fixed["t_star"] == 0.0 and abs(fixed["alpha"] - 1.5) < 1e-9
    # too few points, or none positive
    assert bench.power_law_fit(ts[:3], v[:3], 1500.0) is None
    assert bench.power_law_fit(ts, -v, 1500.0) is None


def test_traffic_lookup_needs_digest_and_variant(tmp_path, monkeypatch):
    (tmp_path / "profiles").mkdir()
    rec = {"kernel": "col_kernel", "workload": "w", "source_digest": bench.source_digest(),
           "variants": [{"points_per_thread": 16, "rows": 1536, "hbm_bytes_per_launch": 1.5e7},
                        {"points_per_thread": 16, "rows": 1536, "streaming": True, "hbm_bytes_per_launch": 1.6e7},
                        {"points_per_thread": 12, "rows": 1536, "streaming": 2, "hbm_bytes_per_launch": 1.7e7},
                        {"points_per_thread": 12, "rows": 2048, "streaming_codes": [1, 2], "hbm_bytes_per_launch": 1.8e7}]}
    (tmp_path / "profiles" / "col_kernel_w_traffic.json").write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "source_digest", lambda: rec["source_digest"])
    assert bench.measured_traffic("col", "w", 16, 1536) == 1.5e7
    assert bench.measured_traffic("col", "w", 16, 1536, streaming=True) == 1.6e7
    assert bench.measured_traffic("col", "w", 8, 1536, streaming=True) is None
    assert bench.measured_traffic("col", "w", 12, 1536, streaming=2) == 1.7e7  # W only non-temporal
    assert bench.measured_traffic("col", "w", 12, 1536, streaming=1) is None
    assert bench.measured_traffic("col", "w", 12, 2048, streaming=1) == 1.8e7  # one kernel serves codes 1 and 2
    assert bench.measured_traffic("col", "w", 12, 2048, streaming=2) == 1.8e7
    assert bench.measured_traffic("col", "w", 12, 2048, streaming=3) is None
    assert bench.measured_traffic("col", "w", 8, 1536) is None
    assert bench.measured_traffic("col", "w", 16, 2048) is None
    assert bench.measured_traffic("row", "w", 16, 1536) is None
    monkeypatch.setattr(bench, "source_digest", lambda: "another build")
    assert bench.measured_traffic("col", "w", 16, 1536) is None


def test_committed_traffic_records_are_well_formed():
    for kern in ("row", "col"):
        path = os.path.join(ROOT, "profiles", f"{kern}_kernel_flame2048x4096_traffic.json")
        rec = json.load(open(path))
        assert rec["variants"] and all(v["hbm_bytes_per_launch"] > 0 for v in rec["variants"])
        for v in rec["variants"]:
            alg = bench.algorithmic_bytes(2048, 4096, v["rows"])[kern]
            assert v["algorithmic_bytes_per_launch"] == alg
            assert 0.95 < v["hbm_bytes_per_launch"] / alg < 1.5


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_row_pass_flops_is_the_nominal_count():
    # per row: 5 L log2 L (inverse complex transform) + 3 L (|z|^2) + 2.5 L log2 L
    # (half of the forward complex transform of two real rows)
    assert bench.row_pass_flops(2, 16) == 2 * (5 * 16 * 4 + 3 * 16 + 2.5 * 16 * 4)
    assert bench.row_pass_flops(1536, 4096) == 1536 * 4096 * (7.5 * 12 + 3)
