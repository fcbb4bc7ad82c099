"""Host-side parts of bench.py that run without a GPU."""
import os
import subprocess
import sys

import torch

from conftest import ROOT

sys.path.insert(0, ROOT)
import bench  # noqa: E402
from paper_1803_11449_amd import traffic  # noqa: E402


def test_cpu_baseline_leg_reports_the_oracle():
    w = traffic.generate(traffic.spec_single_window_1m(), traffic.config_seed(1), device="cpu")
    cb = bench.cpu_baseline_leg(w.pairs, (1024, 14, 5, 6), 1024.0, 20_000, 2)
    assert cb["kind"] == "oracle" and cb["unit"] == "Mpps"
    assert cb["value"] > 0 and cb["cores"] == 2
    assert "20000 pairs" in cb["sample"]
    legs = cb["legs"]
    assert legs["update_1thread"]["threads"] == 1
    assert legs["update_omp"]["threads"] == 2 and legs["update_omp"]["same_sketch_as_1thread"]
    assert legs["restore_2to32_scan"]["threads"] == 2


def test_restore_roofline_arithmetic():
    t = {"hot_scan_ms": 0.01, "rows_ms": 0.02, "join_ms": 0.1, "estimate_ms": 0.01,
         "sort_publish_ms": 0.01, "hot_scan_bytes": 8e7, "join_probes": 1e6,
         "join_outputs": 2e6, "estimate_bytes": 6.4e6, "search": 1, "lattice_points": 0}
    rr = bench.restore_roofline([t, t, t])
    assert rr["hot_scan"]["achieved"] == 8000.0 and rr["hot_scan"]["frac"] == 1.0
    ops = bench.JOIN_LDS_OPS_PER_OUTPUT * 2e6 + bench.JOIN_LDS_OPS_PER_PROBE * 1e6
    cs = rr["candidate_search"]
    assert cs["kind"] == "join" and cs["bound"] == "lds"
    assert abs(cs["achieved"] - ops / 1e-4 / 1e12) < 1e-3
    assert rr["estimate"]["achieved"] == 640.0
    # the lattice search: integer operations per address walked vs the ALU peak
    t2 = dict(t, search=2, join_probes=0, join_outputs=5000, lattice_points=1e8)
    cs = bench.restore_roofline([t2])["candidate_search"]
    assert cs["kind"] == "lattice" and cs["bound"] == "alu"
    assert bench.VALU_LANE_OPS_PEAK == 256 * 64 * 2.4e9
    assert abs(cs["achieved"] - bench.LATTICE_OPS_PER_POINT * 1e8 / 1e-4 / 1e12) < 1e-3
    assert abs(cs["frac"] - bench.LATTICE_OPS_PER_POINT * 1e12 / bench.VALU_LANE_OPS_PEAK) < 1e-5


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in (r.stdout + r.stderr)


def test_workload_choices_are_listed():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--help"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 0
    for w in ("large_window_100m", "batched_64_links", "serving_256_links"):
        assert w in r.stdout


def test_workload_line_has_the_contract_fields(capsys):
    """The --workload modes print one JSON line through bench._line."""
    import json
    bench._line(1234.5678, 5, 1, 52.61, {"workload": "batched_64_links"},
                {"plan_update_launches": 18})
    line = json.loads(capsys.readouterr().out.strip())
    for key in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step",
                "higher_is_better", "scaling", "vs_baseline", "dtype", "data", "config"):
        assert key in line, key
    assert line["value"] == 1234.568 and line["config"]["workload"] == "batched_64_links"
    assert line["plan_update_launches"] == 18
