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
    cb = bench.cpu_baseline_leg(w.pairs, (1024, 14, 5, 6), 1024.0, 20_000)
    assert cb["kind"] == "oracle" and cb["unit"] == "Mpps"
    assert cb["value"] > 0 and cb["cores"] >= 1
    assert "20000 pairs" in cb["sample"]


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
