"""The accuracy study's host logic (CPU) and its ground truth (GPU).

FPR/FNR/TFR follow the paper's definition in Sec. 5: with N true super
points, N+ reported hosts that are not super points and N- super points
not reported, FPR = N+/N, FNR = N-/N, TFR = FPR + FNR. The paper's own
values (its figures and table) come from CAIDA traces that are not
available: the study's numbers are parity unpinned; only the definitions
and the exact ground truth are tested.
"""
import numpy as np
import pytest
import torch

from paper_1803_11449_amd import accuracy


def test_rates_definition():
    truth = [10, 20, 30, 40]
    r = accuracy.rates([20, 30, 99, 98, 97], truth)
    assert (r["N"], r["reported"], r["N_plus"], r["N_minus"]) == (4, 5, 3, 2)
    assert r["FPR"] == 3 / 4 and r["FNR"] == 2 / 4 and r["TFR"] == 5 / 4
    assert accuracy.rates(truth, truth)["TFR"] == 0.0
    assert accuracy.rates([], truth)["FNR"] == 1.0
    assert accuracy.rates([], [])["TFR"] == 0.0


def test_exact_out_degree_cpu():
    # src 1 -> {5, 6, 6, 7}: 3 distinct; src 2 -> {5}: 1; src 0xFFFFFFFF -> {0, 1}: 2
    p = np.array([[1, 5], [2, 5], [1, 6], [1, 6], [-1, 0], [1, 7], [-1, 1]], dtype=np.int32)
    src, deg = accuracy.exact_out_degree(torch.from_numpy(p))
    assert src.tolist() == [1, 2, 0xFFFFFFFF]
    assert deg.tolist() == [3, 1, 2]
    assert accuracy.true_super_points(src, deg, 2.0).tolist() == [1, 0xFFFFFFFF]


def test_exact_out_degree_matches_python_sets():
    rng = np.random.default_rng(5)
    src = rng.integers(0, 50, size=5000)
    dst = rng.integers(0, 300, size=5000)
    p = np.stack([src, dst], 1).astype(np.uint32).view(np.int32)
    s, d = accuracy.exact_out_degree(torch.from_numpy(p))
    ref = {}
    for a, b in zip(src, dst):
        ref.setdefault(int(a), set()).add(int(b))
    assert s.tolist() == sorted(ref)
    assert d.tolist() == [len(ref[a]) for a in sorted(ref)]


@pytest.mark.gpu
def test_planted_super_points_found_at_default_g():
    """On the 1M-pair window every planted host (2000 distinct dsts, about
    twice theta) is reported with the paper's default parameters, and the
    exact ground truth on the device equals the one on the host."""
    from paper_1803_11449_amd import traffic
    dev = torch.device("cuda:0")
    w = traffic.generate(traffic.spec_single_window_1m(), traffic.config_seed(1), device=dev)
    s_gpu, d_gpu = accuracy.exact_out_degree(w.pairs)
    s_cpu, d_cpu = accuracy.exact_out_degree(w.pairs.cpu())
    assert torch.equal(s_gpu.cpu(), s_cpu) and torch.equal(d_gpu.cpu(), d_cpu)
    truth = accuracy.true_super_points(s_gpu, d_gpu, 1024.0)
    assert set(w.planted_src.tolist()) <= set(truth.tolist())
    ips, info = accuracy.detect(w.pairs, 1024, 5, 14, 6, 1024.0)
    r = accuracy.rates(ips, truth)
    assert set(w.planted_src.tolist()) <= set(ips.tolist())
    assert r["FNR"] <= 0.1
