"""Batched and served windows give exactly the results of each window alone."""
import numpy as np
import pytest
import torch

from paper_1803_11449_amd import serving, traffic

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")


@pytest.fixture(scope="module")
def pools():
    print("serving pools: 2 x 16M pairs", flush=True)
    return [serving.pair_pool(16_000_000, s, traffic.config_seed(5, i), DEV)
            for i, s in enumerate((0.9, 1.2))]


def same(a, b):
    assert a.rid == b.rid
    assert np.array_equal(a.records["ip"], b.records["ip"])
    assert np.array_equal(a.records["sz"], b.records["sz"])
    assert np.array_equal(a.records["est"], b.records["est"])


def test_continuous_server_results_equal_alone(pools):
    # a burst: 40 windows of 12 links within 20 ms, so batches form, links repeat
    reqs = serving.poisson_windows(pools, n_links=12, rate_pps=4e10, duration_s=0.02,
                                   lo=100_000, hi=3_000_000, seed=3, theta=(512.0, 1024.0))
    assert len(reqs) >= 20
    alone = serving.serve_alone(reqs)
    with serving.ContinuousServer(budget_bytes=8 << 30, max_batch=16) as srv:
        served = srv.serve(reqs)
    assert max(r.batch for r in served) > 1
    for a, b in zip(served, alone):
        same(a, b)
    with serving.PlainServer(budget_bytes=8 << 30) as srv:
        plain = srv.serve(reqs)
    for a, b in zip(plain, alone):
        same(a, b)


def test_budget_forces_eviction_and_still_matches(pools):
    reqs = serving.poisson_windows(pools, n_links=30, rate_pps=4e10, duration_s=0.01,
                                   lo=1_000_000, hi=6_000_000, seed=9)
    alone = serving.serve_alone(reqs)
    # room for about four resident k=14/15 sketches only
    with serving.ContinuousServer(budget_bytes=80 << 20, max_batch=8) as srv:
        served = srv.serve(reqs)
        assert srv.links.used <= 80 << 20
    for a, b in zip(served, alone):
        same(a, b)
