"""Served windows against the CPU oracle.

Every window a server reports on is compared with the oracle's restore of
that window's own sketch (Alg. 1 then Alg. 2): addresses and SZ bit for bit,
estimates within 1e-6 relative. The same holds for the window alone on a
fresh GPU sketch, so each result is the same alone and in the mix.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_1803_11449_amd import serving, traffic
from test_gpu_parity import assert_spl_equal

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")


@pytest.fixture(scope="module")
def pools():
    print("serving pools: 2 x 16M pairs", flush=True)
    return [serving.pair_pool(16_000_000, s, traffic.config_seed(5, i), DEV)
            for i, s in enumerate((0.9, 1.2))]


def oracle_results(reqs) -> dict:
    """rid -> (ip, sz, est) of the oracle on each window's own sketch."""
    out = {}
    for q in reqs:
        k, alpha = serving.sized_params(q.n_pairs)
        p = oracle.Params(1024, k, 5, alpha, traffic.HASH_SEED)
        pairs = q.pairs.cpu().numpy().view(np.uint32)
        ip, sz, c, _ = oracle.restore(p, oracle.build_sketch(p, pairs), q.theta, mode="brute")
        out[q.rid] = (ip, sz, c)
    return out


def check_against(resps, ref, what):
    assert len(resps) == len(ref), what
    for r in resps:
        assert r.status == 0, (what, r.rid, r.status)
        assert_spl_equal(r.records, *ref[r.rid])


def test_servers_equal_oracle_and_alone(pools):
    # a burst of windows from 12 links within 3 ms, so batches form and links
    # repeat; windows of 1M-6M pairs, so that a batch's work on the device
    # outlasts the host's turn between batches (with windows of 0.1M-3M the
    # device could finish a batch before the host enqueued the next)
    reqs = serving.poisson_windows(pools, n_links=12, rate_pps=4e10, duration_s=0.003,
                                   lo=1_000_000, hi=6_000_000, seed=3, theta=(512.0, 1024.0))
    assert len(reqs) >= 20
    print(f"serving: {len(reqs)} windows, oracle restores", flush=True)
    ref = oracle_results(reqs)
    check_against(serving.serve_alone(reqs), ref, "alone")
    with serving.ContinuousServer(budget_bytes=8 << 30, max_batch=16, trace=True) as srv:
        served = srv.serve(reqs)
        overlapped = srv.overlaps()
        print(f"batches {len(srv.trace)}, overlapped {overlapped}", flush=True)
    assert max(r.batch for r in served) > 1
    check_against(served, ref, "continuous")
    # a later batch's update ran on the device while an earlier batch restored
    assert overlapped >= 1
    with serving.PlainServer(budget_bytes=8 << 30) as srv:
        check_against(srv.serve(reqs), ref, "plain")


def test_budget_forces_eviction_and_still_equals_oracle(pools):
    reqs = serving.poisson_windows(pools, n_links=30, rate_pps=4e10, duration_s=0.0015,
                                   lo=1_000_000, hi=6_000_000, seed=9)
    assert len(reqs) >= 8
    print(f"serving with evictions: {len(reqs)} windows", flush=True)
    ref = oracle_results(reqs)
    # room for about four resident k=14/15 sketches only
    with serving.ContinuousServer(budget_bytes=80 << 20, max_batch=8) as srv:
        served = srv.serve(reqs)
        assert srv.links.used <= 80 << 20
    check_against(served, ref, "continuous, evicting")
