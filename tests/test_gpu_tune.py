"""The autotuner picks a valid launch setting, and a tuned sketch computes
exactly what an untuned one does (options never change a result)."""
import numpy as np
import pytest
import torch

import oracle
from paper_1803_11449_amd import ddhf, tune
from test_gpu_parity import planted, rand_pairs, say, to_dev

pytestmark = pytest.mark.gpu


def test_tuned_setting_is_valid_and_exact(tmp_path, monkeypatch):
    monkeypatch.setattr(tune, "CACHE", str(tmp_path / "tune.json"))
    p = oracle.Params()
    rng = np.random.default_rng(83)
    hosts = rng.choice(2**32, size=6, replace=False).astype(np.uint32)
    pairs = np.concatenate([rand_pairs(rng, 400_000, 12_000)] + planted(rng, hosts, 2500))
    t = to_dev(pairs)
    say("tuning a 415k-pair window")
    best = tune.tune(p.g, p.k, p.r, p.alpha, t, p.seed, trials=1)
    assert best["path"] in (1, 2) and best["ms"] > 0
    assert tune.tune(p.g, p.k, p.r, p.alpha, t, p.seed) == best       # from the cache
    ref = oracle.build_sketch(p, pairs)
    with ddhf.Sketch(p.g, p.k, p.r, p.alpha, p.seed, device=0) as sk:
        tune.apply(sk, best)
        sk.update(t)
        torch.cuda.synchronize()
        assert np.array_equal(sk.download(), ref)
    for opts in tune.candidates(torch.cuda.get_device_properties(0).multi_processor_count,
                                True)[::5]:
        with ddhf.Sketch(p.g, p.k, p.r, p.alpha, p.seed, device=0) as sk:
            tune.apply(sk, opts)
            sk.update(t)
            torch.cuda.synchronize()
            assert np.array_equal(sk.download(), ref), opts


def test_tuned_restore_is_valid_and_exact(tmp_path, monkeypatch):
    """The restore tuner's pick and every candidate it times give the
    oracle's list."""
    monkeypatch.setattr(tune, "CACHE", str(tmp_path / "tune.json"))
    p = oracle.Params()
    rng = np.random.default_rng(89)
    hosts = rng.choice(2**32, size=8, replace=False).astype(np.uint32)
    pairs = np.concatenate([rand_pairs(rng, 500_000, 20_000)] + planted(rng, hosts, 2500))
    theta = 700.0
    ref = oracle.build_sketch(p, pairs)
    ip, sz, c, _ = oracle.restore(p, ref, theta, mode="brute")
    say("tuning the restore of a 520k-pair window")
    with ddhf.Sketch(p.g, p.k, p.r, p.alpha, p.seed, device=0) as sk:
        sk.update(to_dev(pairs))
        best = tune.tune_restore(sk, theta, len(pairs), trials=1)
        assert best["cand"] in (1, 2) and best["ms"] > 0
        recs, _ = sk.restore(theta)
        assert np.array_equal(recs["ip"], ip) and np.array_equal(recs["sz"], sz)
        n_cu = torch.cuda.get_device_properties(0).multi_processor_count
        for opts in tune.restore_candidates(n_cu, p.k):
            tune.apply(sk, opts)
            recs, _ = sk.restore(theta)
            assert np.array_equal(recs["ip"], ip) and np.array_equal(recs["sz"], sz), opts
            np.testing.assert_allclose(recs["est"][np.isfinite(c)], c[np.isfinite(c)], rtol=1e-6)
