"""Restore phase timings (SKETCH_OPT_TIMING): recorded only when asked for,
positive, and with the work counts the restore's own diagnostics imply."""
import numpy as np
import pytest
import torch

import oracle
from paper_1803_11449_amd import ddhf
from test_gpu_parity import make_sketch, planted, rand_pairs, to_dev

pytestmark = pytest.mark.gpu


def test_restore_timings():
    p = oracle.Params(1024, 16, 5, 6)
    rng = np.random.default_rng(101)
    hosts = rng.choice(2**32, size=10, replace=False).astype(np.uint32)
    pairs = np.concatenate([rand_pairs(rng, 2_000_000, 50_000)] + planted(rng, hosts, 3000))
    with make_sketch(p, 2) as sk:
        with pytest.raises(ddhf.SketchError):
            ddhf.sketch_timings(sk.handle)          # nothing timed yet
        sk.set_option(ddhf.SKETCH_OPT_TIMING, 1)
        sk.reset()                 # a window's first binned update keeps the zero counts
        sk.update(to_dev(pairs))
        recs, info = sk.restore(700.0)
        t = ddhf.sketch_timings(sk.handle)
        for name in ("hot_scan_ms", "rows_ms", "join_ms", "estimate_ms", "sort_publish_ms"):
            assert 0 < t[name] < 1000, (name, t[name])
        n_le = p.r << p.k
        # a fresh binned update kept the zero counts: 4 bytes per LE
        assert t["hot_scan_bytes"] == 4 * n_le
        he = info["he_count"]
        assert t["estimate_bytes"] == info["n_candidates"] * p.r * p.g // 8
        assert len(recs) >= len(hosts)
        # each candidate search reports its own work
        for path in (1, 2):
            sk.set_option(ddhf.SKETCH_OPT_CANDIDATES, path)
            again, info = sk.restore(700.0)
            assert np.array_equal(again, recs)
            t = ddhf.sketch_timings(sk.handle)
            parts = info["n_partials"]
            assert t["search"] == path
            if path == 1:
                assert t["join_probes"] == he[0] * he[1] + sum(parts[2:p.r - 1])
                assert t["join_outputs"] == sum(parts[2:p.r - 1]) + info["n_candidates"]
                assert t["lattice_points"] == 0
            else:
                assert t["join_probes"] == 0 and not any(parts)
                assert t["join_outputs"] == info["n_candidates"]
                assert t["lattice_points"] == he[0] << (32 - p.k)
        sk.set_option(ddhf.SKETCH_OPT_CANDIDATES, 0)
        # after a direct update the hot scan reads the sketch itself
        sk.set_option(ddhf.SKETCH_OPT_UPDATE_PATH, 1)
        sk.update(to_dev(pairs[:1000]))
        sk.restore(700.0)
        assert ddhf.sketch_timings(sk.handle)["hot_scan_bytes"] == n_le * p.g // 8
