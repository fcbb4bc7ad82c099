"""sketch_restore_noalloc (the restore on the library's fixed per-GPU work
array) against sketch_restore, through the C ABI.

Bar: the same records (address, SZ bit for bit; estimates within 1e-6
relative, +inf == +inf) and the same info. Two calls in a row, the second
on a smaller window, so the second runs on what the first left in the
shared array; then a list longer than the pinned host buffer, and the
limits.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_1803_11449_amd import ddhf, traffic as T

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")
RTOL = 1e-6


def say(msg):
    print(msg, flush=True)


def assert_same(recs, ref):
    assert np.array_equal(recs["ip"], ref["ip"]), (len(recs), len(ref))
    assert np.array_equal(recs["sz"], ref["sz"])
    a, b = recs["est"], ref["est"]
    assert np.array_equal(np.isinf(a), np.isinf(b))
    fin = ~np.isinf(b)
    np.testing.assert_allclose(a[fin], b[fin], rtol=RTOL, atol=0)


def window_sketch(spec, seed, p):
    w = T.generate(spec, seed, device=DEV)
    sk = ddhf.Sketch(p.g, p.k, p.r, p.alpha, p.seed, device=0)
    sk.update(w.pairs)
    torch.cuda.synchronize()
    return sk, w


def test_noalloc_equals_restore_twice_second_smaller():
    p = oracle.Params()
    say("no-alloc restore: 1M-pair window, then a 300k-pair window")
    big = T.spec_single_window_1m()
    small = T.WindowSpec(n_pairs=300_000, n_sources=30_000, zipf_s=1.1,
                         planted_card=[1500, 2500, 4000], name="small")
    sk1, w1 = window_sketch(big, T.config_seed(1), p)
    sk2, w2 = window_sketch(small, T.config_seed(99), p)
    with sk1, sk2:
        got1, info1 = sk1.restore_noalloc(1024.0)
        got2, info2 = sk2.restore_noalloc(1024.0)
        ref1, rinfo1 = sk1.restore(1024.0)
        ref2, rinfo2 = sk2.restore(1024.0)
        words1 = sk1.download()
    assert len(got1) > len(got2) > 0
    assert_same(got1, ref1)
    assert_same(got2, ref2)
    for a, b in ((info1, rinfo1), (info2, rinfo2)):
        assert a["he_count"] == b["he_count"] and a["n_candidates"] == b["n_candidates"]
        assert a["szmax"] == b["szmax"] and a["zhot"] == b["zhot"]
    # and the first against the oracle's restore of the same sketch
    ip, sz, c, _ = oracle.restore(p, words1, 1024.0)
    assert np.array_equal(got1["ip"], ip) and np.array_equal(got1["sz"], sz)


def test_noalloc_list_longer_than_the_pinned_buffer():
    """More records than the handle's pinned copy holds (4096): the call
    copies them through it a buffer's worth at a time."""
    p = oracle.Params(1024, 18, 5, 5)
    rng = np.random.default_rng(37)
    hosts = rng.choice(2**32, size=6000, replace=False).astype(np.uint32)
    src = np.repeat(hosts, 1300)
    dst = rng.integers(0, 2**32, size=src.size, dtype=np.uint64).astype(np.uint32)
    pairs = np.stack([src, dst], 1)[rng.permutation(src.size)]
    say(f"no-alloc restore: {len(hosts)} planted hosts, k=18")
    d = torch.from_numpy(np.ascontiguousarray(pairs).view(np.int32)).to(DEV)
    with ddhf.Sketch(p.g, p.k, p.r, p.alpha, p.seed, device=0) as sk:
        sk.update(d)
        got, _ = sk.restore_noalloc(1024.0)
        ref, _ = sk.restore(1024.0)
        got_again, _ = sk.restore_noalloc(1024.0)
    assert len(ref) > 4096
    assert_same(got, ref)
    assert_same(got_again, ref)


def test_noalloc_capacity_and_bad_arguments():
    p = oracle.Params()
    sk, _ = window_sketch(T.spec_single_window_1m(), T.config_seed(1), p)
    with sk:
        ref, _ = sk.restore(1024.0)
        # cap too small: CAPACITY with the count needed
        with pytest.raises(ddhf.SketchError) as e:
            ddhf.sketch_restore_noalloc(sk.handle, 1024.0, 1, 0)
        assert e.value.code == ddhf.SKETCH_E_CAPACITY and e.value.n_needed == len(ref)
        with pytest.raises(ddhf.SketchError) as e:
            ddhf.sketch_restore_noalloc(sk.handle, -1.0, 16, 0)
        assert e.value.code == ddhf.SKETCH_E_INVAL
        # the join forced, on the lattice-free path: still the same list
        sk.set_option(ddhf.SKETCH_OPT_CANDIDATES, 1)
        got, _ = sk.restore_noalloc(1024.0)
    assert_same(got, ref)


def test_noalloc_join_beyond_the_array():
    """A crafted sketch with about a thousand hot LEs per row: the join's
    partial addresses (millions) outgrow the fixed array. Forced to the
    join, the call fails with CAPACITY; left to choose, it takes the
    lattice search and gives sketch_restore's list."""
    p = oracle.Params()
    rng = np.random.default_rng(43)
    words = np.zeros(p.words(), dtype=np.uint32).reshape(p.r, 1 << p.k, p.g // 32)
    words[rng.random((p.r, 1 << p.k)) < 0.06] = 0xFFFFFFFF
    with ddhf.Sketch(p.g, p.k, p.r, p.alpha, p.seed, device=0) as sk:
        sk.upload(words.reshape(-1))
        ref, _ = sk.restore(1024.0)
        got, _ = sk.restore_noalloc(1024.0)
        assert_same(got, ref)
        sk.set_option(ddhf.SKETCH_OPT_CANDIDATES, 1)
        with pytest.raises(ddhf.SketchError) as e:
            sk.restore_noalloc(1024.0)
        assert e.value.code == ddhf.SKETCH_E_CAPACITY
        assert "partial addresses" in str(e.value)
        again, _ = sk.restore(1024.0)           # the growing restore still serves it
    assert_same(again, ref)
