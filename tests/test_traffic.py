"""The seeded synthetic traffic generator (inputs only)."""
import numpy as np
import torch

import oracle
from paper_1803_11449_amd import traffic as T

M64 = (1 << 64) - 1


def splitmix_py(key, i):
    z = (key + (i + 1) * 0x9E3779B97F4A7C15) & M64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M64
    return z ^ (z >> 31)


def test_rng_is_splitmix64_stream_with_wrapping_int64():
    key = T.stream_key(123, 4)
    idx = torch.tensor([0, 1, 2, 1000, 2**40 + 7], dtype=torch.int64)
    got = [int(x) & M64 for x in T.rng64(key, idx)]
    assert got == [splitmix_py(key, int(i)) for i in idx]
    # the oracle's SplitMix64 (independent C code) agrees on stream 0
    assert got[:3] == [int(x) for x in oracle.splitmix64(key, 3)]


def test_feistel_is_a_bijection():
    x = torch.arange(1 << 16, dtype=torch.int64) * 65537 % (1 << 32)
    y = T.feistel32(x, T.stream_key(5, 1))
    assert y.unique().numel() == x.numel()
    assert int(y.min()) >= 0 and int(y.max()) < 2**32


def test_window_shape_planted_and_determinism():
    spec = T.WindowSpec(n_pairs=50_000, n_sources=2000, zipf_s=1.1,
                        planted_card=[1500, 1100], n_scanners=2,
                        scanner_len=3000, dup_frac=0.1)
    w1 = T.generate(spec, 77)
    w2 = T.generate(spec, 77)
    assert torch.equal(w1.pairs, w2.pairs)
    assert w1.pairs.shape == (50_000, 2) and w1.pairs.dtype == torch.int32
    pairs = w1.pairs.numpy().view(np.uint32)
    hosts, card = oracle.exact_cardinality(pairs)
    cmap = dict(zip(hosts.tolist(), card.tolist()))
    for s, c in zip(w1.planted_src, w1.planted_card):
        assert cmap[int(s)] == c
    for s in w1.scanner_src:
        assert cmap[int(s)] == 3000
    other = T.generate(spec, 78)
    assert not torch.equal(w1.pairs, other.pairs)


def test_stream_windows_churn_planted_sets():
    a = T.spec_stream_window(0, n_pairs=10_000_000)
    b = T.spec_stream_window(1, n_pairs=10_000_000)
    sa, sb = set(a.planted_ids), set(b.planted_ids)
    assert len(sa) == len(sb) == 1000
    assert len(sa - sb) == 200
    assert all(1024 <= c <= 50000 for c in a.planted_card)
