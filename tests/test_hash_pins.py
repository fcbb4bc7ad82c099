"""The hash family pinned by a second, independent implementation.

The paper leaves H1 and DH0 unspecified (Sec. 3.1 calls H1 a random hash,
Sec. 3.2 gives DH0 only as a random hash into [0, 2^k) and builds DH_i from it
by eq. (2)). Both sides take the multiply-add-shift reading: coefficients are
the first four SplitMix64 outputs of the sketch seed (Steele, Lea and Flood
2014) with the multipliers forced odd, and

    DH0(x)  = ((A0 x + B0) mod 2^64) >> (64 - k)
    H1(y)   = ((A1 y + B1) mod 2^64) >> (64 - log2 g)
    DH_i(x) = DH0(x) xor ((x >> (i-1) alpha) mod 2^k)     (0 past bit 31)

Here the whole family is written again with Python integers (no fixed-width
arithmetic at all), its SplitMix64 is checked against the published vectors,
and the oracle's DH_i and H1 must agree with it element for element on keys
that include 0, 1, 2^31, 2^32 - 1 and sequential runs. A dropped B0, swapped
A0/A1, a wrong SplitMix output index, an unforced odd bit or a wrong shift
fails here.
"""
import numpy as np
import pytest

import oracle
from conftest import golden_path
from paper_1803_11449_amd import traffic

M64 = (1 << 64) - 1


def py_splitmix64(seed: int, n: int) -> list:
    """SplitMix64 from its published definition, in Python integers."""
    out, s = [], seed & M64
    for _ in range(n):
        s = (s + 0x9E3779B97F4A7C15) & M64
        z = s
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M64
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M64
        out.append(z ^ (z >> 31))
    return out


def py_family(g: int, k: int, r: int, alpha: int, seed: int):
    """(dh(i, x), h1(y)) as Python-integer functions."""
    a0, b0, a1, b1 = py_splitmix64(seed, 4)
    a0 |= 1
    a1 |= 1
    log2g = g.bit_length() - 1

    def dh0(x):
        return ((a0 * x + b0) % (1 << 64)) >> (64 - k)

    def dh(i, x):
        if i == 0:
            return dh0(x)
        s = (i - 1) * alpha
        block = (x >> s) % (1 << k) if s < 32 else 0
        return dh0(x) ^ block

    def h1(y):
        return ((a1 * y + b1) % (1 << 64)) >> (64 - log2g)

    return dh, h1


def pin_keys() -> np.ndarray:
    """At least 1000 keys: the edges, sequential runs at 0, 2^31 and the
    top of the space, powers of two, and seeded random keys."""
    edges = [0, 1, 2, 3, 2**31 - 1, 2**31, 2**31 + 1, 2**32 - 2, 2**32 - 1]
    runs = list(range(0, 200)) + list(range(2**31 - 100, 2**31 + 100)) + \
        list(range(2**32 - 200, 2**32))
    pows = [1 << i for i in range(32)] + [(1 << i) - 1 for i in range(1, 33)]
    rnd = np.random.default_rng(1803).integers(0, 2**32, size=400, dtype=np.uint64).tolist()
    keys = np.array(sorted(set(edges + runs + pows + [int(x) for x in rnd])), dtype=np.uint64)
    assert keys.size >= 1000
    return keys.astype(np.uint32)


SETS = [(1024, 14, 5, 6), (1024, 18, 5, 5), (256, 12, 6, 5)]
SEEDS = [traffic.HASH_SEED, 0, 0xDEADBEEFCAFEF00D]


def test_python_splitmix64_matches_published_vectors():
    with open(golden_path("splitmix64_vectors.txt")) as f:
        rows = [l.split() for l in f if l.strip() and not l.startswith("#")]
    assert rows
    for row in rows:
        seed, expect = int(row[0]), [int(x) for x in row[1:]]
        assert py_splitmix64(seed, len(expect)) == expect


@pytest.mark.parametrize("seed", SEEDS)
def test_oracle_coefficients_equal_python(seed):
    a0, b0, a1, b1 = py_splitmix64(seed, 4)
    assert [int(x) for x in oracle.hash_coeffs(seed)] == [a0 | 1, b0, a1 | 1, b1]


@pytest.mark.parametrize("seed", SEEDS)
@pytest.mark.parametrize("shape", SETS)
def test_oracle_dh_and_h1_equal_python(shape, seed):
    g, k, r, alpha = shape
    p = oracle.Params(g, k, r, alpha, seed)
    keys = pin_keys()
    dh, h1 = py_family(g, k, r, alpha, seed)
    ints = [int(x) for x in keys]
    for i in range(r):
        want = np.array([dh(i, x) for x in ints], dtype=np.uint32)
        got = oracle.dh(p, i, keys)
        bad = np.nonzero(got != want)[0]
        assert bad.size == 0, (i, ints[bad[0]], int(got[bad[0]]), int(want[bad[0]]))
    want = np.array([h1(y) for y in ints], dtype=np.uint32)
    got = oracle.h1(p, keys)
    bad = np.nonzero(got != want)[0]
    assert bad.size == 0, (ints[bad[0]], int(got[bad[0]]), int(want[bad[0]]))


def test_python_family_hand_checks():
    """Spot values worked by hand from the definition: DH0(0) is the top k
    bits of B0, H1(0) the top log2 g bits of B1, and DH_1(x) xor DH_0(x) is
    the low k bits of x."""
    g, k, r, alpha = SETS[0]
    seed = traffic.HASH_SEED
    a0, b0, a1, b1 = py_splitmix64(seed, 4)
    dh, h1 = py_family(g, k, r, alpha, seed)
    assert dh(0, 0) == b0 >> (64 - k)
    assert h1(0) == b1 >> (64 - 10)
    x = 0xA5A5F00F
    assert dh(1, x) ^ dh(0, x) == x & ((1 << k) - 1)
    assert dh(4, x) ^ dh(0, x) == (x >> 18) & ((1 << k) - 1)
    # DH0(1) - DH0(0) is the top k bits of the sum A0 + B0, not of B0 alone
    assert dh(0, 1) == ((a0 | 1) + b0) % (1 << 64) >> (64 - k)


def python_sketch(g, k, r, alpha, seed, pairs) -> np.ndarray:
    """The sketch of Alg. 1 built from the Python-integer family (for the
    GPU pin), in the shared word layout."""
    dh, h1 = py_family(g, k, r, alpha, seed)
    words = np.zeros(r * (1 << k) * (g // 32), dtype=np.uint32)
    for a, b in pairs.tolist():
        bit = h1(b)
        for i in range(r):
            w = ((i << k) + dh(i, a)) * (g // 32) + bit // 32
            words[w] |= np.uint32(1 << (bit % 32))
    return words
