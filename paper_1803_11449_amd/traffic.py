"""Seeded synthetic traffic: windows of (src, dst) IPv4 pairs.

This module only makes inputs. It holds none of the sketch's arithmetic and
is the one piece that both the GPU library's callers and the CPU oracle's
callers use. Every random draw comes from a counter-based generator, so a
window is a pure function of (spec, seed) and is identical on the CPU and on
the GPU (integer-only torch ops; the Zipf CDF table is built once in float64
on the host and then used as integers).

Traffic shape (stand-in for the CAIDA OC192 windows the paper measures on,
which are not available): measured sources drawn Zipf(s) over a fixed
population of source IPs with uniform 32-bit destinations; planted super
points that each contact an exact number of distinct destinations; optional
scanner sources hitting sequential destinations; optional duplicate pairs;
all positions shuffled by a seeded permutation.

Generator definitions
  rng(key, i)      SplitMix64 output i of the stream started at key
                   (Steele, Lea and Flood 2014), computed directly from i
  zipf rank        smallest j with u53 < T[j], T[j] = floor(2^53 * CDF(j))
  source IP(rank)  a 4-round keyed Feistel bijection on 32 bits, so ranks
                   give distinct IPs; planted and scanner sources use ranks
                   at or above the Zipf population, so they are disjoint
  planted dst      Feistel(m, key_j) for m < C_j: C_j distinct destinations
  scanner dst      base_j + m (mod 2^32), m < L
  duplicates       copies of uniformly chosen body pairs
  order            ascending (rng >> 33, position): a seeded permutation
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np
import torch

_M64 = (1 << 64) - 1
_GOLDEN = 0x9E3779B97F4A7C15
_MIX1 = 0xBF58476D1CE4E5B9
_MIX2 = 0x94D049BB133111EB

HASH_SEED = 0x1803114490000001
TRAFFIC_SEED = 0x18031144900


def _s64(x: int) -> int:
    """Python int (mod 2^64) as the signed int64 with the same bits."""
    x &= _M64
    return x - (1 << 64) if x >= (1 << 63) else x


def _srl(x: torch.Tensor, s: int) -> torch.Tensor:
    """Logical right shift of int64 bit patterns."""
    return (x >> s) & ((1 << (64 - s)) - 1)


def mix64(x: torch.Tensor) -> torch.Tensor:
    """SplitMix64 output function on int64 bit patterns (wrapping)."""
    x = x ^ _srl(x, 30)
    x = x * _s64(_MIX1)
    x = x ^ _srl(x, 27)
    x = x * _s64(_MIX2)
    return x ^ _srl(x, 31)


def stream_key(seed: int, stream: int) -> int:
    """Start state of an independent stream (python int, mod 2^64)."""
    x = (seed ^ ((stream * 0xD1B54A32D192ED03) & _M64)) & _M64
    # one SplitMix64 step on the host to decorrelate nearby streams
    x = (x + _GOLDEN) & _M64
    z = x
    z = ((z ^ (z >> 30)) * _MIX1) & _M64
    z = ((z ^ (z >> 27)) * _MIX2) & _M64
    return z ^ (z >> 31)


def rng64(key: int, idx: torch.Tensor) -> torch.Tensor:
    """Output idx (0-based) of the SplitMix64 stream started at key."""
    return mix64(idx * _s64(_GOLDEN) + _s64(key + _GOLDEN))


def rng32(key: int, idx: torch.Tensor) -> torch.Tensor:
    """Top 32 bits of rng64 as values in [0, 2^32) (int64)."""
    return _srl(rng64(key, idx), 32)


def feistel32(x: torch.Tensor, key) -> torch.Tensor:
    """Keyed bijection on 32-bit values (int64 tensor in [0,2^32)).

    key is a python int or an int64 tensor broadcastable to x."""
    left = _srl(x, 16) & 0xFFFF
    right = x & 0xFFFF
    for rnd in range(4):
        kr = key + _s64((rnd + 1) * _GOLDEN) if isinstance(key, torch.Tensor) \
            else _s64(key + (rnd + 1) * _GOLDEN)
        f = _srl(mix64(right * 0x10001 ^ kr), 48)
        left, right = right, left ^ f
    return (left << 16) | right


def to_int32_bits(x: torch.Tensor) -> torch.Tensor:
    """int64 values in [0,2^32) to int32 with the same 32-bit pattern."""
    return (x - ((x >> 31) & 1) * (1 << 32)).to(torch.int32)


_zipf_cache: dict = {}


def zipf_table(n: int, s: float, device) -> torch.Tensor:
    """T[j] = floor(2^53 * CDF(j)) for Zipf(s) over ranks 0..n-1."""
    key = (n, float(s), str(device))
    t = _zipf_cache.get(key)
    if t is None:
        w = np.arange(1, n + 1, dtype=np.float64) ** (-float(s))
        cdf = np.cumsum(w)
        cdf /= cdf[-1]
        tab = np.floor(cdf * float(1 << 53)).astype(np.int64)
        tab[-1] = 1 << 53
        t = torch.from_numpy(tab).to(device)
        if len(_zipf_cache) > 8:
            _zipf_cache.clear()
        _zipf_cache[key] = t
    return t


@dataclasses.dataclass
class WindowSpec:
    """One window of traffic."""
    n_pairs: int
    n_sources: int            # Zipf source population
    zipf_s: float
    planted_card: list        # distinct destinations of each planted source
    planted_ids: list | None = None   # identity of each planted source
    n_scanners: int = 0
    scanner_len: int = 0
    dup_frac: float = 0.0
    name: str = ""


@dataclasses.dataclass
class Window:
    pairs: torch.Tensor       # int32 [n, 2]: (src, dst) bit patterns
    planted_src: np.ndarray   # uint32
    planted_card: np.ndarray  # int64
    scanner_src: np.ndarray   # uint32
    spec: WindowSpec


def _loguniform_ints(key: int, n: int, lo: int, hi: int) -> list:
    u = rng64(key, torch.arange(n, dtype=torch.int64))
    u = (_srl(u, 11).double() / float(1 << 53)).numpy()
    return [int(math.floor(math.exp(math.log(lo) + x * (math.log(hi) - math.log(lo)))))
            for x in u]


def generate(spec: WindowSpec, seed: int, device="cpu") -> Window:
    """Make one window as an int32 [n,2] tensor on device."""
    dev = torch.device(device)
    i64 = torch.int64
    ip_key = stream_key(seed, 1)
    card = [int(c) for c in spec.planted_card]
    ids = list(spec.planted_ids) if spec.planted_ids is not None else list(range(len(card)))
    n_planted_pairs = sum(card)
    n_scan_pairs = spec.n_scanners * spec.scanner_len
    n_dup = int(round(spec.dup_frac * spec.n_pairs))
    n_body = spec.n_pairs - n_dup
    n_zipf = n_body - n_planted_pairs - n_scan_pairs
    if n_zipf < 0:
        raise ValueError("planted and scanner pairs exceed the window")

    parts_src, parts_dst = [], []
    # planted super points: rank n_sources + id, C_j distinct destinations
    planted_src = np.zeros(0, dtype=np.uint32)
    if card:
        c_t = torch.tensor(card, dtype=i64, device=dev)
        id_t = torch.tensor(ids, dtype=i64, device=dev)
        src_j = feistel32(spec.n_sources + id_t, ip_key)
        planted_src = src_j.cpu().numpy().astype(np.uint32)
        j = torch.repeat_interleave(torch.arange(len(card), device=dev), c_t)
        start = torch.cumsum(c_t, 0) - c_t
        m = torch.arange(n_planted_pairs, dtype=i64, device=dev) - start[j]
        dkey = _srl(rng64(stream_key(seed, 2), id_t), 1)   # per-source key
        parts_src.append(src_j[j])
        parts_dst.append(feistel32(m, dkey[j]))
    # scanners: sequential destinations from a random base
    scanner_src = np.zeros(0, dtype=np.uint32)
    if n_scan_pairs:
        sid = torch.arange(spec.n_scanners, dtype=i64, device=dev)
        s_src = feistel32(spec.n_sources + 1_000_000_000 + sid, ip_key)
        scanner_src = s_src.cpu().numpy().astype(np.uint32)
        base = rng32(stream_key(seed, 3), sid)
        q = torch.arange(n_scan_pairs, dtype=i64, device=dev)
        parts_src.append(s_src[q // spec.scanner_len])
        parts_dst.append((base[q // spec.scanner_len] + q % spec.scanner_len) & 0xFFFFFFFF)
    # Zipf background
    if n_zipf:
        q = torch.arange(n_zipf, dtype=i64, device=dev)
        u = _srl(rng64(stream_key(seed, 4), q), 11)
        tab = zipf_table(spec.n_sources, spec.zipf_s, dev)
        rank = torch.searchsorted(tab, u, right=True).clamp_(max=spec.n_sources - 1)
        parts_src.append(feistel32(rank, ip_key))
        parts_dst.append(rng32(stream_key(seed, 5), q))
    src = torch.cat(parts_src) if parts_src else torch.zeros(0, dtype=i64, device=dev)
    dst = torch.cat(parts_dst) if parts_dst else torch.zeros(0, dtype=i64, device=dev)
    # duplicates of uniformly chosen body pairs
    if n_dup:
        q = torch.arange(n_dup, dtype=i64, device=dev)
        pick = rng32(stream_key(seed, 6), q) * n_body >> 32
        src = torch.cat([src, src[pick]])
        dst = torch.cat([dst, dst[pick]])
    # seeded permutation of positions
    n = src.numel()
    pos = torch.arange(n, dtype=i64, device=dev)
    order = torch.sort((_srl(rng64(stream_key(seed, 7), pos), 33) << 31) | pos).values
    perm = order & ((1 << 31) - 1)
    del order, pos
    src = src[perm]
    dst = dst[perm]
    pairs = torch.stack([to_int32_bits(src), to_int32_bits(dst)], dim=1).contiguous()
    return Window(pairs=pairs, planted_src=planted_src,
                  planted_card=np.asarray(card, dtype=np.int64),
                  scanner_src=scanner_src, spec=spec)


# ---------------------------------------------------------------- configs

def spec_single_window_1m() -> WindowSpec:
    """1M pairs: 960k Zipf(1.1) over 100k sources, 20 planted x 2000 dsts."""
    return WindowSpec(n_pairs=1_000_000, n_sources=100_000, zipf_s=1.1,
                      planted_card=[2000] * 20, name="single_window_1m")


def spec_large_window_100m(n_pairs: int = 100_000_000) -> WindowSpec:
    """100M pairs: Zipf(1.0) over 4M sources, 500 planted log-uniform in
    [1024, 50000], 50 scanners x 20k sequential dsts, 10% duplicates."""
    card = _loguniform_ints(stream_key(TRAFFIC_SEED + 2, 9), 500, 1024, 50000)
    return WindowSpec(n_pairs=n_pairs, n_sources=4_000_000, zipf_s=1.0,
                      planted_card=card, n_scanners=50, scanner_len=20_000,
                      dup_frac=0.10, name="large_window_100m")


def spec_stream_window(w: int, n_pairs: int = 117_000_000,
                       n_sources: int = 8_000_000, n_planted: int = 1000) -> WindowSpec:
    """Window w of the sustained 117 Mpps stream: Zipf(1.0) over 8M sources,
    1000 planted log-uniform in [1024, 50000], 20% of them replaced each
    window (slot s is renewed when (w + s) % 5 == 0)."""
    ids, card = [], []
    for s in range(n_planted):
        gen = (w + s % 5) // 5
        pid = s + n_planted * gen
        ids.append(pid)
    c = _loguniform_ints(stream_key(TRAFFIC_SEED + 3, 11), max(ids) + 1, 1024, 50000)
    card = [c[i] for i in ids]
    return WindowSpec(n_pairs=n_pairs, n_sources=n_sources, zipf_s=1.0,
                      planted_card=card, planted_ids=ids,
                      name=f"stream_window_{w}")


def spec_link_window(n_pairs: int, zipf_s: float, n_planted: int, key: int) -> WindowSpec:
    """One link's window in a batch of monitored links: Zipf(s) over
    n_pairs/25 sources with uniform destinations, n_planted planted sources
    with cardinalities log-uniform in [1024, 50000] (the list is cut while
    the planted pairs exceed 30% of the window)."""
    card = _loguniform_ints(stream_key(key, 13), n_planted, 1024, 50000)
    while len(card) > 1 and sum(card) > 0.3 * n_pairs:
        card = card[:-1]
    return WindowSpec(n_pairs=n_pairs, n_sources=max(1000, n_pairs // 25), zipf_s=zipf_s,
                      planted_card=card, name="link_window")


def config_seed(config_id: int, window: int = 0) -> int:
    return TRAFFIC_SEED + config_id + (window << 32)
