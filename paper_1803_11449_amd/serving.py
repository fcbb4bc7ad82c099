"""Serving closing windows of many monitored links on one GPU.

A request is the close of one window of one link: its (src,dst) pairs are
already in device memory; the response is the window's super point list
(Alg. 2 restore after Alg. 1 update). Each link keeps a sketch resident on
the device, sized for its windows by the sizing rule (smallest k >= 14 with
n / (g 2^k) <= 0.45 and alpha = ceil((32 - k) / (r - 2)) <= k).

ContinuousServer batches continuously and keeps two batches on the GPU:
each loop iteration admits the requests that have arrived (one per link,
links with a batch still on the GPU wait, and only while the resident
sketches fit the HBM budget), enqueues their updates as one batched update
and their restores as one batched restore on one of two streams of equal
priority, and only then waits for the older batch's restores. So a batch's
update runs on the device while the batch before it restores, and requests
that arrive meanwhile are admitted as soon as a slot frees. PlainServer
handles one request at a time in arrival order (the per-window launch).
Both report every request's close-to-report latency.

The scheduling is host code over the batched C ABI; every step of the
update and the restore runs in the HIP library.
"""
from __future__ import annotations

import dataclasses
import gc
import math
import time
from collections import OrderedDict

import numpy as np
import torch

from . import ddhf, traffic


def sized_params(n_pairs: int, g: int = 1024, r: int = 5, k_min: int = 14,
                 k_max: int = 20, load: float = 0.45):
    """(k, alpha) of the sizing rule for a window of n_pairs pairs. alpha is
    the least that meets (r - 2) alpha + k >= 32; k also grows until
    alpha <= k (for r = 3 that is k >= 16)."""
    def alpha_of(k):
        return max(1, math.ceil((32 - k) / (r - 2)))
    k = k_min
    while k < k_max and (n_pairs / (g * 2 ** k) > load or alpha_of(k) > k):
        k += 1
    return k, alpha_of(k)


def resident_bytes(g: int, k: int, r: int, alpha: int) -> int:
    """Device memory a resident link costs: the sketch plus its per-row
    restore arrays and per-tile update arrays (the large scratch is shared)."""
    n_le = r << k
    sketch = n_le * g // 8
    rows = n_le // 8 + 3 * 4 * n_le + 8 * r * (1 << (k - alpha))
    tiles = max(1, sketch // (160 << 10)) * 4 * (256 + 4)
    return sketch + rows + tiles + (1 << 16)


@dataclasses.dataclass
class Request:
    rid: int
    link: int
    arrival: float            # seconds after the start of serving
    pairs: torch.Tensor       # int32 [n, 2] on the device
    theta: float = 1024.0

    @property
    def n_pairs(self) -> int:
        return self.pairs.shape[0]


@dataclasses.dataclass
class Response:
    rid: int
    link: int
    records: np.ndarray       # sketch records, ascending by address
    info: dict
    arrival: float
    done: float               # seconds after the start of serving
    batch: int                # requests served in the same batch
    n_pairs: int = 0
    status: int = 0           # SKETCH_OK, or the library's error (records empty)

    @property
    def latency(self) -> float:
        return self.done - self.arrival


class _Links:
    """Resident sketches, one per (link, k), under an HBM budget; the least
    recently used ones not in the current batch are evicted first."""

    def __init__(self, budget_bytes: int, g: int, r: int, device: int):
        self.budget = budget_bytes
        self.g, self.r, self.device = g, r, device
        self.sk: OrderedDict = OrderedDict()    # (link, k) -> (Sketch, bytes)
        self.used = 0

    def _key(self, link: int, n_pairs: int):
        k, alpha = sized_params(n_pairs, self.g, self.r)
        return (link, k), alpha

    def need(self, link: int, n_pairs: int) -> int:
        """Bytes a request's sketch still has to take (0 if resident)."""
        key, alpha = self._key(link, n_pairs)
        return 0 if key in self.sk else resident_bytes(self.g, key[1], self.r, alpha)

    def fits(self, need: int, pinned: set, pending: int = 0) -> bool:
        """Whether `need` more bytes fit next to `pending` bytes already
        promised to this batch, evicting sketches of links not in `pinned`."""
        free = self.budget - self.used - pending
        free += sum(b for kk, (_, b) in self.sk.items() if kk[0] not in pinned)
        return need <= free

    def get(self, link: int, n_pairs: int, pinned: set) -> ddhf.Sketch:
        key, alpha = self._key(link, n_pairs)
        cur = self.sk.get(key)
        if cur is not None:
            self.sk.move_to_end(key)
            return cur[0]
        need = resident_bytes(self.g, key[1], self.r, alpha)
        for kk in list(self.sk):
            if self.used + need <= self.budget:
                break
            if kk[0] not in pinned:
                self._drop(kk)
        if self.used + need > self.budget:
            raise MemoryError("link sketches exceed the HBM budget")
        sk = ddhf.Sketch(self.g, key[1], self.r, alpha, traffic.HASH_SEED, device=self.device)
        self.sk[key] = (sk, need)
        self.used += need
        return sk

    def prewarm(self, requests):
        """Create the sketches a list of requests will use (as fits)."""
        for q in requests:
            if self.fits(self.need(q.link, q.n_pairs), set()):
                self.get(q.link, q.n_pairs, set())

    def _drop(self, key):
        sk, b = self.sk.pop(key)
        sk.close()
        self.used -= b

    def close(self):
        for kk in list(self.sk):
            self._drop(kk)


def _response(q: Request, recs, info: dict, done: float, batch: int) -> Response:
    """A request's response; a failed restore (a saturated sketch) gives an
    empty list and its status instead of stopping the server."""
    if recs is None:
        recs = np.zeros(0, dtype=ddhf.SP_DTYPE)
    return Response(q.rid, q.link, recs, info, q.arrival, done, batch, q.n_pairs,
                    int(info.get("status", ddhf.SKETCH_OK)))


class _Server:
    def __init__(self, budget_bytes: int = 64 << 30, g: int = 1024, r: int = 5,
                 device: int = 0):
        self.links = _Links(budget_bytes, g, r, device)
        self.dev = torch.device("cuda", device)

    def close(self):
        self.links.close()

    def serve(self, requests) -> list:
        """Serve the requests (see the class); one response per request, in
        request order. Python's cycle collector is off meanwhile: a full
        collection in the loop would stall every request in flight by
        tens of milliseconds (reference counting still frees what the
        loop drops)."""
        was = gc.isenabled()
        gc.disable()
        try:
            return self._serve(requests)
        finally:
            if was:
                gc.enable()

    def warm(self, requests, n: int = 16):
        """Grow the device's shared buffers (update arena, restore pools)
        before serving: one batched update of the largest windows, one per
        link (at most n, within the budget), their batched restore and each
        one's restore alone. The sketches are reset when their requests are
        served, so results do not change."""
        chosen, links, pending = [], set(), 0
        for q in sorted(requests, key=lambda q: -q.n_pairs):
            if len(chosen) == n:
                break
            need = self.links.need(q.link, q.n_pairs)
            if q.link in links or not self.links.fits(need, links | {q.link}, pending):
                continue
            chosen.append(q)
            links.add(q.link)
            pending += need
        if not chosen:
            return
        sks = [self.links.get(q.link, q.n_pairs, links) for q in chosen]
        for sk in sks:
            sk.reset()
        ddhf.update_batch([(sk, q.pairs) for sk, q in zip(sks, chosen)])
        # the batch grows the pools its jobs land on; one job alone always
        # takes the first pool, so each window is also restored by itself
        ddhf.restore_batch([(sk, q.theta) for sk, q in zip(sks, chosen)], raise_errors=False)
        for sk, q in zip(sks, chosen):
            ddhf.restore_batch([(sk, q.theta)], raise_errors=False)
        torch.cuda.synchronize(self.dev)

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    @staticmethod
    def _wait_until(t0: float, t: float):
        while True:
            now = time.perf_counter() - t0
            if now >= t:
                return
            if t - now > 2e-3:
                time.sleep((t - now) / 2)


# Streams checked to run their work concurrently, per device (see
# concurrent_streams); every server of the process reuses them.
_CONCURRENT: dict = {}


def _spin_pair_s(a, b, cycles: int) -> float:
    """Host seconds for one spin kernel on each of two streams."""
    torch.cuda.synchronize(a.device)
    t0 = time.perf_counter()
    for s in (a, b):
        with torch.cuda.stream(s):
            torch.cuda._sleep(cycles)
    torch.cuda.synchronize(a.device)
    return time.perf_counter() - t0


def concurrent_streams(device: int, n: int = 2, tries: int = 8, cycles: int = 2_000_000):
    """n streams of the default priority whose work runs at the same time.

    HIP runs streams on a few hardware queues per process (four by default)
    and streams that share a queue run their work in submission order, one
    after the other; which queue a new stream gets depends on the streams
    made before it. So each new stream is checked against the ones kept: a
    spin kernel of about a millisecond on both must end in about the time
    of one (below 1.5 times). A stream that fails is dropped and another
    made, up to `tries`; past that the last one is kept (work is still
    correct, only in order). The result is cached per device."""
    if device in _CONCURRENT and len(_CONCURRENT[device]) >= n:
        return _CONCURRENT[device][:n]
    dev = torch.device("cuda", device)
    if not hasattr(torch.cuda, "_sleep"):          # no spin kernel to check with
        kept = list(_CONCURRENT.get(device, []))
        kept += [torch.cuda.Stream(dev) for _ in range(n - len(kept))]
        _CONCURRENT[device] = kept
        return kept[:n]
    kept = list(_CONCURRENT.get(device, []))
    if not kept:
        kept.append(torch.cuda.Stream(dev))
    with torch.cuda.device(dev):
        one = min(_spin_pair_s(kept[0], kept[0], cycles) for _ in range(2)) / 2
        while len(kept) < n:
            cand = None
            for _ in range(tries):
                cand = torch.cuda.Stream(dev)
                if all(_spin_pair_s(k, cand, cycles) < 1.5 * one for k in kept):
                    break
            kept.append(cand)
    _CONCURRENT[device] = kept
    return kept[:n]


class ContinuousServer(_Server):
    """Continuous batching with two batches in flight: see the module
    docstring. With trace=True every batch records timing events on its
    stream (update start and end, restore end) in self.trace."""

    def __init__(self, budget_bytes: int = 64 << 30, g: int = 1024, r: int = 5,
                 device: int = 0, max_batch: int = 64, depth: int = 2, trace: bool = False):
        super().__init__(budget_bytes, g, r, device)
        self.max_batch = max_batch
        self.depth = max(1, depth)
        # streams of the default priority, one per batch in flight, checked
        # to run concurrently
        self.streams = concurrent_streams(device, self.depth)
        self.trace_on = trace
        self.trace = []

    def _event(self, stream):
        if not self.trace_on:
            return None
        e = torch.cuda.Event(enable_timing=True)
        e.record(stream)
        return e

    def _admit(self, waiting, busy: set):
        """Requests of the next batch, in arrival order: one per link, none
        for a link with a batch in flight, within the budget (bytes of new
        sketches promised to the batch count, and the sketches of batches in
        flight are never evicted)."""
        batch, links, pending = [], set(), 0
        for q in waiting:
            if len(batch) == self.max_batch:
                break
            if q.link in links or q.link in busy:
                continue
            need = self.links.need(q.link, q.n_pairs)
            if not self.links.fits(need, links | busy | {q.link}, pending):
                continue
            batch.append(q)
            links.add(q.link)
            pending += need
        if not batch and not busy:     # the oldest request alone may evict anything
            batch = [waiting[0]]
        return batch

    def _serve(self, requests) -> list:
        reqs = sorted(requests, key=lambda q: q.arrival)
        out, waiting, nxt = [], [], 0
        inflight = []         # (batch, PendingRestore, done event, trace events), oldest first
        k = 0
        t0 = time.perf_counter()
        base = self._event(self.streams[0])
        while nxt < len(reqs) or waiting or inflight:
            now = time.perf_counter() - t0
            while nxt < len(reqs) and reqs[nxt].arrival <= now:
                waiting.append(reqs[nxt])
                nxt += 1
            busy = {q.link for b, _, _, _ in inflight for q in b}
            batch = self._admit(waiting, busy) if waiting and len(inflight) < self.depth else []
            if batch:
                taken = {id(q) for q in batch}
                waiting = [q for q in waiting if id(q) not in taken]
                busy |= {q.link for q in batch}
                sks = [self.links.get(q.link, q.n_pairs, busy) for q in batch]
                st = self.streams[k % self.depth]
                k += 1
                e0 = self._event(st)
                for sk in sks:
                    sk.reset(st)
                ddhf.update_batch([(sk, q.pairs) for sk, q in zip(sks, batch)], st)
                e1 = self._event(st)
                pend = ddhf.restore_batch_begin([(sk, q.theta) for sk, q in zip(sks, batch)], st)
                done_ev = torch.cuda.Event()
                done_ev.record(st)
                inflight.append((batch, pend, done_ev, (e0, e1, self._event(st))))
                continue               # admit more while this batch is on the GPU
            if inflight:
                # collect the oldest batch once it is done, or at once when no
                # other batch can start before it is (every slot taken, or no
                # request left to come); else look again shortly for arrivals
                if (len(inflight) == self.depth or nxt == len(reqs)
                        or inflight[0][2].query()):
                    b, pend, _, ev = inflight.pop(0)
                    res = pend.end(raise_errors=False)
                    done = time.perf_counter() - t0
                    for q, (recs, info) in zip(b, res):
                        out.append(_response(q, recs, info, done, len(b)))
                    if self.trace_on:
                        self.trace.append((base, ev, len(b)))
                else:
                    time.sleep(2e-5)
                continue
            if nxt < len(reqs):
                self._wait_until(t0, reqs[nxt].arrival)
        return sorted(out, key=lambda r: r.rid)

    def overlaps(self) -> int:
        """Batches whose work began on the device before the previous batch's
        restore had ended (from the trace's timing events: the start marker
        on the batch's own stream against the previous batch's restore end
        on the other stream): the two batches were on the GPU together."""
        torch.cuda.synchronize(self.dev)
        n = 0
        for (base, ev, _), (_, prev, _) in zip(self.trace[1:], self.trace[:-1]):
            if base.elapsed_time(ev[0]) < base.elapsed_time(prev[2]):
                n += 1
        return n


class PlainServer(_Server):
    """One request at a time, in arrival order: reset, update, restore."""

    def _serve(self, requests) -> list:
        reqs = sorted(requests, key=lambda q: q.arrival)
        out = []
        t0 = time.perf_counter()
        for q in reqs:
            self._wait_until(t0, q.arrival)
            sk = self.links.get(q.link, q.n_pairs, {q.link})
            sk.reset()
            sk.update(q.pairs)
            (recs, info), = ddhf.restore_batch([(sk, q.theta)], raise_errors=False)
            out.append(_response(q, recs, info, time.perf_counter() - t0, 1))
        return sorted(out, key=lambda r: r.rid)


def serve_alone(requests, device: int = 0, g: int = 1024, r: int = 5) -> list:
    """Every request on its own fresh sketch, no timing: the reference
    results a served request must reproduce."""
    out = []
    for q in requests:
        k, alpha = sized_params(q.n_pairs, g, r)
        with ddhf.Sketch(g, k, r, alpha, traffic.HASH_SEED, device=device) as sk:
            sk.update(q.pairs)
            recs, info = sk.restore(q.theta)
        out.append(Response(q.rid, q.link, recs, info, q.arrival, 0.0, 1, q.n_pairs))
    return out


# ------------------------------------------------------------------ loads

def pair_pool(n_pairs: int, zipf_s: float, seed: int, device) -> torch.Tensor:
    """A long stream of synthetic pairs that windows are cut from: Zipf(s)
    sources over n/32 hosts with uniform destinations, 0.05% of the hosts
    planted as super points with log-uniform cardinalities in
    [1024, 50000] (capped at 30% of the pool)."""
    n_src = max(1000, n_pairs // 32)
    n_planted = max(1, int(0.0005 * n_src))
    card = traffic._loguniform_ints(traffic.stream_key(seed, 17), n_planted, 1024, 50000)
    while sum(card) > 0.3 * n_pairs and len(card) > 1:
        card = card[:-1]
    spec = traffic.WindowSpec(n_pairs=n_pairs, n_sources=n_src, zipf_s=zipf_s,
                              planted_card=card, name="pool")
    return traffic.generate(spec, seed, device=device).pairs


def poisson_windows(pools, n_links: int, rate_pps: float, duration_s: float,
                    lo: int, hi: int, seed: int, theta=(1024.0,)) -> list:
    """Closing windows of n_links links: Poisson arrivals whose sizes are
    log-uniform in [lo, hi] pairs, at an aggregate rate_pps pairs per second,
    over duration_s seconds. Window pairs are slices of the given pools."""
    rng = np.random.default_rng(seed)
    mean = (hi - lo) / math.log(hi / lo)
    lam = rate_pps / mean                       # windows per second
    reqs, t, rid = [], 0.0, 0
    while True:
        t += rng.exponential(1.0 / lam)
        if t > duration_s:
            break
        n = int(math.exp(rng.uniform(math.log(lo), math.log(hi))))
        pool = pools[rng.integers(len(pools))]
        off = int(rng.integers(0, pool.shape[0] - n + 1))
        reqs.append(Request(rid, int(rng.integers(n_links)), t, pool[off:off + n],
                            float(theta[rng.integers(len(theta))])))
        rid += 1
    return reqs


def latency_summary(resps) -> dict:
    """Close-to-report latency percentiles and the served pair rate."""
    if not resps:
        return {}
    lat = np.array([r.latency for r in resps]) * 1e3
    span = max(r.done for r in resps) - min(r.arrival for r in resps)
    pairs = sum(r.n_pairs for r in resps)
    return {"requests": len(resps), "pairs": pairs,
            "latency_ms_p50": round(float(np.percentile(lat, 50)), 4),
            "latency_ms_p99": round(float(np.percentile(lat, 99)), 4),
            "latency_ms_max": round(float(lat.max()), 4),
            "span_s": round(span, 4), "served_mpps": round(pairs / span / 1e6, 2),
            "mean_batch": round(float(np.mean([r.batch for r in resps])), 2)}
