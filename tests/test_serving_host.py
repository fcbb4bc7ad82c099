"""Host logic of the serving loop, on the CPU: the sizing rule, the resident
sketch cache under its HBM budget, and the continuous batcher's admission.
The library calls are replaced by stand-ins that record what the server asks
for (the GPU serving tests check the results themselves).
"""
import contextlib

import numpy as np
import pytest
import torch

from paper_1803_11449_amd import ddhf, serving


def test_sizing_rule_meets_the_parameter_constraints():
    """k is the smallest in [14, 20] with n / (g 2^k) <= 0.45 and a valid
    alpha, and every (k, alpha) it gives satisfies the constraints
    sketch_create checks: 5 <= k <= 24, 1 <= alpha <= k,
    (r - 2) alpha + k >= 32, k - alpha <= 20."""
    for r in (3, 4, 5, 6, 8):
        for g in (256, 1024, 4096):
            prev_k = 14
            for n in [0, 1] + [int(x) for x in np.geomspace(2, 2**33, 300)]:
                k, alpha = serving.sized_params(n, g, r)
                assert 14 <= k <= 20 and k >= prev_k
                prev_k = k
                assert 1 <= alpha <= k and (r - 2) * alpha + k >= 32 and k - alpha <= 20
                assert k == 20 or n / (g * 2**k) <= 0.45
                # k - 1 fails the load bound, or no alpha <= k - 1 meets the constraint
                assert k == 14 or n / (g * 2 ** (k - 1)) > 0.45 or (r - 2) * (k - 1) + k - 1 < 32
                assert (r - 2) * (alpha - 1) + k < 32 or alpha == 1   # the least alpha


def test_resident_bytes_cover_the_sketch():
    for k in range(14, 21):
        alpha = serving.sized_params(1024 * 2**k // 3)[1]
        b = serving.resident_bytes(1024, k, 5, alpha)
        assert b >= 5 * 2**k * 1024 // 8
        assert b < 2 * 5 * 2**k * 1024 // 8 + (1 << 20)


class FakeSketch:
    """Stands in for ddhf.Sketch: counts live instances."""
    live = set()

    def __init__(self, g, k, r, alpha, seed, device=0):
        self.k, self.closed = k, False
        FakeSketch.live.add(id(self))

    def reset(self, stream=None):
        assert not self.closed

    def close(self):
        assert not self.closed
        self.closed = True
        FakeSketch.live.discard(id(self))


class Batches(list):
    """The batches the server formed, in order (and the peak number of
    sketches with a restore in flight, as .peak[0])."""


class FakeEvent:
    """Stands in for torch.cuda.Event: the work before it is always done."""

    def __init__(self, enable_timing=False):
        pass

    def record(self, stream=None):
        pass

    def query(self):
        return True


@pytest.fixture
def fake_lib(monkeypatch):
    FakeSketch.live = set()
    batches = Batches()
    inflight = set()          # ids of sketches with a restore begun, not ended
    peak = [0]

    def update_batch(items, stream=None):
        assert all(not sk.closed for sk, _ in items)
        # a sketch is never updated while its last restore is in flight
        assert not inflight & {id(sk) for sk, _ in items}
        batches.append([sk for sk, _ in items])

    def restore_batch(items, stream=None, raise_errors=True):
        assert not raise_errors
        assert [sk for sk, _ in items] == batches[-1]
        return [(np.zeros(0, dtype=ddhf.SP_DTYPE), {"status": ddhf.SKETCH_OK})] * len(items)

    class Pending:
        def __init__(self, items, stream=None):
            assert [sk for sk, _ in items] == batches[-1]
            self.items = items
            inflight.update(id(sk) for sk, _ in items)
            peak[0] = max(peak[0], len(inflight))

        def end(self, raise_errors=True):
            assert not raise_errors
            for sk, _ in self.items:
                inflight.discard(id(sk))
            return [(np.zeros(0, dtype=ddhf.SP_DTYPE), {"status": ddhf.SKETCH_OK})] * \
                len(self.items)

    monkeypatch.setattr(ddhf, "Sketch", FakeSketch)
    monkeypatch.setattr(FakeSketch, "update", lambda sk, pairs: update_batch([(sk, pairs)]),
                        raising=False)
    monkeypatch.setattr(ddhf, "update_batch", update_batch)
    monkeypatch.setattr(ddhf, "restore_batch", restore_batch)
    monkeypatch.setattr(ddhf, "restore_batch_begin", Pending)
    monkeypatch.setattr(serving.torch.cuda, "Stream", lambda device=None: object())
    monkeypatch.setattr(serving.torch.cuda, "Event", FakeEvent)
    monkeypatch.setattr(serving, "concurrent_streams", lambda device, n: [object()] * n)
    batches.peak = peak
    return batches


def one_link_bytes(n_pairs=1000):
    k, alpha = serving.sized_params(n_pairs)
    return serving.resident_bytes(1024, k, 5, alpha)


def test_link_cache_evicts_least_recent_unpinned(fake_lib):
    unit = one_link_bytes()
    links = serving._Links(int(3.5 * unit), 1024, 5, 0)
    a = links.get(0, 1000, {0})
    links.get(1, 1000, {1})
    links.get(2, 1000, {2})
    assert links.used == 3 * unit and len(FakeSketch.live) == 3
    assert links.get(0, 1000, {0}) is a          # resident: no new sketch, now most recent
    assert links.need(0, 1000) == 0 and links.need(3, 1000) == unit
    assert links.fits(unit, {3}) and not links.fits(unit, {0, 1, 2, 3})
    links.get(3, 1000, {3})                        # evicts link 1, the least recent
    assert set(k[0] for k in links.sk) == {0, 2, 3} and links.used == 3 * unit
    links.get(4, 1000, {0, 2, 4})                  # 0 and 2 pinned: evicts 3
    assert set(k[0] for k in links.sk) == {0, 2, 4}
    with pytest.raises(MemoryError):
        links.get(5, 1000, {0, 2, 4, 5})            # nothing left to evict
    # a larger window of the same link is another (link, k) sketch
    big = 1024 * 2**16
    assert serving.sized_params(big)[0] > serving.sized_params(1000)[0]
    assert links.need(0, big) > 0
    links.close()
    assert links.used == 0 and not FakeSketch.live


def requests(n, links, n_pairs=1000, spacing=0.0):
    rng = np.random.default_rng(5)
    return [serving.Request(i, int(rng.integers(0, links)), i * spacing,
                            torch.zeros((n_pairs, 2), dtype=torch.int32))
            for i in range(n)]


@pytest.mark.parametrize("budget_links,max_batch", [(3.5, 64), (100, 4), (1.2, 64)])
def test_continuous_batches_respect_links_budget_and_size(fake_lib, budget_links, max_batch):
    unit = one_link_bytes()
    reqs = requests(40, 8)
    with serving.ContinuousServer(int(budget_links * unit), max_batch=max_batch) as srv:
        used_seen = []
        real_get = srv.links.get

        def get(link, n_pairs, pinned):
            sk = real_get(link, n_pairs, pinned)
            used_seen.append(srv.links.used)
            return sk
        srv.links.get = get
        out = srv.serve(reqs)
    # every request answered once, in rid order, with its link
    assert [r.rid for r in out] == list(range(len(reqs)))
    assert all(r.link == q.link and r.status == ddhf.SKETCH_OK for r, q in zip(out, reqs))
    assert sum(len(b) for b in fake_lib) == len(reqs)
    assert max(used_seen) <= budget_links * unit
    for b in fake_lib:
        assert 1 <= len(b) <= max_batch
        assert len(set(map(id, b))) == len(b)     # one request (one sketch) per link
    # all requests arrive at once: the first batch takes as many links as fit
    first = fake_lib[0]
    assert len(first) == min(max_batch, int(budget_links), len({q.link for q in reqs}))
    assert not FakeSketch.live


def test_requests_of_one_link_keep_arrival_order(fake_lib, monkeypatch):
    reqs = requests(12, 2)
    order = []
    real_response = serving._response

    def response(q, recs, info, done, batch):
        order.append(q.rid)
        return real_response(q, recs, info, done, batch)
    monkeypatch.setattr(serving, "_response", response)
    with serving.ContinuousServer(100 * one_link_bytes()) as srv:
        srv.serve(reqs)
    assert sorted(order) == list(range(12))
    for link in (0, 1):
        rids = [rid for rid in order if reqs[rid].link == link]
        assert rids == sorted(rids)


def test_a_window_larger_than_the_budget_is_refused(fake_lib):
    reqs = requests(2, 1)
    with serving.ContinuousServer(one_link_bytes() // 2) as srv:
        with pytest.raises(MemoryError):
            srv.serve(reqs)


def test_two_batches_in_flight_never_share_a_link(fake_lib, monkeypatch):
    """With two batches in flight, the second is formed from links the
    first does not use, and a link waits until its batch is collected."""
    # completion events say "not done" until the batch was collected, so the
    # server must keep the first batch in flight while it forms the second
    monkeypatch.setattr(FakeEvent, "query", lambda self: False)
    reqs = requests(30, 6)
    with serving.ContinuousServer(100 * one_link_bytes(), max_batch=2) as srv:
        out = srv.serve(reqs)
    assert [r.rid for r in out] == list(range(30))
    # two batches of two sketches were in flight at once; the stand-in
    # update asserts that no batch touched a sketch whose restore was
    # still in flight
    assert fake_lib.peak[0] == 4


def test_plain_server_serves_one_at_a_time(fake_lib):
    reqs = requests(10, 3)
    with serving.PlainServer(2 * one_link_bytes()) as srv:
        out = srv.serve(reqs)
    assert [r.rid for r in out] == list(range(10))
    assert all(len(b) == 1 for b in fake_lib) and len(fake_lib) == 10
    assert all(r.batch == 1 for r in out)


class FakeQueues:
    """Streams on hardware queues in a given order; a pair of spin kernels
    takes 2 units on one queue and 1 on two."""

    def __init__(self, order):
        self.order = list(order)
        self.made = []

    def stream(self, device=None):
        st = type("S", (), {})()
        st.q = self.order[len(self.made) % len(self.order)]
        self.made.append(st)
        return st

    def spin(self, a, b, cycles):
        return 2.0 if a.q == b.q else 1.0


@pytest.mark.parametrize("order", [[0, 1, 2, 3, 3, 2, 1, 0], [2, 2, 2, 1], [0, 0, 0, 0, 0, 3]])
def test_concurrent_streams_skips_streams_on_a_shared_queue(monkeypatch, order):
    fq = FakeQueues(order)
    monkeypatch.setattr(serving, "_CONCURRENT", {})
    monkeypatch.setattr(serving.torch.cuda, "Stream", fq.stream)
    monkeypatch.setattr(serving.torch.cuda, "device", lambda d: contextlib.nullcontext())
    monkeypatch.setattr(serving, "_spin_pair_s", fq.spin)
    a, b = serving.concurrent_streams(0, 2)
    assert a.q != b.q
    # cached: later servers get the same pair without new checks
    made = len(fq.made)
    assert serving.concurrent_streams(0, 2) == [a, b]
    assert len(fq.made) == made


def test_concurrent_streams_gives_up_after_its_tries(monkeypatch):
    fq = FakeQueues([1])                      # one queue: nothing is concurrent
    monkeypatch.setattr(serving, "_CONCURRENT", {})
    monkeypatch.setattr(serving.torch.cuda, "Stream", fq.stream)
    monkeypatch.setattr(serving.torch.cuda, "device", lambda d: contextlib.nullcontext())
    monkeypatch.setattr(serving, "_spin_pair_s", fq.spin)
    streams = serving.concurrent_streams(0, 2, tries=3)
    assert len(streams) == 2 and len(fq.made) == 1 + 3


def test_warm_takes_the_largest_windows_one_per_link_within_budget(fake_lib, monkeypatch):
    """warm() runs one batched update of the largest windows, one per link,
    at most n, only as many as the budget holds at once."""
    monkeypatch.setattr(serving.torch.cuda, "synchronize", lambda dev=None: None)
    restores = []
    monkeypatch.setattr(ddhf, "restore_batch",
                        lambda items, stream=None, raise_errors=True: restores.append(
                            [sk for sk, _ in items]))
    reqs = requests(40, 10)
    with serving.ContinuousServer(4 * one_link_bytes(max(q.n_pairs for q in reqs))) as srv:
        srv.warm(reqs, n=6)
    assert len(fake_lib) == 1                   # one batched update
    batch = fake_lib[0]
    assert 1 <= len(batch) <= 4
    assert len({id(sk) for sk in batch}) == len(batch)
    # their batched restore, then each one alone
    assert restores == [batch] + [[sk] for sk in batch]
