"""Host logic of the autotuner, on the CPU: the candidate settings stay inside
the ranges sketch_set_option accepts, the fastest candidate wins, sketches
past the binned kernels' tile limit get only direct candidates, the restore
tuner offers the lattice search only where it runs (k <= 20) and leaves the
sketch on its best setting, and results are cached by shape and size class
(and theta for the restore). The device queries, the sketch
and the timer are replaced by stand-ins (the GPU tuning test times the real
kernels).
"""
import json

import pytest
import torch

from paper_1803_11449_amd import ddhf, tune

# what sketch_set_option accepts for each option the tuner sets
VALID = {
    "path": lambda v: v in (1, 2),
    "grid": lambda v: 1 <= v <= 1 << 20,
    "check": lambda v: v in (0, 1),
    "ppt": lambda v: v in (2, 4, 6),
    "blocks": lambda v: 1 <= v <= 1024,
    "cand": lambda v: v in (0, 1, 2),
    "jblocks": lambda v: 0 <= v <= 4 * 1024,     # at most four per compute unit
}


@pytest.mark.parametrize("n_cu", [80, 256, 304])
def test_candidates_are_valid_settings(n_cu):
    for binned_ok in (True, False):
        cands = tune.candidates(n_cu, binned_ok)
        assert cands and len({json.dumps(c, sort_keys=True) for c in cands}) == len(cands)
        for c in cands:
            assert set(c) <= set(tune.OPTION)
            assert all(VALID[k](v) for k, v in c.items()), c
        assert any(c["path"] == 2 for c in cands) == binned_ok


def test_size_class_rounds_log2():
    assert [tune.size_class(n) for n in (0, 1, 2, 3, 5, 6, 1 << 20, 3 << 19)] == \
        [0, 0, 1, 2, 2, 3, 20, 21]


class FakeSketch:
    made = []

    def __init__(self, g, k, r, alpha, seed, device=0):
        self.shape, self.opts = (g, k, r, alpha), {}
        FakeSketch.made.append(self)

    def set_option(self, option, value):
        self.opts[option] = value

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        pass


class Props:
    multi_processor_count = 256


@pytest.fixture
def fake_device(monkeypatch, tmp_path):
    FakeSketch.made = []
    timed = []

    def time_update(sk, pairs, trials=3):
        o = {name: sk.opts.get(opt) for name, opt in tune.OPTION.items()}
        timed.append(o)
        # a made-up cost: binned beats direct; 6 pairs per thread and 256 blocks are best
        if o["path"] == 2:
            return 1.0 + abs(o["ppt"] - 6) * 0.1 + abs(o["blocks"] - 256) / 1000
        return 5.0 + o["check"] + 256 / o["grid"]

    monkeypatch.setattr(tune, "CACHE", str(tmp_path / "tune.json"))
    monkeypatch.setattr(tune, "time_update", time_update)
    monkeypatch.setattr(ddhf, "Sketch", FakeSketch)
    monkeypatch.setattr(torch.cuda, "get_device_name", lambda dev=None: "Test GPU")
    monkeypatch.setattr(torch.cuda, "get_device_properties", lambda dev=None: Props())
    return timed


def test_fastest_setting_is_kept_and_cached(fake_device):
    timed = fake_device
    pairs = torch.zeros((3 << 20, 2), dtype=torch.int32)
    best = tune.tune(1024, 18, 5, 5, pairs)
    assert (best["path"], best["ppt"], best["blocks"]) == (2, 6, 256)
    assert best["ms"] == pytest.approx(1.0)
    n_cands = len(tune.candidates(256, True))
    assert len(timed) == n_cands
    db = json.load(open(tune.CACHE))
    assert list(db) == ["Test_GPU/g1024_k18_r5_a5/n2^22"] and db[list(db)[0]] == best
    # the same shape and size class: from the cache, nothing timed
    again = tune.tune(1024, 18, 5, 5, torch.zeros((3 << 20) + 5, 2, dtype=torch.int32))
    assert again == best and len(timed) == n_cands
    # another size class is tuned afresh and cached beside the first
    tune.tune(1024, 18, 5, 5, torch.zeros((1 << 20, 2), dtype=torch.int32))
    assert len(timed) == 2 * n_cands and len(json.load(open(tune.CACHE))) == 2


def test_apply_sets_each_named_option(fake_device):
    sk = FakeSketch(1024, 14, 5, 6, 0)
    tune.apply(sk, {"ms": 0.5, "path": 2, "ppt": 4, "blocks": 128})
    assert sk.opts == {ddhf.SKETCH_OPT_UPDATE_PATH: 2, ddhf.SKETCH_OPT_SCATTER_PPT: 4,
                       ddhf.SKETCH_OPT_BINNED_BLOCKS: 128}


def test_past_the_tile_limit_only_direct_settings(fake_device):
    """g = 65536, k = 14, r = 5: 5 * 2^14 LEs of 2^16 bits = 640 MiB, 4096
    tiles of 160 KiB, more than the binned kernels' 3276."""
    timed = fake_device
    best = tune.tune(65536, 14, 5, 6, torch.zeros((1000, 2), dtype=torch.int32), use_cache=False)
    assert best["path"] == 1 and all(o["path"] == 1 for o in timed)
    assert len(timed) == len(tune.candidates(256, False))


@pytest.mark.parametrize("n_cu", [80, 256, 304])
@pytest.mark.parametrize("k", [14, 20, 21])
def test_restore_candidates_are_valid_settings(n_cu, k):
    cands = tune.restore_candidates(n_cu, k)
    assert len({json.dumps(c, sort_keys=True) for c in cands}) == len(cands)
    for c in cands:
        assert set(c) <= set(tune.OPTION)
        assert all(VALID[name](v) for name, v in c.items()), c
        assert c["jblocks"] <= 4 * n_cu
    assert any(c["cand"] == 2 for c in cands) == (k <= 20)
    assert any(c["cand"] == 1 for c in cands)


class RestoreSketch:
    def __init__(self, k):
        self.params = ddhf.sketch_params_t(1024, k, 5, 5, 1, 0)
        self.device = 0
        self.opts = {}
        self.restores = 0

    def set_option(self, option, value):
        self.opts[option] = value

    def restore(self, theta):
        self.restores += 1


@pytest.mark.parametrize("k,lattice_fast", [(18, True), (18, False), (21, False)])
def test_tune_restore_picks_the_fastest_and_keeps_it(monkeypatch, tmp_path, k, lattice_fast):
    monkeypatch.setattr(tune, "CACHE", str(tmp_path / "tune.json"))
    monkeypatch.setattr(torch.cuda, "get_device_name", lambda dev=None: "Test GPU")
    monkeypatch.setattr(torch.cuda, "get_device_properties", lambda dev=None: Props())

    def time_restore(sk, theta, trials=3):
        cand = sk.opts[ddhf.SKETCH_OPT_CANDIDATES]
        jb = sk.opts[ddhf.SKETCH_OPT_JOIN_BLOCKS]
        if cand == 2:
            return 0.1 if lattice_fast else 0.9
        return 0.3 + abs(jb - 512) / 10000        # the join is best at 512 blocks

    monkeypatch.setattr(tune, "time_restore", time_restore)
    sk = RestoreSketch(k)
    best = tune.tune_restore(sk, 512.0, 1 << 20)
    want = {"cand": 2, "jblocks": 0} if (lattice_fast and k <= 20) else {"cand": 1, "jblocks": 512}
    assert {n: best[n] for n in ("cand", "jblocks")} == want
    assert sk.opts == {ddhf.SKETCH_OPT_CANDIDATES: want["cand"],
                       ddhf.SKETCH_OPT_JOIN_BLOCKS: want["jblocks"]}
    # cached per theta: the same key skips the sweep, another theta does not
    calls = []
    monkeypatch.setattr(tune, "time_restore", lambda sk, th, trials=3: calls.append(th) or 1.0)
    again = RestoreSketch(k)
    assert tune.tune_restore(again, 512.0, (1 << 20) + 7) == best and not calls
    assert again.opts[ddhf.SKETCH_OPT_CANDIDATES] == want["cand"]
    tune.tune_restore(RestoreSketch(k), 1024.0, 1 << 20)
    assert calls
