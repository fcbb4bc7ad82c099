"""Autotuner for the update's and the restore's launch options
(sketch_set_option).

For one sketch shape (g, k, r, alpha) and one window size it times the
update under each candidate setting on the device and keeps the fastest:

  direct   UPDATE_GRID (blocks) x UPDATE_CHECK (test the bit first or not)
  binned   SCATTER_PPT (pairs per thread per LDS batch) x BINNED_BLOCKS
           (blocks of the count and scatter passes)

and whether the window takes the direct or the binned kernels. Each
setting is timed with HIP events on the stream the update runs on, as the
median of a few updates of the same pairs into a freshly reset sketch.

For the restore of a window at one theta it times the candidate search
each way: the join of Algs. 3-4 at JOIN_BLOCKS of one, two or four per
compute unit, and the lattice search (k <= 20), as the host time from the
call to the list, the median of a few restores of the same sketch. Both
searches give the same candidates; the choice only moves time.

Results are cached in a JSON file keyed by device name, shape and size
class (the window size rounded to a power of two; for the restore also
theta), so a process pays for a sweep once per key.
"""
from __future__ import annotations

import json
import math
import os
import statistics
import time

import torch

from . import ddhf

CACHE = os.environ.get("DDHF_TUNE_CACHE",
                       os.path.join(os.path.expanduser("~"), ".cache", "ddhf", "tune.json"))

OPTION = {"path": ddhf.SKETCH_OPT_UPDATE_PATH, "grid": ddhf.SKETCH_OPT_UPDATE_GRID,
          "check": ddhf.SKETCH_OPT_UPDATE_CHECK, "ppt": ddhf.SKETCH_OPT_SCATTER_PPT,
          "blocks": ddhf.SKETCH_OPT_BINNED_BLOCKS, "cand": ddhf.SKETCH_OPT_CANDIDATES,
          "jblocks": ddhf.SKETCH_OPT_JOIN_BLOCKS}


def size_class(n_pairs: int) -> int:
    return max(0, round(math.log2(max(1, n_pairs))))


def _key(dev: int, g, k, r, alpha, n_pairs) -> str:
    name = torch.cuda.get_device_name(dev).replace(" ", "_")
    return f"{name}/g{g}_k{k}_r{r}_a{alpha}/n2^{size_class(n_pairs)}"


def candidates(n_cu: int, binned_ok: bool) -> list:
    out = [{"path": 1, "grid": n_cu * m, "check": c} for m in (4, 8, 16) for c in (1, 0)]
    if binned_ok:
        out += [{"path": 2, "ppt": ppt, "blocks": b}
                for ppt in (2, 4, 6) for b in (n_cu // 2, n_cu, 2 * n_cu)]
    return out


def restore_candidates(n_cu: int, k: int) -> list:
    out = [{"cand": 1, "jblocks": n_cu * m} for m in (1, 2, 4)]
    if k <= 20:
        out.append({"cand": 2, "jblocks": 0})
    return out


def apply(sk: ddhf.Sketch, opts: dict) -> None:
    """Set a tuned setting on a sketch (options not named keep their value)."""
    for name, v in opts.items():
        if name in OPTION:
            sk.set_option(OPTION[name], int(v))


def time_update(sk: ddhf.Sketch, pairs: torch.Tensor, trials: int = 3) -> float:
    """Median milliseconds of one update of pairs into the reset sketch."""
    stream = torch.cuda.current_stream(pairs.device)
    ts = []
    for _ in range(trials + 1):
        sk.reset(stream)
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(stream)
        sk.update(pairs, stream)
        b.record(stream)
        b.synchronize()
        ts.append(a.elapsed_time(b))
    return statistics.median(ts[1:])        # the first run warms caches and buffers


def _load() -> dict:
    try:
        with open(CACHE) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _save(db: dict) -> None:
    try:
        os.makedirs(os.path.dirname(CACHE), exist_ok=True)
        tmp = CACHE + f".{os.getpid()}"
        with open(tmp, "w") as f:
            json.dump(db, f, indent=1, sort_keys=True)
        os.replace(tmp, CACHE)
    except OSError:
        pass                                 # a read-only home: tune again next time


def tune(g: int, k: int, r: int, alpha: int, pairs: torch.Tensor, seed: int = ddhf.DEFAULT_SEED,
         trials: int = 3, use_cache: bool = True) -> dict:
    """The fastest setting for windows like `pairs` (int32 [n, 2] on the
    device) on a (g, k, r, alpha) sketch: {"ms": ..., option: value, ...}."""
    dev = pairs.device.index or 0
    key = _key(dev, g, k, r, alpha, pairs.shape[0])
    db = _load() if use_cache else {}
    if key in db:
        return db[key]
    n_cu = torch.cuda.get_device_properties(dev).multi_processor_count
    words = (r << k) * g // 32
    binned_ok = -(-words // 40960) <= 3276             # the binned kernels' limit: 160 KiB tiles
    best = None
    with ddhf.Sketch(g, k, r, alpha, seed, device=dev) as sk:
        for opts in candidates(n_cu, binned_ok):
            apply(sk, opts)
            ms = time_update(sk, pairs, trials)
            if best is None or ms < best["ms"]:
                best = {"ms": round(ms, 5), **opts}
    db = _load()
    db[key] = best
    if use_cache:
        _save(db)
    return best


def time_restore(sk: ddhf.Sketch, theta: float, trials: int = 3) -> float:
    """Median milliseconds from the restore call to the list on the host."""
    ts = []
    for _ in range(trials + 1):
        torch.cuda.synchronize(sk.device)
        t0 = time.perf_counter()
        sk.restore(theta)
        ts.append((time.perf_counter() - t0) * 1e3)
    return statistics.median(ts[1:])        # the first run grows buffers


def tune_restore(sk: ddhf.Sketch, theta: float, n_pairs: int, trials: int = 5,
                 use_cache: bool = True) -> dict:
    """The fastest candidate search for windows like the one sk holds now
    (updated, not reset) at theta: {"ms": ..., "cand": ..., "jblocks": ...}.
    The sketch keeps the best setting."""
    p = sk.params
    key = _key(sk.device, p.g, p.k, p.r, p.alpha, n_pairs) + f"/restore_theta{theta:g}"
    db = _load() if use_cache else {}
    if key in db:
        apply(sk, db[key])
        return db[key]
    n_cu = torch.cuda.get_device_properties(sk.device).multi_processor_count
    best = None
    for opts in restore_candidates(n_cu, p.k):
        apply(sk, opts)
        ms = time_restore(sk, theta, trials)
        if best is None or ms < best["ms"]:
            best = {"ms": round(ms, 5), **opts}
    apply(sk, best)
    db = _load()
    db[key] = best
    if use_cache:
        _save(db)
    return best
