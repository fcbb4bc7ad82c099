"""Benchmark: one DDHF window end to end on one MI355X.

A step is the whole hot path over one window: reset the sketch, stream the
window's (src,dst) pairs into it (Alg. 1), restore the super points
(Alg. 2 / Algs. 3-4 / eq. (4)) and hand the list to the host. The window is
the 100M-pair large window (Zipf(1.0) over 4M sources, 500 planted super
points log-uniform in [1024, 50000], 50 sequential scanners, 10% duplicate
pairs, theta = 1024) on a k = 18, alpha = 5 sketch (160 MiB); the pairs are
generated on the device and are resident in HBM before timing starts.

Prints one JSON line. value = pairs per second over the whole step (reset +
update + restore, wall clock, inputs in HBM), in Mpps. Also reported: the
update's own rate (HIP events around it in the timed steps), the restore
latency (window close to super point list on the host) p50/p99 over
separate runs after the timed steps, each started on an idle device, the
roofline of the dominant kernel and the CPU oracle's rate on the same
window.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "sketch update Mpps + restore ms/window; p50/p99 window-to-report latency"
HBM_PEAK_GBS = 8000.0     # MI355X HBM3E, published
PAIR_BYTES = 8


def sized_k(n_pairs: int, g: int = 1024) -> tuple[int, int]:
    """Smallest k >= 14 with n/(g 2^k) <= 0.45; alpha = ceil((32-k)/(r-2)), r=5."""
    k = 14
    while n_pairs / (g * 2**k) > 0.45:
        k += 1
    return k, math.ceil((32 - k) / 3)


TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "large_window_100m_hbm_traffic.md")
UPDATE_SRC = os.path.join(ROOT, "paper_1803_11449_amd", "csrc", "update.hip")


def measured_update_traffic():
    """HBM bytes of one 100M-pair update from the committed counter profile,
    or None if the update source changed since the counters were taken."""
    import hashlib
    try:
        text = open(TRAFFIC_PROFILE).read()
        src = hashlib.sha256(open(UPDATE_SRC, "rb").read()).hexdigest()[:16]
    except OSError:
        return None
    vals = dict(line.split(": ", 1) for line in text.splitlines() if ": " in line
                and line.split(": ", 1)[0] in ("update_traffic_bytes", "update_source_sha256"))
    if vals.get("update_source_sha256", "").strip() != src:
        return None
    return float(vals["update_traffic_bytes"])


def percentile(xs, q):
    xs = sorted(xs)
    if not xs:
        return float("nan")
    i = min(len(xs) - 1, max(0, int(math.ceil(q / 100 * len(xs))) - 1))
    return xs[i]


def cpu_threads() -> int:
    env = os.environ.get("OMP_NUM_THREADS")
    n = len(os.sched_getaffinity(0))
    if env and env.isdigit():
        n = min(n, int(env))
    return max(1, min(n, 16))


def cpu_baseline_leg(pairs, shape, theta, n_sample, threads):
    """The oracle as it stands on the host, over the first n_sample pairs
    of the window (pairs: int32 [n, 2] tensor on the device):
      update      Alg. 1, sequential loop, 1 thread
      update_omp  the same on `threads` threads (atomic OR after the test)
      restore     candidates by scanning all 2^32 addresses on `threads`
                  threads, eq. (4) estimates
    value = sample pairs / (update_omp + restore) seconds, the whole job on
    `threads` host threads (cores)."""
    import numpy as np
    import oracle
    from paper_1803_11449_amd import traffic
    host = pairs[:n_sample].cpu().numpy().view(np.uint32).reshape(-1)
    g, k, r, alpha = shape
    p = oracle.Params(g, k, r, alpha, traffic.HASH_SEED)
    t0 = time.perf_counter()
    sk1 = oracle.build_sketch(p, host)
    t1 = time.perf_counter()
    skn = oracle.update_omp(p, oracle.new_sketch(p), host, nthreads=threads)
    t2 = time.perf_counter()
    same = bool(np.array_equal(sk1, skn))
    del sk1
    try:
        oracle.restore(p, skn, theta, mode="brute", nthreads=threads)
    except oracle.OracleError:
        pass
    t3 = time.perf_counter()
    return {
        "value": round(n_sample / ((t2 - t1) + (t3 - t2)) / 1e6, 3), "unit": "Mpps",
        "cores": threads, "kind": "oracle",
        "sample": (f"first {n_sample} pairs of the same window: Alg. 1 on {threads} threads "
                   f"{t2 - t1:.2f} s, restore by 2^32 scan on {threads} threads {t3 - t2:.2f} s; "
                   f"Alg. 1 on 1 thread {t1 - t0:.2f} s"),
        "legs": {"update_1thread": {"threads": 1, "s": round(t1 - t0, 3),
                                    "mpps": round(n_sample / (t1 - t0) / 1e6, 2)},
                 "update_omp": {"threads": threads, "s": round(t2 - t1, 3),
                                "mpps": round(n_sample / (t2 - t1) / 1e6, 2),
                                "same_sketch_as_1thread": same},
                 "restore_2to32_scan": {"threads": threads, "s": round(t3 - t2, 3)}},
    }


def direct_kernel_rate(ddhf, traffic, pairs, shape, stream):
    """The direct update kernel with its bit test off issues exactly one
    global atomicOr per (pair, row): its rate on this window is the random
    global-atomic throughput of the chip for this sketch size. It is a
    measured reference, not a ceiling of the binned update, which moves
    every bit set into LDS."""
    import torch
    g, k, r, alpha = shape
    sk = ddhf.Sketch(g, k, r, alpha, traffic.HASH_SEED, device=0)
    sk.set_option(ddhf.SKETCH_OPT_UPDATE_PATH, 1)
    sk.set_option(ddhf.SKETCH_OPT_UPDATE_CHECK, 0)
    ms = []
    for i in range(4):
        sk.reset()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(stream)
        sk.update(pairs)
        b.record(stream)
        b.synchronize()
        if i:
            ms.append(a.elapsed_time(b))
    sk.close()
    n = pairs.shape[0]
    rate = n / (sorted(ms)[len(ms) // 2] / 1e3) / 1e6
    return {"kind": "direct kernel, one global atomicOr per (pair, row), bit test off",
            "atomics_per_s": round(rate * 1e6 * r, 1), "mpps": round(rate, 2)}


# LDS of one compute unit: 32 banks of 4 bytes, one access per bank per
# clock (a wave's 64 lanes in two halves), at the 2.4 GHz peak clock
LDS_LANE_OPS_PEAK = 256 * 32 * 2.4e9
# LDS lane operations per join output and per probe, counted in k_join:
# per probe the two bucket-offset reads; per output slot the owner write and
# read, three ds_bpermute, the entry's top-bits read and the append counter
JOIN_LDS_OPS_PER_OUTPUT = 6
JOIN_LDS_OPS_PER_PROBE = 2
# Integer vector ALU of the chip: 256 compute units, 4 SIMDs of 16 lanes
# each, one 32-bit operation per lane per clock, at 2.4 GHz
VALU_LANE_OPS_PEAK = 256 * 4 * 16 * 2.4e9
# The lattice search's integer operations per address walked: the step to
# the next address, its row-1 LE (xor, and), the LE's bitmap word (shift),
# the bit's test (shift, and)
LATTICE_OPS_PER_POINT = 6


def restore_roofline(timings: list) -> dict:
    """Restore-side rooflines from the phase timings of the latency runs
    (median of each phase): the hot scan against HBM bandwidth; the
    candidate search, the lattice walk's integer operations against the
    vector ALU peak or the join's LDS lane operations against the LDS peak;
    the estimate's LE gathers against HBM bandwidth."""
    med = {k: percentile([t[k] for t in timings], 50) for k in timings[0]}
    hs = med["hot_scan_bytes"] / (med["hot_scan_ms"] / 1e3) / 1e9
    eg = med["estimate_bytes"] / (med["estimate_ms"] / 1e3) / 1e9
    search_s = med["join_ms"] / 1e3
    if int(med["search"]) == 2:
        ops = LATTICE_OPS_PER_POINT * med["lattice_points"] / search_s
        search = {"kind": "lattice", "bound": "alu", "points": int(med["lattice_points"]),
                  "outputs": int(med["join_outputs"]),
                  "points_per_s": round(med["lattice_points"] / search_s, 1),
                  "achieved": round(ops / 1e12, 4),
                  "peak": round(VALU_LANE_OPS_PEAK / 1e12, 2),
                  "unit": "T int32 lane-ops/s", "frac": round(ops / VALU_LANE_OPS_PEAK, 5)}
    else:
        lds_ops = (JOIN_LDS_OPS_PER_OUTPUT * med["join_outputs"] +
                   JOIN_LDS_OPS_PER_PROBE * med["join_probes"])
        jr = lds_ops / search_s
        search = {"kind": "join", "bound": "lds", "probes": int(med["join_probes"]),
                  "outputs": int(med["join_outputs"]),
                  "probes_per_s": round(med["join_probes"] / search_s, 1),
                  "achieved": round(jr / 1e12, 4), "peak": round(LDS_LANE_OPS_PEAK / 1e12, 2),
                  "unit": "T LDS lane-ops/s", "frac": round(jr / LDS_LANE_OPS_PEAK, 5)}
    return {
        "phase_ms": {k: round(med[k], 4) for k in ("hot_scan_ms", "rows_ms", "join_ms",
                                                     "estimate_ms", "sort_publish_ms")},
        "hot_scan": {"bound": "hbm", "bytes": int(med["hot_scan_bytes"]),
                     "achieved": round(hs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(hs / HBM_PEAK_GBS, 5)},
        "candidate_search": search,
        "estimate": {"bound": "hbm", "bytes": int(med["estimate_bytes"]),
                     "achieved": round(eg, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(eg / HBM_PEAK_GBS, 5)},
    }


def headline(args, dev) -> dict:
    """The 100M-pair window: timed steps, update events, restore latency
    with phase timings, rooflines, the direct kernel's atomic rate and the
    CPU baseline. Returns the JSON line's fields."""
    import torch
    from paper_1803_11449_amd import ddhf, traffic
    spec = traffic.spec_large_window_100m(args.pairs)
    k, alpha = sized_k(spec.n_pairs)
    g, r = 1024, 5
    log(f"generating {spec.n_pairs} pairs on {dev}")
    w = traffic.generate(spec, traffic.config_seed(2), device=dev)
    pairs = w.pairs
    torch.cuda.synchronize()

    if args.copy_calibration:
        n = args.copy_calibration * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.int32, device=dev)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    sk = ddhf.Sketch(g, k, r, alpha, traffic.HASH_SEED, device=0)
    if args.update_path:
        sk.set_option(ddhf.SKETCH_OPT_UPDATE_PATH, args.update_path)
    stream = torch.cuda.current_stream(dev)
    n = spec.n_pairs

    def step(record=None):
        """Reset, update, restore: what a monitor does per window. The update
        is bracketed by events on its stream (no wait); the restore returns
        with the list on the host."""
        sk.reset()
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        ev0.record(stream)
        sk.update(pairs)
        ev1.record(stream)
        recs, info = sk.restore(args.theta)
        if record is not None:
            record["events"].append((ev0, ev1))
            record["n_sp"] = len(recs)
            record["info"] = info
        return recs

    def latency_step(record):
        """Window close to report: the restore alone, timed from the moment
        every pair of the window is in the sketch (its phases timed by the
        library's events)."""
        sk.reset()
        sk.update(pairs)
        torch.cuda.synchronize()
        t_close = time.perf_counter()
        sk.restore(args.theta)
        record["restore_ms"].append((time.perf_counter() - t_close) * 1e3)
        record["phases"].append(ddhf.sketch_timings(sk.handle))

    log("warmup")
    for _ in range(args.warmup):
        step()
    # the restore's candidate search as the autotuner picks it for this
    # window (the sketch holds the window after the warmup)
    from paper_1803_11449_amd import tune
    rtuned = tune.tune_restore(sk, args.theta, n, use_cache=False)
    log(f"restore tuned: {rtuned}")

    # the monitor's loop: two sketches and two streams, so window w+1 is
    # reset and updated while window w's restore runs (Sec. 4's cycle:
    # each period's data comes in while the last period is processed); a
    # step still takes every pair of its window through update and restore
    # to the list on the host
    from paper_1803_11449_amd import serving
    sk2 = ddhf.Sketch(g, k, r, alpha, traffic.HASH_SEED, device=0)
    if args.update_path:
        sk2.set_option(ddhf.SKETCH_OPT_UPDATE_PATH, args.update_path)
    tune.apply(sk2, rtuned)
    pipe = [sk, sk2]
    streams = serving.concurrent_streams(0, 2)

    def piped_steps(steps, record=None):
        pending = None
        for i in range(steps):
            s_, st_ = pipe[i % 2], streams[i % 2]
            s_.reset(st_)
            s_.update(pairs, st_)
            nxt = ddhf.restore_batch_begin([(s_, args.theta)], st_)
            if pending is not None:
                recs, info = pending.end()[0]
                if record is not None:
                    record["piped_sp"] = len(recs)
            pending = nxt
        recs, info = pending.end()[0]
        if record is not None:
            record["piped_sp"] = len(recs)

    piped_steps(max(2, args.warmup))
    rec = {"events": [], "restore_ms": [], "phases": []}
    # as a serving loop would, keep Python's cycle collector out of the
    # timed loops (reference counting still frees what they drop)
    import gc
    gc.collect()
    gc.disable()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    piped_steps(args.steps, rec)
    torch.cuda.synchronize()
    total = time.perf_counter() - t0
    log(f"{args.steps} pipelined steps in {total:.3f} s")
    # the same steps one after another on one stream (no overlap); the
    # update's events come from these, where nothing runs beside it
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step(rec)
    torch.cuda.synchronize()
    serial = time.perf_counter() - t0
    sk2.close()
    assert rec["piped_sp"] == rec["n_sp"], "pipelined and serial lists differ in length"
    rec["update_ms"] = [a.elapsed_time(b) for a, b in rec["events"]]
    # 200 latency samples at the default 50 steps, so that p99 is not the
    # maximum of a few dozen
    sk.set_option(ddhf.SKETCH_OPT_TIMING, 1)
    for _ in range(max(20, min(4 * args.steps, 200))):
        latency_step(rec)
    sk.set_option(ddhf.SKETCH_OPT_TIMING, 0)
    gc.enable()

    ms_per_step = total / args.steps * 1e3
    upd_ms = percentile(rec["update_ms"], 50)
    upd_mean = sum(rec["update_ms"]) / len(rec["update_ms"])
    update_mpps = n / (upd_mean / 1e3) / 1e6
    achieved = n * PAIR_BYTES / (upd_mean / 1e3) / 1e9
    info = rec["info"]
    hbm_traffic = measured_update_traffic() if n == 100_000_000 else None
    out = {
        "metric": METRIC,
        "value": round(n * args.steps / total / 1e6, 3),
        "unit": "Mpps",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": "large_window_100m", "n_pairs": n, "g": g, "k": k,
                   "r": r, "alpha": alpha, "theta": args.theta,
                   "zipf_s": spec.zipf_s, "sources": spec.n_sources,
                   "planted": len(spec.planted_card), "scanners": spec.n_scanners,
                   "dup_frac": spec.dup_frac},
        "update_mpps": round(update_mpps, 2),
        "update_ms_p50": round(upd_ms, 4),
        "restore_ms_p50": round(percentile(rec["restore_ms"], 50), 4),
        "restore_ms_p99": round(percentile(rec["restore_ms"], 99), 4),
        "latency_ms_p50": round(percentile(rec["restore_ms"], 50), 4),
        "latency_ms_p99": round(percentile(rec["restore_ms"], 99), 4),
        "latency_samples": len(rec["restore_ms"]),
        "super_points": rec["n_sp"],
        "candidates": info["n_candidates"],
        "he_count": info["he_count"][:r],
        "psi": round(info["psi"], 6),
        "roofline": {"kernel": "sketch_update (k_bin_count, k_bin_scan_cols, "
                               "k_bin_layout, k_bin_scatter, k_bin_items, "
                               "k_item_offsets, k_bin_apply, k_bin_merge)",
                     "bound": "hbm",
                     "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 5),
                     "traffic": hbm_traffic},
        "restore_roofline": restore_roofline(rec["phases"]),
        "restore_tuned": rtuned,
        "serial_ms_per_step": round(serial / args.steps * 1e3, 4),
        "serial_mpps": round(n * args.steps / serial / 1e6, 3),
    }
    if hbm_traffic:
        out["roofline"]["traffic_gbs"] = round(hbm_traffic / (upd_mean / 1e3) / 1e9, 1)
    out["direct_kernel_atomics"] = direct_kernel_rate(ddhf, traffic, pairs, (g, k, r, alpha),
                                                      stream)
    sk.close()
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        out["cpu_baseline"] = cpu_baseline_leg(pairs, (g, k, r, alpha), args.theta,
                                               min(args.cpu_sample, n), cpu_threads())
    del pairs, w
    torch.cuda.empty_cache()
    return out


def config1_oracle_leg(pairs, gpu_recs) -> dict:
    """The oracle on one host thread over the whole 1M-pair window: Alg. 1
    as a sequential loop, then Alg. 2's restore with the candidates from
    the join of Algs. 3-4 (the paper's own restore, not the 2^32 scan),
    and whether its list equals the GPU's."""
    import numpy as np
    import oracle
    from paper_1803_11449_amd import traffic
    host = pairs.cpu().numpy().view(np.uint32).reshape(-1)
    p = oracle.Params(1024, 14, 5, 6, traffic.HASH_SEED)
    t0 = time.perf_counter()
    sk = oracle.build_sketch(p, host)
    t1 = time.perf_counter()
    ip, sz, _, _ = oracle.restore(p, sk, 1024.0, mode="join", nthreads=1)
    t2 = time.perf_counter()
    same = bool(np.array_equal(ip, gpu_recs["ip"]) and np.array_equal(sz, gpu_recs["sz"]))
    return {"kind": "oracle", "threads": 1, "update_s": round(t1 - t0, 4),
            "restore_join_s": round(t2 - t1, 4),
            "step_mpps": round(len(host) / 2 / (t2 - t0) / 1e6, 3),
            "same_list_as_gpu": same}


def config1_run(args, dev) -> dict:
    """The 1M-pair single window on the default sketch, with the update and
    the restore tuned for it first (as the other workloads are): update
    rate (HIP events, median of 30), restore latency (window close to list
    on the host) and whole steps."""
    import torch
    from paper_1803_11449_amd import ddhf, traffic, tune
    w = traffic.generate(traffic.spec_single_window_1m(), traffic.config_seed(1), device=dev)
    stream = torch.cuda.current_stream(dev)
    n = w.pairs.shape[0]
    upd, lat = [], []
    utuned = tune.tune(1024, 14, 5, 6, w.pairs, traffic.HASH_SEED, use_cache=False)
    with ddhf.Sketch(1024, 14, 5, 6, traffic.HASH_SEED, device=0) as sk:
        tune.apply(sk, utuned)
        sk.update(w.pairs)
        rtuned = tune.tune_restore(sk, 1024.0, n, use_cache=False)
        for i in range(33):
            sk.reset()
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record(stream)
            sk.update(w.pairs)
            b.record(stream)
            b.synchronize()
            t = time.perf_counter()
            recs, _ = sk.restore(1024.0)
            if i >= 3:
                upd.append(a.elapsed_time(b))
                lat.append((time.perf_counter() - t) * 1e3)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(30):
            sk.reset()
            sk.update(w.pairs)
            sk.restore(1024.0)
        step = (time.perf_counter() - t0) / 30
    out = {}
    if not args.no_cpu_baseline:
        out["cpu_oracle"] = config1_oracle_leg(w.pairs, recs)
    return {"workload": "single_window_1m", "n_pairs": n, "g": 1024, "k": 14, "r": 5,
            "alpha": 6, "theta": 1024.0, **out,
            "update_ms_p50": round(percentile(upd, 50), 4),
            "update_mpps": round(n / (percentile(upd, 50) / 1e3) / 1e6, 1),
            "restore_ms_p50": round(percentile(lat, 50), 4),
            "restore_ms_p99": round(percentile(lat, 99), 4),
            "step_ms": round(step * 1e3, 4), "step_mpps": round(n / step / 1e6, 1),
            "super_points": len(recs), "update_tuned": utuned, "restore_tuned": rtuned}


def stream_run(args, dev) -> dict:
    """The sustained stream: consecutive windows of 117M pairs (Zipf(1.0)
    over 8M sources, 1000 planted with 20% replaced each window), each
    generated on the device from its own seed before timing, then processed
    back to back on one k = 18 sketch: reset, update, restore with the list
    on the host; then the same windows double-buffered on two sketches and
    two streams. Sustained rates against the 117 Mpps line rate (750 Gb/s
    at 800-byte packets)."""
    import torch
    from paper_1803_11449_amd import ddhf, traffic
    nw = args.stream_windows
    wins = []
    t0 = time.perf_counter()
    for i in range(nw):
        wins.append(traffic.generate(traffic.spec_stream_window(i), traffic.config_seed(3, i),
                                     device=dev).pairs)
        if i % 10 == 9 or i == nw - 1:
            torch.cuda.synchronize()
            log(f"stream: {i + 1} of {nw} windows generated ({time.perf_counter() - t0:.1f} s)")
    n = wins[0].shape[0]
    k, alpha = sized_k(n)
    sps = []
    with ddhf.Sketch(1024, k, 5, alpha, traffic.HASH_SEED, device=0) as sk:
        for p in wins[:2]:                                  # warm up
            sk.reset()
            sk.update(p)
            sk.restore(1024.0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for p in wins:
            sk.reset()
            sk.update(p)
            recs, _ = sk.restore(1024.0)
            sps.append(len(recs))
        dt = time.perf_counter() - t0
    # the same windows double-buffered, as a monitor would run them: two
    # sketches on two streams, window w+1 reset and updated while window w
    # restores (the headline step's pipelining)
    from paper_1803_11449_amd import serving
    streams = serving.concurrent_streams(0, 2)
    piped_sps = []
    with ddhf.Sketch(1024, k, 5, alpha, traffic.HASH_SEED, device=0) as s0, \
            ddhf.Sketch(1024, k, 5, alpha, traffic.HASH_SEED, device=0) as s1:
        pipe = [s0, s1]

        def piped(ws, out):
            pending = None
            for i, p in enumerate(ws):
                s_, st_ = pipe[i % 2], streams[i % 2]
                s_.reset(st_)
                s_.update(p, st_)
                nxt = ddhf.restore_batch_begin([(s_, 1024.0)], st_)
                if pending is not None:
                    out.append(len(pending.end()[0][0]))
                pending = nxt
            out.append(len(pending.end()[0][0]))

        piped(wins[:2], [])                                 # warm up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        piped(wins, piped_sps)
        torch.cuda.synchronize()
        dt_piped = time.perf_counter() - t0
    assert piped_sps == sps, "pipelined and serial stream lists differ in length"
    del wins
    torch.cuda.empty_cache()
    total = n * nw
    return {"workload": "stream_117m_windows", "windows": nw, "pairs_per_window": n,
            "k": k, "alpha": alpha, "theta": 1024.0,
            "sustained_mpps": round(total / dt / 1e6, 1),
            "line_rate_mpps": 117.0,
            "x_line_rate": round(total / dt / 1e6 / 117.0, 1),
            "ms_per_window": round(dt / nw * 1e3, 4),
            "pipelined_mpps": round(total / dt_piped / 1e6, 1),
            "pipelined_x_line_rate": round(total / dt_piped / 1e6 / 117.0, 1),
            "pipelined_ms_per_window": round(dt_piped / nw * 1e3, 4),
            "super_points_mean": round(sum(sps) / len(sps), 1)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--pairs", type=int, default=100_000_000)
    ap.add_argument("--theta", type=float, default=1024.0)
    ap.add_argument("--cpu-sample", type=int, default=100_000_000,
                    help="pairs of the window the oracle baseline processes")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--update-path", type=int, default=0, choices=(0, 1, 2),
                    help="0 = library's choice by size, 1 = direct, 2 = binned")
    ap.add_argument("--workload", default="large_window_100m",
                    choices=("large_window_100m", "batched_64_links", "serving_256_links"),
                    help="large_window_100m (default, the headline); batched_64_links: 64 "
                         "links of uneven windows in one batched launch vs one launch per "
                         "window; serving_256_links: Poisson window closes from 256 links, "
                         "continuous batching vs one window at a time")
    ap.add_argument("--extras", default="config1,stream,batched,serving",
                    help="sub-objects of the default line (comma list; empty for none)")
    ap.add_argument("--stream-windows", type=int, default=60)
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="also run one plain device copy of this many MiB "
                         "(for scaling HBM counters)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(the sketch would shard by an OR all-reduce, not built here).",
              file=sys.stderr)
        sys.exit(2)

    import torch

    dev = torch.device("cuda:0")
    if args.workload == "batched_64_links":
        b = batched_run(args, dev)
        return _line(b.pop("plan_mpps"), b.pop("steps"), args.warmup, b.pop("plan_ms_per_step"),
                     b.pop("config"), b)
    if args.workload == "serving_256_links":
        s = serving_run(args, dev)
        ov = s["runs"]["overload_40gpps_continuous"]
        return _line(ov["served_mpps"], 1, 0, ov["span_s"] * 1e3, s.pop("config"),
                     {"latency_ms_p50": ov["latency_ms_p50"],
                      "latency_ms_p99": ov["latency_ms_p99"], "runs": s["runs"]})

    out = headline(args, dev)
    extras = [x for x in args.extras.split(",") if x]
    for name, fn in (("config1", config1_run), ("stream", stream_run),
                     ("batched", batched_run), ("serving", serving_run)):
        if name in extras:
            log(f"{name}")
            t = time.perf_counter()
            out[name] = fn(args, dev)
            log(f"{name} done in {time.perf_counter() - t:.1f} s")
    print(json.dumps(out), flush=True)


def log(msg):
    print(f"bench: {msg}", file=sys.stderr, flush=True)


def _line(value, steps, warmup, ms_per_step, config, extra) -> None:
    """The one JSON line of a --workload run other than the headline: value
    in Mpps for that workload, its config, and its own fields."""
    out = {"metric": METRIC, "value": round(value, 3), "unit": "Mpps", "n_gpus": 1,
           "steps": steps, "warmup": warmup, "ms_per_step": round(ms_per_step, 4),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u32",
           "data": "synthetic", "config": config}
    out.update(extra)
    print(json.dumps(out), flush=True)


def batched_links(dev, n_links=64, seed=0x640):
    """The links of the batched workload: (n_pairs, zipf_s, n_planted, theta,
    pairs tensor) each, windows log-uniform in [1e6, 2e8] pairs."""
    import math as _m
    import numpy as np
    from paper_1803_11449_amd import traffic
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n_links):
        n = int(_m.exp(rng.uniform(_m.log(1e6), _m.log(2e8))))
        s = float(rng.uniform(0.8, 1.3))
        planted = int(rng.integers(10, 501))
        theta = float(rng.choice([512.0, 1024.0]))
        key = traffic.config_seed(4, i)
        spec = traffic.spec_link_window(n, s, planted, key)
        out.append((n, s, planted, theta, traffic.generate(spec, key, device=dev).pairs))
    return out


def batched_run(args, dev) -> dict:
    """64 links, each with its own sketch and one window (sizes log-uniform
    in [1M, 200M] pairs, Zipf exponent uniform in [0.8, 1.3], 10..500
    planted super points, theta 512 or 1024, sizing rule with k <= 19).
    Update options per (sketch shape, size class) come from the autotuner.
    A step is one window cycle of every link: reset, update, restore. The
    plan runs the whole cycle as one HIP graph; the same cycle as eager
    batched calls and as one reset/update/restore per window in turn are
    timed beside it, and all three must agree."""
    import numpy as np
    import torch
    from paper_1803_11449_amd import ddhf, serving, traffic, tune
    log("generating 64 link windows")
    links = batched_links(dev)
    total = sum(x[0] for x in links)
    sks, tuned = [], {}
    for n, s, planted, theta, pairs in links:
        k, alpha = serving.sized_params(n, k_max=19)
        key = (k, tune.size_class(n))
        if key not in tuned:
            log(f"tuning k={k} n~2^{key[1]}")
            tuned[key] = tune.tune(1024, k, 5, alpha, pairs, traffic.HASH_SEED, use_cache=False)
        sk = ddhf.Sketch(1024, k, 5, alpha, traffic.HASH_SEED, device=0)
        tune.apply(sk, tuned[key])
        sks.append(sk)
    items = [(sk, x[4], x[3]) for sk, x in zip(sks, links)]
    # the restore's candidate search per (shape, size class, theta), tuned
    # on the first link of each class with its window in the sketch
    rtuned = {}
    for (n, s, planted, theta, pairs), sk in zip(links, sks):
        key = (sk.params.k, tune.size_class(n), theta)
        if key not in rtuned:
            log(f"tuning the restore k={key[0]} n~2^{key[1]} theta={theta:g}")
            sk.reset()
            sk.update(pairs)
            rtuned[key] = tune.tune_restore(sk, theta, n, use_cache=False)
        else:
            tune.apply(sk, rtuned[key])

    def batched():
        for sk in sks:
            sk.reset()
        ddhf.update_batch([(sk, p) for sk, p, _ in items])
        return ddhf.restore_batch([(sk, th) for sk, _, th in items])

    def plain():
        res = []
        for sk, p, th in items:
            sk.reset()
            sk.update(p)
            res.append(sk.restore(th))
        return res

    plan = ddhf.Plan(items)

    def planned():
        plan.run()
        return plan.results()

    # the eager calls grow the shared buffers to this batch's needs; the plan
    # runs last so that its graph is captured against the grown buffers once
    log("batched warmup")
    for _ in range(max(1, args.warmup)):
        rb = batched()
        rp = plain()
        rg = planned()
    rg = planned()
    for (n, s, planted, theta, _), sk, (recs, info) in zip(links, sks, rg):
        log(f"link n={n} s={s:.2f} planted={planted} theta={theta:g} k={sk.params.k} "
            f"he={info['he_count'][:5]} partials={info['n_partials'][2:4]} "
            f"cand={info['n_candidates']} spl={len(recs)} psi={info['psi']:.3f}")
    differ = sum(not (np.array_equal(a[0], b[0]) and np.array_equal(a[0], c[0]))
                 for a, b, c in zip(rg, rb, rp))
    steps = max(1, min(args.steps, 5))

    def timed(fn):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / steps

    tg, tb, tp = timed(planned), timed(batched), timed(plain)

    # where an eager cycle's time goes: the batched update by events on its
    # stream, then (after it has finished) the batched restore of every link
    # from the call to the lists on the host
    stream = torch.cuda.current_stream(dev)
    upd_ms, rst_ms = [], []
    for _ in range(steps):
        for sk in sks:
            sk.reset()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        ddhf.update_batch([(sk, p) for sk, p, _ in items])
        e1.record(stream)
        e1.synchronize()
        upd_ms.append(e0.elapsed_time(e1))
        t0 = time.perf_counter()
        ddhf.restore_batch([(sk, th) for sk, _, th in items])
        rst_ms.append((time.perf_counter() - t0) * 1e3)
    out = {"config": {"workload": "batched_64_links", "links": 64, "pairs": total,
                      "window_pairs": "log-uniform [1e6, 2e8]", "zipf_s": "U[0.8, 1.3]",
                      "planted": "U{10..500}", "theta": "512 or 1024", "k_max": 19},
           "steps": steps,
           "plan_mpps": round(total / tg / 1e6, 2), "plan_ms_per_step": round(tg * 1e3, 3),
           "plan_update_launches": plan.launches,
           "eager_batched_mpps": round(total / tb / 1e6, 2),
           "eager_batched_ms_per_step": round(tb * 1e3, 3),
           "plain_mpps": round(total / tp / 1e6, 2), "plain_ms_per_step": round(tp * 1e3, 3),
           "speedup_vs_plain": round(tp / tg, 3),
           "eager_update_ms_p50": round(percentile(upd_ms, 50), 3),
           "eager_restore_ms_p50": round(percentile(rst_ms, 50), 3),
           "windows_differing": differ,
           "super_points": int(sum(len(r[0]) for r in rg)),
           "tuned": {f"k{k}_n2^{c}": v for (k, c), v in sorted(tuned.items())},
           "restore_tuned": {f"k{k}_n2^{c}_theta{t:g}": v
                             for (k, c, t), v in sorted(rtuned.items())}}
    plan.close()
    for sk in sks:
        sk.close()
    del links, items
    torch.cuda.empty_cache()
    return out


def serving_run(args, dev) -> dict:
    """256 links whose windows close at Poisson times: sizes log-uniform in
    [1e5, 5e7] pairs, Zipf(1.0) sources with 0.05% planted, theta 1024, 64 GB
    HBM budget for resident sketches. Runs at the nominal aggregate rate of
    150 Mpps and at 20 and 40 G pairs/s (the second past what one window
    at a time can serve); for each, continuous
    batching (two batches in flight) and one window at a time, with
    close-to-report latency."""
    import torch
    from paper_1803_11449_amd import serving, traffic
    log("generating 2 pools of 2^27 pairs")
    pools = [serving.pair_pool(1 << 27, 1.0, traffic.config_seed(5, i), dev) for i in range(2)]
    res = {}
    for name, rate, dur in (("nominal_150mpps", 1.5e8, 3.0), ("overload_20gpps", 2e10, 0.25),
                            ("overload_40gpps", 4e10, 0.25)):
        reqs = serving.poisson_windows(pools, 256, rate, dur, 100_000, 50_000_000,
                                       seed=0x256, theta=(1024.0,))
        for mode, cls in (("continuous", serving.ContinuousServer), ("plain", serving.PlainServer)):
            log(f"{name} {mode}: {len(reqs)} windows")
            kw = {"trace": True} if cls is serving.ContinuousServer else {}
            with cls(budget_bytes=64 << 30, **kw) as srv:
                srv.links.prewarm(reqs)
                srv.warm(reqs)
                out = srv.serve(reqs)
                summ = serving.latency_summary(out)
                if kw:
                    summ["batches"] = len(srv.trace)
                    summ["batches_overlapping_previous"] = srv.overlaps()
            res[f"{name}_{mode}"] = summ
    del pools
    torch.cuda.empty_cache()
    return {"config": {"workload": "serving_256_links", "links": 256,
                       "window_pairs": "log-uniform [1e5, 5e7]", "hbm_budget_gb": 64,
                       "theta": 1024},
            "runs": res}


if __name__ == "__main__":
    main()
