"""A plan (one HIP graph per window cycle) gives, on every replay, what the
eager calls give and what the oracle computes."""
import numpy as np
import pytest
import torch

import oracle
from paper_1803_11449_amd import ddhf
from test_gpu_parity import (DEV, assert_spl_equal, make_sketch, planted, rand_pairs, say,
                             to_dev)

pytestmark = pytest.mark.gpu


def windows(seed, specs):
    rng = np.random.default_rng(seed)
    out = []
    for p, n, m in specs:
        hosts = rng.choice(2**32, size=m, replace=False).astype(np.uint32)
        pairs = np.concatenate([rand_pairs(rng, n, max(1, n // 30))] + planted(rng, hosts, 2500))
        out.append((p, pairs))
    return out


def test_plan_replays_match_oracle_and_eager():
    specs = [(oracle.Params(), 600_000, 8), (oracle.Params(1024, 18, 5, 5), 3_000_000, 12),
             (oracle.Params(256, 12, 6, 5), 300_000, 4), (oracle.Params(), 1_000, 0)]
    data = windows(61, specs)
    theta = [0.7 * p.g for p, _ in data]
    refs = [oracle.restore(p, oracle.build_sketch(p, x), th) for (p, x), th in zip(data, theta)]
    sks = [make_sketch(p) for p, _ in data]
    # the second window starts 8 bytes into its buffer (first pair peeled)
    bufs = [to_dev(x) for _, x in data]
    big = to_dev(np.concatenate([np.zeros((1, 2), np.uint32), data[1][1]]))
    bufs[1] = big[1:]
    extra = make_sketch(oracle.Params())
    noise = to_dev(rand_pairs(np.random.default_rng(7), 200_000, 5000))
    try:
        with ddhf.Plan([(sk, b, th) for sk, b, th in zip(sks, bufs, theta)]) as plan:
            assert plan.launches >= 2          # direct and binned launches
            for rep in range(3):
                say(f"plan replay {rep}")
                for sk in sks:                 # stale contents: the plan resets
                    sk.update(noise)
                plan.run()
                res = plan.results()
                for (recs, info), (ip, sz, c, _) in zip(res, refs):
                    assert_spl_equal(recs, ip, sz, c)
                assert np.array_equal(sks[2].download(), oracle.build_sketch(*data[2]))
                # eager work and a sync between replays
                extra.update(noise)
                torch.cuda.synchronize()
        eager = ddhf.restore_batch([(sk, th) for sk, th in zip(sks, theta)])
        for (a, _), (b, _) in zip(eager, res):
            assert np.array_equal(a, b)
    finally:
        for sk in sks + [extra]:
            sk.close()


def test_plan_buffers_grow_and_graph_is_rebuilt():
    """Plan buffers start at 16 entries: the first run's results come from
    eager reruns, the next runs from the rebuilt graph; all match. Six jobs
    spread over all four restore pools, each of which starts small."""
    p = oracle.Params()
    data = windows(67, [(p, 400_000, m) for m in (6, 10, 14, 18, 24, 30)])
    refs = [oracle.restore(p, oracle.build_sketch(p, x), 0.7 * p.g) for _, x in data]
    sks = [make_sketch(p) for _ in data]
    bufs = [to_dev(x) for _, x in data]
    sks[0].set_option(ddhf.SKETCH_OPT_TRIM_POOLS, 16)
    try:
        with ddhf.Plan([(sk, b, 0.7 * p.g) for sk, b in zip(sks, bufs)]) as plan:
            for rep in range(3):
                say(f"plan run {rep}")
                plan.run()
                for (recs, _), (ip, sz, c, _) in zip(plan.results(), refs):
                    assert_spl_equal(recs, ip, sz, c)
    finally:
        sks[0].set_option(ddhf.SKETCH_OPT_TRIM_POOLS, 0)
        for sk in sks:
            sk.close()


def test_plan_rejects_bad_jobs():
    p = oracle.Params()
    with make_sketch(p) as sk:
        t = to_dev(rand_pairs(np.random.default_rng(2), 1000, 10))
        for items, flags in (([], 3), ([(sk.handle, t.data_ptr(), 1000, 0.0)], 3),
                             ([(sk.handle, t.data_ptr(), 1000, 1.0)] * 2, 3),
                             ([(sk.handle, t.data_ptr(), 1000, 1.0)], 8)):
            with pytest.raises(ddhf.SketchError) as e:
                ddhf.sketch_plan_create(items, flags)
            assert e.value.code == ddhf.SKETCH_E_INVAL


def test_plan_update_in_rounds_and_without_restore():
    """A window cut into several binned rounds inside one graph, and a plan
    that only resets and updates: the sketch equals the oracle's."""
    p = oracle.Params(1024, 16, 5, 6)
    data = windows(71, [(p, 3_000_000, 10)])
    _, pairs = data[0]
    ref = oracle.build_sketch(p, pairs)
    with make_sketch(p) as sk:
        sk.set_option(ddhf.SKETCH_OPT_UPDATE_PATH, 2)
        sk.set_option(ddhf.SKETCH_OPT_BINNED_ROUND, 1 << 20)     # 3 rounds
        buf = to_dev(pairs)
        with ddhf.Plan([(sk, buf, 0.7 * p.g)], restore=False) as plan:
            assert plan.launches >= 3
            for rep in range(2):
                say(f"update-only plan run {rep}")
                plan.run()
                torch.cuda.synchronize()
                assert np.array_equal(sk.download(), ref)
            with pytest.raises(ddhf.SketchError) as e:
                plan.results()
            assert e.value.code == ddhf.SKETCH_E_INVAL


# The 64-link batch's shape at reduced sizes: link windows from the same
# generator (Zipf sources over n/25 hosts, planted log-uniform in
# [1024, 50000]), exponents across [0.8, 1.3], theta 512 and 1024, one
# k = 19 sketch (2048 tiles of 160 KiB, the most the scatter's 2048-tile
# variant takes) next to k = 14..15 ones, autotuned update options.
LINKS = [  # (n_pairs, zipf_s, planted, theta, forced (k, alpha) or None)
    (2_000_000, 0.80, 10, 512.0, None),
    (9_000_000, 0.85, 200, 512.0, None),
    (4_000_000, 1.30, 500, 1024.0, None),
    (12_000_000, 1.00, 50, 1024.0, (19, 5)),
    (1_000_000, 1.10, 30, 1024.0, None),
    (6_000_000, 0.90, 100, 512.0, (18, 5)),
]


def test_link_batch_shape_plan_equals_oracle_per_link():
    from paper_1803_11449_amd import serving, traffic, tune
    links, refs = [], []
    for i, (n, s, m, theta, forced) in enumerate(LINKS):
        key = traffic.config_seed(4, 1000 + i)
        spec = traffic.spec_link_window(n, s, m, key)
        w = traffic.generate(spec, key, device=DEV)
        k, alpha = forced or serving.sized_params(n, k_max=19)
        p = oracle.Params(1024, k, 5, alpha, traffic.HASH_SEED)
        say(f"link {i}: n={n} s={s} planted={len(spec.planted_card)} theta={theta:g} k={k}")
        hp = w.pairs.cpu().numpy().view(np.uint32)
        refs.append(oracle.restore(p, oracle.build_sketch(p, hp), theta, mode="brute"))
        links.append((p, w.pairs, theta))
    sks = []
    tuned = {}
    try:
        for p, pairs, theta in links:
            sk = make_sketch(p)
            tk = (p.k, tune.size_class(pairs.shape[0]))
            if tk not in tuned:
                tuned[tk] = tune.tune(p.g, p.k, p.r, p.alpha, pairs, p.seed, trials=1,
                                      use_cache=False)
            tune.apply(sk, tuned[tk])
            sks.append(sk)
        items = [(sk, pairs, theta) for sk, (_, pairs, theta) in zip(sks, links)]
        with ddhf.Plan(items) as plan:
            for rep in range(2):
                say(f"link plan run {rep}")
                plan.run()
                for i, ((recs, info), (ip, sz, c, _)) in enumerate(zip(plan.results(), refs)):
                    assert len(ip) > 0, i
                    assert_spl_equal(recs, ip, sz, c)
        say("link batch, eager")
        for sk in sks:
            sk.reset()
        ddhf.update_batch([(sk, pairs) for sk, pairs, _ in items])
        for (recs, _), (ip, sz, c, _) in zip(
                ddhf.restore_batch([(sk, th) for sk, _, th in items]), refs):
            assert_spl_equal(recs, ip, sz, c)
    finally:
        for sk in sks:
            sk.close()
