"""GPU tests of the serving loop: requests from many host threads, continuous
batching over in-flight slots, the HBM cache under a byte budget, and that
every served block is byte-identical to the oracle's (alone or in the mix)."""
import sys
import threading

import numpy as np
import pytest

import meshgen
import oracle

pytestmark = pytest.mark.gpu

REL = (1, 2, 4)


def _gale():
    from paper_2507_15230_amd import gale
    return gale


def _say(*a):
    from tests.conftest import say
    say(*a)


def _expected(orc, ncl, mask):
    return {(k, rel): orc.block(k, rel) for k in range(ncl) for rel in REL if mask & rel}


def _consumer(ctx, seq, mask, exp, errors, tid):
    try:
        for ids in seq:
            tk = ctx.submit(ids, mask)
            ctx.poll(tk)
            for k in np.unique(ids):
                for rel in REL:
                    if not (mask & rel):
                        continue
                    got = ctx.block(tk, int(k), rel)
                    e = exp[(int(k), rel)]
                    if not all(np.array_equal(g, x) for g, x in zip(got, e)):
                        errors.append((tid, int(k), rel))
            ctx.release(tk)
    except Exception as ex:  # reported by the main thread
        errors.append((tid, "exception", repr(ex)))


@pytest.mark.parametrize("budget_mb,slots", [(256, 2), (1, 4)])
def test_serve_many_threads_match_oracle(budget_mb, slots):
    """16 threads, each requesting single clusters and small sets with re-access;
    a 1 MiB budget forces evictions."""
    gale = _gale()
    m = meshgen.grid_mesh(20, 100, seed=3)
    _say("serve", m.nclusters, "clusters, budget MiB", budget_mb, "slots", slots)
    orc = oracle.Oracle.of(m)
    exp = _expected(orc, m.nclusters, 7)
    rng = np.random.default_rng(5)
    seqs = []
    for t in range(16):
        seq = []
        for i in range(12):
            if i % 3 == 2:
                seq.append(rng.choice(m.nclusters, size=3, replace=False).astype(np.int32))
            else:
                seq.append(np.array([rng.integers(0, m.nclusters)], dtype=np.int32))
        seqs.append(seq)
    with gale.Context(mode="serve", cache_budget_bytes=budget_mb << 20, max_inflight=slots) as ctx:
        ctx.load(m.tets, m.cluster, m.nclusters)
        errors = []
        th = [threading.Thread(target=_consumer, args=(ctx, seqs[t], 7, exp, errors, t)) for t in range(16)]
        for x in th:
            x.start()
        for x in th:
            x.join()
        assert not errors, errors[:10]
        st = ctx.stats()
        _say("stats", {k: st[k] for k in ("cache_hits", "cache_misses", "evictions", "batches",
                                           "mean_batch_clusters", "lat_p50_us", "lat_p99_us")})
        assert st["lat_count"] == 16 * 12
        assert st["cache_hits"] + st["cache_misses"] >= 16 * 12
        assert st["batches"] >= 1
        if budget_mb == 1:
            assert st["evictions"] > 0
        else:
            assert st["cache_hits"] > 0


def test_serve_masks_and_alone_vs_mix():
    """The same cluster requested alone, in a mix, and with different masks gives
    the same bytes."""
    gale = _gale()
    m = meshgen.random_small(7, n=6, nclusters=8, drop=0.25, isolated=3, empty_clusters=2)
    orc = oracle.Oracle.of(m)
    with gale.Context(mode="serve", max_inflight=3) as ctx:
        ctx.load(m.tets, m.cluster, m.nclusters)
        for mask in (1, 2, 4, 3, 5, 6, 7):
            exp = _expected(orc, m.nclusters, mask)
            tks = [ctx.submit([k], mask) for k in range(m.nclusters)]
            tk_all = ctx.submit(np.arange(m.nclusters, dtype=np.int32), mask)
            for k, tk in enumerate(tks):
                ctx.poll(tk)
                for rel in REL:
                    if mask & rel:
                        assert all(np.array_equal(g, e) for g, e in zip(ctx.block(tk, k, rel), exp[(k, rel)]))
            ctx.poll(tk_all)
            for k in range(m.nclusters):
                for rel in REL:
                    if mask & rel:
                        assert all(np.array_equal(g, e)
                                   for g, e in zip(ctx.block(tk_all, k, rel), exp[(k, rel)]))
            for tk in tks + [tk_all]:
                ctx.release(tk)


def test_serve_queue_full_and_errors():
    gale = _gale()
    m = meshgen.grid_mesh(10, 50, seed=1)
    with gale.Context(mode="serve", max_queue=1, max_inflight=1) as ctx:
        ctx.load(m.tets, m.cluster, m.nclusters)
        # a burst larger than the queue: some submissions may see EAGAIN, none fail otherwise
        tks, again = [], 0
        for i in range(64):
            st, tk = ctx.try_submit([i % m.nclusters], 7)
            if st == gale.EAGAIN:
                again += 1
            else:
                assert st == gale.OK
                tks.append(tk)
        for tk in tks:
            ctx.poll(tk)
            ctx.release(tk)
        with pytest.raises(gale.GaleError) as ei:
            ctx.submit([m.nclusters], 7)
        assert ei.value.status == gale.EINVAL
        with pytest.raises(gale.GaleError) as ei:
            ctx.release(123456789)
        assert ei.value.status == gale.ENOENT
        _say("EAGAIN seen", again)


def test_serve_block_larger_than_budget_is_enomem():
    gale = _gale()
    m = meshgen.grid_mesh(12, 1728, seed=2)  # one cluster holding the whole mesh
    with gale.Context(mode="serve", cache_budget_bytes=64 << 10) as ctx:
        ctx.load(m.tets, m.cluster, m.nclusters)
        tk = ctx.submit([0], 7)
        with pytest.raises(gale.GaleError) as ei:
            ctx.poll(tk)
        assert ei.value.status == gale.ENOMEM
        ctx.release(tk)


def test_serve_destroy_with_requests_in_flight():
    gale = _gale()
    m = meshgen.grid_mesh(16, 64, seed=4)
    ctx = gale.Context(mode="serve", max_inflight=2)
    ctx.load(m.tets, m.cluster, m.nclusters)
    for k in range(m.nclusters):
        ctx.submit([k], 7)
    ctx.close()  # drains in-flight batches, fails what is still queued


def test_consumers_classify_like_the_oracle():
    """The serving workload (consumer threads, Zipf re-access, a budget that
    forces evictions): every access's critical-point labels equal those from the
    oracle's blocks, and re-accesses reproduce them."""
    gale = _gale()
    from paper_2507_15230_amd import workload
    m = meshgen.grid_mesh(16, 64, seed=6)
    field = meshgen.gauss_field(m.coords.astype(np.float64), 16, np.random.default_rng(2))
    orc = oracle.Oracle.of(m)
    exp = {}
    for k in range(m.nclusters):
        vt, vv = orc.block(k, 1), orc.block(k, 2)
        exp[k] = gale.lowerstar_classify(vt[0], vt, vv, m.tets, field)
    with gale.Context(mode="serve", cache_budget_bytes=256 << 10, max_inflight=3) as ctx:
        ctx.load(m.tets, m.cluster, m.nclusters)
        got = {}
        base = workload.served_request(ctx)

        def request(c):
            vt, vv, release = base(c)
            lab = gale.lowerstar_classify(vt[0], vt, vv, m.tets, field)
            got.setdefault(c, []).append(lab)
            return vt, vv, release
        res = workload.run_consumers(request, m.tets, field, range(m.nclusters), threads=12, seed=3)
        st = ctx.stats()
    _say("consumers", {k: res[k] for k in ("accesses", "reaccesses", "mismatches", "clusters")},
         "evictions", st["evictions"])
    assert not res["errors"], res["errors"]
    assert res["mismatches"] == 0
    assert res["clusters"] == m.nclusters
    assert res["reaccesses"] > 0
    for c, labs in got.items():
        for lab in labs:
            assert np.array_equal(lab, exp[c])


@pytest.mark.parametrize("mode", ["serve", "plain"])
def test_native_consumers_count_like_the_oracle(mode):
    """Native consumer threads (gale_consumer_run) through the serving loop and
    through plain per-cluster launches: no errors, no label changes between
    accesses, and the critical points counted at each cluster's first access
    equal those from the oracle's blocks."""
    gale = _gale()
    m = meshgen.grid_mesh(16, 64, seed=8)
    field = meshgen.gauss_field(m.coords.astype(np.float64), 16, np.random.default_rng(4))
    orc = oracle.Oracle.of(m)
    tot = np.zeros(4, np.int64)
    for k in range(m.nclusters):
        vt, vv = orc.block(k, 1), orc.block(k, 2)
        tot += np.bincount(gale.lowerstar_classify(vt[0], vt, vv, m.tets, field), minlength=4)
    kw = dict(mode="serve", cache_budget_bytes=256 << 10, max_inflight=3) if mode == "serve" else \
        dict(mode="direct", form="plain")
    with gale.Context(**kw) as ctx:
        ctx.load(m.tets, m.cluster, m.nclusters)
        res = gale.consumer_run(ctx, m.tets, field, np.arange(m.nclusters), threads=24, seed=5)
    _say(mode, {k: res[k] for k in ("accesses", "reaccesses", "mismatches", "errors", "lat_p50_us", "lat_p99_us")})
    assert res["errors"] == 0 and res["first_error"] == 0
    assert res["mismatches"] == 0
    assert res["clusters"] == m.nclusters
    assert [res["regular"], res["minima"], res["maxima"], res["saddles"]] == tot.tolist()


def _block_bytes(info, mask):
    """Bytes the serving cache reserves for a block of this cluster before it
    is built: the block layout with the default capacities (exact VT, 4 TT
    entries per row, the VV bound), each array on a 32-word boundary."""
    al = lambda w: (w + 31) // 32 * 32
    nV, nT, nvt, cvv = info["nV"], info["nT"], info["nnzVT"], info["cap_vv"]
    w = al(8)
    if mask & 3:
        w = al(w + nV)
    if mask & 1:
        w = al(w + nV + 1)
        w = al(w + nvt)
    if mask & 4:
        w = al(w + nT)
        w = al(w + nT + 1)
        w = al(w + 4 * nT)
    if mask & 2:
        w = al(w + nV + 1)
        w = al(w + cvv)
    return (4 * w + 255) // 256 * 256


def test_prefetch_blocks_equal_oracle_and_are_evicted_first():
    """Speculative builds of the clusters following a request (the leader's
    proactive precomputation, prefetch_depth 2): a later request for one of
    them is a hit on a block equal to the oracle's, and when space runs out
    speculative blocks are evicted before the block a request used."""
    gale = _gale()
    m = meshgen.grid_mesh(20, 100, seed=3)
    orc = oracle.Oracle.of(m)
    with gale.Context(mode="direct") as probe:
        probe.load(m.tets, m.cluster, m.nclusters)
        info = {k: probe.cluster_info(k) for k in range(m.nclusters)}
    need = _block_bytes(info[10], 7) + _block_bytes(info[50], 7) + \
        max(_block_bytes(info[11], 7), _block_bytes(info[12], 7))
    with gale.Context(mode="serve", cache_budget_bytes=need + 256, max_inflight=2, prefetch_depth=2) as ctx:
        ctx.load(m.tets, m.cluster, m.nclusters)
        tk = ctx.submit([10], 7)
        ctx.poll(tk)
        ctx.release(tk)
        st = ctx.stats()
        _say("after 10", {k: st[k] for k in ("prefetch_built", "prefetch_hits", "evictions", "cache_misses")})
        assert st["prefetch_built"] >= 1
        # cluster 11 was built ahead of this request
        tk = ctx.submit([11], 7)
        ctx.poll(tk)
        for rel in REL:
            assert all(np.array_equal(g, e) for g, e in zip(ctx.block(tk, 11, rel), orc.block(11, rel)))
        ctx.release(tk)
        st = ctx.stats()
        assert st["prefetch_hits"] >= 1 and st["cache_misses"] == 1
        # a far cluster needs space: speculative blocks go, the used ones stay
        tk = ctx.submit([50], 7)
        ctx.poll(tk)
        for rel in REL:
            assert all(np.array_equal(g, e) for g, e in zip(ctx.block(tk, 50, rel), orc.block(50, rel)))
        ctx.release(tk)
        st = ctx.stats()
        _say("after 50", {k: st[k] for k in ("prefetch_built", "prefetch_evicted", "demand_evictions", "evictions")})
        assert st["prefetch_evicted"] >= 1
        before = st["cache_misses"]
        tk = ctx.submit([10], 7)
        ctx.poll(tk)
        for rel in REL:
            assert all(np.array_equal(g, e) for g, e in zip(ctx.block(tk, 10, rel), orc.block(10, rel)))
        ctx.release(tk)
        assert ctx.stats()["cache_misses"] == before  # still resident


@pytest.mark.parametrize("budget_mb", [256, 1])
def test_per_relation_front_end_matches_oracle(budget_mb):
    """The per-relation front end (one queue and one leader thread per
    relation, each request split into one part per relation): 16 threads
    with mixed masks, every block equal to the oracle's; a 1 MiB budget
    forces evictions."""
    gale = _gale()
    m = meshgen.grid_mesh(20, 100, seed=3)
    orc = oracle.Oracle.of(m)
    exp = _expected(orc, m.nclusters, 7)
    rng = np.random.default_rng(9)
    masks = [7, 3, 1, 2, 4, 6, 5]
    with gale.Context(mode="serve", cache_budget_bytes=budget_mb << 20, max_inflight=2,
                      front_end="per_relation") as ctx:
        ctx.load(m.tets, m.cluster, m.nclusters)
        assert ctx.stats()["front_end"] == gale.FRONT_PER_RELATION
        errors = []

        def worker(t):
            r = np.random.default_rng(100 + t)
            for i in range(10):
                mask = masks[(t + i) % len(masks)]
                ids = r.choice(m.nclusters, size=1 + (i % 3), replace=False).astype(np.int32)
                _consumer(ctx, [ids], mask, exp, errors, t)
        th = [threading.Thread(target=worker, args=(t,)) for t in range(16)]
        for x in th:
            x.start()
        for x in th:
            x.join()
        assert not errors, errors[:10]
        st = ctx.stats()
        _say("per-relation", {k: st[k] for k in ("cache_hits", "cache_misses", "evictions", "batches",
                                                 "lat_p50_us", "lat_p99_us", "queue_depth_mean")})
        assert st["lat_count"] == 160
        if budget_mb == 1:
            assert st["evictions"] > 0


def test_per_relation_native_consumers():
    gale = _gale()
    m = meshgen.grid_mesh(16, 64, seed=8)
    field = meshgen.gauss_field(m.coords.astype(np.float64), 16, np.random.default_rng(4))
    orc = oracle.Oracle.of(m)
    tot = np.zeros(4, np.int64)
    for k in range(m.nclusters):
        vt, vv = orc.block(k, 1), orc.block(k, 2)
        tot += np.bincount(gale.lowerstar_classify(vt[0], vt, vv, m.tets, field), minlength=4)
    with gale.Context(mode="serve", cache_budget_bytes=256 << 10, max_inflight=2, front_end="per_relation") as ctx:
        ctx.load(m.tets, m.cluster, m.nclusters)
        res = gale.consumer_run(ctx, m.tets, field, np.arange(m.nclusters), threads=24, seed=5)
        st = ctx.stats()
    _say("per-relation native", {k: res[k] for k in ("accesses", "mismatches", "errors", "lat_p50_us")},
         {k: st[k] for k in ("stage_push_us", "stage_queue_us", "stage_prep_us", "stage_kernel_copy_us",
                              "wait_queue_s_max")})
    assert res["errors"] == 0 and res["mismatches"] == 0
    assert [res["regular"], res["minima"], res["maxima"], res["saddles"]] == tot.tolist()


def test_borrowed_arena_from_torch():
    """The HBM cache in device memory the caller owns (a torch tensor)."""
    import torch
    gale = _gale()
    torch.cuda.set_device(0)
    arena = torch.empty(8 << 20, dtype=torch.uint8, device="cuda")
    m = meshgen.grid_mesh(12, 100, seed=5)
    orc = oracle.Oracle.of(m)
    exp = _expected(orc, m.nclusters, 7)
    with gale.Context(mode="serve", dev_arena=arena.data_ptr(), arena_bytes=arena.numel(),
                      cache_budget_bytes=4 << 20) as ctx:
        ctx.load(m.tets, m.cluster, m.nclusters)
        assert ctx.stats()["cache_budget"] == 4 << 20
        errors = []
        _consumer(ctx, [np.array([k], np.int32) for k in range(m.nclusters)], 7, exp, errors, 0)
        assert not errors, errors[:5]
    with pytest.raises(gale.GaleError) as ei:
        gale.Context(mode="direct", dev_arena=arena.data_ptr(), arena_bytes=arena.numel())
    assert ei.value.status == gale.EINVAL
    del arena


def test_stage_breakdown_and_queue_depth():
    """The paper's five waiting stages and the queue depth at admission are
    reported, consistent with the total latency."""
    gale = _gale()
    m = meshgen.grid_mesh(16, 64, seed=8)
    field = meshgen.gauss_field(m.coords.astype(np.float64), 16, np.random.default_rng(4))
    with gale.Context(mode="serve", cache_budget_bytes=1 << 20, max_inflight=3) as ctx:
        ctx.load(m.tets, m.cluster, m.nclusters)
        res = gale.consumer_run(ctx, m.tets, field, np.arange(m.nclusters), threads=16, seed=2)
        st = ctx.stats()
    parts = st["stage_push_us"] + (st["stage_queue_us"] - st["stage_push_us"]) + st["stage_prep_us"] + \
        st["stage_kernel_copy_us"] + st["stage_integration_us"]
    _say("stages", {k: round(st[k], 1) for k in st if k.startswith("stage_")}, "mean", st["lat_mean_us"],
         "depth", st["queue_depth_mean"], st["queue_depth_max"])
    assert res["errors"] == 0
    assert abs(parts - st["lat_mean_us"]) <= 0.02 * st["lat_mean_us"] + 1.0
    assert st["queue_depth_max"] >= 1 and st["queue_depth_mean"] >= 1.0
    assert st["wait_queue_s_max"] > 0 and st["wait_kernel_copy_s_max"] > 0


@pytest.mark.timeout(900)
def test_config4_served_blocks_with_evictions():
    """The config-4 mesh (the refined 256^3 mesh with its scalar field)
    served with the 4 GB cache budget: 40 native consumer threads walk
    24,000 clusters in Morton order with Zipf re-access (more block bytes
    than the budget holds, so blocks are evicted) while four Python threads
    request a seeded sample of the same clusters in the mix; every sampled
    block equals the oracle's and no consumer label changes."""
    gale = _gale()
    m = meshgen.config(4)
    _say("config 4", m.nv, m.nt, m.nclusters)
    orc = oracle.Oracle.of(m)
    ncur = 24000
    rng = np.random.default_rng(41)
    sample = np.sort(rng.choice(ncur, 1200, replace=False)).astype(np.int32)
    with gale.Context(mode="serve", cache_budget_bytes=4 << 30, max_inflight=4) as ctx:
        ctx.load(m.tets, m.cluster, m.nclusters)
        _say("loaded")
        errors, done = [], []

        def sampler(t):
            part = sample[t::4]
            for c0 in range(0, len(part), 50):
                ids = part[c0:c0 + 50]
                exp = orc.blocks([(int(k), rel) for k in ids for rel in REL], threads=4)
                i = 0
                for k in ids:
                    try:
                        tk = ctx.submit([int(k)], 7)
                        ctx.poll(tk)
                        for rel in REL:
                            got = ctx.block(tk, int(k), rel)
                            if not all(np.array_equal(g, x) for g, x in zip(got, exp[i])):
                                errors.append((int(k), rel))
                            i += 1
                        ctx.release(tk)
                    except Exception as ex:
                        errors.append((int(k), repr(ex)))
                        return
            done.append(t)
        th = [threading.Thread(target=sampler, args=(t,)) for t in range(4)]
        for x in th:
            x.start()
        res = gale.consumer_run(ctx, m.tets, m.scalar, np.arange(ncur, dtype=np.int32), threads=40, seed=0)
        _say("consumers", {k: res[k] for k in ("accesses", "reaccesses", "mismatches", "errors", "lat_p50_us",
                                               "lat_p99_us")})
        for x in th:
            x.join()
        st = ctx.stats()
        _say("cache", {k: st[k] for k in ("cache_hits", "cache_misses", "evictions", "cache_bytes_resident",
                                          "cache_budget", "queue_depth_mean", "tt_exhaustive_blocks")})
    assert not errors, errors[:10]
    assert len(done) == 4
    assert res["errors"] == 0 and res["mismatches"] == 0
    assert st["evictions"] > 0
    assert st["tt_exhaustive_blocks"] == 0
