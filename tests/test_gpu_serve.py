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
    print(*a, flush=True)
    sys.stdout.flush()


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
