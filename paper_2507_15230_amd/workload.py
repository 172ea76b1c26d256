"""Consumer workload for the serving form: host threads that walk the clusters,
request their relations and classify critical points (include/gale_lowerstar.h).

Each consumer thread draws k from a Zipf(s) law truncated to {1..64} after
every access: k = 1 takes the next cluster from a shared cursor over the
cluster ids (Morton order), k >= 2 re-accesses the thread's (k-1)-th most
recent cluster (or the next new one when there are fewer).  Every access
requests VT, VV and TT for one cluster, classifies its vertices from VT and VV
and releases the ticket.  The first labels computed for a cluster are kept;
every later access must reproduce them (the same bytes alone and in the mix).
"""
from __future__ import annotations

import threading
import time
from collections import deque

import numpy as np

from . import gale


class _Cursor:
    def __init__(self, ids):
        self.ids = list(ids)
        self.i = 0
        self.mu = threading.Lock()

    def next(self):
        with self.mu:
            if self.i >= len(self.ids):
                return None
            c = self.ids[self.i]
            self.i += 1
            return c


def zipf_cdf(s: float = 1.1, kmax: int = 64) -> np.ndarray:
    w = 1.0 / np.arange(1, kmax + 1, dtype=np.float64) ** s
    return np.cumsum(w) / w.sum()


def run_consumers(request, tets, field, cluster_ids, threads: int = 40, seed: int = 0, s: float = 1.1):
    """Run the workload.  request(c) -> (vt, vv, release) performs one access
    (vt, vv as (rows, offsets, entries); release() frees it) and is called from
    many threads.  Returns a dict with per-access latencies (seconds), counts
    and label mismatches."""
    cur = _Cursor(cluster_ids)
    cdf = zipf_cdf(s)
    first = {}
    first_mu = threading.Lock()
    lat = [[] for _ in range(threads)]
    counts = {"accesses": 0, "reaccesses": 0, "mismatches": 0, "minima": 0, "maxima": 0, "saddles": 0}
    cmu = threading.Lock()
    errors = []

    def worker(tid):
        rng = np.random.default_rng((seed, tid))
        recent = deque(maxlen=64)
        acc = re = mis = 0
        cp = [0, 0, 0, 0]
        try:
            while True:
                k = int(np.searchsorted(cdf, rng.random(), side="right")) + 1
                if k >= 2 and len(recent) >= k - 1:
                    c = recent[-(k - 1)]
                    re += 1
                else:
                    c = cur.next()
                    if c is None:
                        break
                t0 = time.perf_counter()
                vt, vv, release = request(c)
                lat[tid].append(time.perf_counter() - t0)
                labels = gale.lowerstar_classify(vt[0], vt, vv, tets, field)
                release()
                acc += 1
                key = bytes(labels.tobytes()) + bytes(np.asarray(vt[0], np.int32).tobytes())
                with first_mu:
                    prev = first.get(c)
                    if prev is None:
                        first[c] = key
                        for v in labels:
                            cp[int(v)] += 1
                    elif prev != key:
                        mis += 1
                recent.append(c)
        except Exception as ex:  # reported to the caller
            errors.append(repr(ex))
        with cmu:
            counts["accesses"] += acc
            counts["reaccesses"] += re
            counts["mismatches"] += mis
            counts["minima"] += cp[1]
            counts["maxima"] += cp[2]
            counts["saddles"] += cp[3]

    th = [threading.Thread(target=worker, args=(i,)) for i in range(threads)]
    t0 = time.perf_counter()
    for x in th:
        x.start()
    for x in th:
        x.join()
    wall = time.perf_counter() - t0
    all_lat = np.array([v for l in lat for v in l], dtype=np.float64)
    counts.update({"wall_s": wall, "latencies_s": all_lat, "errors": errors, "clusters": len(first)})
    return counts


def served_request(ctx: "gale.Context", mask: int = 7):
    """An access through a serving context: submit, wait, read VT and VV."""
    def request(c):
        tk = ctx.submit([c], mask)
        ctx.poll(tk)
        vt = ctx.block(tk, c, 1)
        vv = ctx.block(tk, c, 2)
        return vt, vv, (lambda: ctx.release(tk))
    return request


def plain_request(ctx: "gale.Context", mask: int = 7):
    """An access through a DIRECT plain-form context: per-cluster launches, no
    cache; gale_submit returns when the blocks are on the host."""
    return served_request(ctx, mask)
