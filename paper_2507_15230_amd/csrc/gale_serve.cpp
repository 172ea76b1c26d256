// gale_serve.cpp -- the serving loop: continuous batching over an HBM cache.
//
// The paper's consumers push (segment, consumer) requests into per-relation
// queues; a leader thread per queue pops every pending request, adds the
// following segments for proactive precomputation, launches one kernel for
// the whole batch into preallocated GPU memory, copies the results back and
// wakes the consumers through semaphores; kernels of different leaders run
// concurrently (Sections 4.2, 4.4, 4.5).  Here:
//   * gale_submit appends the request to a lane's pending queue and returns.
//     A lane is one leader: a queue, a service thread and its in-flight slots.
//     The single front end has one lane, and a request's relations are built
//     by one kernel; the per-relation front end (the paper's design) has one
//     lane per relation, and a request is split into one part per relation;
//   * a lane's thread admits every pending request whose blocks fit: a block
//     already resident in the HBM cache is a hit, one being built is joined,
//     a missing one gets space in the cache arena (least-recently-used
//     unpinned blocks are evicted until it fits the byte budget) and goes into
//     the next batch;
//   * with prefetch_depth > 0 the batch also builds the clusters following
//     each requested one (cluster ids follow the clustering's Morton order) as
//     speculative entries: they take free space or evict other speculative
//     blocks only, and are evicted before any block a request has used;
//   * a batch is one persistent-kernel launch writing straight into the
//     arena, on one of max_inflight slots (streams), so requests that arrive
//     while earlier batches run are admitted into the next free slot and their
//     work overlaps on the device;
//   * when all of a request's blocks are resident they are copied to a pinned
//     host buffer (one copy per block on the lane's copy stream) and the
//     request becomes ready; gale_poll waits on a condition variable.
// Blocks stay pinned while a request waits for or copies them.  The same
// kernel and the same block layout as the direct path make every served
// block byte-identical to a block built alone.  One mutex guards the cache
// and the queues; no thread holds it while it waits for the device or while
// it launches a batch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <functional>

#include "gale_ctx.h"

namespace gale {

// ---------------------------------------------------------------------------
// latency histogram
// ---------------------------------------------------------------------------
namespace {
constexpr double kHistLo = 0.1;      // microseconds
constexpr double kHistStep = 1.005;  // bucket width ratio
}  // namespace

int LatHist::bucket(double us) {
    if (!(us > kHistLo)) return 0;
    const int b = (int)(std::log(us / kHistLo) / std::log(kHistStep));
    return std::min(std::max(b, 0), kBuckets - 1);
}

double LatHist::lower(int b) { return kHistLo * std::pow(kHistStep, (double)b); }

void LatHist::add(double us) {
    n[bucket(us)]++;
    count++;
    sum += us;
    mx = std::max(mx, us);
}

// value at rank p*(count-1) (linear between ranks, as over sorted samples),
// each sample read as the geometric middle of its bucket (clamped to the max)
double LatHist::percentile(double p) const {
    if (count == 0) return 0.0;
    const double x = p * (double)(count - 1);
    const uint64_t i = (uint64_t)x;
    const double f = x - (double)i;
    auto at = [&](uint64_t rank) -> double {
        uint64_t c = 0;
        for (int b = 0; b < kBuckets; ++b) {
            c += n[b];
            if (c > rank) return std::min(mx, std::sqrt(lower(b) * lower(b + 1)));
        }
        return mx;
    };
    const double a = at(i);
    return i + 1 < count ? a * (1 - f) + at(i + 1) * f : a;
}

void LatHist::clear() {
    std::fill(n.begin(), n.end(), 0);
    count = 0;
    sum = 0.0;
    mx = 0.0;
}

namespace {

constexpr int64_t kArenaAlign = 256;

int64_t round_up(int64_t b, int64_t a) { return (b + a - 1) / a * a; }

int64_t cache_key(int32_t cluster, uint32_t mask) { return (int64_t)cluster * 8 + (int64_t)mask; }

double us_between(Clock::time_point a, Clock::time_point b) {
    return std::chrono::duration<double, std::micro>(b - a).count();
}

int64_t arena_alloc(Serve &s, int64_t bytes) {
    bytes = round_up(bytes, kArenaAlign);
    for (auto it = s.free_map.begin(); it != s.free_map.end(); ++it) {
        if (it->second >= bytes) {
            const int64_t off = it->first, rem = it->second - bytes;
            s.free_map.erase(it);
            if (rem > 0) s.free_map[off + bytes] = rem;
            return off;
        }
    }
    return -1;
}

void arena_free(Serve &s, int64_t off, int64_t bytes) {
    bytes = round_up(bytes, kArenaAlign);
    auto it = s.free_map.emplace(off, bytes).first;
    auto nx = std::next(it);
    if (nx != s.free_map.end() && it->first + it->second == nx->first) {
        it->second += nx->second;
        s.free_map.erase(nx);
    }
    if (it != s.free_map.begin()) {
        auto pv = std::prev(it);
        if (pv->first + pv->second == it->first) {
            pv->second += it->second;
            s.free_map.erase(it);
        }
    }
}

int64_t block_bytes(const ClusterMeta &m, uint32_t mask, int32_t cap_vv, int32_t cap_tt) {
    return block_layout(mask, m.nV, m.nT, m.nnzVT, cap_vv, cap_tt).total * 4;
}

void lru_remove(Serve &s, CacheEntry &e) {
    if (e.lru_kind == 1) s.lru.erase(e.lru_it);
    if (e.lru_kind == 2) s.spec_lru.erase(e.lru_it);
    e.lru_kind = 0;
}

// a resident, unpinned entry goes to the back of its list
void lru_insert(Serve &s, int64_t key, CacheEntry &e) {
    lru_remove(s, e);
    std::list<int64_t> &l = e.spec ? s.spec_lru : s.lru;
    l.push_back(key);
    e.lru_it = std::prev(l.end());
    e.lru_kind = e.spec ? 2 : 1;
}

void unpin(Serve &s, int64_t key) {
    auto it = s.cache.find(key);
    if (it == s.cache.end()) return;
    CacheEntry &e = it->second;
    if (--e.pins == 0 && e.state == 1) lru_insert(s, key, e);
}

void pin(Serve &s, CacheEntry &e) {
    if (e.pins++ == 0) lru_remove(s, e);
}

void drop_entry(Serve &s, std::unordered_map<int64_t, CacheEntry>::iterator it) {
    lru_remove(s, it->second);
    if (it->second.off >= 0) arena_free(s, it->second.off, it->second.bytes);
    if (it->second.state == 1) s.resident_bytes -= it->second.bytes;
    s.cache.erase(it);
}

// Evict the least recently used unpinned block: speculative ones first;
// demand blocks only when allowed.
bool evict_one(Serve &s, bool demand_too) {
    std::list<int64_t> *l = !s.spec_lru.empty() ? &s.spec_lru : (demand_too && !s.lru.empty() ? &s.lru : nullptr);
    if (!l) return false;
    const int64_t key = l->front();
    auto it = s.cache.find(key);
    if (it == s.cache.end()) {
        l->pop_front();
        return true;
    }
    if (it->second.lru_kind == 2)
        s.prefetch_evicted++;
    else
        s.demand_evictions++;
    s.evictions++;
    drop_entry(s, it);
    return true;
}

// allocate with eviction; -1 if it cannot fit now
int64_t alloc_evicting(Serve &s, int64_t bytes, bool demand_too) {
    int64_t off = arena_alloc(s, bytes);
    while (off < 0 && evict_one(s, demand_too)) off = arena_alloc(s, bytes);
    return off;
}

// stage_sum: queue (submit -> admitted), build (admitted -> blocks resident),
// copy (resident -> ready), then the paper's five: push, in queue, data
// preparation, kernel + transfer back, integration
void record_stages(Serve &s, const ServeReq *r) {
    const double v[8] = {us_between(r->t_submit, r->t_admit),   us_between(r->t_admit, r->t_built),
                         us_between(r->t_built, r->t_ready),    us_between(r->t_submit, r->t_pushed),
                         us_between(r->t_pushed, r->t_admit),   us_between(r->t_admit, r->t_launched),
                         us_between(r->t_launched, r->t_copied), us_between(r->t_copied, r->t_ready)};
    for (int i = 0; i < 8; ++i) s.stage_sum[i] += v[i];
    s.n_stage++;
    auto &pt = s.per_thread[r->thread_key];
    for (int i = 0; i < 5; ++i) pt[i] += v[3 + i] * 1e-6;
}

void finish_request(gale_ctx *ctx, ServeReq *r, gale_status st);

void finish_parent(gale_ctx *ctx, ServeReq *p, const ServeReq *last) {
    Serve &s = ctx->serve;
    p->ready = true;
    p->t_ready = Clock::now();
    if (p->status == GALE_OK) {
        // the stages of the part that finished last (the request's critical path)
        p->t_pushed = last->t_pushed;
        p->t_admit = last->t_admit;
        p->t_launched = last->t_launched;
        p->t_built = last->t_built;
        p->t_copied = last->t_copied;
        s.lat.add(us_between(p->t_submit, p->t_ready));
        record_stages(s, p);
    }
}

void finish_request(gale_ctx *ctx, ServeReq *r, gale_status st) {
    Serve &s = ctx->serve;
    if (r->ready) return;
    for (int64_t k : r->keys) {
        auto it = s.cache.find(k);
        if (it != s.cache.end()) {
            auto &w = it->second.waiters;
            w.erase(std::remove(w.begin(), w.end(), r), w.end());
        }
        unpin(s, k);
    }
    r->keys.clear();
    r->status = st;
    r->ready = true;
    r->t_ready = Clock::now();
    if (r->t_copied.time_since_epoch().count() == 0) r->t_copied = r->t_ready;
    if (r->parent) {
        ServeReq *p = r->parent;
        if (st != GALE_OK && p->status == GALE_OK) p->status = st;
        if (--p->parts_left == 0) finish_parent(ctx, p, r);
    } else if (st == GALE_OK) {
        s.lat.add(us_between(r->t_submit, r->t_ready));
        record_stages(s, r);
    }
    s.cv_done.notify_all();
}

// all blocks of r are resident: copy them to a pinned host buffer
void start_copy(gale_ctx *ctx, Lane &ln, ServeReq *r) {
    Serve &s = ctx->serve;
    r->t_built = Clock::now();
    if (r->t_launched.time_since_epoch().count() == 0) r->t_launched = r->t_built;
    const size_t n = r->clusters.size();
    r->snap.resize(n);
    r->host_word.assign(n, 0);
    int64_t words = 0;
    for (size_t i = 0; i < n; ++i) {
        const CacheEntry &e = s.cache[cache_key(r->clusters[i], r->mask)];
        r->snap[i].cluster = e.cluster;
        r->snap[i].mask = e.mask;
        r->snap[i].cap_vv = e.hdr[4];  // exact count: VV tail is not copied
        r->snap[i].cap_tt = e.cap_tt;
        std::memcpy(r->snap[i].hdr, e.hdr, sizeof(e.hdr));
        r->host_word[i] = words;
        words += block_bytes(ctx->meta[e.cluster], e.mask, r->snap[i].cap_vv, e.cap_tt) / 4;
    }
    hipError_t err;
    r->host = ctx->pin_pool.acquire((size_t)words * 4 + 256, &err);
    if (!r->host) {
        finish_request(ctx, r, fail(GALE_ENOMEM, "pinned host buffer"));
        return;
    }
    uint64_t bytes = 0, ent = 0;
    for (size_t i = 0; i < n && err == hipSuccess; ++i) {
        const CacheEntry &e = s.cache[cache_key(r->clusters[i], r->mask)];
        const int64_t b = block_bytes(ctx->meta[e.cluster], e.mask, r->snap[i].cap_vv, e.cap_tt);
        err = hipMemcpyAsync((int32_t *)r->host->ptr + r->host_word[i], (char *)s.arena + e.off, (size_t)b,
                             hipMemcpyDeviceToHost, ln.copy_stream);
        bytes += (uint64_t)b;
        if (e.mask & kRelVT) ent += (uint64_t)e.hdr[3];
        if (e.mask & kRelVV) ent += (uint64_t)e.hdr[4];
        if (e.mask & kRelTT) ent += (uint64_t)e.hdr[5];
    }
    if (err == hipSuccess && !r->copy_done) err = hipEventCreateWithFlags(&r->copy_done, hipEventDisableTiming);
    if (err == hipSuccess) err = hipEventRecord(r->copy_done, ln.copy_stream);
    if (err != hipSuccess) {
        ctx->poisoned = true;
        finish_request(ctx, r, fail(GALE_EDEVICE, std::string("copy: ") + hipGetErrorString(err)));
        return;
    }
    ctx->n_bytes_d2h += bytes;
    ctx->n_delivered += ent;
    r->copying = true;
    ln.copying.push_back(r);
}

void fail_waiters(gale_ctx *ctx, CacheEntry &e, gale_status st) {
    std::vector<ServeReq *> w;
    w.swap(e.waiters);
    for (ServeReq *r : w)
        if (!r->ready) finish_request(ctx, r, st);
}

void release_slot_buffers(gale_ctx *ctx, Slot &sl) {
    ctx->dev_pool.release(sl.batch.dev_items);
    ctx->dev_pool.release(sl.batch.dev_hdr);
    ctx->dev_pool.release(sl.batch.ws);
    ctx->pin_pool.release(sl.batch.host_items);
    ctx->pin_pool.release(sl.batch.host_hdr);
    sl.batch = Batch();
    sl.keys.clear();
}

// A slot's batch finished on the GPU (kernels and the header copy: the
// header copy is queued on the slot stream before its done event).
void complete_slot(gale_ctx *ctx, Lane &ln, Slot &sl) {
    Serve &s = ctx->serve;
    const int n = (int)sl.batch.items.size();
    const int32_t *hdr = (const int32_t *)sl.batch.host_hdr->ptr;
    for (int i = 0; i < n; ++i) {
        auto it = s.cache.find(sl.keys[i]);
        if (it == s.cache.end()) continue;
        CacheEntry &e = it->second;
        const int32_t *h = hdr + (size_t)i * 8;
        if (ctx->poisoned || (h[0] & kStInconsistent)) {
            ctx->poisoned = true;
            fail_waiters(ctx, e, fail(GALE_EDEVICE, ctx->poisoned && !(h[0] & kStInconsistent)
                                                        ? std::string("context poisoned by a device error")
                                                        : std::string("stream metadata mismatch")));
            drop_entry(s, it);
            continue;
        }
        const ClusterMeta &m = ctx->meta[e.cluster];
        if (h[0] & (kStVVOverflow | kStTTOverflow)) {
            // rebuild with exact capacities in the lane's next batch
            arena_free(s, e.off, e.bytes);
            e.cap_vv = (e.mask & kRelVV) ? std::max(h[4], 0) : 0;
            e.cap_tt = (e.mask & kRelTT) ? std::max(h[5], default_cap_tt(m)) : 0;
            e.bytes = round_up(block_bytes(m, e.mask, e.cap_vv, e.cap_tt), kArenaAlign);
            e.off = -1;
            ln.rebuild.push_back(sl.keys[i]);
            ctx->n_overflow++;
            continue;
        }
        std::memcpy(e.hdr, h, sizeof(e.hdr));
        if (h[0] & kStTTFallback) ctx->n_tt_exhaustive++;
        e.state = 1;
        // give back the unused VV tail
        const int64_t used = round_up(block_bytes(m, e.mask, (e.mask & kRelVV) ? h[4] : 0, e.cap_tt), kArenaAlign);
        if (used < e.bytes) {
            arena_free(s, e.off + used, e.bytes - used);
            e.bytes = used;
        }
        s.resident_bytes += e.bytes;
        if (e.pins == 0) lru_insert(s, sl.keys[i], e);
        if (e.mask & kRelVT) ctx->n_entries += (uint64_t)h[3];
        if (e.mask & kRelVV) ctx->n_entries += (uint64_t)h[4];
        if (e.mask & kRelTT) ctx->n_entries += (uint64_t)h[5];
        ctx->n_blocks++;
        std::vector<ServeReq *> w;
        w.swap(e.waiters);
        for (ServeReq *r : w) {
            if (r->ready) continue;
            if (--r->waiting == 0) start_copy(ctx, *s.lanes[r->lane], r);
        }
    }
    release_slot_buffers(ctx, sl);
    sl.busy = false;
}

// Fail everything a lane has not finished, after a device error poisoned the
// context: pending requests, blocks waiting for a rebuild (their arena space
// is freed) and the requests waiting on them.
void fail_lane(gale_ctx *ctx, Lane &ln, gale_status st) {
    Serve &s = ctx->serve;
    while (!ln.pending.empty()) {
        ServeReq *r = ln.pending.front();
        ln.pending.pop_front();
        finish_request(ctx, r, st);
    }
    for (int64_t key : ln.rebuild) {
        auto it = s.cache.find(key);
        if (it == s.cache.end()) continue;
        fail_waiters(ctx, it->second, st);
        it->second.off = -1;  // already given back when the rebuild was scheduled
        drop_entry(s, it);
    }
    ln.rebuild.clear();
}

bool any_busy(const Serve &s) {
    for (const auto &l : s.lanes)
        for (const Slot &x : l->slots)
            if (x.busy || x.launching) return true;
    return false;
}

// Admit pending requests and launch one batch on slot sl.  Returns true if
// anything was admitted or launched.  Called with the lock held; releases it
// while the batch is launched.
bool admit_round(gale_ctx *ctx, Lane &ln, Slot &sl, std::unique_lock<std::mutex> &lk) {
    Serve &s = ctx->serve;
    std::vector<int64_t> build_keys;
    bool progressed = false;
    // blocks to rebuild with exact capacities come first
    std::vector<int64_t> still;
    for (int64_t key : ln.rebuild) {
        auto it = s.cache.find(key);
        if (it == s.cache.end()) continue;
        CacheEntry &e = it->second;
        const int64_t off = alloc_evicting(s, e.bytes, true);
        if (off < 0) {
            still.push_back(key);
            continue;
        }
        e.off = off;
        build_keys.push_back(key);
    }
    ln.rebuild.swap(still);
    if (!ln.pending.empty()) {
        const int depth = (int)ln.pending.size();
        s.admissions++;
        s.depth_sum += depth;
        s.depth_max = std::max(s.depth_max, depth);
    }
    std::vector<ServeReq *> admitted;
    while (!ln.pending.empty()) {
        ServeReq *r = ln.pending.front();
        // phase 1: pin hits and joins, allocate misses
        std::vector<int64_t> held, fresh;
        bool ok = true;
        gale_status why = GALE_OK;
        for (int32_t k : r->clusters) {
            const int64_t key = cache_key(k, r->mask);
            auto it = s.cache.find(key);
            if (it != s.cache.end()) {
                if (it->second.spec) {
                    it->second.spec = false;
                    s.prefetch_hits++;
                    if (it->second.lru_kind == 2) lru_remove(s, it->second);
                }
                pin(s, it->second);
                held.push_back(key);
                continue;
            }
            const ClusterMeta &m = ctx->meta[k];
            const int32_t cvv = (r->mask & kRelVV) ? m.cap_vv : 0;
            const int32_t ctt = (r->mask & kRelTT) ? default_cap_tt(m) : 0;
            const int64_t bytes = round_up(block_bytes(m, r->mask, cvv, ctt), kArenaAlign);
            if (bytes > s.arena_bytes) {
                ok = false;
                why = fail(GALE_ENOMEM, "block of cluster " + std::to_string(k) + " exceeds the cache budget");
                break;
            }
            const int64_t off = alloc_evicting(s, bytes, true);
            if (off < 0) {
                ok = false;
                break;
            }
            CacheEntry e;
            e.cluster = k;
            e.mask = r->mask;
            e.off = off;
            e.bytes = bytes;
            e.state = 0;
            e.pins = 1;
            e.cap_vv = cvv;
            e.cap_tt = ctt;
            s.cache.emplace(key, e);
            held.push_back(key);
            fresh.push_back(key);
        }
        if (!ok) {
            // roll back this request's holds; fresh entries are dropped
            for (int64_t key : fresh) {
                auto it = s.cache.find(key);
                if (it != s.cache.end()) drop_entry(s, it);
            }
            for (int64_t key : held)
                if (std::find(fresh.begin(), fresh.end(), key) == fresh.end()) unpin(s, key);
            bool others_hold = any_busy(s);
            for (auto &kv : s.cache)
                if (kv.second.pins > 0) others_hold = true;
            if (why != GALE_OK || (!others_hold && build_keys.empty())) {
                ln.pending.pop_front();
                finish_request(ctx, r, why != GALE_OK ? why
                                                      : fail(GALE_ENOMEM, "request does not fit the cache budget"));
                progressed = true;
                continue;
            }
            break;  // wait for space; keep FIFO order
        }
        ln.pending.pop_front();
        progressed = true;
        r->admitted = true;
        r->t_admit = Clock::now();
        r->keys = held;
        r->waiting = 0;
        for (int64_t key : held) {
            CacheEntry &e = s.cache[key];
            if (e.state == 0) {
                e.waiters.push_back(r);
                r->waiting++;
            }
        }
        for (int64_t key : fresh) build_keys.push_back(key);
        s.hits += held.size() - fresh.size();
        s.misses += fresh.size();
        if (r->waiting == 0) {
            r->t_launched = r->t_admit;
            start_copy(ctx, ln, r);
        } else {
            admitted.push_back(r);
        }
    }
    // proactive precomputation of the clusters that follow each requested one
    const int depth = ctx->cfg.prefetch_depth;
    if (depth > 0) {
        bool room = true;
        for (ServeReq *r : admitted) {
            for (size_t ci = 0; ci < r->clusters.size() && room; ++ci) {
                for (int j = 1; j <= depth && room; ++j) {
                    const int32_t c = r->clusters[ci] + j;
                    if (c >= ctx->ncl) break;
                    const int64_t key = cache_key(c, r->mask);
                    if (s.cache.count(key)) continue;
                    const ClusterMeta &m = ctx->meta[c];
                    const int32_t cvv = (r->mask & kRelVV) ? m.cap_vv : 0;
                    const int32_t ctt = (r->mask & kRelTT) ? default_cap_tt(m) : 0;
                    const int64_t bytes = round_up(block_bytes(m, r->mask, cvv, ctt), kArenaAlign);
                    const int64_t off = bytes <= s.arena_bytes ? alloc_evicting(s, bytes, false) : -1;
                    if (off < 0) {
                        room = false;
                        break;
                    }
                    CacheEntry e;
                    e.cluster = c;
                    e.mask = r->mask;
                    e.off = off;
                    e.bytes = bytes;
                    e.state = 0;
                    e.pins = 0;
                    e.spec = true;
                    e.cap_vv = cvv;
                    e.cap_tt = ctt;
                    s.cache.emplace(key, e);
                    build_keys.push_back(key);
                    s.prefetch_built++;
                }
            }
        }
    }
    if (build_keys.empty()) return progressed;

    // the batch: largest streams first
    Batch &b = sl.batch;
    b = Batch();
    std::vector<int> order(build_keys.size());
    for (size_t i = 0; i < order.size(); ++i) order[i] = (int)i;
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
        const ClusterMeta &a = ctx->meta[s.cache[build_keys[x]].cluster], &c = ctx->meta[s.cache[build_keys[y]].cluster];
        return (int64_t)a.ns + a.nh > (int64_t)c.ns + c.nh;
    });
    sl.keys.clear();
    for (int i : order) {
        const CacheEntry &e = s.cache[build_keys[i]];
        WorkItem it{};
        it.cluster = e.cluster;
        it.mask = e.mask;
        it.cap_vv = e.cap_vv;
        it.cap_tt = e.cap_tt;
        it.out_word = e.off / 4;
        it.hdr_index = (int32_t)b.items.size();
        b.items.push_back(it);
        sl.keys.push_back(build_keys[i]);
    }
    const int n = (int)b.items.size();
    s.batches++;
    s.batch_clusters += (uint64_t)n;
    // launch without the lock: the batch's entries are in state 0 (not
    // evictable) and the slot is marked as launching
    sl.launching = true;
    lk.unlock();
    hipError_t err;
    gale_status st = GALE_OK;
    b.host_hdr = ctx->pin_pool.acquire((size_t)n * 32 + 64, &err);
    if (!b.host_hdr) st = fail(GALE_ENOMEM, "serving batch buffers");
    if (st == GALE_OK)
        st = upload_and_launch(ctx, GALE_FORM_BATCHED, b.items, (int32_t *)s.arena, b.dev_items, b.dev_hdr,
                               b.host_items, b.ws, sl.stream);
    if (st == GALE_OK) {
        err = hipMemcpyAsync(b.host_hdr->ptr, b.dev_hdr->ptr, (size_t)n * 32, hipMemcpyDeviceToHost, sl.stream);
        if (err == hipSuccess) err = hipEventRecord(sl.done, sl.stream);
        if (err != hipSuccess) st = fail(GALE_EDEVICE, std::string("batch: ") + hipGetErrorString(err));
    }
    const Clock::time_point launched = Clock::now();
    lk.lock();
    sl.launching = false;
    if (st != GALE_OK) {
        if (st == GALE_EDEVICE) ctx->poisoned = true;
        for (int64_t key : sl.keys) {
            auto it = s.cache.find(key);
            if (it == s.cache.end()) continue;
            fail_waiters(ctx, it->second, st);
            drop_entry(s, it);
        }
        release_slot_buffers(ctx, sl);
        return true;
    }
    for (ServeReq *r : admitted)
        if (!r->ready) r->t_launched = launched;
    sl.busy = true;
    return true;
}

void lane_loop(gale_ctx *ctx, Lane *lnp) {
    Serve &s = ctx->serve;
    Lane &ln = *lnp;
    (void)hipSetDevice(ctx->cfg.device);
    std::unique_lock<std::mutex> lk(s.mu);
    while (true) {
        bool busy = false;
        for (auto &sl : ln.slots) busy |= sl.busy || sl.launching;
        if (s.stop || ctx->poisoned) {
            fail_lane(ctx, ln, s.stop ? fail(GALE_ESTATE, "context destroyed")
                                      : fail(GALE_EDEVICE, "context poisoned by a device error"));
            if (s.stop && !busy && ln.copying.empty()) break;
        }
        bool progressed = false;
        for (auto &sl : ln.slots) {
            if (!sl.busy) continue;
            const hipError_t q = hipEventQuery(sl.done);
            if (q == hipSuccess) {
                complete_slot(ctx, ln, sl);
                progressed = true;
            } else if (q != hipErrorNotReady) {
                ctx->poisoned = true;
                for (int64_t key : sl.keys) {
                    auto it = s.cache.find(key);
                    if (it == s.cache.end()) continue;
                    fail_waiters(ctx, it->second, fail(GALE_EDEVICE, hipGetErrorString(q)));
                    drop_entry(s, it);
                }
                release_slot_buffers(ctx, sl);
                sl.busy = false;
                progressed = true;
            }
        }
        for (size_t i = 0; i < ln.copying.size();) {
            ServeReq *r = ln.copying[i];
            const hipError_t q = hipEventQuery(r->copy_done);
            if (q == hipSuccess || q != hipErrorNotReady) {
                ln.copying.erase(ln.copying.begin() + (long)i);
                r->copying = false;
                r->t_copied = Clock::now();
                if (q != hipSuccess) ctx->poisoned = true;
                finish_request(ctx, r, q == hipSuccess ? GALE_OK : fail(GALE_EDEVICE, hipGetErrorString(q)));
                progressed = true;
            } else {
                ++i;
            }
        }
        if (!s.stop && !ctx->poisoned && (!ln.pending.empty() || !ln.rebuild.empty())) {
            for (auto &sl : ln.slots) {
                if (sl.busy || sl.launching) continue;
                if (admit_round(ctx, ln, sl, lk)) progressed = true;
                break;
            }
        }
        if (!progressed) {
            busy = false;
            for (auto &sl : ln.slots) busy |= sl.busy || sl.launching;
            if (busy || !ln.copying.empty())
                ln.cv_work.wait_for(lk, std::chrono::microseconds(20));
            else
                // (after a device error fail_lane empties both lists at the top
                // of every round, so this waits for new work or the stop)
                ln.cv_work.wait(lk, [&] { return s.stop || !ln.pending.empty() || !ln.rebuild.empty(); });
        }
    }
    // nothing of this lane is on the device any more: requests still waiting
    // for a block this lane would have built are failed
    for (auto &kv : s.reqs) {
        ServeReq *r = kv.second;
        if (r->parts.empty()) {
            if (r->lane == ln.index && !r->ready) finish_request(ctx, r, fail(GALE_ESTATE, "context destroyed"));
        } else {
            for (ServeReq *p : r->parts)
                if (p->lane == ln.index && !p->ready) finish_request(ctx, p, fail(GALE_ESTATE, "context destroyed"));
        }
    }
    s.cv_done.notify_all();
}

void delete_req(gale_ctx *ctx, ServeReq *r) {
    for (ServeReq *p : r->parts) delete_req(ctx, p);
    ctx->pin_pool.release(r->host);
    if (r->copy_done) (void)hipEventDestroy(r->copy_done);
    delete r;
}

// a caller inside serve_poll / serve_block / serve_release
struct CallerGuard {
    Serve &s;
    explicit CallerGuard(Serve &x) : s(x) { s.callers++; }
    ~CallerGuard() {
        if (--s.callers == 0) s.cv_idle.notify_all();
    }
};

}  // namespace

gale_status serve_start(gale_ctx *ctx) {
    Serve &s = ctx->serve;
    uint64_t budget = ctx->cfg.cache_budget_bytes ? ctx->cfg.cache_budget_bytes : (1ull << 30);
    if (ctx->cfg.dev_arena) {
        budget = ctx->cfg.cache_budget_bytes ? std::min(ctx->cfg.cache_budget_bytes, ctx->cfg.arena_bytes)
                                             : ctx->cfg.arena_bytes;
        s.arena = ctx->cfg.dev_arena;
        s.own_arena = false;
    } else {
        hipError_t e = hipMalloc(&s.arena, (size_t)budget);
        if (e != hipSuccess) return fail(GALE_ENOMEM, std::string("cache arena: ") + hipGetErrorString(e));
        s.own_arena = true;
    }
    s.arena_bytes = (int64_t)budget / kArenaAlign * kArenaAlign;
    s.free_map.clear();
    s.free_map[0] = s.arena_bytes;
    int k = ctx->cfg.max_inflight > 0 ? ctx->cfg.max_inflight : 2;
    k = std::max(1, std::min(k, 8));
    const bool per_rel = ctx->cfg.front_end == GALE_FRONT_PER_RELATION;
    const int nl = per_rel ? 3 : 1;
    for (int li = 0; li < nl; ++li) {
        auto ln = std::make_unique<Lane>();
        ln->index = li;
        ln->accept = per_rel ? (1u << li) : 7u;
        ln->slots.resize(k);
        for (auto &sl : ln->slots) {
            hipError_t e = hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking);
            if (e == hipSuccess) e = hipEventCreateWithFlags(&sl.done, hipEventDisableTiming);
            if (e != hipSuccess) return fail(GALE_EDEVICE, std::string("slot stream: ") + hipGetErrorString(e));
        }
        hipError_t e = hipStreamCreateWithFlags(&ln->copy_stream, hipStreamNonBlocking);
        if (e != hipSuccess) return fail(GALE_EDEVICE, std::string("copy stream: ") + hipGetErrorString(e));
        s.lanes.push_back(std::move(ln));
    }
    s.stop = false;
    for (auto &ln : s.lanes) ln->th = std::thread(lane_loop, ctx, ln.get());
    return GALE_OK;
}

void serve_stop(gale_ctx *ctx) {
    Serve &s = ctx->serve;
    {
        std::lock_guard<std::mutex> g(s.mu);
        s.stop = true;
    }
    for (auto &ln : s.lanes) ln->cv_work.notify_all();
    for (auto &ln : s.lanes)
        if (ln->th.joinable()) ln->th.join();
    std::unique_lock<std::mutex> lk(s.mu);
    // every request is finished now; wake its waiters and let them leave
    for (auto &kv : s.reqs)
        if (!kv.second->ready) {
            for (ServeReq *p : kv.second->parts) finish_request(ctx, p, GALE_ESTATE);
            finish_request(ctx, kv.second, GALE_ESTATE);
        }
    s.cv_done.notify_all();
    s.cv_idle.wait(lk, [&] { return s.callers == 0; });
    for (auto &kv : s.reqs) delete_req(ctx, kv.second);
    s.reqs.clear();
    for (auto &ln : s.lanes) {
        for (auto &sl : ln->slots) {
            if (sl.done) (void)hipEventDestroy(sl.done);
            if (sl.stream) (void)hipStreamDestroy(sl.stream);
        }
        if (ln->copy_stream) (void)hipStreamDestroy(ln->copy_stream);
    }
    s.lanes.clear();
    if (s.arena && s.own_arena) (void)hipFree(s.arena);
    s.arena = nullptr;
}

gale_status serve_submit(gale_ctx *ctx, const int32_t *ids, int32_t n, uint32_t mask, uint64_t *ticket) {
    gale_status st = check_request(ctx, ids, n, mask);
    if (st) return st;
    if (ctx->poisoned) return fail(GALE_EDEVICE, "context poisoned by an earlier device error");
    auto *r = new ServeReq();
    r->t_submit = Clock::now();
    r->clusters.assign(ids, ids + n);
    std::sort(r->clusters.begin(), r->clusters.end());
    r->clusters.erase(std::unique(r->clusters.begin(), r->clusters.end()), r->clusters.end());
    r->mask = mask;
    r->thread_key = std::hash<std::thread::id>()(std::this_thread::get_id());
    Serve &s = ctx->serve;
    const bool per_rel = s.lanes.size() > 1;
    std::vector<int> lanes;
    {
        std::lock_guard<std::mutex> g(s.mu);
        if (s.stop) {
            delete r;
            return fail(GALE_ESTATE, "context is being destroyed");
        }
        const int maxq = ctx->cfg.max_queue > 0 ? ctx->cfg.max_queue : 65536;
        for (auto &ln : s.lanes) {
            if ((ln->accept & mask) && (int)ln->pending.size() >= maxq) {
                delete r;
                return fail(GALE_EAGAIN, "serving queue full");
            }
        }
        {
            std::lock_guard<std::mutex> g2(ctx->tick_mu);
            r->id = ++ctx->next_ticket;
        }
        s.reqs[r->id] = r;
        if (!per_rel) {
            r->lane = 0;
            s.lanes[0]->pending.push_back(r);
            lanes.push_back(0);
        } else {
            for (int li = 0; li < (int)s.lanes.size(); ++li) {
                if (!(mask & s.lanes[li]->accept)) continue;
                auto *p = new ServeReq();
                p->id = r->id;
                p->clusters = r->clusters;
                p->mask = s.lanes[li]->accept;
                p->lane = li;
                p->parent = r;
                p->thread_key = r->thread_key;
                p->t_submit = r->t_submit;
                r->parts.push_back(p);
                r->parts_left++;
                s.lanes[li]->pending.push_back(p);
                lanes.push_back(li);
            }
        }
        const Clock::time_point now = Clock::now();
        r->t_pushed = now;
        for (ServeReq *p : r->parts) p->t_pushed = now;
        *ticket = r->id;
    }
    ctx->n_requests++;
    for (int li : lanes) s.lanes[li]->cv_work.notify_one();
    return GALE_OK;
}

gale_status serve_poll(gale_ctx *ctx, uint64_t ticket, int64_t timeout_ns) {
    Serve &s = ctx->serve;
    std::unique_lock<std::mutex> lk(s.mu);
    CallerGuard cg(s);
    auto it = s.reqs.find(ticket);
    if (it == s.reqs.end()) return fail(GALE_ENOENT, "unknown ticket");
    ServeReq *r = it->second;
    if (!r->ready) {
        if (timeout_ns == 0) return GALE_EAGAIN;
        if (timeout_ns < 0)
            s.cv_done.wait(lk, [&] { return r->ready; });
        else if (!s.cv_done.wait_for(lk, std::chrono::nanoseconds(timeout_ns), [&] { return r->ready; }))
            return GALE_EAGAIN;
    }
    return r->status ? fail(r->status, "request failed") : GALE_OK;
}

gale_status serve_block(gale_ctx *ctx, uint64_t ticket, int32_t cluster, uint32_t rel, gale_csr *out) {
    Serve &s = ctx->serve;
    std::lock_guard<std::mutex> g(s.mu);
    CallerGuard cg(s);
    auto it = s.reqs.find(ticket);
    if (it == s.reqs.end()) return fail(GALE_ENOENT, "unknown ticket");
    const ServeReq *r = it->second;
    if (!r->ready) return fail(GALE_EAGAIN, "ticket not ready");
    if (r->status) return fail(r->status, "request failed");
    if (!(r->mask & rel)) return fail(GALE_ENOENT, "relation not in ticket");
    for (const ServeReq *p : r->parts)
        if (p->mask == rel) r = p;
    auto pos = std::lower_bound(r->clusters.begin(), r->clusters.end(), cluster);
    if (pos == r->clusters.end() || *pos != cluster) return fail(GALE_ENOENT, "cluster not in ticket");
    const size_t i = (size_t)(pos - r->clusters.begin());
    const CacheEntry &e = r->snap[i];
    const ClusterMeta &m = ctx->meta[cluster];
    const BlockLayout lay = block_layout(e.mask, m.nV, m.nT, m.nnzVT, e.cap_vv, e.cap_tt);
    const int32_t *base = (const int32_t *)r->host->ptr + r->host_word[i];
    out->cluster = cluster;
    out->rel = rel;
    out->pad = 0;
    if (rel == GALE_REL_VT) {
        out->nrows = m.nV; out->nnz = e.hdr[3];
        out->row_ids = base + lay.vrows; out->offsets = base + lay.vt_off; out->entries = base + lay.vt_ent;
    } else if (rel == GALE_REL_VV) {
        out->nrows = m.nV; out->nnz = e.hdr[4];
        out->row_ids = base + lay.vrows; out->offsets = base + lay.vv_off; out->entries = base + lay.vv_ent;
    } else {
        out->nrows = m.nT; out->nnz = e.hdr[5];
        out->row_ids = base + lay.trows; out->offsets = base + lay.tt_off; out->entries = base + lay.tt_ent;
    }
    return GALE_OK;
}

gale_status serve_release(gale_ctx *ctx, uint64_t ticket) {
    Serve &s = ctx->serve;
    std::unique_lock<std::mutex> lk(s.mu);
    ServeReq *r = nullptr;
    {
        CallerGuard cg(s);
        auto it = s.reqs.find(ticket);
        if (it == s.reqs.end()) return fail(GALE_ENOENT, "unknown or released ticket");
        r = it->second;
        s.cv_done.wait(lk, [&] { return r->ready; });
        s.reqs.erase(ticket);
    }
    delete_req(ctx, r);
    return GALE_OK;
}

void serve_stats(gale_ctx *ctx, gale_stats *out) {
    Serve &s = ctx->serve;
    std::lock_guard<std::mutex> g(s.mu);
    out->cache_hits = s.hits;
    out->cache_misses = s.misses;
    out->evictions = s.evictions;
    out->cache_bytes_resident = (uint64_t)s.resident_bytes;
    out->cache_budget = (uint64_t)s.arena_bytes;
    out->batches = s.batches;
    out->mean_batch_clusters = s.batches ? (double)s.batch_clusters / (double)s.batches : 0.0;
    out->queue_depth_mean = s.admissions ? (double)s.depth_sum / (double)s.admissions : 0.0;
    out->queue_depth_max = s.depth_max;
    out->lat_p50_us = s.lat.percentile(0.50);
    out->lat_p99_us = s.lat.percentile(0.99);
    out->lat_mean_us = s.lat.count ? s.lat.sum / (double)s.lat.count : 0.0;
    out->lat_max_us = s.lat.mx;
    out->lat_count = s.lat.count;
    const double n = s.n_stage ? (double)s.n_stage : 1.0;
    out->stage_queue_us = s.stage_sum[0] / n;
    out->stage_build_us = s.stage_sum[1] / n;
    out->stage_copy_us = s.stage_sum[2] / n;
    out->stage_push_us = s.stage_sum[3] / n;
    out->stage_prep_us = s.stage_sum[5] / n;
    out->stage_kernel_copy_us = s.stage_sum[6] / n;
    out->stage_integration_us = s.stage_sum[7] / n;
    double mx[5] = {0, 0, 0, 0, 0};
    for (auto &kv : s.per_thread)
        for (int i = 0; i < 5; ++i) mx[i] = std::max(mx[i], kv.second[i]);
    out->wait_push_s_max = mx[0];
    out->wait_queue_s_max = mx[1];
    out->wait_prep_s_max = mx[2];
    out->wait_kernel_copy_s_max = mx[3];
    out->wait_integration_s_max = mx[4];
    out->prefetch_built = s.prefetch_built;
    out->prefetch_hits = s.prefetch_hits;
    out->prefetch_evicted = s.prefetch_evicted;
    out->demand_evictions = s.demand_evictions;
}

void serve_reset_stats(gale_ctx *ctx) {
    Serve &s = ctx->serve;
    std::lock_guard<std::mutex> g(s.mu);
    s.hits = s.misses = s.evictions = s.batches = s.batch_clusters = 0;
    s.admissions = s.depth_sum = 0;
    s.depth_max = 0;
    s.prefetch_built = s.prefetch_hits = s.prefetch_evicted = s.demand_evictions = 0;
    s.lat.clear();
    s.n_stage = 0;
    for (double &x : s.stage_sum) x = 0.0;
    s.per_thread.clear();
}

}  // namespace gale
