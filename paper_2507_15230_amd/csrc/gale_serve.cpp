// gale_serve.cpp -- the serving loop: continuous batching over an HBM cache.
//
// The paper's consumers push (segment, consumer) requests into per-relation
// queues; a leader thread per queue pops every pending request, launches one
// kernel for the whole batch into preallocated GPU memory, copies the results
// back and wakes the consumers through semaphores; kernels of different
// leaders run concurrently (Sections 4.2, 4.4, 4.5).  Here:
//   * gale_submit appends the request to one pending queue and returns;
//   * a service thread admits every pending request whose blocks fit: a block
//     already resident in the HBM cache is a hit, one being built is joined,
//     a missing one gets space in the cache arena (least-recently-used
//     unpinned blocks are evicted until it fits the byte budget) and goes into
//     the next batch;
//   * a batch is one persistent-kernel launch writing straight into the
//     arena, on one of max_inflight slots (streams), so requests that arrive
//     while earlier batches run are admitted into the next free slot and their
//     work overlaps on the device;
//   * when all of a request's blocks are resident they are copied to a pinned
//     host buffer (one copy per block on a copy stream) and the request
//     becomes ready; gale_poll waits on a condition variable.
// Blocks stay pinned while a request waits for or copies them.  The same
// kernel and the same block layout as the direct path make every served
// block byte-identical to a block built alone.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>

#include "gale_ctx.h"

namespace gale {

namespace {

constexpr int64_t kArenaAlign = 256;

int64_t round_up(int64_t b, int64_t a) { return (b + a - 1) / a * a; }

int64_t cache_key(int32_t cluster, uint32_t mask) { return (int64_t)cluster * 8 + (int64_t)mask; }

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

void unpin(Serve &s, int64_t key) {
    auto it = s.cache.find(key);
    if (it == s.cache.end()) return;
    CacheEntry &e = it->second;
    if (--e.pins == 0 && e.state == 1) {
        s.lru.push_back(key);
        e.lru_it = std::prev(s.lru.end());
        e.in_lru = true;
    }
}

void pin(Serve &s, CacheEntry &e) {
    if (e.pins++ == 0 && e.in_lru) {
        s.lru.erase(e.lru_it);
        e.in_lru = false;
    }
}

bool evict_one(Serve &s) {
    if (s.lru.empty()) return false;
    const int64_t key = s.lru.front();
    s.lru.pop_front();
    auto it = s.cache.find(key);
    if (it != s.cache.end()) {
        arena_free(s, it->second.off, it->second.bytes);
        s.resident_bytes -= it->second.bytes;
        s.cache.erase(it);
        s.evictions++;
    }
    return true;
}

// allocate with eviction; -1 if it cannot fit now
int64_t alloc_evicting(Serve &s, int64_t bytes) {
    int64_t off = arena_alloc(s, bytes);
    while (off < 0 && evict_one(s)) off = arena_alloc(s, bytes);
    return off;
}

void finish_request(gale_ctx *ctx, ServeReq *r, gale_status st) {
    Serve &s = ctx->serve;
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
    if (st == GALE_OK) {
        auto us = [](Clock::time_point a, Clock::time_point b) {
            return std::chrono::duration<double, std::micro>(b - a).count();
        };
        s.lat_us.push_back(us(r->t_submit, r->t_ready));
        s.q_us.push_back(us(r->t_submit, r->t_admit));
        s.b_us.push_back(us(r->t_admit, r->t_built));
        s.c_us.push_back(us(r->t_built, r->t_ready));
    }
    s.cv_done.notify_all();
}

// all blocks of r are resident: copy them to a pinned host buffer
void start_copy(gale_ctx *ctx, ServeReq *r) {
    Serve &s = ctx->serve;
    r->t_built = Clock::now();
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
                             hipMemcpyDeviceToHost, s.copy_stream);
        bytes += (uint64_t)b;
        if (e.mask & kRelVT) ent += (uint64_t)e.hdr[3];
        if (e.mask & kRelVV) ent += (uint64_t)e.hdr[4];
        if (e.mask & kRelTT) ent += (uint64_t)e.hdr[5];
    }
    if (err == hipSuccess && !r->copy_done) err = hipEventCreateWithFlags(&r->copy_done, hipEventDisableTiming);
    if (err == hipSuccess) err = hipEventRecord(r->copy_done, s.copy_stream);
    if (err != hipSuccess) {
        ctx->poisoned = true;
        finish_request(ctx, r, fail(GALE_EDEVICE, std::string("copy: ") + hipGetErrorString(err)));
        return;
    }
    ctx->n_bytes_d2h += bytes;
    ctx->n_delivered += ent;
    r->copying = true;
    s.copying.push_back(r);
}

void fail_waiters(gale_ctx *ctx, CacheEntry &e, gale_status st) {
    std::vector<ServeReq *> w;
    w.swap(e.waiters);
    for (ServeReq *r : w)
        if (!r->ready) finish_request(ctx, r, st);
}

// a slot's batch finished on the GPU
void complete_slot(gale_ctx *ctx, Slot &sl, std::vector<int64_t> &rebuild) {
    Serve &s = ctx->serve;
    const int n = (int)sl.batch.items.size();
    hipError_t err = hipMemcpyAsync(sl.batch.host_hdr->ptr, sl.batch.dev_hdr->ptr, (size_t)n * 32,
                                    hipMemcpyDeviceToHost, sl.stream);
    if (err == hipSuccess) err = hipStreamSynchronize(sl.stream);
    const int32_t *hdr = (const int32_t *)sl.batch.host_hdr->ptr;
    for (int i = 0; i < n; ++i) {
        auto it = s.cache.find(sl.keys[i]);
        if (it == s.cache.end()) continue;
        CacheEntry &e = it->second;
        const int32_t *h = hdr + (size_t)i * 8;
        if (err != hipSuccess || (h[0] & kStInconsistent)) {
            ctx->poisoned = true;
            fail_waiters(ctx, e, fail(GALE_EDEVICE, err != hipSuccess ? std::string(hipGetErrorString(err))
                                                                      : std::string("stream metadata mismatch")));
            continue;
        }
        const ClusterMeta &m = ctx->meta[e.cluster];
        if (h[0] & (kStVVOverflow | kStTTOverflow)) {
            // rebuild with exact capacities in the next batch
            arena_free(s, e.off, e.bytes);
            e.cap_vv = (e.mask & kRelVV) ? std::max(h[4], 0) : 0;
            e.cap_tt = (e.mask & kRelTT) ? std::max(h[5], default_cap_tt(m)) : 0;
            e.bytes = round_up(block_bytes(m, e.mask, e.cap_vv, e.cap_tt), kArenaAlign);
            e.off = -1;
            rebuild.push_back(sl.keys[i]);
            ctx->n_overflow++;
            continue;
        }
        std::memcpy(e.hdr, h, sizeof(e.hdr));
        if (h[0] & kStTTFallback) ctx->n_tt_exhaustive++;
        e.state = 1;
        if (e.pins == 0 && !e.in_lru) {
            s.lru.push_back(sl.keys[i]);
            e.lru_it = std::prev(s.lru.end());
            e.in_lru = true;
        }
        // give back the unused VV tail
        const int64_t used = round_up(block_bytes(m, e.mask, (e.mask & kRelVV) ? h[4] : 0, e.cap_tt), kArenaAlign);
        if (used < e.bytes) {
            arena_free(s, e.off + used, e.bytes - used);
            e.bytes = used;
        }
        s.resident_bytes += e.bytes;
        if (e.mask & kRelVT) ctx->n_entries += (uint64_t)h[3];
        if (e.mask & kRelVV) ctx->n_entries += (uint64_t)h[4];
        if (e.mask & kRelTT) ctx->n_entries += (uint64_t)h[5];
        ctx->n_blocks++;
        std::vector<ServeReq *> w;
        w.swap(e.waiters);
        for (ServeReq *r : w) {
            if (r->ready) continue;
            if (--r->waiting == 0) start_copy(ctx, r);
        }
    }
    ctx->dev_pool.release(sl.batch.dev_items);
    ctx->dev_pool.release(sl.batch.dev_hdr);
    ctx->dev_pool.release(sl.batch.ws);
    ctx->pin_pool.release(sl.batch.host_items);
    ctx->pin_pool.release(sl.batch.host_hdr);
    sl.batch = Batch();
    sl.keys.clear();
    sl.busy = false;
}

// Admit pending requests and launch one batch on slot sl.  Returns true if a
// batch was launched.
bool admit_round(gale_ctx *ctx, Slot &sl, std::vector<int64_t> &rebuild) {
    Serve &s = ctx->serve;
    std::vector<int64_t> build_keys;
    // blocks to rebuild with exact capacities come first
    std::vector<int64_t> still;
    for (int64_t key : rebuild) {
        auto it = s.cache.find(key);
        if (it == s.cache.end()) continue;
        CacheEntry &e = it->second;
        const int64_t off = alloc_evicting(s, e.bytes);
        if (off < 0) {
            still.push_back(key);
            continue;
        }
        e.off = off;
        build_keys.push_back(key);
    }
    rebuild.swap(still);
    if (!s.pending.empty()) {
        const int depth = (int)s.pending.size();
        s.admissions++;
        s.depth_sum += depth;
        s.depth_max = std::max(s.depth_max, depth);
    }
    while (!s.pending.empty()) {
        ServeReq *r = s.pending.front();
        // phase 1: pin hits and joins, allocate misses
        std::vector<int64_t> held, fresh;
        bool ok = true;
        gale_status why = GALE_OK;
        for (int32_t k : r->clusters) {
            const int64_t key = cache_key(k, r->mask);
            auto it = s.cache.find(key);
            if (it != s.cache.end()) {
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
            const int64_t off = alloc_evicting(s, bytes);
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
                if (it != s.cache.end()) {
                    arena_free(s, it->second.off, it->second.bytes);
                    s.cache.erase(it);
                }
            }
            for (int64_t key : held)
                if (std::find(fresh.begin(), fresh.end(), key) == fresh.end()) unpin(s, key);
            bool others_hold = false;
            for (auto &kv : s.cache)
                if (kv.second.pins > 0) others_hold = true;
            for (auto &x : s.slots)
                if (x.busy) others_hold = true;
            if (why != GALE_OK || (!others_hold && build_keys.empty())) {
                s.pending.pop_front();
                finish_request(ctx, r, why != GALE_OK ? why
                                                      : fail(GALE_ENOMEM, "request does not fit the cache budget"));
                continue;
            }
            break;  // wait for space; keep FIFO order
        }
        s.pending.pop_front();
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
        if (r->waiting == 0) start_copy(ctx, r);
    }
    if (build_keys.empty()) return false;

    // launch
    Batch &b = sl.batch;
    b = Batch();
    for (int64_t key : build_keys) {
        const CacheEntry &e = s.cache[key];
        WorkItem it{};
        it.cluster = e.cluster;
        it.mask = e.mask;
        it.cap_vv = e.cap_vv;
        it.cap_tt = e.cap_tt;
        it.out_word = e.off / 4;
        b.items.push_back(it);
    }
    // largest streams first
    std::vector<int> order(b.items.size());
    for (size_t i = 0; i < order.size(); ++i) order[i] = (int)i;
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
        const ClusterMeta &a = ctx->meta[b.items[x].cluster], &c = ctx->meta[b.items[y].cluster];
        return (int64_t)a.ns + a.nh > (int64_t)c.ns + c.nh;
    });
    std::vector<WorkItem> items;
    sl.keys.clear();
    for (int i : order) {
        items.push_back(b.items[i]);
        sl.keys.push_back(build_keys[i]);
    }
    for (size_t i = 0; i < items.size(); ++i) items[i].hdr_index = (int32_t)i;
    b.items = items;
    const int n = (int)items.size();
    hipError_t err;
    gale_status st = GALE_OK;
    b.host_hdr = ctx->pin_pool.acquire((size_t)n * 32 + 64, &err);
    if (!b.host_hdr) st = fail(GALE_ENOMEM, "serving batch buffers");
    if (st == GALE_OK)
        st = upload_and_launch(ctx, GALE_FORM_BATCHED, items, (int32_t *)s.arena, b.dev_items, b.dev_hdr,
                               b.host_items, b.ws, sl.stream);
    if (st == GALE_OK) {
        err = hipEventRecord(sl.done, sl.stream);
        if (err != hipSuccess) st = fail(GALE_EDEVICE, std::string("event: ") + hipGetErrorString(err));
    }
    if (st != GALE_OK) {
        if (st == GALE_EDEVICE) ctx->poisoned = true;
        for (int64_t key : sl.keys) {
            auto it = s.cache.find(key);
            if (it == s.cache.end()) continue;
            fail_waiters(ctx, it->second, st);
            arena_free(s, it->second.off, it->second.bytes);
            s.cache.erase(it);
        }
        ctx->dev_pool.release(b.dev_items);
        ctx->dev_pool.release(b.dev_hdr);
        ctx->dev_pool.release(b.ws);
        ctx->pin_pool.release(b.host_items);
        ctx->pin_pool.release(b.host_hdr);
        b = Batch();
        sl.keys.clear();
        return false;
    }
    s.batches++;
    s.batch_clusters += (uint64_t)n;
    sl.busy = true;
    return true;
}

void service_loop(gale_ctx *ctx) {
    Serve &s = ctx->serve;
    (void)hipSetDevice(ctx->cfg.device);
    std::vector<int64_t> rebuild;
    std::unique_lock<std::mutex> lk(s.mu);
    while (true) {
        bool busy = false;
        for (auto &sl : s.slots) busy |= sl.busy;
        if (s.stop) {
            while (!s.pending.empty()) {
                ServeReq *r = s.pending.front();
                s.pending.pop_front();
                finish_request(ctx, r, fail(GALE_ESTATE, "context destroyed"));
            }
            if (!busy && s.copying.empty()) break;
        }
        bool progressed = false;
        for (auto &sl : s.slots) {
            if (!sl.busy) continue;
            const hipError_t q = hipEventQuery(sl.done);
            if (q == hipSuccess) {
                complete_slot(ctx, sl, rebuild);
                progressed = true;
            } else if (q != hipErrorNotReady) {
                ctx->poisoned = true;
                for (int64_t key : sl.keys) {
                    auto it = s.cache.find(key);
                    if (it != s.cache.end()) fail_waiters(ctx, it->second, fail(GALE_EDEVICE, hipGetErrorString(q)));
                }
                sl.busy = false;
                progressed = true;
            }
        }
        for (size_t i = 0; i < s.copying.size();) {
            ServeReq *r = s.copying[i];
            const hipError_t q = hipEventQuery(r->copy_done);
            if (q == hipSuccess || q != hipErrorNotReady) {
                s.copying.erase(s.copying.begin() + (long)i);
                r->copying = false;
                finish_request(ctx, r, q == hipSuccess ? GALE_OK : fail(GALE_EDEVICE, hipGetErrorString(q)));
                progressed = true;
            } else {
                ++i;
            }
        }
        if (!s.stop && (!s.pending.empty() || !rebuild.empty())) {
            for (auto &sl : s.slots) {
                if (sl.busy) continue;
                if (admit_round(ctx, sl, rebuild)) progressed = true;
                break;
            }
        }
        if (!progressed) {
            busy = false;
            for (auto &sl : s.slots) busy |= sl.busy;
            if (busy || !s.copying.empty())
                s.cv_work.wait_for(lk, std::chrono::microseconds(20));
            else
                s.cv_work.wait(lk, [&] { return s.stop || !s.pending.empty() || !rebuild.empty(); });
        }
    }
}

double percentile(std::vector<double> v, double p) {
    if (v.empty()) return 0.0;
    std::sort(v.begin(), v.end());
    const double x = p * (double)(v.size() - 1);
    const size_t i = (size_t)x;
    const double f = x - (double)i;
    return i + 1 < v.size() ? v[i] * (1 - f) + v[i + 1] * f : v[i];
}

double mean(const std::vector<double> &v) {
    if (v.empty()) return 0.0;
    double s = 0;
    for (double x : v) s += x;
    return s / (double)v.size();
}

}  // namespace

gale_status serve_start(gale_ctx *ctx) {
    Serve &s = ctx->serve;
    const uint64_t budget = ctx->cfg.cache_budget_bytes ? ctx->cfg.cache_budget_bytes : (1ull << 30);
    hipError_t e = hipMalloc(&s.arena, (size_t)budget);
    if (e != hipSuccess) return fail(GALE_ENOMEM, std::string("cache arena: ") + hipGetErrorString(e));
    s.arena_bytes = (int64_t)budget / kArenaAlign * kArenaAlign;
    s.free_map.clear();
    s.free_map[0] = s.arena_bytes;
    int k = ctx->cfg.max_inflight > 0 ? ctx->cfg.max_inflight : 2;
    k = std::max(1, std::min(k, 8));
    s.slots.resize(k);
    for (auto &sl : s.slots) {
        e = hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&sl.done, hipEventDisableTiming);
        if (e != hipSuccess) return fail(GALE_EDEVICE, std::string("slot stream: ") + hipGetErrorString(e));
    }
    e = hipStreamCreateWithFlags(&s.copy_stream, hipStreamNonBlocking);
    if (e != hipSuccess) return fail(GALE_EDEVICE, std::string("copy stream: ") + hipGetErrorString(e));
    s.stop = false;
    s.th = std::thread(service_loop, ctx);
    return GALE_OK;
}

void serve_stop(gale_ctx *ctx) {
    Serve &s = ctx->serve;
    if (!s.th.joinable()) return;
    {
        std::lock_guard<std::mutex> g(s.mu);
        s.stop = true;
    }
    s.cv_work.notify_all();
    s.th.join();
    std::lock_guard<std::mutex> g(s.mu);
    for (auto &kv : s.reqs) {
        ServeReq *r = kv.second;
        if (r->copy_done) (void)hipEventDestroy(r->copy_done);
        delete r;
    }
    s.reqs.clear();
    for (auto &sl : s.slots) {
        if (sl.done) (void)hipEventDestroy(sl.done);
        if (sl.stream) (void)hipStreamDestroy(sl.stream);
    }
    s.slots.clear();
    if (s.copy_stream) (void)hipStreamDestroy(s.copy_stream);
    if (s.arena) (void)hipFree(s.arena);
    s.arena = nullptr;
}

gale_status serve_submit(gale_ctx *ctx, const int32_t *ids, int32_t n, uint32_t mask, uint64_t *ticket) {
    gale_status st = check_request(ctx, ids, n, mask);
    if (st) return st;
    if (ctx->poisoned) return fail(GALE_EDEVICE, "context poisoned by an earlier device error");
    auto *r = new ServeReq();
    r->clusters.assign(ids, ids + n);
    std::sort(r->clusters.begin(), r->clusters.end());
    r->clusters.erase(std::unique(r->clusters.begin(), r->clusters.end()), r->clusters.end());
    r->mask = mask;
    r->t_submit = Clock::now();
    Serve &s = ctx->serve;
    {
        std::lock_guard<std::mutex> g(s.mu);
        if (s.stop) {
            delete r;
            return fail(GALE_ESTATE, "context is being destroyed");
        }
        const int maxq = ctx->cfg.max_queue > 0 ? ctx->cfg.max_queue : 65536;
        if ((int)s.pending.size() >= maxq) {
            delete r;
            return fail(GALE_EAGAIN, "serving queue full");
        }
        std::lock_guard<std::mutex> g2(ctx->tick_mu);
        r->id = ++ctx->next_ticket;
        s.reqs[r->id] = r;
        s.pending.push_back(r);
        *ticket = r->id;
    }
    ctx->n_requests++;
    s.cv_work.notify_one();
    return GALE_OK;
}

gale_status serve_poll(gale_ctx *ctx, uint64_t ticket, int64_t timeout_ns) {
    Serve &s = ctx->serve;
    std::unique_lock<std::mutex> lk(s.mu);
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
    auto it = s.reqs.find(ticket);
    if (it == s.reqs.end()) return fail(GALE_ENOENT, "unknown ticket");
    ServeReq *r = it->second;
    if (!r->ready) return fail(GALE_EAGAIN, "ticket not ready");
    if (r->status) return fail(r->status, "request failed");
    if (!(r->mask & rel)) return fail(GALE_ENOENT, "relation not in ticket");
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
    auto it = s.reqs.find(ticket);
    if (it == s.reqs.end()) return fail(GALE_ENOENT, "unknown or released ticket");
    ServeReq *r = it->second;
    s.cv_done.wait(lk, [&] { return r->ready; });
    s.reqs.erase(it);
    ctx->pin_pool.release(r->host);
    if (r->copy_done) (void)hipEventDestroy(r->copy_done);
    delete r;
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
    out->lat_p50_us = percentile(s.lat_us, 0.50);
    out->lat_p99_us = percentile(s.lat_us, 0.99);
    out->lat_mean_us = mean(s.lat_us);
    out->lat_max_us = s.lat_us.empty() ? 0.0 : *std::max_element(s.lat_us.begin(), s.lat_us.end());
    out->lat_count = s.lat_us.size();
    out->stage_queue_us = mean(s.q_us);
    out->stage_build_us = mean(s.b_us);
    out->stage_copy_us = mean(s.c_us);
}

void serve_reset_stats(gale_ctx *ctx) {
    Serve &s = ctx->serve;
    std::lock_guard<std::mutex> g(s.mu);
    s.hits = s.misses = s.evictions = s.batches = s.batch_clusters = 0;
    s.admissions = s.depth_sum = 0;
    s.depth_max = 0;
    s.lat_us.clear();
    s.q_us.clear();
    s.b_us.clear();
    s.c_us.clear();
}

}  // namespace gale
