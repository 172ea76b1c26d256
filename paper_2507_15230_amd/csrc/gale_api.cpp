// gale_api.cpp -- the C ABI: context, mesh load, requests, tickets, views.
//
// A request names cluster ids and a relation mask (the paper's consumer
// request carries a segment and its consumer, Section 4.4).  DIRECT mode runs
// it on the caller's thread: the plain form launches one kernel per
// (cluster, relation), the batched form one persistent kernel over a device
// work queue holding every requested cluster, largest first (the leader's
// batch of all pending requests, Section 4.5).  SERVE mode (gale_serve.cpp)
// queues requests for a service thread with an HBM cache.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "gale_ctx.h"

namespace gale {

thread_local std::string t_last_error;

gale_status fail(gale_status s, const std::string &msg) {
    t_last_error = msg;
    return s;
}

// ---------------------------------------------------------------------------
// buffer pools (grow-only; buffers are reused by size)
// ---------------------------------------------------------------------------
Buf *Pool::acquire(size_t bytes, hipError_t *err) {
    *err = hipSuccess;
    std::lock_guard<std::mutex> g(mu);
    Buf *best = nullptr;
    for (Buf *b : free_list)
        if (b->bytes >= bytes && (!best || b->bytes < best->bytes)) best = b;
    if (best) {
        free_list.erase(std::find(free_list.begin(), free_list.end(), best));
        return best;
    }
    Buf *b = new Buf();
    b->bytes = std::max<size_t>(bytes, 256);
    b->pinned = pinned;
    *err = pinned ? hipHostMalloc(&b->ptr, b->bytes, hipHostMallocDefault) : hipMalloc(&b->ptr, b->bytes);
    if (*err != hipSuccess) {
        delete b;
        return nullptr;
    }
    all.push_back(b);
    return b;
}

void Pool::release(Buf *b) {
    if (!b) return;
    std::lock_guard<std::mutex> g(mu);
    free_list.push_back(b);
}

void Pool::clear() {
    std::lock_guard<std::mutex> g(mu);
    for (Buf *b : all) {
        if (b->pinned)
            (void)hipHostFree(b->ptr);
        else
            (void)hipFree(b->ptr);
        delete b;
    }
    all.clear();
    free_list.clear();
}

// ---------------------------------------------------------------------------
// batch building (shared by DIRECT and SERVE)
// ---------------------------------------------------------------------------
int32_t default_cap_tt(const ClusterMeta &m) { return 4 * m.nT; }

// Fill items (out_word relative to out_base_word) for the requested
// (cluster, mask) pairs.  Returns the total words needed.
int64_t lay_out_items(const gale_ctx *ctx, std::vector<WorkItem> &items, int64_t out_base_word) {
    int64_t w = out_base_word;
    for (size_t i = 0; i < items.size(); ++i) {
        WorkItem &it = items[i];
        const ClusterMeta &m = ctx->meta[it.cluster];
        if (it.cap_vv < 0) it.cap_vv = (it.mask & kRelVV) ? m.cap_vv : 0;
        if (it.cap_tt < 0) it.cap_tt = (it.mask & kRelTT) ? default_cap_tt(m) : 0;
        const BlockLayout lay = block_layout(it.mask, m.nV, m.nT, m.nnzVT, it.cap_vv, it.cap_tt);
        it.out_word = w;
        it.hdr_index = (int32_t)i;
        w += lay.total;
    }
    return w - out_base_word;
}

bool item_on_lds_path(const gale_ctx *ctx, const WorkItem &it) {
    return lds_plan(ctx->meta[it.cluster], it.mask, ctx->lds_budget, ctx->block_threads).ok != 0;
}

int64_t workspace_bytes(const gale_ctx *ctx, const std::vector<WorkItem> &items, int *n_global) {
    int64_t need = 0;
    int ng = 0;
    for (const WorkItem &it : items) {
        if (!item_on_lds_path(ctx, it)) {
            const Plan gp = ws_plan(ctx->meta[it.cluster], it.mask, ctx->block_threads);
            need = std::max<int64_t>(need, gp.bytes);
            ++ng;
        }
    }
    if (n_global) *n_global = ng;
    return align16(need);
}

KArgs base_args(const gale_ctx *ctx) {
    KArgs a{};
    a.s.tets = reinterpret_cast<const char *>(ctx->d_tets);
    a.s.tid = ctx->d_tid;
    a.s.lverts = ctx->d_lverts;
    a.s.meta = ctx->d_meta;
    a.lds_budget = (int32_t)ctx->lds_budget;
    return a;
}

void destroy_ticket_events(Ticket *t) {
    for (hipEvent_t &e : t->batch.kev) {
        if (e) (void)hipEventDestroy(e);
        e = nullptr;
    }
}

// Launch items already uploaded in launch order: the first n_lds take the
// LDS path, the next n_glob the global-workspace path.  PLAIN: one launch per
// item; BATCHED: one persistent launch per path, each with its own queue word.
gale_status launch_batch(gale_ctx *ctx, int form, int32_t *d_out, int32_t *d_hdr, const WorkItem *d_items,
                         int n_lds, int n_glob, int32_t *d_queue, char *d_ws, int64_t ws_stride, hipStream_t st,
                         const hipEvent_t *kev, bool *kev_recorded) {
    KArgs a = base_args(ctx);
    a.out = d_out;
    a.hdr = d_hdr;
    a.ws = d_ws;
    a.ws_stride = ws_stride;
    hipError_t e = hipSuccess;
    if (form == GALE_FORM_PLAIN) {
        for (int i = 0; i < n_lds + n_glob && e == hipSuccess; ++i) {
            a.items = d_items + i;
            a.nitems = 1;
            e = launch_items(a, i < n_lds, ctx->block_threads, 1, ctx->lds_budget, st);
            ctx->n_launches++;
        }
    } else {
        if (n_lds > 0) {
            a.items = d_items;
            a.nitems = n_lds;
            a.queue = d_queue;
            if (kev) e = hipEventRecord(kev[0], st);
            if (e == hipSuccess)
                e = launch_persistent(a, true, ctx->block_threads, std::min<int>(n_lds, ctx->grid_lds),
                                      ctx->lds_budget, st);
            if (kev && e == hipSuccess) e = hipEventRecord(kev[1], st);
            if (kev && kev_recorded && e == hipSuccess) *kev_recorded = true;
            ctx->n_launches++;
        }
        if (n_glob > 0 && e == hipSuccess) {
            a.items = d_items + n_lds;
            a.nitems = n_glob;
            a.queue = d_queue + 1;
            e = launch_persistent(a, false, ctx->block_threads, std::min<int>(n_glob, ctx->grid_glob), 0, st);
            ctx->n_launches++;
        }
    }
    if (e != hipSuccess) return fail(GALE_EDEVICE, std::string("kernel launch: ") + hipGetErrorString(e));
    return GALE_OK;
}

// Upload items (layout order in `items`, with out_word and hdr_index set) in
// launch order with two zero queue words, and launch.  Buffers come from the
// pools; the caller releases them.
gale_status upload_and_launch(gale_ctx *ctx, int form, const std::vector<WorkItem> &items, int32_t *d_out,
                              Buf *&dev_items, Buf *&dev_hdr, Buf *&host_items, Buf *&ws, hipStream_t st,
                              const hipEvent_t *kev, bool *kev_recorded) {
    hipError_t e;
    const int n = (int)items.size();
    std::vector<WorkItem> order;
    order.reserve(n);
    for (const WorkItem &it : items)
        if (item_on_lds_path(ctx, it)) order.push_back(it);
    const int n_lds = (int)order.size();
    for (const WorkItem &it : items)
        if (!item_on_lds_path(ctx, it)) order.push_back(it);
    const int n_glob = n - n_lds;
    const int64_t wsb = workspace_bytes(ctx, items, nullptr);
    ctx->n_global_blocks += n_glob;
    const int slots = form == GALE_FORM_PLAIN ? 1 : std::min<int>(std::max(n_glob, 1), ctx->grid_glob);
    dev_items = ctx->dev_pool.acquire((size_t)n * sizeof(WorkItem) + 64, &e);
    dev_hdr = ctx->dev_pool.acquire((size_t)n * 32 + 64, &e);
    host_items = ctx->pin_pool.acquire((size_t)n * sizeof(WorkItem) + 64, &e);
    if (!dev_items || !dev_hdr || !host_items) return fail(GALE_ENOMEM, "batch buffers");
    if (n_glob > 0) {
        ws = ctx->dev_pool.acquire((size_t)wsb * slots, &e);
        if (!ws) return fail(GALE_ENOMEM, "workspace");
    }
    char *hi = (char *)host_items->ptr;
    std::memset(hi, 0, 64);
    std::memcpy(hi + 64, order.data(), (size_t)n * sizeof(WorkItem));
    e = hipMemcpyAsync(dev_items->ptr, hi, (size_t)n * sizeof(WorkItem) + 64, hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return fail(GALE_EDEVICE, std::string("work list copy: ") + hipGetErrorString(e));
    char *di = (char *)dev_items->ptr;
    return launch_batch(ctx, form, d_out, (int32_t *)dev_hdr->ptr, (const WorkItem *)(di + 64), n_lds, n_glob,
                        (int32_t *)di, ws ? (char *)ws->ptr : nullptr, wsb, st, kev, kev_recorded);
}

// Lay out the batch's items in a fresh output buffer and launch them.
gale_status run_items(gale_ctx *ctx, Batch &b, int form, hipStream_t st) {
    hipError_t e;
    const int n = (int)b.items.size();
    b.out_words = lay_out_items(ctx, b.items, 0);
    b.out = ctx->dev_pool.acquire((size_t)b.out_words * 4 + 256, &e);
    if (!b.out) return fail(GALE_ENOMEM, "device output buffer");
    b.host_hdr = ctx->pin_pool.acquire((size_t)n * 32 + 64, &e);
    if (!b.host_hdr) return fail(GALE_ENOMEM, "batch buffers");
    if (n == 0) return GALE_OK;
    return upload_and_launch(ctx, form, b.items, (int32_t *)b.out->ptr, b.dev_items, b.dev_hdr, b.host_items, b.ws,
                             st, b.kev[0] ? b.kev : nullptr, &b.kev_recorded);
}

void release_batch(gale_ctx *ctx, Batch &b) {
    ctx->dev_pool.release(b.out);
    ctx->dev_pool.release(b.dev_items);
    ctx->dev_pool.release(b.dev_hdr);
    ctx->dev_pool.release(b.ws);
    ctx->pin_pool.release(b.host_items);
    ctx->pin_pool.release(b.host_hdr);
    ctx->pin_pool.release(b.host_out);
    b.out = b.dev_items = b.dev_hdr = b.ws = b.host_items = b.host_hdr = b.host_out = nullptr;
}

// After the batch's kernels finished: read the headers, rebuild the blocks
// whose capacity bound was exceeded with exact capacities, and check
// consistency.  Synchronous on st.
gale_status finalize_batch(gale_ctx *ctx, Batch &b, hipStream_t st) {
    const int n = (int)b.items.size();
    hipError_t e = n ? hipMemcpyAsync(b.host_hdr->ptr, b.dev_hdr->ptr, (size_t)n * 32, hipMemcpyDeviceToHost, st)
                     : hipSuccess;
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return fail(GALE_EDEVICE, std::string("header copy: ") + hipGetErrorString(e));
    b.hdr.assign((int32_t *)b.host_hdr->ptr, (int32_t *)b.host_hdr->ptr + (size_t)n * 8);
    b.loc.assign(n, BlockLoc{b.out, 0});
    for (int i = 0; i < n; ++i) b.loc[i].word = b.items[i].out_word;
    std::vector<int> redo;
    for (int i = 0; i < n; ++i) {
        const int32_t *h = &b.hdr[(size_t)i * 8];
        if (h[0] & kStInconsistent)
            return fail(GALE_EDEVICE, "stream metadata of cluster " + std::to_string(b.items[i].cluster) +
                                          " disagrees with the kernel's counts");
        if (h[0] & (kStVVOverflow | kStTTOverflow)) redo.push_back(i);
        if (h[0] & kStTTFallback) ctx->n_tt_exhaustive++;
    }
    if (!redo.empty()) {
        Batch r;
        for (int i : redo) {
            WorkItem it = b.items[i];
            const int32_t *h = &b.hdr[(size_t)i * 8];
            it.cap_vv = (it.mask & kRelVV) ? std::max(h[4], 0) : 0;
            it.cap_tt = (it.mask & kRelTT) ? std::max(h[5], default_cap_tt(ctx->meta[it.cluster])) : 0;
            r.items.push_back(it);
        }
        gale_status s = run_items(ctx, r, GALE_FORM_PLAIN, st);
        if (s) return s;
        e = hipMemcpyAsync(r.host_hdr->ptr, r.dev_hdr->ptr, r.items.size() * 32, hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) return fail(GALE_EDEVICE, std::string("rebuild: ") + hipGetErrorString(e));
        for (size_t j = 0; j < redo.size(); ++j) {
            const int i = redo[j];
            const int32_t *h = (const int32_t *)r.host_hdr->ptr + j * 8;
            if (h[0] & (kStInconsistent | kStVVOverflow | kStTTOverflow))
                return fail(GALE_EDEVICE, "rebuild with exact capacities failed");
            std::memcpy(&b.hdr[(size_t)i * 8], h, 32);
            b.items[i].cap_vv = r.items[j].cap_vv;
            b.items[i].cap_tt = r.items[j].cap_tt;
            b.loc[i] = BlockLoc{r.out, r.items[j].out_word};
        }
        ctx->n_overflow += redo.size();
        // keep the rebuild's output buffer with this batch
        b.extra.push_back(r.out);
        r.out = nullptr;
        release_batch(ctx, r);
    }
    uint64_t ent = 0;
    for (int i = 0; i < n; ++i) {
        const int32_t *h = &b.hdr[(size_t)i * 8];
        if (b.items[i].mask & kRelVT) ent += (uint64_t)h[3];
        if (b.items[i].mask & kRelVV) ent += (uint64_t)h[4];
        if (b.items[i].mask & kRelTT) ent += (uint64_t)h[5];
    }
    ctx->n_entries += ent;
    ctx->n_blocks += n;
    return GALE_OK;
}

// Copy every block of a finalized batch to pinned host memory (synchronous).
gale_status copy_batch_to_host(gale_ctx *ctx, Batch &b, hipStream_t st) {
    // one host buffer laid out like the device buffers, blocks at their words
    int64_t words = 0;
    const int n = (int)b.items.size();
    b.host_word.assign(n, 0);
    for (int i = 0; i < n; ++i) {
        const ClusterMeta &m = ctx->meta[b.items[i].cluster];
        const int32_t *h = &b.hdr[(size_t)i * 8];
        // exact used size: VV is last, so its tail beyond the real count is skipped
        const int32_t used_vv = (b.items[i].mask & kRelVV) ? h[4] : 0;
        const BlockLayout lay = block_layout(b.items[i].mask, m.nV, m.nT, m.nnzVT, used_vv, b.items[i].cap_tt);
        b.host_word[i] = words;
        words += lay.total;
    }
    hipError_t e;
    b.host_out = ctx->pin_pool.acquire((size_t)words * 4 + 256, &e);
    if (!b.host_out) return fail(GALE_ENOMEM, "pinned host buffer");
    uint64_t bytes = 0;
    for (int i = 0; i < n; ++i) {
        const ClusterMeta &m = ctx->meta[b.items[i].cluster];
        const int32_t *h = &b.hdr[(size_t)i * 8];
        const int32_t used_vv = (b.items[i].mask & kRelVV) ? h[4] : 0;
        const BlockLayout lay = block_layout(b.items[i].mask, m.nV, m.nT, m.nnzVT, used_vv, b.items[i].cap_tt);
        const int32_t *src = (const int32_t *)b.loc[i].buf->ptr + b.loc[i].word;
        int32_t *dst = (int32_t *)b.host_out->ptr + b.host_word[i];
        e = hipMemcpyAsync(dst, src, (size_t)lay.total * 4, hipMemcpyDeviceToHost, st);
        if (e != hipSuccess) return fail(GALE_EDEVICE, std::string("block copy: ") + hipGetErrorString(e));
        bytes += (uint64_t)lay.total * 4;
    }
    e = hipStreamSynchronize(st);
    if (e != hipSuccess) return fail(GALE_EDEVICE, std::string("block copy: ") + hipGetErrorString(e));
    ctx->n_bytes_d2h += bytes;
    uint64_t ent = 0;
    for (int i = 0; i < n; ++i) {
        const int32_t *h = &b.hdr[(size_t)i * 8];
        if (b.items[i].mask & kRelVT) ent += (uint64_t)h[3];
        if (b.items[i].mask & kRelVV) ent += (uint64_t)h[4];
        if (b.items[i].mask & kRelTT) ent += (uint64_t)h[5];
    }
    ctx->n_delivered += ent;
    b.host_ready = true;
    return GALE_OK;
}

// view of block i of a finalized batch
gale_status block_view(const gale_ctx *ctx, const Batch &b, int i, uint32_t rel, bool host, gale_csr *out) {
    const WorkItem &it = b.items[i];
    const ClusterMeta &m = ctx->meta[it.cluster];
    const int32_t *h = &b.hdr[(size_t)i * 8];
    const int32_t *base;
    BlockLayout lay;
    if (host) {
        if (!b.host_ready) return fail(GALE_ESTATE, "ticket has no host copy (made with gale_build)");
        const int32_t used_vv = (it.mask & kRelVV) ? h[4] : 0;
        lay = block_layout(it.mask, m.nV, m.nT, m.nnzVT, used_vv, it.cap_tt);
        base = (const int32_t *)b.host_out->ptr + b.host_word[i];
    } else {
        lay = block_layout(it.mask, m.nV, m.nT, m.nnzVT, it.cap_vv, it.cap_tt);
        base = (const int32_t *)b.loc[i].buf->ptr + b.loc[i].word;
    }
    out->cluster = it.cluster;
    out->rel = rel;
    out->pad = 0;
    if (rel == GALE_REL_VT) {
        out->nrows = m.nV;
        out->nnz = h[3];
        out->row_ids = base + lay.vrows;
        out->offsets = base + lay.vt_off;
        out->entries = base + lay.vt_ent;
    } else if (rel == GALE_REL_VV) {
        out->nrows = m.nV;
        out->nnz = h[4];
        out->row_ids = base + lay.vrows;
        out->offsets = base + lay.vv_off;
        out->entries = base + lay.vv_ent;
    } else {
        out->nrows = m.nT;
        out->nnz = h[5];
        out->row_ids = base + lay.trows;
        out->offsets = base + lay.tt_off;
        out->entries = base + lay.tt_ent;
    }
    return GALE_OK;
}

// ---------------------------------------------------------------------------
// tickets (DIRECT mode)
// ---------------------------------------------------------------------------
gale_status check_request(const gale_ctx *ctx, const int32_t *ids, int32_t n, uint32_t mask) {
    if (!ctx->loaded) return fail(GALE_ESTATE, "no mesh loaded");
    if (n < 0 || (n > 0 && !ids)) return fail(GALE_EINVAL, "bad cluster id list");
    if (mask == 0 || (mask & ~GALE_REL_ALL)) return fail(GALE_EINVAL, "relation mask must be a non-empty subset of VT|VV|TT");
    for (int32_t i = 0; i < n; ++i)
        if (ids[i] < 0 || ids[i] >= ctx->ncl)
            return fail(GALE_EINVAL, "cluster id " + std::to_string(ids[i]) + " out of range");
    return GALE_OK;
}

// items for the unique ids: BATCHED = one item per cluster with the whole mask,
// ordered by decreasing stream length; PLAIN = one item per (cluster, relation)
std::vector<WorkItem> make_items(const gale_ctx *ctx, const int32_t *ids, int32_t n, uint32_t mask, int form) {
    std::vector<int32_t> u(ids, ids + n);
    std::sort(u.begin(), u.end());
    u.erase(std::unique(u.begin(), u.end()), u.end());
    std::vector<WorkItem> items;
    auto mk = [&](int32_t k, uint32_t m) {
        WorkItem it{};
        it.cluster = k;
        it.mask = m;
        it.cap_vv = -1;
        it.cap_tt = -1;
        items.push_back(it);
    };
    if (form == GALE_FORM_PLAIN) {
        for (int32_t k : u)
            for (uint32_t bit : {kRelVT, kRelVV, kRelTT})
                if (mask & bit) mk(k, bit);
    } else {
        std::stable_sort(u.begin(), u.end(), [&](int32_t x, int32_t y) {
            const int64_t cx = (int64_t)ctx->meta[x].ns + ctx->meta[x].nh;
            const int64_t cy = (int64_t)ctx->meta[y].ns + ctx->meta[y].nh;
            return cx > cy;
        });
        for (int32_t k : u) mk(k, mask);
    }
    return items;
}

gale_status direct_build(gale_ctx *ctx, const int32_t *ids, int32_t n, uint32_t mask, int form, bool host,
                         uint64_t *ticket_out) {
    gale_status s = check_request(ctx, ids, n, mask);
    if (s) return s;
    if (form != GALE_FORM_PLAIN && form != GALE_FORM_BATCHED) return fail(GALE_EINVAL, "unknown form");
    if (ctx->poisoned) return fail(GALE_EDEVICE, "context poisoned by an earlier device error");
    auto *t = new Ticket();
    t->batch.items = make_items(ctx, ids, n, mask, form);
    t->mask = mask;
    t->host = host;
    for (size_t i = 0; i < t->batch.items.size(); ++i)
        t->by_cluster[t->batch.items[i].cluster].push_back((int)i);
    std::lock_guard<std::mutex> g(ctx->direct_mu);
    if (form == GALE_FORM_BATCHED) {
        // kernel timing: events around the persistent LDS-path launch
        if (hipEventCreate(&t->batch.kev[0]) != hipSuccess || hipEventCreate(&t->batch.kev[1]) != hipSuccess)
            destroy_ticket_events(t);
    }
    s = run_items(ctx, t->batch, form, ctx->stream);
    if (s == GALE_OK) {
        hipError_t e = hipEventCreateWithFlags(&t->done, hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventRecord(t->done, ctx->stream);
        if (e != hipSuccess) s = fail(GALE_EDEVICE, std::string("event: ") + hipGetErrorString(e));
    }
    if (s) {
        if (s == GALE_EDEVICE) ctx->poisoned = true;
        release_batch(ctx, t->batch);
        if (t->done) (void)hipEventDestroy(t->done);
        destroy_ticket_events(t);
        delete t;
        return s;
    }
    ctx->n_requests++;
    std::lock_guard<std::mutex> g2(ctx->tick_mu);
    const uint64_t id = ++ctx->next_ticket;
    ctx->tickets[id] = t;
    *ticket_out = id;
    return GALE_OK;
}

gale_status direct_poll(gale_ctx *ctx, Ticket *t, int64_t timeout_ns) {
    if (t->ready) return t->status;
    const auto t0 = std::chrono::steady_clock::now();
    while (true) {
        hipError_t q = hipEventQuery(t->done);
        if (q == hipSuccess) break;
        if (q != hipErrorNotReady) {
            ctx->poisoned = true;
            return fail(GALE_EDEVICE, std::string("kernel: ") + hipGetErrorString(q));
        }
        if (timeout_ns == 0) return GALE_EAGAIN;
        if (timeout_ns > 0 &&
            std::chrono::duration_cast<std::chrono::nanoseconds>(std::chrono::steady_clock::now() - t0).count() >=
                timeout_ns)
            return GALE_EAGAIN;
        std::this_thread::sleep_for(std::chrono::microseconds(20));
    }
    std::lock_guard<std::mutex> g(ctx->direct_mu);
    if (t->ready) return t->status;
    if (t->batch.kev_recorded) {
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, t->batch.kev[0], t->batch.kev[1]) == hipSuccess) {
            ctx->kernel_ms += ms;
            ctx->n_timed++;
        }
    }
    gale_status s = finalize_batch(ctx, t->batch, ctx->stream);
    if (s == GALE_OK && t->host) s = copy_batch_to_host(ctx, t->batch, ctx->stream);
    if (s == GALE_EDEVICE) ctx->poisoned = true;
    t->status = s;
    t->ready = true;
    return s;
}

}  // namespace gale

using namespace gale;

// ---------------------------------------------------------------------------
// exported C functions
// ---------------------------------------------------------------------------
extern "C" {

const char *gale_strerror(gale_status s) {
    switch (s) {
        case GALE_OK: return "ok";
        case GALE_EINVAL: return "invalid argument";
        case GALE_ENOMEM: return "out of memory";
        case GALE_EAGAIN: return "not ready / queue full";
        case GALE_ENOENT: return "unknown ticket or block";
        case GALE_ESTATE: return "call out of order";
        case GALE_EDEVICE: return "device error";
        default: return "unknown status";
    }
}

const char *gale_last_error(void) { return t_last_error.c_str(); }

gale_status gale_create(const gale_config *cfg_in, gale_ctx **out) {
    if (!out) return fail(GALE_EINVAL, "out is NULL");
    *out = nullptr;
    gale_config cfg{};
    if (cfg_in) cfg = *cfg_in;
    if (cfg.mode != GALE_MODE_DIRECT && cfg.mode != GALE_MODE_SERVE) return fail(GALE_EINVAL, "unknown mode");
    if (cfg.form != GALE_FORM_PLAIN && cfg.form != GALE_FORM_BATCHED) return fail(GALE_EINVAL, "unknown form");
    if (cfg.block_threads != 0 && cfg.block_threads != 256 && cfg.block_threads != 512 && cfg.block_threads != 1024)
        return fail(GALE_EINVAL, "block_threads must be 256, 512 or 1024");
    int ndev = 0;
    hipError_t e = hipGetDeviceCount(&ndev);
    if (e != hipSuccess || ndev <= 0) return fail(GALE_EDEVICE, "no HIP device");
    if (cfg.device < 0 || cfg.device >= ndev) return fail(GALE_EINVAL, "device ordinal out of range");
    e = hipSetDevice(cfg.device);
    if (e != hipSuccess) return fail(GALE_EDEVICE, std::string("hipSetDevice: ") + hipGetErrorString(e));
    auto *ctx = new gale_ctx();
    ctx->cfg = cfg;
    ctx->dev_pool.pinned = false;
    ctx->pin_pool.pinned = true;
    hipDeviceProp_t prop;
    e = hipGetDeviceProperties(&prop, cfg.device);
    if (e != hipSuccess) {
        delete ctx;
        return fail(GALE_EDEVICE, std::string("device properties: ") + hipGetErrorString(e));
    }
    ctx->num_cus = prop.multiProcessorCount;
    ctx->block_threads = cfg.block_threads ? cfg.block_threads : 1024;
    // LDS: the device limit minus what the kernels declare statically
    int64_t static_lds = 0;
    e = static_lds_bytes(&static_lds);
    if (e != hipSuccess) {
        delete ctx;
        return fail(GALE_EDEVICE, std::string("kernel attributes: ") + hipGetErrorString(e));
    }
    int64_t budget = (int64_t)prop.sharedMemPerBlock - static_lds;
    if (cfg.lds_bytes > 0) budget = std::min<int64_t>(budget, cfg.lds_bytes);
    ctx->lds_budget = std::max<int64_t>(budget, 0);
    e = set_lds_limits((size_t)std::max<int64_t>(ctx->lds_budget, 1));
    if (e != hipSuccess) {
        delete ctx;
        return fail(GALE_EDEVICE, std::string("LDS limit: ") + hipGetErrorString(e));
    }
    int occ = 0;
    e = persistent_occupancy(ctx->block_threads, true, (size_t)ctx->lds_budget, &occ);
    if (e != hipSuccess || occ <= 0) occ = 1;
    ctx->grid_lds = ctx->num_cus * occ;
    occ = 0;
    e = persistent_occupancy(ctx->block_threads, false, 0, &occ);
    if (e != hipSuccess || occ <= 0) occ = 1;
    ctx->grid_glob = ctx->num_cus * occ;
    if (cfg.hip_stream) {
        ctx->stream = (hipStream_t)cfg.hip_stream;
        ctx->own_stream = false;
    } else {
        e = hipStreamCreateWithFlags(&ctx->stream, hipStreamNonBlocking);
        if (e != hipSuccess) {
            delete ctx;
            return fail(GALE_EDEVICE, std::string("stream: ") + hipGetErrorString(e));
        }
        ctx->own_stream = true;
    }
    *out = ctx;
    return GALE_OK;
}

gale_status gale_load(gale_ctx *ctx, int32_t nv, int64_t nt, const int32_t *tv, const int32_t *cl, int32_t ncl) {
    if (!ctx) return fail(GALE_EINVAL, "ctx is NULL");
    if (ctx->loaded) return fail(GALE_ESTATE, "a mesh is already loaded");
    const auto t0 = std::chrono::steady_clock::now();
    HostStreams hs;
    std::string err;
    gale_status s = prepare_streams(nv, nt, tv, cl, ncl, hs, err);
    if (s) return fail(s, err);
    hipError_t e = hipSetDevice(ctx->cfg.device);
    auto up = [&](void **dst, const void *src, size_t bytes) -> hipError_t {
        hipError_t r = hipMalloc(dst, std::max<size_t>(bytes, 16));
        if (r != hipSuccess) return r;
        if (bytes) r = hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice);
        return r;
    };
    if (e == hipSuccess) e = up((void **)&ctx->d_tets, hs.tets.data(), hs.tets.size());
    if (e == hipSuccess) e = up((void **)&ctx->d_tid, hs.tid.data(), hs.tid.size() * 4);
    if (e == hipSuccess) e = up((void **)&ctx->d_lverts, hs.lverts.data(), hs.lverts.size() * 4);
    if (e == hipSuccess) e = up((void **)&ctx->d_meta, hs.meta.data(), hs.meta.size() * sizeof(ClusterMeta));
    if (e != hipSuccess) {
        ctx->poisoned = true;
        return fail(e == hipErrorOutOfMemory ? GALE_ENOMEM : GALE_EDEVICE,
                    std::string("mesh upload: ") + hipGetErrorString(e));
    }
    ctx->mesh_bytes = hs.tets.size() + (hs.tid.size() + hs.lverts.size()) * 4 + hs.meta.size() * sizeof(ClusterMeta);
    ctx->stream_tets = (int64_t)hs.tid.size();
    ctx->meta = std::move(hs.meta);
    ctx->nv = nv;
    ctx->nt = nt;
    ctx->ncl = ncl;
    ctx->loaded = true;
    ctx->load_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (ctx->cfg.mode == GALE_MODE_SERVE) {
        s = serve_start(ctx);
        if (s) return s;
    }
    return GALE_OK;
}

gale_status gale_build(gale_ctx *ctx, const int32_t *ids, int32_t n, uint32_t mask, int32_t form,
                       uint64_t *ticket_out) {
    if (!ctx || !ticket_out) return fail(GALE_EINVAL, "NULL argument");
    if (ctx->cfg.mode != GALE_MODE_DIRECT) return fail(GALE_ESTATE, "gale_build needs DIRECT mode");
    return direct_build(ctx, ids, n, mask, form, false, ticket_out);
}

gale_status gale_submit(gale_ctx *ctx, const int32_t *ids, int32_t n, uint32_t mask, uint64_t *ticket_out) {
    if (!ctx || !ticket_out) return fail(GALE_EINVAL, "NULL argument");
    if (ctx->cfg.mode == GALE_MODE_SERVE) return serve_submit(ctx, ids, n, mask, ticket_out);
    uint64_t tk = 0;
    gale_status s = direct_build(ctx, ids, n, mask, ctx->cfg.form, true, &tk);
    if (s) return s;
    Ticket *t;
    {
        std::lock_guard<std::mutex> g(ctx->tick_mu);
        t = ctx->tickets[tk];
    }
    s = direct_poll(ctx, t, -1);
    if (s) {
        gale_release(ctx, tk);
        return s;
    }
    *ticket_out = tk;
    return GALE_OK;
}

gale_status gale_poll(gale_ctx *ctx, uint64_t ticket, int64_t timeout_ns) {
    if (!ctx) return fail(GALE_EINVAL, "ctx is NULL");
    if (ctx->cfg.mode == GALE_MODE_SERVE) return serve_poll(ctx, ticket, timeout_ns);
    Ticket *t;
    {
        std::lock_guard<std::mutex> g(ctx->tick_mu);
        auto it = ctx->tickets.find(ticket);
        if (it == ctx->tickets.end()) return fail(GALE_ENOENT, "unknown ticket");
        t = it->second;
    }
    return direct_poll(ctx, t, timeout_ns);
}

static gale_status view(gale_ctx *ctx, uint64_t ticket, int32_t cluster, uint32_t rel, bool host, gale_csr *out) {
    if (!ctx || !out) return fail(GALE_EINVAL, "NULL argument");
    if (rel != GALE_REL_VT && rel != GALE_REL_VV && rel != GALE_REL_TT) return fail(GALE_EINVAL, "rel must be one bit");
    if (ctx->cfg.mode == GALE_MODE_SERVE) {
        if (!host) return fail(GALE_ESTATE, "SERVE mode tickets have host views only");
        return serve_block(ctx, ticket, cluster, rel, out);
    }
    std::lock_guard<std::mutex> g(ctx->tick_mu);
    auto it = ctx->tickets.find(ticket);
    if (it == ctx->tickets.end()) return fail(GALE_ENOENT, "unknown ticket");
    Ticket *t = it->second;
    if (!t->ready) return fail(GALE_EAGAIN, "ticket not ready");
    if (t->status) return fail(t->status, "ticket failed");
    auto c = t->by_cluster.find(cluster);
    if (c == t->by_cluster.end()) return fail(GALE_ENOENT, "cluster not in ticket");
    for (int i : c->second)
        if (t->batch.items[i].mask & rel) return block_view(ctx, t->batch, i, rel, host, out);
    return fail(GALE_ENOENT, "relation not in ticket");
}

gale_status gale_block(gale_ctx *ctx, uint64_t ticket, int32_t cluster, uint32_t rel, gale_csr *out) {
    return view(ctx, ticket, cluster, rel, true, out);
}

gale_status gale_block_device(gale_ctx *ctx, uint64_t ticket, int32_t cluster, uint32_t rel, gale_csr *out) {
    return view(ctx, ticket, cluster, rel, false, out);
}

gale_status gale_release(gale_ctx *ctx, uint64_t ticket) {
    if (!ctx) return fail(GALE_EINVAL, "ctx is NULL");
    if (ctx->cfg.mode == GALE_MODE_SERVE) return serve_release(ctx, ticket);
    Ticket *t;
    {
        std::lock_guard<std::mutex> g(ctx->tick_mu);
        auto it = ctx->tickets.find(ticket);
        if (it == ctx->tickets.end()) return fail(GALE_ENOENT, "unknown or released ticket");
        t = it->second;
        ctx->tickets.erase(it);
    }
    if (!t->ready) (void)hipEventSynchronize(t->done);
    if (t->done) (void)hipEventDestroy(t->done);
    destroy_ticket_events(t);
    for (Buf *b : t->batch.extra) ctx->dev_pool.release(b);
    release_batch(ctx, t->batch);
    delete t;
    return GALE_OK;
}

void *gale_stream(gale_ctx *ctx) { return ctx ? (void *)ctx->stream : nullptr; }

gale_status gale_get_stats(gale_ctx *ctx, gale_stats *out) {
    if (!ctx || !out) return fail(GALE_EINVAL, "NULL argument");
    std::memset(out, 0, sizeof(*out));
    out->nv = ctx->nv;
    out->nclusters = ctx->ncl;
    out->nt = ctx->nt;
    out->stream_tets = ctx->stream_tets;
    out->device_mesh_bytes = ctx->mesh_bytes;
    out->load_seconds = ctx->load_seconds;
    out->requests = ctx->n_requests;
    out->blocks_built = ctx->n_blocks;
    out->entries_built = ctx->n_entries;
    out->kernel_launches = ctx->n_launches;
    out->overflow_reruns = ctx->n_overflow;
    out->global_path_blocks = ctx->n_global_blocks;
    out->tt_exhaustive_blocks = ctx->n_tt_exhaustive;
    out->entries_delivered = ctx->n_delivered;
    out->bytes_d2h = ctx->n_bytes_d2h;
    {
        std::lock_guard<std::mutex> g(ctx->direct_mu);
        out->timed_launches = ctx->n_timed;
        out->kernel_ms_total = ctx->kernel_ms;
    }
    if (ctx->cfg.mode == GALE_MODE_SERVE) serve_stats(ctx, out);
    return GALE_OK;
}

gale_status gale_reset_stats(gale_ctx *ctx) {
    if (!ctx) return fail(GALE_EINVAL, "ctx is NULL");
    {
        std::lock_guard<std::mutex> g(ctx->direct_mu);
        ctx->n_timed = 0;
        ctx->kernel_ms = 0.0;
    }
    if (ctx->cfg.mode == GALE_MODE_SERVE) serve_reset_stats(ctx);
    return GALE_OK;
}

void gale_destroy(gale_ctx *ctx) {
    if (!ctx) return;
    if (ctx->cfg.mode == GALE_MODE_SERVE) serve_stop(ctx);
    (void)hipSetDevice(ctx->cfg.device);
    (void)hipStreamSynchronize(ctx->stream);
    {
        std::lock_guard<std::mutex> g(ctx->tick_mu);
        for (auto &kv : ctx->tickets) {
            Ticket *t = kv.second;
            if (t->done) (void)hipEventDestroy(t->done);
            destroy_ticket_events(t);
            delete t;
        }
        ctx->tickets.clear();
    }
    ctx->dev_pool.clear();
    ctx->pin_pool.clear();
    if (ctx->d_tets) (void)hipFree(ctx->d_tets);
    if (ctx->d_tid) (void)hipFree(ctx->d_tid);
    if (ctx->d_lverts) (void)hipFree(ctx->d_lverts);
    if (ctx->d_meta) (void)hipFree(ctx->d_meta);
    if (ctx->own_stream) (void)hipStreamDestroy(ctx->stream);
    delete ctx;
}

}  // extern "C"
