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
#include <cstdio>
#include <cstdlib>
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
        it.out_word = w;
        it.hdr_index = (int32_t)i;
        if (it.mask & kRelExt) {  // edge / triangle relations: their own block
            it.cap_vv = it.cap_tt = 0;
            w += ext_layout(it.mask, m, ctx->sx.ext[it.cluster]).total;
            continue;
        }
        if (it.cap_vv < 0) it.cap_vv = (it.mask & kRelVV) ? m.cap_vv : 0;
        if (it.cap_tt < 0) it.cap_tt = (it.mask & kRelTT) ? default_cap_tt(m) : 0;
        const BlockLayout lay = block_layout(it.mask, m.nV, m.nT, m.nnzVT, it.cap_vv, it.cap_tt);
        w += lay.total;
    }
    return w - out_base_word;
}

// Launch classes: the configured shape with the whole budget, then the
// smaller shapes the mask enables (half and a quarter of the LDS).
void setup_classes(gale_ctx *ctx, int mask) {
    ctx->classes.clear();
    ctx->classes.push_back({ctx->block_threads, ctx->lds_budget, ctx->grid_lds});
    const struct {
        int bit, bt, div;
    } shapes[] = {{2, 512, 2}, {4, 256, 4}};
    for (const auto &sh : shapes) {
        if (!(mask & sh.bit)) continue;
        int64_t b = ctx->shared_per_block / sh.div - ctx->static_lds;
        b = std::min<int64_t>(b, ctx->lds_budget);
        if (b < 4096) continue;
        int o = 0;
        if (persistent_occupancy(sh.bt, true, (size_t)b, &o) != hipSuccess || o <= 0) o = 1;
        ctx->classes.push_back({sh.bt, b, ctx->num_cus * o});
    }
    ctx->class_mask = mask;
}

// Global-path launches: bt threads per workgroup, as many workgroups per CU as
// the registers allow, each with its share of the CU's LDS for the hybrid
// form (none when bit 3 of the configured launch classes keeps every array in
// global memory).
void setup_global(gale_ctx *ctx, int bt) {
    ctx->glob_bt = bt;
    int occ = 0;
    hipError_t e = persistent_occupancy(bt, false, 0, &occ);
    if (e != hipSuccess || occ <= 0) occ = 1;
    ctx->glob_lds = 0;
    if (!(ctx->cfg.launch_classes & 8)) {
        int64_t g = ctx->shared_per_block / occ - ctx->static_lds;
        g = std::min<int64_t>(g, ctx->lds_budget) / 16 * 16;
        ctx->glob_lds = std::max<int64_t>(g, 0);
    }
    int occ2 = 0;
    e = persistent_occupancy(bt, false, (size_t)ctx->glob_lds, &occ2);
    ctx->grid_glob = ctx->num_cus * ((e != hipSuccess || occ2 <= 0) ? 1 : occ2);
}

// The workgroup shape of an item: the smallest (last) launch class whose LDS
// plan fits, or -1 for the global-workspace path.
int item_class(const gale_ctx *ctx, const WorkItem &it) {
    if (ctx->cfg.launch_classes & 16) return -1;  // every cluster on the global path (tests)
    for (int c = (int)ctx->classes.size() - 1; c >= 0; --c) {
        const gale_ctx::LaunchClass &lc = ctx->classes[c];
        if (lds_plan(ctx->meta[it.cluster], it.mask, lc.budget, lc.bt).ok) return c;
    }
    return -1;
}

bool item_on_lds_path(const gale_ctx *ctx, const WorkItem &it) { return item_class(ctx, it) >= 0; }

int64_t workspace_bytes(const gale_ctx *ctx, const std::vector<WorkItem> &items, int *n_global) {
    int64_t need = 0;
    int ng = 0;
    for (const WorkItem &it : items) {
        if (item_class(ctx, it) < 0) {
            const Plan gp = ws_plan(ctx->meta[it.cluster], it.mask, ctx->glob_bt);
            const Plan hp = hyb_plan(ctx->meta[it.cluster], it.mask, ctx->glob_lds, ctx->glob_bt);
            need = std::max<int64_t>(need, hp.ok ? hp.ws_bytes : gp.bytes);
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
    a.x.ext = ctx->d_ext;
    a.x.eoff = ctx->d_eoff;
    a.x.eidx = ctx->d_eidx;
    a.x.foff = ctx->d_foff;
    a.x.fidx = ctx->d_fidx;
    a.lds_budget = (int32_t)ctx->lds_budget;
    return a;
}

void destroy_ticket_events(Ticket *t) {
    for (hipEvent_t &e : t->batch.kev) {
        if (e) (void)hipEventDestroy(e);
        e = nullptr;
    }
}

// Launch items already uploaded in launch order: first the items of launch
// class 0, then class 1, ... (ncls[c] each), then the n_glob items of the
// global-workspace path, with ncls[classes] workgroups (stage_items).  PLAIN: one launch per item; BATCHED: one persistent
// launch per class and one for the global path, each with its own queue word
// (d_queue[c], d_queue[classes]).  fork: run the launches on the auxiliary
// streams, forked from and joined back into st (DIRECT mode); otherwise one
// after another on st.  kev, when given, brackets all of them on st.
gale_status launch_batch(gale_ctx *ctx, int form, int32_t *d_out, int32_t *d_hdr, const WorkItem *d_items,
                         const std::vector<int> &ncls, int n_glob, int32_t *d_queue, char *d_ws, int64_t ws_stride,
                         hipStream_t st, bool fork, const hipEvent_t *kev, bool *kev_recorded) {
    KArgs a = base_args(ctx);
    a.out = d_out;
    a.hdr = d_hdr;
    a.ws = d_ws;
    a.ws_stride = ws_stride;
    hipError_t e = hipSuccess;
    const int ncl = (int)ctx->classes.size();
    if (form == GALE_FORM_PLAIN) {
        int i = 0;
        for (int c = 0; c < ncl && e == hipSuccess; ++c) {
            const gale_ctx::LaunchClass &lc = ctx->classes[c];
            a.lds_budget = (int32_t)lc.budget;
            for (int j = 0; j < ncls[c] && e == hipSuccess; ++j, ++i) {
                a.items = d_items + i;
                a.nitems = 1;
                e = launch_items(a, true, lc.bt, 1, (size_t)lc.budget, st);
                ctx->n_launches++;
            }
        }
        a.lds_budget = (int32_t)ctx->glob_lds;
        for (int j = 0; j < n_glob && e == hipSuccess; ++j, ++i) {
            a.items = d_items + i;
            a.nitems = 1;
            e = launch_items(a, false, ctx->glob_bt, 1, (size_t)ctx->glob_lds, st);
            ctx->n_launches++;
        }
    } else {
        // the launches to make: (class or -1, first item, count)
        struct L {
            int c, first, n;
        };
        std::vector<L> ls;
        int first = 0;
        for (int c = 0; c < ncl; ++c) {
            if (ncls[c] > 0) ls.push_back({c, first, ncls[c]});
            first += ncls[c];
        }
        // the global launch goes last, or first when it is given only a share
        // of the CUs (its workgroups then take theirs at once and the classes
        // fill the others)
        const int gg = (int)ncls.size() > ncl ? ncls[ncl] : ctx->grid_glob;
        if (n_glob > 0) {
            if (gg < ctx->grid_glob)
                ls.insert(ls.begin(), L{-1, first, n_glob});
            else
                ls.push_back({-1, first, n_glob});
        }
        const bool use_aux = fork && ls.size() > 1 && ctx->aux.size() >= ls.size() - 1;
        if (kev) e = hipEventRecord(kev[0], st);
        if (use_aux && e == hipSuccess) e = hipEventRecord(ctx->fork_ev, st);
        for (size_t li = 0; li < ls.size() && e == hipSuccess; ++li) {
            const L &l = ls[li];
            hipStream_t s2 = st;
            if (use_aux && li > 0) {
                s2 = ctx->aux[li - 1];
                e = hipStreamWaitEvent(s2, ctx->fork_ev, 0);
                if (e != hipSuccess) break;
            }
            a.items = d_items + l.first;
            a.nitems = l.n;
            a.queue = d_queue + (l.c >= 0 ? l.c : ncl);
            if (l.c >= 0) {
                const gale_ctx::LaunchClass &lc = ctx->classes[l.c];
                a.lds_budget = (int32_t)lc.budget;
                e = launch_persistent(a, true, lc.bt, std::min<int>(l.n, lc.grid), (size_t)lc.budget, s2);
            } else {
                a.lds_budget = (int32_t)ctx->glob_lds;
                e = launch_persistent(a, false, ctx->glob_bt, std::min<int>(l.n, gg), (size_t)ctx->glob_lds, s2);
            }
            ctx->n_launches++;
            if (e == hipSuccess && use_aux && li > 0) {
                e = hipEventRecord(ctx->join_ev[li - 1], s2);
                if (e == hipSuccess) e = hipStreamWaitEvent(st, ctx->join_ev[li - 1], 0);
            }
        }
        if (kev && e == hipSuccess) e = hipEventRecord(kev[1], st);
        if (kev && kev_recorded && e == hipSuccess) *kev_recorded = true;
    }
    if (e != hipSuccess) return fail(GALE_EDEVICE, std::string("kernel launch: ") + hipGetErrorString(e));
    return GALE_OK;
}

// Order items by launch class (then the global path), largest cluster first
// within each: order receives the launch order, ncls the items per class
// followed by the global launch's workgroups, n_glob the global-path items,
// wsb the workspace bytes per global-path workgroup.  Host logic only.
void order_items(gale_ctx *ctx, const std::vector<WorkItem> &items, std::vector<WorkItem> &order,
                 std::vector<int> &ncls, int &n_glob, int64_t &wsb) {
    const int n = (int)items.size();
    const int ncl = (int)ctx->classes.size();
    std::vector<int> cls(n);
    ncls.assign(ncl, 0);
    for (int i = 0; i < n; ++i) {
        cls[i] = item_class(ctx, items[i]);
        if (cls[i] >= 0) ncls[cls[i]]++;
    }
    // within a launch, the largest clusters first: workgroups take items in
    // list order, so the last ones to start are the cheapest (a shorter tail)
    auto largest_first = [&](std::vector<WorkItem> &v) {
        std::stable_sort(v.begin(), v.end(), [&](const WorkItem &x, const WorkItem &y) {
            const ClusterMeta &a = ctx->meta[x.cluster], &b = ctx->meta[y.cluster];
            return (int64_t)a.ns + a.nh + a.nnzVT > (int64_t)b.ns + b.nh + b.nnzVT;
        });
    };
    order.clear();
    order.reserve(n);
    for (int c = 0; c < ncl; ++c) {
        std::vector<WorkItem> part;
        for (int i = 0; i < n; ++i)
            if (cls[i] == c) part.push_back(items[i]);
        largest_first(part);
        order.insert(order.end(), part.begin(), part.end());
    }
    std::vector<WorkItem> glob;
    for (int i = 0; i < n; ++i)
        if (cls[i] < 0) glob.push_back(items[i]);
    largest_first(glob);
    n_glob = (int)glob.size();
    order.insert(order.end(), glob.begin(), glob.end());
    // workgroups of the global launch: a global-path workgroup takes a whole
    // CU; when LDS-path classes run beside it (DIRECT mode forks the launches
    // onto streams of their own), it gets the context's share of the CUs
    // (gale_autotune sets it); alone or one launch after another, every CU
    int glob_grid = ctx->grid_glob;
    const bool side_by_side = ctx->cfg.mode == GALE_MODE_DIRECT && !ctx->aux.empty();
    if (n_glob > 0 && n_glob < n && side_by_side)
        glob_grid = std::max(1, (int)(ctx->glob_share * ctx->grid_glob + 0.5));
    ncls.push_back(glob_grid);
    wsb = workspace_bytes(ctx, glob, nullptr);
}

// Order the items (order_items), acquire the work-list buffers and copy the
// list with zeroed queue words to the device.
gale_status stage_items(gale_ctx *ctx, int form, const std::vector<WorkItem> &items, Buf *&dev_items,
                        Buf *&dev_hdr, Buf *&host_items, Buf *&ws, hipStream_t st, std::vector<int> &ncls,
                        int &n_glob, int64_t &wsb) {
    hipError_t e;
    const int n = (int)items.size();
    std::vector<WorkItem> order;
    order_items(ctx, items, order, ncls, n_glob, wsb);
    const int glob_grid = ncls.back();
    ctx->n_global_blocks += n_glob;
    for (int i = n - n_glob; i < n; ++i)
        if (hyb_plan(ctx->meta[order[i].cluster], order[i].mask, ctx->glob_lds, ctx->glob_bt).ok)
            ctx->n_hybrid_blocks++;
    const int slots = form == GALE_FORM_PLAIN ? 1 : std::min<int>(std::max(n_glob, 1), glob_grid);
    // headers are written at each item's hdr_index, which may range over a
    // batch's edge / triangle items too
    size_t nh = (size_t)n;
    for (const WorkItem &it : items) nh = std::max(nh, (size_t)it.hdr_index + 1);
    dev_items = ctx->dev_pool.acquire((size_t)n * sizeof(WorkItem) + 64, &e);
    if (!dev_hdr) dev_hdr = ctx->dev_pool.acquire(nh * 32 + 64, &e);
    host_items = ctx->pin_pool.acquire((size_t)n * sizeof(WorkItem) + 64, &e);
    if (!dev_items || !dev_hdr || !host_items) return fail(GALE_ENOMEM, "batch buffers");
    if (n_glob > 0) {
        ws = ctx->dev_pool.acquire((size_t)wsb * slots, &e);
        if (!ws) return fail(GALE_ENOMEM, "workspace");
    }
    char *hi = (char *)host_items->ptr;
    std::memset(hi, 0, 64);  // the queue words, one per class and one for the global path
    std::memcpy(hi + 64, order.data(), (size_t)n * sizeof(WorkItem));
    e = hipMemcpyAsync(dev_items->ptr, hi, (size_t)n * sizeof(WorkItem) + 64, hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return fail(GALE_EDEVICE, std::string("work list copy: ") + hipGetErrorString(e));
    return GALE_OK;
}

// Stage items (layout order in `items`, with out_word and hdr_index set) and
// launch them.  Buffers come from the pools; the caller releases them.
gale_status upload_and_launch(gale_ctx *ctx, int form, const std::vector<WorkItem> &items, int32_t *d_out,
                              Buf *&dev_items, Buf *&dev_hdr, Buf *&host_items, Buf *&ws, hipStream_t st,
                              const hipEvent_t *kev, bool *kev_recorded) {
    std::vector<int> ncls;
    int n_glob = 0;
    int64_t wsb = 0;
    gale_status s = stage_items(ctx, form, items, dev_items, dev_hdr, host_items, ws, st, ncls, n_glob, wsb);
    if (s) return s;
    char *di = (char *)dev_items->ptr;
    return launch_batch(ctx, form, d_out, (int32_t *)dev_hdr->ptr, (const WorkItem *)(di + 64), ncls, n_glob,
                        (int32_t *)di, ws ? (char *)ws->ptr : nullptr, wsb, st, ctx->cfg.mode == GALE_MODE_DIRECT,
                        kev, kev_recorded);
}

// Edge / triangle relation items (laid out, hdr_index set): their work list
// with one queue word per launch copied to the device, a workspace slice per
// workgroup, then one persistent launch over all of them (BATCHED) or one
// launch per item (PLAIN), after whatever st already holds.
gale_status launch_ext_items(gale_ctx *ctx, Batch &b, int form, const std::vector<WorkItem> &items, hipStream_t st) {
    hipError_t e = hipSuccess;
    const int n = (int)items.size();
    if (n == 0) return GALE_OK;
    const int nq = form == GALE_FORM_PLAIN ? n : 1;
    const size_t qbytes = ((size_t)nq * 4 + 63) / 64 * 64;
    int64_t wsb = 256;
    for (const WorkItem &it : items)
        wsb = std::max<int64_t>(wsb, ext_workspace_bytes(ctx->meta[it.cluster], ctx->sx.ext[it.cluster], it.mask));
    int occ = 4;
    const int grid = form == GALE_FORM_PLAIN ? 1 : std::max(1, std::min(n, ctx->num_cus * occ));
    b.ext_items = ctx->dev_pool.acquire(qbytes + (size_t)n * sizeof(WorkItem), &e);
    b.ext_host = ctx->pin_pool.acquire(qbytes + (size_t)n * sizeof(WorkItem), &e);
    b.ext_ws = ctx->dev_pool.acquire((size_t)wsb * grid, &e);
    if (!b.ext_items || !b.ext_host || !b.ext_ws) return fail(GALE_ENOMEM, "edge / triangle work buffers");
    char *hi = (char *)b.ext_host->ptr;
    std::memset(hi, 0, qbytes);
    std::memcpy(hi + qbytes, items.data(), (size_t)n * sizeof(WorkItem));
    e = hipMemcpyAsync(b.ext_items->ptr, hi, qbytes + (size_t)n * sizeof(WorkItem), hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return fail(GALE_EDEVICE, std::string("work list copy: ") + hipGetErrorString(e));
    KArgs a = base_args(ctx);
    a.out = (int32_t *)b.out->ptr;
    a.hdr = (int32_t *)b.dev_hdr->ptr;
    a.ws = (char *)b.ext_ws->ptr;
    a.ws_stride = wsb;
    const WorkItem *di = (const WorkItem *)((char *)b.ext_items->ptr + qbytes);
    int32_t *dq = (int32_t *)b.ext_items->ptr;
    for (int l = 0; l < nq && e == hipSuccess; ++l) {
        a.items = di + (form == GALE_FORM_PLAIN ? l : 0);
        a.nitems = form == GALE_FORM_PLAIN ? 1 : n;
        a.queue = dq + l;
        e = launch_ext(a, grid, st);
        ctx->n_launches++;
    }
    if (e != hipSuccess) return fail(GALE_EDEVICE, std::string("kernel launch: ") + hipGetErrorString(e));
    return GALE_OK;
}

// Batched form, DIRECT mode: the VT / VV / TT items of tiled clusters are
// replaced in `base` by one item per tile, whose blocks are laid out from
// word `words` on (header slots from `nh` on); `stitch` receives the
// clusters to assemble and `tiles` the tile items in stitch order.
void expand_tiles(const gale_ctx *ctx, std::vector<WorkItem> &base, int64_t &words, int &nh,
                  std::vector<StitchItem> &stitch, std::vector<WorkItem> &tiles) {
    if (ctx->ntiles == 0) return;
    std::vector<WorkItem> out;
    out.reserve(base.size());
    for (const WorkItem &it : base) {
        const int32_t c = it.cluster;
        if (c >= ctx->ncl || ctx->tile_count[c] == 0) {
            out.push_back(it);
            continue;
        }
        // one stitch item per relation (bits 8.. of mask name it)
        for (uint32_t rel : {kRelVT, kRelVV, kRelTT}) {
            if (!(it.mask & rel)) continue;
            StitchItem si{};
            si.out_word = it.out_word;
            si.cluster = c;
            si.mask = it.mask | (rel << 8);
            si.cap_vv = it.cap_vv;
            si.cap_tt = it.cap_tt;
            si.hdr_index = it.hdr_index;
            si.tiles = (int32_t)tiles.size();
            stitch.push_back(si);
        }
        for (int32_t j = 0; j < ctx->tile_count[c]; ++j) {
            WorkItem ti{};
            ti.cluster = ctx->ncl + ctx->tile_first[c] + j;
            ti.mask = it.mask;
            const ClusterMeta &m = ctx->meta[ti.cluster];
            ti.cap_vv = (it.mask & kRelVV) ? m.cap_vv : 0;
            ti.cap_tt = (it.mask & kRelTT) ? default_cap_tt(m) : 0;
            ti.out_word = words;
            ti.hdr_index = nh++;
            words += block_layout(ti.mask, m.nV, m.nT, m.nnzVT, ti.cap_vv, ti.cap_tt).total;
            tiles.push_back(ti);
            out.push_back(ti);
        }
    }
    base.swap(out);
}

// The stitch launch over `stitch` (after the tiles' launches on st): work
// list = queue word, stitch items, tile items; into the batch's buffers.
gale_status launch_stitch_items(gale_ctx *ctx, Batch &b, const std::vector<StitchItem> &stitch,
                                const std::vector<WorkItem> &tiles, hipStream_t st, bool upload) {
    hipError_t e = hipSuccess;
    const int ns = (int)stitch.size();
    if (ns == 0) return GALE_OK;
    const size_t bytes = 64 + (size_t)ns * sizeof(StitchItem) + tiles.size() * sizeof(WorkItem);
    if (upload) {
        b.st_items = ctx->dev_pool.acquire(bytes, &e);
        b.st_host = ctx->pin_pool.acquire(bytes, &e);
        if (!b.st_items || !b.st_host) return fail(GALE_ENOMEM, "stitch work list");
        char *h = (char *)b.st_host->ptr;
        std::memset(h, 0, 64);
        std::memcpy(h + 64, stitch.data(), (size_t)ns * sizeof(StitchItem));
        std::memcpy(h + 64 + (size_t)ns * sizeof(StitchItem), tiles.data(), tiles.size() * sizeof(WorkItem));
        e = hipMemcpyAsync(b.st_items->ptr, h, bytes, hipMemcpyHostToDevice, st);
        if (e != hipSuccess) return fail(GALE_EDEVICE, std::string("stitch list copy: ") + hipGetErrorString(e));
    }
    char *d = (char *)b.st_items->ptr;
    SArgs a{};
    a.meta = ctx->d_meta;
    a.sm = ctx->d_sm;
    a.maps = ctx->d_maps;
    a.out = (int32_t *)b.out->ptr;
    a.hdr = (int32_t *)b.dev_hdr->ptr;
    a.items = (const StitchItem *)(d + 64);
    a.tiles = (const WorkItem *)(d + 64 + (size_t)ns * sizeof(StitchItem));
    a.nitems = ns;
    a.queue = (int32_t *)d;
    const int grid = std::max(1, std::min(ns, ctx->num_cus * 8));
    e = launch_stitch(a, grid, st);
    ctx->n_launches++;
    if (e != hipSuccess) return fail(GALE_EDEVICE, std::string("stitch launch: ") + hipGetErrorString(e));
    return GALE_OK;
}

// Lay out the batch's items in a fresh output buffer and launch them.
gale_status run_items(gale_ctx *ctx, Batch &b, int form, hipStream_t st) {
    hipError_t e;
    const int n = (int)b.items.size();
    b.out_words = lay_out_items(ctx, b.items, 0);
    std::vector<WorkItem> base, ext, tiles;
    std::vector<StitchItem> stitch;
    for (const WorkItem &it : b.items) ((it.mask & kRelExt) ? ext : base).push_back(it);
    int64_t words = b.out_words;
    int nh = n;
    if (form == GALE_FORM_BATCHED && ctx->cfg.mode == GALE_MODE_DIRECT)
        expand_tiles(ctx, base, words, nh, stitch, tiles);
    b.out = ctx->dev_pool.acquire((size_t)words * 4 + 256, &e);
    if (!b.out) return fail(GALE_ENOMEM, "device output buffer");
    b.host_hdr = ctx->pin_pool.acquire((size_t)n * 32 + 64, &e);
    if (!b.host_hdr) return fail(GALE_ENOMEM, "batch buffers");
    if (n == 0) return GALE_OK;
    if (!ext.empty() || nh > n) {
        b.dev_hdr = ctx->dev_pool.acquire((size_t)nh * 32 + 64, &e);
        if (!b.dev_hdr) return fail(GALE_ENOMEM, "batch buffers");
    }
    gale_status s = GALE_OK;
    if (!base.empty())
        s = upload_and_launch(ctx, form, base, (int32_t *)b.out->ptr, b.dev_items, b.dev_hdr, b.host_items, b.ws, st,
                              b.kev[0] ? b.kev : nullptr, &b.kev_recorded);
    if (!s && !stitch.empty()) {
        s = launch_stitch_items(ctx, b, stitch, tiles, st, true);
        // the kernel-time events bracket the stitch too
        if (!s && b.kev[1] && hipEventRecord(b.kev[1], st) != hipSuccess)
            s = fail(GALE_EDEVICE, "event record");
    }
    if (!s) s = launch_ext_items(ctx, b, form, ext, st);
    return s;
}

void release_batch(gale_ctx *ctx, Batch &b) {
    if (b.borrowed) {  // a graph ticket: the buffers belong to the prepared request
        b.out = b.dev_items = b.dev_hdr = b.ws = b.host_items = b.host_hdr = b.host_out = nullptr;
        return;
    }
    ctx->dev_pool.release(b.ext_items);
    ctx->dev_pool.release(b.ext_ws);
    ctx->pin_pool.release(b.ext_host);
    ctx->dev_pool.release(b.st_items);
    ctx->pin_pool.release(b.st_host);
    b.ext_items = b.ext_ws = b.ext_host = b.st_items = b.st_host = nullptr;
    ctx->dev_pool.release(b.out);
    ctx->dev_pool.release(b.dev_items);
    ctx->dev_pool.release(b.dev_hdr);
    ctx->dev_pool.release(b.ws);
    ctx->pin_pool.release(b.host_items);
    ctx->pin_pool.release(b.host_hdr);
    ctx->pin_pool.release(b.host_out);
    b.out = b.dev_items = b.dev_hdr = b.ws = b.host_items = b.host_hdr = b.host_out = nullptr;
}

// relation entries of a finalized batch's blocks (from their headers)
uint64_t batch_entries(const Batch &b) {
    uint64_t ent = 0;
    for (size_t i = 0; i < b.items.size(); ++i) {
        const int32_t *h = &b.hdr[i * 8];
        const uint32_t mk = b.items[i].mask;
        if (mk & kRelExt) {
            for (int r = 0; r < 5; ++r)
                if (mk & (kRelVE << r)) ent += (uint64_t)h[1 + r];
            continue;
        }
        if (mk & kRelVT) ent += (uint64_t)h[3];
        if (mk & kRelVV) ent += (uint64_t)h[4];
        if (mk & kRelTT) ent += (uint64_t)h[5];
    }
    return ent;
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
    ctx->n_entries += batch_entries(b);
    ctx->n_blocks += n;
    return GALE_OK;
}

// Copy every block of a finalized batch to pinned host memory (synchronous).
gale_status copy_batch_to_host(gale_ctx *ctx, Batch &b, hipStream_t st) {
    // one host buffer laid out like the device buffers, blocks at their words
    int64_t words = 0;
    const int n = (int)b.items.size();
    b.host_word.assign(n, 0);
    // exact used size: VV is last, so its tail beyond the real count is
    // skipped; an edge / triangle block is copied whole
    auto used_words = [&](int i) -> int64_t {
        const WorkItem &it = b.items[i];
        const ClusterMeta &m = ctx->meta[it.cluster];
        if (it.mask & kRelExt) return ext_layout(it.mask, m, ctx->sx.ext[it.cluster]).total;
        const int32_t *h = &b.hdr[(size_t)i * 8];
        const int32_t used_vv = (it.mask & kRelVV) ? h[4] : 0;
        return block_layout(it.mask, m.nV, m.nT, m.nnzVT, used_vv, it.cap_tt).total;
    };
    for (int i = 0; i < n; ++i) {
        b.host_word[i] = words;
        words += used_words(i);
    }
    hipError_t e;
    b.host_out = ctx->pin_pool.acquire((size_t)words * 4 + 256, &e);
    if (!b.host_out) return fail(GALE_ENOMEM, "pinned host buffer");
    uint64_t bytes = 0;
    for (int i = 0; i < n; ++i) {
        const int64_t wds = used_words(i);
        const int32_t *src = (const int32_t *)b.loc[i].buf->ptr + b.loc[i].word;
        int32_t *dst = (int32_t *)b.host_out->ptr + b.host_word[i];
        e = hipMemcpyAsync(dst, src, (size_t)wds * 4, hipMemcpyDeviceToHost, st);
        if (e != hipSuccess) return fail(GALE_EDEVICE, std::string("block copy: ") + hipGetErrorString(e));
        bytes += (uint64_t)wds * 4;
    }
    e = hipStreamSynchronize(st);
    if (e != hipSuccess) return fail(GALE_EDEVICE, std::string("block copy: ") + hipGetErrorString(e));
    ctx->n_bytes_d2h += bytes;
    ctx->n_delivered += batch_entries(b);
    b.host_ready = true;
    return GALE_OK;
}

// view of block i of a finalized batch
gale_status block_view(const gale_ctx *ctx, const Batch &b, int i, uint32_t rel, bool host, gale_csr *out) {
    const WorkItem &it = b.items[i];
    const ClusterMeta &m = ctx->meta[it.cluster];
    const int32_t *h = &b.hdr[(size_t)i * 8];
    if (it.mask & kRelExt) {
        if (host && !b.host_ready) return fail(GALE_ESTATE, "ticket has no host copy (made with gale_build)");
        const ExtLayout lay = ext_layout(it.mask, m, ctx->sx.ext[it.cluster]);
        const int32_t *base = host ? (const int32_t *)b.host_out->ptr + b.host_word[i]
                                   : (const int32_t *)b.loc[i].buf->ptr + b.loc[i].word;
        int r = 0;
        while (r < 5 && rel != (kRelVE << r)) ++r;
        out->cluster = it.cluster;
        out->rel = rel;
        out->pad = 0;
        out->nrows = lay.nrows[r];
        out->nnz = h[1 + r];
        out->row_ids = base + lay.rows[r];
        out->offsets = base + lay.off[r];
        out->entries = base + lay.ent[r];
        return GALE_OK;
    }
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
    if (mask == 0 || (mask & ~(GALE_REL_ALL | GALE_REL_EXT)))
        return fail(GALE_EINVAL, "relation mask must be a non-empty subset of VT|VV|TT|VE|VF|EF|ET|FT");
    if ((mask & GALE_REL_EXT) && !ctx->has_simplices)
        return fail(GALE_ESTATE, "edge / triangle relations need gale_config.simplex_lists at load");
    if ((mask & GALE_REL_EXT) && ctx->cfg.mode == GALE_MODE_SERVE)
        return fail(GALE_EINVAL, "SERVE mode builds VT, VV and TT");
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
            for (uint32_t bit : {kRelVT, kRelVV, kRelTT, kRelVE, kRelVF, kRelEF, kRelET, kRelFT})
                if (mask & bit) mk(k, bit);
    } else {
        std::stable_sort(u.begin(), u.end(), [&](int32_t x, int32_t y) {
            const int64_t cx = (int64_t)ctx->meta[x].ns + ctx->meta[x].nh;
            const int64_t cy = (int64_t)ctx->meta[y].ns + ctx->meta[y].nh;
            return cx > cy;
        });
        // VT / VV / TT in one item per cluster, the edge and triangle
        // relations in another (a kernel of their own)
        if (mask & kRelBase)
            for (int32_t k : u) mk(k, mask & kRelBase);
        if (mask & kRelExt)
            for (int32_t k : u) mk(k, mask & kRelExt);
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

// ---- tune table --------------------------------------------------------------
// A JSON file with one object per tuned (mesh, relation mask):
//   {"gale_tune_table": 1, "entries": [
//     {"nv": .., "nt": .., "nclusters": .., "rel_mask": .., "launch_classes": ..,
//      "global_cu_share": .., "global_threads": .., "kernel_ms": ..,
//      "class_ms": [.., .., .., ..]}, ...]}
// Only this writer's format is read back: each entry object on a line of its own.
namespace {

bool json_number(const std::string &obj, const char *key, double &out) {
    const std::string k = std::string("\"") + key + "\"";
    const size_t p = obj.find(k);
    if (p == std::string::npos) return false;
    size_t q = obj.find(':', p + k.size());
    if (q == std::string::npos) return false;
    ++q;
    while (q < obj.size() && (obj[q] == ' ' || obj[q] == '\t')) ++q;
    char *end = nullptr;
    const double v = std::strtod(obj.c_str() + q, &end);
    if (end == obj.c_str() + q) return false;
    out = v;
    return true;
}

// the entry objects of a table file, one string each
std::vector<std::string> tune_objects(const std::string &path) {
    std::vector<std::string> objs;
    FILE *f = std::fopen(path.c_str(), "r");
    if (!f) return objs;
    std::string line;
    char buf[4096];
    while (std::fgets(buf, sizeof(buf), f)) {
        line += buf;
        if (line.empty() || line.back() != '\n') continue;
        const size_t a = line.find("{\"nv\"");
        const size_t b = line.rfind('}');
        if (a != std::string::npos && b != std::string::npos && b > a) objs.push_back(line.substr(a, b - a + 1));
        line.clear();
    }
    std::fclose(f);
    return objs;
}

bool entry_of(const std::string &o, TuneEntry &te) {
    double nv, nt, ncl, mask, lc, share = 1.0, gt = 1024, kms = 0;
    if (!json_number(o, "nv", nv) || !json_number(o, "nt", nt) || !json_number(o, "nclusters", ncl) ||
        !json_number(o, "rel_mask", mask) || !json_number(o, "launch_classes", lc))
        return false;
    json_number(o, "global_cu_share", share);
    json_number(o, "global_threads", gt);
    json_number(o, "kernel_ms", kms);
    te.nv = (int64_t)nv;
    te.nt = (int64_t)nt;
    te.ncl = (int64_t)ncl;
    te.rel_mask = (int)mask;
    te.launch_classes = (int)lc;
    te.global_cu_share = share;
    te.global_threads = (int)gt;
    te.kernel_ms = kms;
    return true;
}

std::string entry_json(const TuneEntry &te) {
    char buf[512];
    std::snprintf(buf, sizeof(buf),
                  "{\"nv\": %lld, \"nt\": %lld, \"nclusters\": %lld, \"rel_mask\": %d, \"launch_classes\": %d, "
                  "\"global_cu_share\": %.4f, \"global_threads\": %d, \"kernel_ms\": %.4f, "
                  "\"class_ms\": [%.4f, %.4f, %.4f, %.4f]}",
                  (long long)te.nv, (long long)te.nt, (long long)te.ncl, te.rel_mask, te.launch_classes,
                  te.global_cu_share, te.global_threads, te.kernel_ms, te.class_ms[0], te.class_ms[1],
                  te.class_ms[2], te.class_ms[3]);
    return buf;
}

}  // namespace

// The entry for a mesh of this size and cluster count; the relation mask 7
// entry is preferred, else the first match.
bool read_tune_entry(const std::string &path, int64_t nv, int64_t nt, int64_t ncl, TuneEntry &out) {
    bool found = false;
    for (const std::string &o : tune_objects(path)) {
        TuneEntry te;
        if (!entry_of(o, te) || te.nv != nv || te.nt != nt || te.ncl != ncl) continue;
        if (!found || te.rel_mask == 7) out = te;
        found = true;
    }
    return found;
}

// Replace (or add) the entry for the same mesh and mask; written to a
// temporary file first and renamed over the table.
bool write_tune_entry(const std::string &path, const TuneEntry &te) {
    std::vector<std::string> keep;
    for (const std::string &o : tune_objects(path)) {
        TuneEntry x;
        if (entry_of(o, x) && x.nv == te.nv && x.nt == te.nt && x.ncl == te.ncl && x.rel_mask == te.rel_mask)
            continue;
        keep.push_back(o);
    }
    keep.push_back(entry_json(te));
    const std::string tmp = path + ".tmp";
    FILE *f = std::fopen(tmp.c_str(), "w");
    if (!f) return false;
    std::fprintf(f, "{\"gale_tune_table\": 1,\n \"entries\": [\n");
    for (size_t i = 0; i < keep.size(); ++i)
        std::fprintf(f, "  %s%s\n", keep[i].c_str(), i + 1 < keep.size() ? "," : "");
    std::fprintf(f, " ]}\n");
    const bool ok = std::fclose(f) == 0;
    return ok && std::rename(tmp.c_str(), path.c_str()) == 0;
}

// ---- prepared (graph) requests --------------------------------------------
gale_status graph_create(gale_ctx *ctx, const int32_t *ids, int32_t n, uint32_t mask, uint64_t *out) {
    gale_status s = check_request(ctx, ids, n, mask);
    if (s) return s;
    if (mask & kRelExt) return fail(GALE_EINVAL, "graphs capture VT, VV and TT requests");
    if (ctx->poisoned) return fail(GALE_EDEVICE, "context poisoned by an earlier device error");
    auto *g = new Prepared();
    g->batch.items = make_items(ctx, ids, n, mask, GALE_FORM_BATCHED);
    g->mask = mask;
    for (size_t i = 0; i < g->batch.items.size(); ++i) g->by_cluster[g->batch.items[i].cluster].push_back((int)i);
    std::lock_guard<std::mutex> lk(ctx->direct_mu);
    Batch &b = g->batch;
    hipError_t e = hipSuccess;
    const int ni = (int)b.items.size();
    b.out_words = lay_out_items(ctx, b.items, 0);
    // tiled clusters: their tiles' items launched, the stitch captured after
    std::vector<WorkItem> launch(b.items), tiles;
    std::vector<StitchItem> stitch;
    int64_t words = b.out_words;
    int nh = ni;
    expand_tiles(ctx, launch, words, nh, stitch, tiles);
    b.out = ctx->dev_pool.acquire((size_t)words * 4 + 256, &e);
    b.host_hdr = ctx->pin_pool.acquire((size_t)ni * 32 + 64, &e);
    if (nh > ni) b.dev_hdr = ctx->dev_pool.acquire((size_t)nh * 32 + 64, &e);
    if (!b.out || !b.host_hdr || (nh > ni && !b.dev_hdr)) s = fail(GALE_ENOMEM, "prepared request buffers");
    std::vector<int> ncls;
    int n_glob = 0;
    int64_t wsb = 0;
    if (!s && ni > 0)
        s = stage_items(ctx, GALE_FORM_BATCHED, launch, b.dev_items, b.dev_hdr, b.host_items, b.ws, ctx->stream,
                        ncls, n_glob, wsb);
    if (!s && !stitch.empty()) {
        // the stitch work list goes up now; the capture only zeroes its queue word
        b.st_items = ctx->dev_pool.acquire(64 + stitch.size() * sizeof(StitchItem) + tiles.size() * sizeof(WorkItem), &e);
        b.st_host = ctx->pin_pool.acquire(64 + stitch.size() * sizeof(StitchItem) + tiles.size() * sizeof(WorkItem), &e);
        if (!b.st_items || !b.st_host) s = fail(GALE_ENOMEM, "stitch work list");
        if (!s) {
            char *h = (char *)b.st_host->ptr;
            std::memset(h, 0, 64);
            std::memcpy(h + 64, stitch.data(), stitch.size() * sizeof(StitchItem));
            std::memcpy(h + 64 + stitch.size() * sizeof(StitchItem), tiles.data(), tiles.size() * sizeof(WorkItem));
            if (hipMemcpyAsync(b.st_items->ptr, h, 64 + stitch.size() * sizeof(StitchItem) +
                                                      tiles.size() * sizeof(WorkItem),
                               hipMemcpyHostToDevice, ctx->stream) != hipSuccess)
                s = fail(GALE_EDEVICE, "stitch list copy");
        }
    }
    if (!s && hipStreamSynchronize(ctx->stream) != hipSuccess) s = fail(GALE_EDEVICE, "work list copy");
    if (!s && ni > 0) {
        // capture: zero the queue words, then the launches (forked over the
        // auxiliary streams and joined back), then the stitch
        e = hipStreamBeginCapture(ctx->stream, hipStreamCaptureModeThreadLocal);
        if (e == hipSuccess) e = launch_zero((int32_t *)b.dev_items->ptr, 16, ctx->stream);
        if (e == hipSuccess && b.st_items) e = launch_zero((int32_t *)b.st_items->ptr, 16, ctx->stream);
        gale_status ls = GALE_OK;
        if (e == hipSuccess) {
            char *di = (char *)b.dev_items->ptr;
            ls = launch_batch(ctx, GALE_FORM_BATCHED, (int32_t *)b.out->ptr, (int32_t *)b.dev_hdr->ptr,
                              (const WorkItem *)(di + 64), ncls, n_glob, (int32_t *)di,
                              b.ws ? (char *)b.ws->ptr : nullptr, wsb, ctx->stream, true, nullptr, nullptr);
            if (ls == GALE_OK && !stitch.empty()) ls = launch_stitch_items(ctx, b, stitch, tiles, ctx->stream, false);
        }
        hipGraph_t graph = nullptr;
        const hipError_t e2 = hipStreamEndCapture(ctx->stream, &graph);
        if (e == hipSuccess) e = e2;
        if (e == hipSuccess && ls == GALE_OK) e = hipGraphInstantiate(&g->exec, graph, nullptr, nullptr, 0);
        g->graph = graph;
        if (ls) s = ls;
        else if (e != hipSuccess) s = fail(GALE_EDEVICE, std::string("graph capture: ") + hipGetErrorString(e));
    }
    if (s) {
        if (g->exec) (void)hipGraphExecDestroy(g->exec);
        if (g->graph) (void)hipGraphDestroy(g->graph);
        release_batch(ctx, b);
        delete g;
        return s;
    }
    *out = ++ctx->next_graph;
    ctx->graphs[*out] = g;
    return GALE_OK;
}

gale_status graph_launch(gale_ctx *ctx, uint64_t gid, uint64_t *ticket_out) {
    if (ctx->poisoned) return fail(GALE_EDEVICE, "context poisoned by an earlier device error");
    auto *t = new Ticket();
    {
        std::lock_guard<std::mutex> lk(ctx->direct_mu);
        auto it = ctx->graphs.find(gid);
        if (it == ctx->graphs.end()) {
            delete t;
            return fail(GALE_ENOENT, "unknown graph");
        }
        Prepared *g = it->second;
        t->batch.items = g->batch.items;
        t->batch.out_words = g->batch.out_words;
        t->batch.out = g->batch.out;
        t->batch.dev_items = g->batch.dev_items;
        t->batch.dev_hdr = g->batch.dev_hdr;
        t->batch.host_hdr = g->batch.host_hdr;
        t->batch.borrowed = true;
        t->graph = gid;
        t->mask = g->mask;
        t->host = false;
        t->by_cluster = g->by_cluster;
        hipError_t e = hipSuccess;
        if (hipEventCreate(&t->batch.kev[0]) != hipSuccess || hipEventCreate(&t->batch.kev[1]) != hipSuccess)
            destroy_ticket_events(t);
        if (t->batch.kev[0]) e = hipEventRecord(t->batch.kev[0], ctx->stream);
        if (e == hipSuccess && g->exec) e = hipGraphLaunch(g->exec, ctx->stream);
        if (e == hipSuccess && t->batch.kev[1]) {
            e = hipEventRecord(t->batch.kev[1], ctx->stream);
            t->batch.kev_recorded = e == hipSuccess;
        }
        if (e == hipSuccess) e = hipEventCreateWithFlags(&t->done, hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventRecord(t->done, ctx->stream);
        if (e != hipSuccess) {
            ctx->poisoned = true;
            if (t->done) (void)hipEventDestroy(t->done);
            destroy_ticket_events(t);
            delete t;
            return fail(GALE_EDEVICE, std::string("graph launch: ") + hipGetErrorString(e));
        }
        ctx->n_requests++;
        g->live++;
    }
    std::lock_guard<std::mutex> g2(ctx->tick_mu);
    const uint64_t id = ++ctx->next_ticket;
    ctx->tickets[id] = t;
    *ticket_out = id;
    return GALE_OK;
}

gale_status graph_destroy(gale_ctx *ctx, uint64_t gid) {
    std::lock_guard<std::mutex> lk(ctx->direct_mu);
    auto it = ctx->graphs.find(gid);
    if (it == ctx->graphs.end()) return fail(GALE_ENOENT, "unknown graph");
    Prepared *g = it->second;
    if (g->live > 0)
        return fail(GALE_ESTATE, std::to_string(g->live) + " ticket(s) of this graph are not released");
    (void)hipStreamSynchronize(ctx->stream);
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    release_batch(ctx, g->batch);
    delete g;
    ctx->graphs.erase(it);
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
    if (!(cfg.global_cu_share >= 0.0 && cfg.global_cu_share <= 1.0))
        return fail(GALE_EINVAL, "global_cu_share must be in [0, 1]");
    if (cfg.dev_arena && cfg.mode != GALE_MODE_SERVE) return fail(GALE_EINVAL, "dev_arena is for SERVE mode only");
    if (cfg.dev_arena && cfg.arena_bytes < (1ull << 20)) return fail(GALE_EINVAL, "arena_bytes must be >= 1 MiB");
    if (cfg.dev_arena && ((uintptr_t)cfg.dev_arena & 255u)) return fail(GALE_EINVAL, "dev_arena must be 256-byte aligned");
    if (cfg.prefetch_depth < 0 || cfg.prefetch_depth > 64) return fail(GALE_EINVAL, "prefetch_depth must be in 0..64");
    if (cfg.front_end != GALE_FRONT_SINGLE && cfg.front_end != GALE_FRONT_PER_RELATION)
        return fail(GALE_EINVAL, "unknown front_end");
    int ndev = 0;
    hipError_t e = hipGetDeviceCount(&ndev);
    if (e != hipSuccess || ndev <= 0) return fail(GALE_EDEVICE, "no HIP device");
    if (cfg.device < 0 || cfg.device >= ndev) return fail(GALE_EINVAL, "device ordinal out of range");
    e = hipSetDevice(cfg.device);
    if (e != hipSuccess) return fail(GALE_EDEVICE, std::string("hipSetDevice: ") + hipGetErrorString(e));
    // the static scratch of gale_build_static: its address on this device, once
    gale_status ss = static_scratch_setup(cfg.device);
    if (ss) return ss;
    auto *ctx = new gale_ctx();
    ctx->cfg = cfg;
    if (cfg.tune_table_path) ctx->tune_path = cfg.tune_table_path;
    ctx->cfg.tune_table_path = nullptr;  // the copy above is the one used
    ctx->glob_share = cfg.global_cu_share > 0.0 ? cfg.global_cu_share : 1.0;
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
    ctx->static_lds = static_lds;
    ctx->shared_per_block = (int64_t)prop.sharedMemPerBlock;
    setup_classes(ctx, cfg.launch_classes);
    setup_global(ctx, ctx->block_threads);
    if (cfg.mode == GALE_MODE_DIRECT) {
        // streams for the launches of one batch beyond the first (classes and
        // the global path run side by side), default priority
        const int naux = 3;  // up to two more classes and the global path
        for (int i = 0; i < naux; ++i) {
            hipStream_t s2 = nullptr;
            hipEvent_t ev = nullptr;
            if (hipStreamCreateWithFlags(&s2, hipStreamNonBlocking) != hipSuccess ||
                hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) {
                if (s2) (void)hipStreamDestroy(s2);
                break;
            }
            ctx->aux.push_back(s2);
            ctx->join_ev.push_back(ev);
        }
        if (hipEventCreateWithFlags(&ctx->fork_ev, hipEventDisableTiming) != hipSuccess) ctx->fork_ev = nullptr;
        if (!ctx->fork_ev) {
            for (hipStream_t s2 : ctx->aux) (void)hipStreamDestroy(s2);
            for (hipEvent_t ev : ctx->join_ev) (void)hipEventDestroy(ev);
            ctx->aux.clear();
            ctx->join_ev.clear();
        }
    }
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
    // tiles of the clusters that do not fit a 1024-thread workgroup's LDS
    // (DIRECT mode): their streams are prepared as pseudo-clusters and
    // appended after the clusters' own, their metadata after the clusters'
    std::vector<StitchMeta> smeta;
    std::vector<int32_t> smaps;
    if (ctx->cfg.mode == GALE_MODE_DIRECT && ctx->cfg.tile_entries >= 0) {
        const int64_t tile_vt = ctx->cfg.tile_entries > 0 ? ctx->cfg.tile_entries : 10000;
        std::vector<ClusterMeta> want(hs.meta);
        for (ClusterMeta &m : want)
            if (lds_plan(m, kRelBase, ctx->lds_budget, 1024).ok) m.nnzVT = 0;  // fits: not tiled
        TilePlan tp;
        s = plan_tiles(nv, nt, tv, cl, ncl, want, tile_vt, tp);
        if (s) return fail(s, "tile plan");
        if (tp.ntiles > 0) {
            HostStreams ts;
            s = prepare_streams(nv, nt, tv, tp.pseudo.data(), tp.npseudo, ts, err, &tp.keep);
            if (s) return fail(s, err);
            stitch_maps(tp, ts, ncl, smeta, smaps);
            const int64_t tb0 = (int64_t)hs.tets.size(), tid0 = (int64_t)hs.tid.size(),
                          lv0 = (int64_t)hs.lverts.size();
            int64_t tbn = 0, tidn = 0, lvn = 0;
            for (int32_t i = 0; i < tp.ntiles; ++i) {
                const ClusterMeta &m = ts.meta[tp.pseudo_of_tile[i]];
                const int64_t ntot = (int64_t)m.ns + m.nh;
                tbn += (ntot * ((m.flags & kMetaWide) ? 16 : 8) + 15) / 16 * 16;
                tidn += ntot;
                lvn += m.L;
            }
            hs.tets.resize((size_t)(tb0 + tbn));
            hs.tid.resize((size_t)(tid0 + tidn));
            hs.lverts.resize((size_t)(lv0 + lvn));
            int64_t tb = tb0, ti = tid0, lv = lv0;
            for (int32_t i = 0; i < tp.ntiles; ++i) {
                ClusterMeta m = ts.meta[tp.pseudo_of_tile[i]];
                const int64_t ntot = (int64_t)m.ns + m.nh;
                const int64_t tbytes = (ntot * ((m.flags & kMetaWide) ? 16 : 8) + 15) / 16 * 16;
                std::memcpy(hs.tets.data() + tb, ts.tets.data() + m.tb_off, (size_t)tbytes);
                std::memcpy(hs.tid.data() + ti, ts.tid.data() + m.tet_off, (size_t)ntot * 4);
                std::memcpy(hs.lverts.data() + lv, ts.lverts.data() + m.lv_off, (size_t)m.L * 4);
                m.tb_off = tb;
                m.tet_off = ti;
                m.lv_off = lv;
                tb += tbytes;
                ti += ntot;
                lv += m.L;
                hs.meta.push_back(m);
            }
            ctx->ntiles = tp.ntiles;
            ctx->tile_first = tp.tile_first;
            ctx->tile_count = tp.tile_count;
        }
    }
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
    if (e == hipSuccess && ctx->ntiles > 0) {
        e = up((void **)&ctx->d_sm, smeta.data(), smeta.size() * sizeof(StitchMeta));
        if (e == hipSuccess) e = up((void **)&ctx->d_maps, smaps.data(), smaps.size() * 4);
    }
    if (e != hipSuccess) {
        ctx->poisoned = true;
        return fail(e == hipErrorOutOfMemory ? GALE_ENOMEM : GALE_EDEVICE,
                    std::string("mesh upload: ") + hipGetErrorString(e));
    }
    ctx->mesh_bytes = hs.tets.size() + (hs.tid.size() + hs.lverts.size()) * 4 + hs.meta.size() * sizeof(ClusterMeta);
    if (ctx->cfg.simplex_lists) {
        // the edge and triangle lists (Section 4.3), their index by smallest
        // vertex and the per-cluster ranges, on the GPU; E, F and the
        // interval arrays stay on the host for gale_get_simplices
        s = enumerate_simplices(hs, ctx->sx, err);
        if (s) return fail(s, err);
        HostSimplices &x = ctx->sx;
        e = up((void **)&ctx->d_ext, x.ext.data(), x.ext.size() * sizeof(ExtMeta));
        if (e == hipSuccess) e = up((void **)&ctx->d_eoff, x.eoff.data(), x.eoff.size() * 4);
        if (e == hipSuccess) e = up((void **)&ctx->d_eidx, x.eidx.data(), x.eidx.size() * 4);
        if (e == hipSuccess) e = up((void **)&ctx->d_foff, x.foff.data(), x.foff.size() * 4);
        if (e == hipSuccess) e = up((void **)&ctx->d_fidx, x.fidx.data(), x.fidx.size() * 4);
        if (e != hipSuccess) {
            ctx->poisoned = true;
            return fail(e == hipErrorOutOfMemory ? GALE_ENOMEM : GALE_EDEVICE,
                        std::string("edge / triangle list upload: ") + hipGetErrorString(e));
        }
        ctx->mesh_bytes += (x.eoff.size() + x.eidx.size() + x.foff.size() + x.fidx.size()) * 4 +
                           x.ext.size() * sizeof(ExtMeta);
        std::vector<int32_t>().swap(x.eoff);
        std::vector<int32_t>().swap(x.eidx);
        std::vector<int32_t>().swap(x.foff);
        std::vector<int32_t>().swap(x.fidx);
        ctx->has_simplices = true;
    }
    ctx->stream_tets = (int64_t)hs.tid.size();
    ctx->meta = std::move(hs.meta);
    ctx->nv = nv;
    ctx->nt = nt;
    ctx->ncl = ncl;
    ctx->loaded = true;
    ctx->load_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (!ctx->tune_path.empty()) {
        TuneEntry te;
        if (read_tune_entry(ctx->tune_path, nv, nt, ncl, te)) {
            setup_classes(ctx, te.launch_classes);
            if (ctx->block_threads == 1024 && (te.global_threads == 512 || te.global_threads == 1024))
                setup_global(ctx, te.global_threads);
            if (te.global_cu_share > 0.0 && te.global_cu_share <= 1.0) ctx->glob_share = te.global_cu_share;
            ctx->tune_applied = true;
        }
    }
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
    if (rel == 0 || (rel & (rel - 1)) || (rel & ~(GALE_REL_ALL | GALE_REL_EXT)))
        return fail(GALE_EINVAL, "rel must be one relation bit");
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
    if (t->graph) {
        std::lock_guard<std::mutex> g(ctx->direct_mu);
        auto it = ctx->graphs.find(t->graph);
        if (it != ctx->graphs.end()) it->second->live--;
    }
    for (Buf *b : t->batch.extra) ctx->dev_pool.release(b);
    release_batch(ctx, t->batch);
    delete t;
    return GALE_OK;
}

void *gale_stream(gale_ctx *ctx) { return ctx ? (void *)ctx->stream : nullptr; }

gale_status gale_autotune(gale_ctx *ctx, const int32_t *ids, int32_t n, uint32_t mask, int32_t reps,
                          int32_t *chosen_out, double *ms_out) {
    if (!ctx) return fail(GALE_EINVAL, "ctx is NULL");
    if (ctx->cfg.mode != GALE_MODE_DIRECT) return fail(GALE_ESTATE, "autotune needs a DIRECT mode context");
    if (reps < 1) return fail(GALE_EINVAL, "reps must be >= 1");
    gale_status st = check_request(ctx, ids, n, mask);
    if (st) return st;
    if (mask & kRelExt) return fail(GALE_EINVAL, "autotune times VT, VV and TT requests");
    const int candidates[4] = {0, 2, 4, 6};
    double ms[4] = {0, 0, 0, 0};
    uint64_t saved_n;
    double saved_ms;
    {
        std::lock_guard<std::mutex> g(ctx->direct_mu);
        saved_n = ctx->n_timed;
        saved_ms = ctx->kernel_ms;
    }
    int best = -1;
    // mean kernel milliseconds of the request under the current settings
    auto time_it = [&]() -> double {
        for (int r = 0; r <= reps && st == GALE_OK; ++r) {
            if (r == 1) {
                std::lock_guard<std::mutex> g(ctx->direct_mu);
                ctx->n_timed = 0;
                ctx->kernel_ms = 0.0;
            }
            uint64_t tk = 0;
            st = gale_build(ctx, ids, n, mask, GALE_FORM_BATCHED, &tk);
            if (st == GALE_OK) st = gale_poll(ctx, tk, -1);
            if (tk) (void)gale_release(ctx, tk);
        }
        std::lock_guard<std::mutex> g(ctx->direct_mu);
        return ctx->n_timed ? ctx->kernel_ms / (double)ctx->n_timed : 0.0;
    };
    const double saved_share = ctx->glob_share;
    const int saved_bt = ctx->glob_bt;
    ctx->glob_share = 1.0;
    // 1. workgroup shapes (launch classes)
    for (int ci = 0; ci < 4 && st == GALE_OK; ++ci) {
        {
            std::lock_guard<std::mutex> g(ctx->direct_mu);
            setup_classes(ctx, candidates[ci]);
        }
        ms[ci] = time_it();
        if (st == GALE_OK && (best < 0 || ms[ci] < ms[best])) best = ci;
    }
    {
        std::lock_guard<std::mutex> g(ctx->direct_mu);
        setup_classes(ctx, best >= 0 ? candidates[best] : ctx->cfg.launch_classes);
    }
    double best_ms = best >= 0 ? ms[best] : 0.0;
    // 2. and 3. for requests with clusters on the global path: its workgroup
    // size, then its share of the CUs when LDS-path classes run beside it
    int nglob = 0;
    if (st == GALE_OK) {
        for (int32_t i = 0; i < n; ++i) {
            WorkItem it{};
            it.cluster = ids[i];
            it.mask = mask;
            nglob += item_class(ctx, it) < 0;
        }
    }
    if (st == GALE_OK && nglob > 0 && ctx->block_threads == 1024) {
        setup_global(ctx, 512);
        const double t = time_it();
        if (st == GALE_OK && t < best_ms)
            best_ms = t;
        else
            setup_global(ctx, 1024);
    }
    if (st == GALE_OK && nglob > 0 && nglob < n) {
        const double shares[3] = {0.8, 0.65, 0.5};
        double best_share = 1.0;
        for (int si = 0; si < 3 && st == GALE_OK; ++si) {
            ctx->glob_share = shares[si];
            const double t = time_it();
            if (st == GALE_OK && t < best_ms) {
                best_ms = t;
                best_share = shares[si];
            }
        }
        ctx->glob_share = best_share;
    }
    if (st != GALE_OK) {
        ctx->glob_share = saved_share;
        setup_global(ctx, saved_bt);
    }
    {
        std::lock_guard<std::mutex> g(ctx->direct_mu);
        ctx->n_timed = saved_n;
        ctx->kernel_ms = saved_ms;
    }
    if (st != GALE_OK) return st;
    if (chosen_out) *chosen_out = candidates[best];
    if (ms_out)
        for (int i = 0; i < 4; ++i) ms_out[i] = ms[i];
    if (!ctx->tune_path.empty()) {
        TuneEntry te;
        te.nv = ctx->nv;
        te.nt = ctx->nt;
        te.ncl = ctx->ncl;
        te.rel_mask = (int)mask;
        te.launch_classes = candidates[best];
        te.global_cu_share = ctx->glob_share;
        te.global_threads = ctx->glob_bt;
        te.kernel_ms = best_ms;
        for (int i = 0; i < 4; ++i) te.class_ms[i] = ms[i];
        if (!write_tune_entry(ctx->tune_path, te))
            return fail(GALE_ENOENT, "cannot write the tune table " + ctx->tune_path);
    }
    return GALE_OK;
}

gale_status gale_graph_create(gale_ctx *ctx, const int32_t *ids, int32_t n, uint32_t mask, uint64_t *graph_out) {
    if (!ctx || !graph_out) return fail(GALE_EINVAL, "NULL argument");
    if (ctx->cfg.mode != GALE_MODE_DIRECT) return fail(GALE_ESTATE, "graphs need a DIRECT mode context");
    return graph_create(ctx, ids, n, mask, graph_out);
}

gale_status gale_graph_launch(gale_ctx *ctx, uint64_t graph, uint64_t *ticket_out) {
    if (!ctx || !ticket_out) return fail(GALE_EINVAL, "NULL argument");
    if (ctx->cfg.mode != GALE_MODE_DIRECT) return fail(GALE_ESTATE, "graphs need a DIRECT mode context");
    return graph_launch(ctx, graph, ticket_out);
}

gale_status gale_graph_destroy(gale_ctx *ctx, uint64_t graph) {
    if (!ctx) return fail(GALE_EINVAL, "ctx is NULL");
    if (ctx->cfg.mode != GALE_MODE_DIRECT) return fail(GALE_ESTATE, "graphs need a DIRECT mode context");
    return graph_destroy(ctx, graph);
}

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
    out->hybrid_path_blocks = ctx->n_hybrid_blocks;
    out->global_cu_share = ctx->glob_share;
    out->tt_exhaustive_blocks = ctx->n_tt_exhaustive;
    out->front_end = ctx->cfg.front_end;
    out->tune_applied = ctx->tune_applied ? 1 : 0;
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

gale_status gale_get_cluster_info(gale_ctx *ctx, int32_t cluster, gale_cluster_info *out) {
    if (!ctx || !out) return fail(GALE_EINVAL, "NULL argument");
    if (!ctx->loaded) return fail(GALE_ESTATE, "no mesh loaded");
    if (cluster < 0 || cluster >= ctx->ncl) return fail(GALE_EINVAL, "cluster id out of range");
    const ClusterMeta &m = ctx->meta[cluster];
    out->cluster = cluster;
    out->nV = m.nV;
    out->nT = m.nT;
    out->ns = m.ns;
    out->nh = m.nh;
    out->L = m.L;
    out->nnzVT = m.nnzVT;
    out->cap_vv = m.cap_vv;
    return GALE_OK;
}

gale_status gale_get_simplices(gale_ctx *ctx, gale_simplices *out) {
    if (!ctx || !out) return fail(GALE_EINVAL, "NULL argument");
    if (!ctx->loaded || !ctx->has_simplices)
        return fail(GALE_ESTATE, "no mesh loaded with gale_config.simplex_lists");
    const HostSimplices &x = ctx->sx;
    out->ne = (int64_t)x.e.size() / 2;
    out->nf = (int64_t)x.f.size() / 3;
    out->ncl = ctx->ncl;
    out->pad = 0;
    out->e = x.e.data();
    out->f = x.f.data();
    out->ie = x.ie.data();
    out->if_ = x.if_.data();
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
    for (auto &kv : ctx->graphs) {
        if (kv.second->exec) (void)hipGraphExecDestroy(kv.second->exec);
        if (kv.second->graph) (void)hipGraphDestroy(kv.second->graph);
        delete kv.second;
    }
    ctx->graphs.clear();
    ctx->dev_pool.clear();
    ctx->pin_pool.clear();
    if (ctx->d_tets) (void)hipFree(ctx->d_tets);
    if (ctx->d_tid) (void)hipFree(ctx->d_tid);
    if (ctx->d_lverts) (void)hipFree(ctx->d_lverts);
    if (ctx->d_meta) (void)hipFree(ctx->d_meta);
    if (ctx->d_sm) (void)hipFree(ctx->d_sm);
    if (ctx->d_maps) (void)hipFree(ctx->d_maps);
    for (void *p : {(void *)ctx->d_ext, (void *)ctx->d_eoff, (void *)ctx->d_eidx, (void *)ctx->d_foff,
                    (void *)ctx->d_fidx})
        if (p) (void)hipFree(p);
    for (hipStream_t s2 : ctx->aux) (void)hipStreamDestroy(s2);
    for (hipEvent_t ev : ctx->join_ev) (void)hipEventDestroy(ev);
    if (ctx->fork_ev) (void)hipEventDestroy(ctx->fork_ev);
    if (ctx->own_stream) (void)hipStreamDestroy(ctx->stream);
    delete ctx;
}

}  // extern "C"
