// gale_static.cpp -- gale_build_static: the batched build with no device
// allocation.  Every device buffer of a batched build other than the caller's
// output (the work list with its queue words, the block headers and the
// global path's workspace slices) lives in one file-scope static array,
// `scratch`, of kStaticScratchBytes per GPU.
//
// Host code never passes `scratch` itself to a kernel or a copy: in host code
// the name is a host-side stand-in, not a device address.  The device address
// of each GPU's copy is looked up once per device with hipGetSymbolAddress
// (gale_create calls static_scratch_setup with the device current) and kept in
// g_scratch[device]; only that pointer is used afterwards.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "gale_ctx.h"

namespace gale {

constexpr int kMaxDevices = 64;

static __device__ __align__(256) char scratch[kStaticScratchBytes];

namespace {
std::mutex g_setup_mu;
char *g_scratch[kMaxDevices] = {nullptr};
// calls on one GPU share its array: one at a time per device in this process
std::mutex g_dev_mu[kMaxDevices];

constexpr int64_t kQueueBytes = 64;  // one queue word per launch class and the global launch

int64_t align256(int64_t b) { return (b + 255) / 256 * 256; }
}  // namespace

gale_status static_scratch_setup(int device) {
    if (device < 0 || device >= kMaxDevices) return fail(GALE_EINVAL, "device ordinal beyond the static scratch table");
    std::lock_guard<std::mutex> g(g_setup_mu);
    if (g_scratch[device]) return GALE_OK;
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
        return fail(GALE_EDEVICE, std::string("static scratch address: ") + hipGetErrorString(e));
    g_scratch[device] = (char *)p;
    return GALE_OK;
}

}  // namespace gale

using namespace gale;

extern "C" gale_status gale_build_static(gale_ctx *ctx, const int32_t *ids, int32_t n, uint32_t mask,
                                         int32_t *dev_out, int64_t out_words, int64_t *block_words) {
    if (!ctx) return fail(GALE_EINVAL, "ctx is NULL");
    if (!block_words) return fail(GALE_EINVAL, "block_words is NULL");
    if (ctx->cfg.mode != GALE_MODE_DIRECT) return fail(GALE_ESTATE, "gale_build_static is for DIRECT mode");
    gale_status s = check_request(ctx, ids, n, mask);
    if (s) return s;
    if (mask & GALE_REL_EXT) return fail(GALE_EINVAL, "gale_build_static builds VT, VV and TT");
    {
        std::vector<int32_t> u(ids, ids + n);
        std::sort(u.begin(), u.end());
        if (std::adjacent_find(u.begin(), u.end()) != u.end())
            return fail(GALE_EINVAL, "repeated cluster id (block i is cluster_ids[i])");
    }
    if (ctx->poisoned) return fail(GALE_EDEVICE, "context poisoned by an earlier device error");
    const int dev = ctx->cfg.device;
    char *sp = (dev >= 0 && dev < kMaxDevices) ? g_scratch[dev] : nullptr;
    if (!sp) return fail(GALE_ESTATE, "static scratch not set up for this device");

    // one item per cluster, in the caller's order, with gale_build's
    // capacities, or the exact sizes an earlier call found for the cluster
    std::vector<WorkItem> items(n);
    {
        std::lock_guard<std::mutex> g(ctx->direct_mu);
        for (int32_t i = 0; i < n; ++i) {
            WorkItem it{};
            it.cluster = ids[i];
            it.mask = mask;
            it.cap_vv = -1;
            it.cap_tt = -1;
            const auto x = ctx->static_caps.find(ids[i]);
            if (x != ctx->static_caps.end()) {
                const ClusterMeta &m = ctx->meta[ids[i]];
                it.cap_vv = (mask & kRelVV) ? std::max(m.cap_vv, x->second.first) : 0;
                it.cap_tt = (mask & kRelTT) ? std::max(default_cap_tt(m), x->second.second) : 0;
            }
            items[i] = it;
        }
    }
    const int64_t total = lay_out_items(ctx, items, 0);
    for (int32_t i = 0; i < n; ++i) block_words[i] = items[i].out_word;
    block_words[n] = total;
    if (!dev_out || out_words < total) return fail(GALE_ENOMEM, "output buffer smaller than block_words[n] words");
    if (n == 0) return GALE_OK;

    std::lock_guard<std::mutex> g(ctx->direct_mu);
    std::lock_guard<std::mutex> gd(g_dev_mu[dev]);
    std::vector<WorkItem> order;
    std::vector<int> ncls;
    int n_glob = 0;
    int64_t wsb = 0;
    order_items(ctx, items, order, ncls, n_glob, wsb);

    // scratch: queue words | work list | headers | workspace slices
    const int64_t items_off = kQueueBytes;
    const int64_t hdr_off = align256(items_off + (int64_t)n * (int64_t)sizeof(WorkItem));
    const int64_t ws_off = align256(hdr_off + (int64_t)n * 32);
    const int64_t ws_stride = align256(std::max<int64_t>(wsb, 16));
    int64_t slots = 0;
    if (ws_off <= kStaticScratchBytes) slots = (kStaticScratchBytes - ws_off) / ws_stride;
    if (ws_off > kStaticScratchBytes || (n_glob > 0 && slots < 1))
        return fail(GALE_EINVAL, "request needs " + std::to_string(ws_off + (n_glob > 0 ? ws_stride : 0)) +
                                     " bytes of static scratch, more than its " +
                                     std::to_string((long long)kStaticScratchBytes));
    if (n_glob > 0) ncls.back() = (int)std::min<int64_t>(ncls.back(), slots);

    // the work list with zeroed queue words, copied into the scratch
    std::vector<char> &hs = ctx->static_host;
    hs.assign((size_t)items_off + (size_t)n * sizeof(WorkItem), 0);
    std::memcpy(hs.data() + items_off, order.data(), (size_t)n * sizeof(WorkItem));
    hipStream_t st = ctx->stream;
    hipError_t e = hipMemcpyAsync(sp, hs.data(), hs.size(), hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return fail(GALE_EDEVICE, std::string("work list copy: ") + hipGetErrorString(e));
    ctx->n_global_blocks += n_glob;
    s = launch_batch(ctx, GALE_FORM_BATCHED, dev_out, (int32_t *)(sp + hdr_off), (const WorkItem *)(sp + items_off),
                     ncls, n_glob, (int32_t *)sp, n_glob > 0 ? sp + ws_off : nullptr, ws_stride, st, true, nullptr,
                     nullptr);
    if (s) {
        ctx->poisoned = true;
        return s;
    }
    // headers: in the order the items were launched (hdr_index = position in `items`)
    std::vector<int32_t> &hh = ctx->static_hdr;
    hh.assign((size_t)n * 8, 0);
    e = hipMemcpyAsync(hh.data(), sp + hdr_off, (size_t)n * 32, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) {
        ctx->poisoned = true;
        return fail(GALE_EDEVICE, std::string("static build: ") + hipGetErrorString(e));
    }
    bool grow = false;
    uint64_t ent = 0;
    for (int32_t i = 0; i < n; ++i) {
        const int32_t *h = &hh[(size_t)i * 8];
        if (h[0] & kStInconsistent)
            return fail(GALE_EDEVICE, "stream metadata of cluster " + std::to_string(ids[i]) +
                                          " disagrees with the kernel's counts");
        if (h[0] & kStTTFallback) ctx->n_tt_exhaustive++;
        if (h[0] & (kStVVOverflow | kStTTOverflow)) {
            // the kernel counted the exact sizes; kept for this cluster's later calls
            grow = true;
            auto &c = ctx->static_caps[ids[i]];
            if (mask & kRelVV) c.first = std::max(c.first, h[4]);
            if (mask & kRelTT) c.second = std::max(c.second, h[5]);
            WorkItem &it = items[i];
            const ClusterMeta &m = ctx->meta[it.cluster];
            it.cap_vv = (mask & kRelVV) ? std::max(m.cap_vv, c.first) : 0;
            it.cap_tt = (mask & kRelTT) ? std::max(default_cap_tt(m), c.second) : 0;
        }
        if (mask & kRelVT) ent += (uint64_t)h[3];
        if (mask & kRelVV) ent += (uint64_t)h[4];
        if (mask & kRelTT) ent += (uint64_t)h[5];
    }
    if (grow) {
        // exact capacities for the blocks that overflowed: the caller builds
        // again into a buffer of the new size (the next call lays them out so)
        const int64_t t2 = lay_out_items(ctx, items, 0);
        for (int32_t i = 0; i < n; ++i) block_words[i] = items[i].out_word;
        block_words[n] = t2;
        ctx->n_overflow++;
        return fail(GALE_ENOMEM, "a block exceeded its capacity bound; block_words holds the exact layout");
    }
    ctx->n_requests++;
    ctx->n_blocks += n;
    ctx->n_entries += ent;
    return GALE_OK;
}
