// gale_ctx.h -- the context object and the runtime's internal types.
#pragma once
#include <hip/hip_runtime.h>

#include <array>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <list>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "gale_host.h"

namespace gale {

struct Buf {
    void *ptr = nullptr;
    size_t bytes = 0;
    bool pinned = false;
};

// Grow-only pool of device or pinned host buffers, reused by size so that
// repeated requests of the same shape allocate nothing.
struct Pool {
    bool pinned = false;
    std::mutex mu;
    std::vector<Buf *> all, free_list;
    Buf *acquire(size_t bytes, hipError_t *err);
    void release(Buf *b);
    void clear();
};

struct BlockLoc {
    Buf *buf;
    int64_t word;
};

// One set of work items built together, with its buffers.
struct Batch {
    std::vector<WorkItem> items;
    int64_t out_words = 0;
    Buf *out = nullptr, *dev_items = nullptr, *dev_hdr = nullptr, *ws = nullptr;
    Buf *host_items = nullptr, *host_hdr = nullptr, *host_out = nullptr;
    std::vector<Buf *> extra;           // rebuild outputs owned by this batch
    std::vector<int32_t> hdr;           // 8 words per item, after finalize
    std::vector<BlockLoc> loc;          // where each item's block lives, after finalize
    std::vector<int64_t> host_word;     // host copy offsets
    bool host_ready = false;
    hipEvent_t kev[2] = {nullptr, nullptr};  // around the persistent launches (DIRECT, BATCHED)
    bool kev_recorded = false;
    bool borrowed = false;  // buffers owned by a prepared (graph) request, not by this batch
    // edge / triangle relation items (their own work list and workspace)
    Buf *ext_items = nullptr, *ext_host = nullptr, *ext_ws = nullptr;
    // stitch of tiled clusters (work list: queue word, stitch items, tile items)
    Buf *st_items = nullptr, *st_host = nullptr;
};

struct Ticket {
    Batch batch;
    uint64_t graph = 0;  // the prepared request whose buffers the batch borrows (0: none)
    uint32_t mask = 0;
    bool host = false;
    bool ready = false;
    gale_status status = GALE_OK;
    hipEvent_t done = nullptr;
    std::unordered_map<int32_t, std::vector<int>> by_cluster;
};

// A batched request prepared for repeated builds: its blocks' buffer and work
// list stay in device memory and its launches are captured in a HIP graph.
struct Prepared {
    Batch batch;
    uint32_t mask = 0;
    std::unordered_map<int32_t, std::vector<int>> by_cluster;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int live = 0;  // tickets of this graph not yet released (they borrow its buffers)
};

// ---- serving -------------------------------------------------------------
using Clock = std::chrono::steady_clock;

struct ServeReq;

// Request latencies in microseconds, in log-spaced buckets (0.5 % wide) from
// 0.1 us to 1e9 us: bounded memory however many requests are served;
// percentiles are read to within the bucket width, count / mean / max exactly.
struct LatHist {
    static constexpr int kBuckets = 5600;
    std::vector<uint64_t> n = std::vector<uint64_t>(kBuckets, 0);
    uint64_t count = 0;
    double sum = 0.0, mx = 0.0;
    static int bucket(double us);
    static double lower(int b);
    void add(double us);
    double percentile(double p) const;
    void clear();
};

struct CacheEntry {
    int32_t cluster = 0;
    uint32_t mask = 0;
    int64_t off = 0;        // bytes into the arena
    int64_t bytes = 0;      // bytes allocated
    int state = 0;          // 0 = building, 1 = resident
    int pins = 0;           // requests holding it (waiting or copying)
    int32_t cap_vv = 0, cap_tt = 0;
    int32_t hdr[8] = {0};
    int lru_kind = 0;       // 0 = in no list, 1 = demand LRU, 2 = speculative LRU
    bool spec = false;      // built ahead of any request (prefetch) and not used by one yet
    std::list<int64_t>::iterator lru_it;
    std::vector<ServeReq *> waiters;
};

struct ServeReq {
    uint64_t id = 0;
    std::vector<int32_t> clusters;
    uint32_t mask = 0;
    int lane = 0;                       // the leader (lane) that admits it
    ServeReq *parent = nullptr;         // per-relation front end: the request this part belongs to
    std::vector<ServeReq *> parts;      // per-relation front end: one part per relation of the mask
    int parts_left = 0;
    size_t thread_key = 0;              // the submitting thread
    Clock::time_point t_submit, t_pushed, t_admit, t_launched, t_built, t_copied, t_ready;
    int waiting = 0;
    bool admitted = false, copying = false, ready = false;
    gale_status status = GALE_OK;
    std::vector<int64_t> keys;          // cache keys held (pinned)
    Buf *host = nullptr;
    std::vector<int64_t> host_word;     // per cluster (same order as clusters)
    std::vector<CacheEntry> snap;       // header / capacities of each block at copy time
    hipEvent_t copy_done = nullptr;
};

struct Slot {
    bool busy = false;                  // a batch is on the GPU
    bool launching = false;             // the lane is launching a batch (lock released meanwhile)
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;          // after the kernels and the header copy
    Batch batch;
    std::vector<int64_t> keys;          // cache keys built by this batch, per item
};

// One leader: a pending queue, a service thread and its in-flight slots.  The
// single front end has one lane taking every relation mask; the per-relation
// front end one lane per relation (the paper's queue and leader per relation).
struct Lane {
    int index = 0;
    uint32_t accept = 7;
    std::thread th;
    std::condition_variable cv_work;
    std::deque<ServeReq *> pending;
    std::vector<Slot> slots;
    std::vector<int64_t> rebuild;       // blocks to rebuild with exact capacities
    std::vector<ServeReq *> copying;
    hipStream_t copy_stream = nullptr;
};

struct Serve {
    std::mutex mu;
    std::condition_variable cv_done, cv_idle;
    bool stop = false;
    int callers = 0;                    // threads inside serve_poll / serve_block / serve_release
    std::vector<std::unique_ptr<Lane>> lanes;
    std::unordered_map<uint64_t, ServeReq *> reqs;
    std::unordered_map<int64_t, CacheEntry> cache;
    std::list<int64_t> lru;             // unpinned resident keys some request used, least recent first
    std::list<int64_t> spec_lru;        // unpinned resident speculative keys, evicted first
    std::map<int64_t, int64_t> free_map;  // arena free ranges offset -> bytes
    void *arena = nullptr;
    bool own_arena = true;
    int64_t arena_bytes = 0, resident_bytes = 0;
    // statistics
    uint64_t hits = 0, misses = 0, evictions = 0, batches = 0, batch_clusters = 0;
    uint64_t admissions = 0, depth_sum = 0;
    int32_t depth_max = 0;
    uint64_t prefetch_built = 0, prefetch_hits = 0, prefetch_evicted = 0, demand_evictions = 0;
    LatHist lat;
    uint64_t n_stage = 0;
    // sums (microseconds) of: queue, build, copy, push, in queue, preparation, kernel + copy, integration
    double stage_sum[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    // per submitting thread: push, queue, prep, kernel+copy, integration (seconds)
    std::unordered_map<size_t, std::array<double, 5>> per_thread;
};

}  // namespace gale

struct gale_ctx {
    gale_config cfg{};
    hipStream_t stream = nullptr;
    bool own_stream = false;
    std::atomic<bool> poisoned{false};
    int num_cus = 0, grid_lds = 1, grid_glob = 1, block_threads = 256;
    int glob_bt = 1024;  // threads per workgroup of the global-path launches
    int64_t lds_budget = 0;
    // dynamic LDS of a global-path workgroup (the hybrid form's arrays), 0
    // when the global path keeps every array in global memory
    int64_t glob_lds = 0;
    // share of the CUs the global launch takes when LDS-path classes run
    // beside it (gale_autotune)
    double glob_share = 1.0;
    // workgroup shapes for LDS-path clusters, largest LDS first; a cluster
    // takes the last (smallest) one its working set fits
    struct LaunchClass {
        int bt;          // threads per workgroup
        int64_t budget;  // dynamic LDS bytes
        int grid;        // persistent workgroups (CUs x occupancy)
    };
    std::vector<LaunchClass> classes;
    int class_mask = 0;
    int64_t static_lds = 0, shared_per_block = 0;
    std::vector<hipStream_t> aux;  // DIRECT mode: streams the classes' launches run on, joined back
    hipEvent_t fork_ev = nullptr;
    std::vector<hipEvent_t> join_ev;
    // mesh
    bool loaded = false;
    int32_t nv = 0, ncl = 0;
    int64_t nt = 0, stream_tets = 0;
    uint64_t mesh_bytes = 0;
    double load_seconds = 0;
    std::vector<gale::ClusterMeta> meta;
    uint8_t *d_tets = nullptr;
    int32_t *d_tid = nullptr, *d_lverts = nullptr;
    gale::ClusterMeta *d_meta = nullptr;
    // tiles of large clusters (batched form): metadata entries ncl ..
    // ncl + ntiles - 1 of meta / d_meta are tiles; per cluster its first tile
    // and count (0: not tiled), the stitch metadata and maps on the device
    int32_t ntiles = 0;
    std::vector<int32_t> tile_first, tile_count;
    gale::StitchMeta *d_sm = nullptr;
    int32_t *d_maps = nullptr;
    // edge and triangle lists (gale_config.simplex_lists): host copies of E,
    // F and the interval arrays, the per-cluster ranges, and the device index
    bool has_simplices = false;
    gale::HostSimplices sx;
    gale::ExtMeta *d_ext = nullptr;
    int32_t *d_eoff = nullptr, *d_eidx = nullptr, *d_foff = nullptr, *d_fidx = nullptr;
    // pools and tickets
    gale::Pool dev_pool, pin_pool;
    std::mutex direct_mu, tick_mu;
    std::unordered_map<uint64_t, gale::Ticket *> tickets;
    uint64_t next_ticket = 0;
    std::unordered_map<uint64_t, gale::Prepared *> graphs;  // under direct_mu
    uint64_t next_graph = 0;
    // counters
    std::atomic<uint64_t> n_requests{0}, n_blocks{0}, n_entries{0}, n_launches{0}, n_overflow{0},
        n_global_blocks{0}, n_hybrid_blocks{0}, n_delivered{0}, n_bytes_d2h{0}, n_tt_exhaustive{0};
    std::string tune_path;    // gale_config.tune_table_path, copied
    bool tune_applied = false;
    uint64_t n_timed = 0;     // timed persistent launches (under direct_mu)
    double kernel_ms = 0.0;   // their total duration
    // gale_build_static: host staging of the work list and headers (reused),
    // and exact (VV, TT) sizes of clusters whose blocks exceeded a bound
    std::vector<char> static_host;
    std::vector<int32_t> static_hdr;
    std::unordered_map<int32_t, std::pair<int32_t, int32_t>> static_caps;
    gale::Serve serve;
};

namespace gale {
// one entry of the tune table (gale_config.tune_table_path)
struct TuneEntry {
    int64_t nv = 0, nt = 0, ncl = 0;
    int rel_mask = 7, launch_classes = 0, global_threads = 1024;
    double global_cu_share = 1.0, kernel_ms = 0.0;
    double class_ms[4] = {0, 0, 0, 0};
};
bool read_tune_entry(const std::string &path, int64_t nv, int64_t nt, int64_t ncl, TuneEntry &out);
bool write_tune_entry(const std::string &path, const TuneEntry &te);
int item_class(const gale_ctx *ctx, const WorkItem &it);

gale_status fail(gale_status s, const std::string &msg);
int32_t default_cap_tt(const ClusterMeta &m);
int64_t lay_out_items(const gale_ctx *ctx, std::vector<WorkItem> &items, int64_t out_base_word);
int64_t workspace_bytes(const gale_ctx *ctx, const std::vector<WorkItem> &items, int *n_global);
std::vector<WorkItem> make_items(const gale_ctx *ctx, const int32_t *ids, int32_t n, uint32_t mask, int form);
void order_items(gale_ctx *ctx, const std::vector<WorkItem> &items, std::vector<WorkItem> &order,
                 std::vector<int> &ncls, int &n_glob, int64_t &wsb);
gale_status launch_batch(gale_ctx *ctx, int form, int32_t *d_out, int32_t *d_hdr, const WorkItem *d_items,
                         const std::vector<int> &ncls, int n_glob, int32_t *d_queue, char *d_ws, int64_t ws_stride,
                         hipStream_t st, bool fork, const hipEvent_t *kev, bool *kev_recorded);
void setup_classes(gale_ctx *ctx, int mask);
void setup_global(gale_ctx *ctx, int bt);
gale_status upload_and_launch(gale_ctx *ctx, int form, const std::vector<WorkItem> &items, int32_t *d_out,
                              Buf *&dev_items, Buf *&dev_hdr, Buf *&host_items, Buf *&ws, hipStream_t st,
                              const hipEvent_t *kev = nullptr, bool *kev_recorded = nullptr);
gale_status check_request(const gale_ctx *ctx, const int32_t *ids, int32_t n, uint32_t mask);

// gale_build_static's device scratch: bytes per GPU, and the once-per-device
// lookup of its address (gale_create, with the device current)
constexpr int64_t kStaticScratchBytes = 64ll << 20;
gale_status static_scratch_setup(int device);

gale_status serve_start(gale_ctx *ctx);
void serve_stop(gale_ctx *ctx);
gale_status serve_submit(gale_ctx *ctx, const int32_t *ids, int32_t n, uint32_t mask, uint64_t *ticket);
gale_status serve_poll(gale_ctx *ctx, uint64_t ticket, int64_t timeout_ns);
gale_status serve_block(gale_ctx *ctx, uint64_t ticket, int32_t cluster, uint32_t rel, gale_csr *out);
gale_status serve_release(gale_ctx *ctx, uint64_t ticket);
void serve_stats(gale_ctx *ctx, gale_stats *out);
void serve_reset_stats(gale_ctx *ctx);
}  // namespace gale
