/*
 * gale.h -- C ABI of the MI355X localized-relation builder.
 *
 * A tetrahedral mesh is given in the paper's top-simplex encoding: an indexed
 * list T of tetrahedra (four vertex ids each, the TV relation) and a map S that
 * assigns every vertex to exactly one segment, here called a cluster (paper,
 * Section 4.3, "Input data").  For any requested cluster the library builds, on
 * the GPU, three relations restricted to that cluster as CSR blocks:
 *
 *   VT  rows = the cluster's vertices; entries = the tetrahedra incident to the
 *       vertex (a coboundary relation, Section 2.2, Table 1).
 *   VV  rows = the cluster's vertices; entries = the vertices sharing an edge
 *       with it, the vertex itself excluded (adjacency relation, Section 2.2;
 *       Fig. 1 gives VV(v0) = [v1, v2, v3]).
 *   TT  rows = the tetrahedra internal to the cluster; entries = the
 *       tetrahedra sharing a triangle with it (adjacency relation, Section 2.2).
 *       A tetrahedron is internal to the cluster of its lowest vertex
 *       (Section 4.3), read as: the smallest cluster id among its four
 *       vertices.  Every tetrahedron is a TT row of exactly one cluster, and
 *       its entries are the global face neighbours, also those outside the
 *       cluster's own tetrahedra.
 *
 * Every block is canonical: rows in ascending original id (listed explicitly in
 * row_ids), offsets starting at 0, each row's entries in ascending original id
 * without repeats.  The result is the same byte string whichever way it was
 * built (one launch per cluster, a batched launch, or the serving loop) and
 * whichever other clusters or relations were requested with it.
 *
 * Ids are int32, 0-based (the paper's segments are 1-based, Section 4.3).
 * Every call returns a gale_status; 0 is success.  No C++ exception crosses
 * this boundary.
 */
#ifndef GALE_H
#define GALE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t gale_status;
#define GALE_OK        0
#define GALE_EINVAL  (-1)  /* bad argument: id out of range, repeated vertex in a tetrahedron, nclusters <= 0, unknown relation bit */
#define GALE_ENOMEM  (-2)  /* host or device allocation failed, or a block does not fit the cache budget */
#define GALE_EAGAIN  (-3)  /* not ready yet (gale_poll), or the serving queue is full (gale_submit) */
#define GALE_ENOENT  (-4)  /* unknown or already released ticket; cluster/relation not part of the ticket */
#define GALE_ESTATE  (-5)  /* call made in the wrong order (e.g. submit before load) or in the wrong mode */
#define GALE_EDEVICE (-6)  /* HIP runtime error or GPU-side consistency failure; the context is poisoned and only gale_destroy is valid */

/* Relation bits of a request mask */
#define GALE_REL_VT 1u
#define GALE_REL_VV 2u
#define GALE_REL_TT 4u
#define GALE_REL_ALL 7u

/* How gale_submit / gale_build execute a request. */
#define GALE_FORM_PLAIN   0  /* one kernel launch per (cluster, relation) */
#define GALE_FORM_BATCHED 1  /* one persistent launch over all requested clusters, taken from a device work queue */

/* Context modes */
#define GALE_MODE_DIRECT 0   /* gale_submit runs the request on the caller's thread (PLAIN or BATCHED form) */
#define GALE_MODE_SERVE  1   /* gale_submit queues the request for the serving loop (continuous batching + HBM cache) */

typedef struct gale_ctx gale_ctx;

typedef struct {
    int32_t  device;              /* HIP device ordinal */
    int32_t  mode;                /* GALE_MODE_DIRECT or GALE_MODE_SERVE */
    int32_t  form;                /* DIRECT mode: GALE_FORM_PLAIN or GALE_FORM_BATCHED */
    int32_t  block_threads;       /* threads per workgroup, 256, 512 or 1024; 0 = tuned default */
    int32_t  lds_bytes;           /* LDS budget per workgroup in bytes; 0 = tuned default; small values force the
                                     global-memory path (used by tests) */
    int32_t  max_inflight;        /* SERVE: batches on the GPU at once (1..8); 0 = 2 */
    uint64_t cache_budget_bytes;  /* SERVE: bytes of device memory for resident blocks; 0 = 1 GiB */
    int32_t  max_queue;           /* SERVE: pending requests accepted before EAGAIN; 0 = 65536 */
    int32_t  launch_classes;      /* BATCHED form: which workgroup shapes clusters may use, bit 0 = 1024 threads with
                                     the whole LDS, bit 1 = 512 threads with half, bit 2 = 256 threads with a
                                     quarter (several workgroups per CU); each cluster takes the smallest shape its
                                     working set fits.  0 = the 1024-thread shape only.  Bit 3 (all forms): the
                                     global-memory path keeps every working array in global memory instead of
                                     placing its most used ones in LDS when they fit (used by tests). */
    void    *hip_stream;          /* borrowed hipStream_t for DIRECT mode work, or NULL for a library-owned stream.
                                     Must outlive the context. */
    double   global_cu_share;     /* DIRECT mode, BATCHED form: share of the CUs (0 < s <= 1) the global-path
                                     launch takes when LDS-path launch classes run beside it (it is then launched
                                     first); 0 = 1.  gale_autotune may change it.  SERVE mode runs a batch's
                                     launches one after another and always gives the global launch every CU. */
} gale_config;

/* A read-only view of one CSR block.  For gale_block the pointers are host
 * memory owned by the library; for gale_block_device they are device memory.
 * Either way they stay valid until gale_release(ticket). */
typedef struct {
    int32_t        cluster;
    uint32_t       rel;      /* one of GALE_REL_VT / VV / TT */
    int32_t        nrows;
    int32_t        pad;
    int64_t        nnz;
    const int32_t *row_ids;  /* nrows original ids, ascending */
    const int32_t *offsets;  /* nrows + 1, offsets[0] = 0, offsets[nrows] = nnz */
    const int32_t *entries;  /* nnz original ids */
} gale_csr;

typedef struct {
    /* mesh */
    int32_t  nv, nclusters;
    int64_t  nt;
    int64_t  stream_tets;           /* tetrahedra in all clusters' star + halo streams */
    uint64_t device_mesh_bytes;     /* device memory held by the loaded mesh streams */
    double   load_seconds;          /* wall time of gale_load (host preparation + copy to the GPU) */
    /* work */
    uint64_t requests;              /* gale_submit / gale_build calls accepted */
    uint64_t blocks_built;          /* (cluster, relation-mask) blocks built on the GPU */
    uint64_t entries_built;         /* sum of nnz over built blocks, all relations */
    uint64_t kernel_launches;
    uint64_t overflow_reruns;       /* blocks rebuilt because a capacity bound was exceeded */
    uint64_t global_path_blocks;    /* blocks whose working set did not fit LDS */
    uint64_t tt_exhaustive_blocks;  /* blocks whose TT face table could not pair every face (non-manifold face or
                                       full table) and whose TT rows were built by exhaustive pairing */
    /* serving */
    uint64_t cache_hits, cache_misses, evictions;
    uint64_t cache_bytes_resident, cache_budget;
    uint64_t entries_delivered;     /* sum of nnz copied to host views */
    uint64_t bytes_d2h;
    uint64_t batches;               /* serving batches launched */
    double   mean_batch_clusters;   /* clusters per serving batch */
    double   queue_depth_mean;      /* pending requests seen at each admission */
    int32_t  queue_depth_max;
    int32_t  pad;
    /* request latency (submit -> ready), microseconds, over all completed requests */
    double   lat_p50_us, lat_p99_us, lat_mean_us, lat_max_us;
    uint64_t lat_count;
    /* mean per-request stage times, microseconds: queued (submit -> admitted),
       build (admitted -> kernel done), copy (kernel done -> host copy done) */
    double   stage_queue_us, stage_build_us, stage_copy_us;
    /* DIRECT mode, BATCHED form: duration of the persistent LDS-path kernel
       launches, from HIP events recorded around each launch on the context
       stream */
    uint64_t timed_launches;
    double   kernel_ms_total;
    uint64_t hybrid_path_blocks;    /* of global_path_blocks, those run with their most used arrays in LDS */
    double   global_cu_share;       /* share of the CUs the global-path launch takes when LDS-path launch classes
                                       run beside it (1 unless gale_autotune chose less) */
} gale_stats;

/* Create a context on cfg->device.  cfg may be NULL for defaults. */
gale_status gale_create(const gale_config *cfg, gale_ctx **out);

/* Load a mesh (host arrays; copied, the caller keeps ownership).
 * tv: nt*4 vertex ids, row-major; cluster_of_vertex: nv cluster ids in
 * [0, nclusters); nv and nt at most 2^30.  Validates (EINVAL), prepares every
 * cluster's star and halo
 * stream and copies them to device memory.  May be called once per context. */
gale_status gale_load(gale_ctx *ctx, int32_t nv, int64_t nt, const int32_t *tv,
                      const int32_t *cluster_of_vertex, int32_t nclusters);

/* Request the relations in rel_mask for n cluster ids (duplicates allowed and
 * built once).  DIRECT mode: builds on the GPU and copies the blocks to host
 * memory before returning (the ticket is ready).  SERVE mode: queues the
 * request and returns at once; EAGAIN if the queue is full.  Thread-safe. */
gale_status gale_submit(gale_ctx *ctx, const int32_t *cluster_ids, int32_t n, uint32_t rel_mask,
                        uint64_t *ticket_out);

/* Build into device memory only (no copy to the host), asynchronously on the
 * context stream, in the given form.  Returns a ticket whose blocks are read
 * with gale_block_device after gale_poll reports it ready.  DIRECT mode only. */
gale_status gale_build(gale_ctx *ctx, const int32_t *cluster_ids, int32_t n, uint32_t rel_mask,
                       int32_t form, uint64_t *ticket_out);

/* Choose the workgroup shapes for batched work by measurement (batch
 * formation with cluster buckets; Section 4.5 batches every pending request,
 * these buckets decide how each cluster of a batch runs).  Each candidate
 * value of gale_config.launch_classes (0, 2, 4, 6) builds the clusters
 * ids[0..n) with rel_mask in the BATCHED form, device only, once to warm up
 * and then `reps` times; the one with the shortest mean kernel time is kept
 * for the context's later batched work.  When the request then runs both
 * LDS-path classes and the global path, the share of the CUs the global
 * launch takes (1, 0.8, 0.65, 0.5) is chosen the same way
 * (gale_stats.global_cu_share).  DIRECT mode with a mesh loaded; no
 * other call may use the context meanwhile.  chosen_out (may be NULL)
 * receives the chosen value, ms_out (may be NULL; 4 doubles) the mean
 * milliseconds of each candidate in the order above.  EINVAL, ESTATE,
 * EDEVICE as gale_build. */
gale_status gale_autotune(gale_ctx *ctx, const int32_t *cluster_ids, int32_t n, uint32_t rel_mask, int32_t reps,
                          int32_t *chosen_out, double *ms_out);

/* hipGraph-captured submit for a request built again and again (the same
 * clusters and relations, e.g. every step of an iterative analysis).
 * gale_graph_create lays the request's blocks out in one device buffer, copies
 * its work list to the device and captures its launches (queue reset and the
 * persistent kernels of every workgroup shape) in a HIP graph; DIRECT mode.
 * gale_graph_launch replays the graph on the context stream and returns a
 * ticket read with gale_poll and gale_block_device and freed with
 * gale_release; all tickets of one graph share its buffer, so a ticket's
 * blocks are valid until the next gale_graph_launch of the same graph.
 * gale_graph_destroy waits for the context stream and frees the graph and its
 * buffer (its tickets must be released first).  EINVAL, ESTATE, ENOENT
 * (unknown graph), ENOMEM, EDEVICE. */
gale_status gale_graph_create(gale_ctx *ctx, const int32_t *cluster_ids, int32_t n, uint32_t rel_mask,
                              uint64_t *graph_out);
gale_status gale_graph_launch(gale_ctx *ctx, uint64_t graph, uint64_t *ticket_out);
gale_status gale_graph_destroy(gale_ctx *ctx, uint64_t graph);

/* Wait up to timeout_ns (0 = just test, <0 = forever) for the ticket.
 * OK = ready; EAGAIN = not yet; ENOENT = unknown ticket. */
gale_status gale_poll(gale_ctx *ctx, uint64_t ticket, int64_t timeout_ns);

/* Host view of one block of a ready ticket (submitted with gale_submit). */
gale_status gale_block(gale_ctx *ctx, uint64_t ticket, int32_t cluster_id, uint32_t rel, gale_csr *out);

/* Device view of one block of a ready ticket made with gale_build. */
gale_status gale_block_device(gale_ctx *ctx, uint64_t ticket, int32_t cluster_id, uint32_t rel, gale_csr *out);

/* Release a ticket: its views become invalid and its memory is reused. */
gale_status gale_release(gale_ctx *ctx, uint64_t ticket);

gale_status gale_get_stats(gale_ctx *ctx, gale_stats *out);

/* Set the serving-loop latency statistics back to zero (between benchmark phases). */
gale_status gale_reset_stats(gale_ctx *ctx);

/* The hipStream_t the context launches DIRECT-mode work on. */
void *gale_stream(gale_ctx *ctx);

const char *gale_strerror(gale_status s);
/* Detail of the last error raised on the calling thread ("" if none). */
const char *gale_last_error(void);

/* Drain in-flight work, fail pending polls with ESTATE, free everything. */
void gale_destroy(gale_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif /* GALE_H */
