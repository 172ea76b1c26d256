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
/* The further coboundary relations (Section 2.2, Table 1), DIRECT mode, with
 * gale_config.simplex_lists set:
 *   VE  rows = the cluster's vertices; entries = ids of the edges containing
 *       the vertex.
 *   VF  rows = the cluster's vertices; entries = ids of the triangles
 *       containing it.
 *   EF  rows = the edges internal to the cluster (the smallest cluster among
 *       an edge's vertices owns it, as for tetrahedra), listed by their ids;
 *       entries = ids of the triangles containing the edge.
 *   ET  rows as EF; entries = the tetrahedra containing the edge.
 *   FT  rows = the triangles internal to the cluster; entries = the
 *       tetrahedra containing the triangle.
 * Edge and triangle ids are positions in the lists E and F of
 * gale_get_simplices; entries ascending without repeats, as for VT/VV/TT. */
#define GALE_REL_VE  8u
#define GALE_REL_VF 16u
#define GALE_REL_EF 32u
#define GALE_REL_ET 64u
#define GALE_REL_FT 128u
#define GALE_REL_EXT 248u

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
    uint64_t cache_budget_bytes;  /* SERVE: bytes of device memory for resident blocks; 0 = 1 GiB (or arena_bytes
                                     when dev_arena is given) */
    int32_t  max_queue;           /* SERVE: pending requests accepted before EAGAIN; 0 = 65536 */
    int32_t  launch_classes;      /* BATCHED form: which workgroup shapes clusters may use, bit 0 = 1024 threads with
                                     the whole LDS, bit 1 = 512 threads with half, bit 2 = 256 threads with a
                                     quarter (several workgroups per CU); each cluster takes the smallest shape its
                                     working set fits.  0 = the 1024-thread shape only.  Bit 3 (all forms): the
                                     global-memory path keeps every working array in global memory instead of
                                     placing its most used ones in LDS when they fit (used by tests).  Bit 4
                                     (all forms): every cluster takes the global path, with that placement
                                     when it fits (used by tests). */
    void    *hip_stream;          /* borrowed hipStream_t for DIRECT mode work, or NULL for a library-owned stream.
                                     Must outlive the context. */
    double   global_cu_share;     /* DIRECT mode, BATCHED form: share of the CUs (0 < s <= 1) the global-path
                                     launch takes when LDS-path launch classes run beside it (it is then launched
                                     first); 0 = 1.  gale_autotune may change it.  SERVE mode runs a batch's
                                     launches one after another and always gives the global launch every CU. */
    void    *dev_arena;           /* SERVE: borrowed device memory (e.g. the storage of a torch tensor on
                                     `device`) that holds the HBM relation cache instead of a library allocation;
                                     NULL = the library allocates the cache.  Must outlive the context; 256-byte
                                     aligned.  DIRECT mode: must be NULL. */
    uint64_t arena_bytes;         /* bytes at dev_arena (at least 1 MiB); the cache budget is then
                                     min(arena_bytes, cache_budget_bytes) with 0 read as arena_bytes */
    const char *tune_table_path;  /* JSON tune table, or NULL.  gale_load reads it when the file exists and
                                     applies the entry recorded for a mesh of the same size and cluster count
                                     (launch classes, CU share of the global launch, VV lanes per row);
                                     gale_autotune writes its choice there.  The string is copied. */
    int32_t  prefetch_depth;      /* SERVE: also build the next prefetch_depth clusters (by id, which is the
                                     Morton order of the generator's clusterings) after each requested one, as
                                     speculative cache entries evicted before any requested block (0..64; 0 =
                                     none).  The paper's leader computes each request's following segments too,
                                     Section 4.5. */
    int32_t  front_end;           /* SERVE: GALE_FRONT_SINGLE (one queue, one service thread, a request's relations
                                     built by one kernel) or GALE_FRONT_PER_RELATION (one queue and one leader
                                     thread per relation, each building only its relation, Section 4.5) */
    int32_t  simplex_lists;       /* nonzero: gale_load also enumerates the edge and triangle lists E, F and
                                     their interval arrays (Section 4.3: built only when an algorithm needs edge
                                     or triangle relations), which the VE, VF, EF, ET and FT relations and
                                     gale_get_simplices need */
    int32_t  tile_entries;        /* DIRECT mode, BATCHED form: a cluster whose working set does not fit the LDS of
                                     a 1024-thread workgroup is built as tiles of about this many VT entries (its
                                     vertices split in breadth-first layers), each on the LDS path like a cluster
                                     of its own, then assembled into the cluster's block; 0 = 10000, < 0 = never
                                     (such clusters then run on the global-memory path) */
} gale_config;

#define GALE_FRONT_SINGLE       0
#define GALE_FRONT_PER_RELATION 1

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
    uint64_t tt_exhaustive_blocks;  /* blocks whose TT face table could not pair every face: a non-manifold face
                                       (TT rows then built by chains of the tetrahedra on each face) or a table
                                       that stays full (every row against every stream tetrahedron) */
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
    /* serving: the paper's waiting-time breakdown (Section 5.3: request push, request in queue, data
       preparation, kernel computation and transfer back, data integration), mean microseconds per request;
       the id mapping the paper does on the host after the copy is fused into the kernel's stores here,
       so "integration" is the time from the block copy's completion to the request being ready */
    double   stage_push_us, stage_prep_us, stage_kernel_copy_us, stage_integration_us;
    /* the same stages summed per submitting thread, seconds, maximum over threads (the paper's
       aggregation for many consumers, Section 5.3) */
    double   wait_push_s_max, wait_queue_s_max, wait_prep_s_max, wait_kernel_copy_s_max, wait_integration_s_max;
    /* serving: speculative builds of following clusters (gale_config.prefetch_depth) */
    uint64_t prefetch_built;        /* speculative blocks built */
    uint64_t prefetch_hits;         /* requests that found a speculative block resident or in flight */
    uint64_t prefetch_evicted;      /* speculative blocks evicted before any request used them */
    uint64_t demand_evictions;      /* evictions of blocks some request had used */
    int32_t  front_end;             /* GALE_FRONT_SINGLE or GALE_FRONT_PER_RELATION */
    int32_t  tune_applied;          /* 1 when gale_load applied an entry of the tune table */
} gale_stats;

/* Sizes of one cluster's prepared lists (the per-segment internal and
 * external tetrahedra and vertex interval of the initialization step,
 * Section 4.3, plus this library's halo), as gale_get_cluster_info reports
 * them. */
typedef struct {
    int32_t cluster;
    int32_t nV;       /* vertices of the cluster: VT and VV rows */
    int32_t nT;       /* tetrahedra internal to the cluster: TT rows */
    int32_t ns;       /* tetrahedra with a vertex in the cluster (internal and external) */
    int32_t nh;       /* halo: tetrahedra outside that set sharing a triangle with an internal one */
    int32_t L;        /* distinct vertices of those tetrahedra and of the cluster */
    int32_t nnzVT;    /* entries of the cluster's VT block */
    int32_t cap_vv;   /* bound on the entries of its VV block (exact count known after a build) */
} gale_cluster_info;

/* Create a context on cfg->device (cfg may be NULL for defaults).  The
 * context stands for the paper's producer side: it owns the leader role
 * (batching requests and launching kernels) and the memory it preallocates
 * (Section 4.2, overview of the consumer / leader / worker model; Section 4.5,
 * preallocated GPU memory).  Ownership: *out belongs to the caller until
 * gale_destroy.  Errors: EINVAL (bad field, e.g. block_threads not 256/512/1024,
 * global_cu_share outside [0, 1], dev_arena in DIRECT mode, arena_bytes below
 * 1 MiB, prefetch_depth outside 0..64, unknown front_end), EDEVICE (no HIP
 * device or a runtime failure); *out is NULL on error. */
gale_status gale_create(const gale_config *cfg, gale_ctx **out);

/* Load a mesh: the paper's input (V, T, S; here T and S, since no kernel reads
 * coordinates) and its initialization step, which prepares per-segment
 * internal and external tetrahedron lists and interval arrays on the CPU and
 * copies them to GPU memory (Section 4.3, "Input data" and "Initialization").
 * tv: nt*4 vertex ids, row-major; cluster_of_vertex: nv cluster ids in
 * [0, nclusters); nv and nt at most 2^30.  Both arrays are host memory, read
 * during the call and copied; the caller keeps ownership.  Errors: EINVAL
 * (id out of range, repeated vertex in a tetrahedron, nclusters <= 0),
 * ENOMEM (device memory), ESTATE (a mesh is already loaded: once per
 * context), EDEVICE.  When cfg.tune_table_path names an existing table with
 * an entry for this mesh's (nv, nt, nclusters), that entry is applied. */
gale_status gale_load(gale_ctx *ctx, int32_t nv, int64_t nt, const int32_t *tv,
                      const int32_t *cluster_of_vertex, int32_t nclusters);

/* Request the relations in rel_mask for n cluster ids: the consumer's request
 * for a coboundary or adjacency relation of a whole segment (Section 4.4).
 * cluster_ids is host memory, read during the call; duplicates are allowed
 * and built once.  DIRECT mode: builds on the GPU in cfg.form and copies the
 * blocks to pinned host memory before returning (the ticket is ready).  SERVE
 * mode: queues the request for the serving loop and returns at once.
 * *ticket_out identifies the request until gale_release.  Errors: EINVAL (id
 * out of range, mask empty or with unknown bits, NULL pointer), ESTATE (no
 * mesh loaded, context being destroyed), EAGAIN (SERVE: queue full),
 * ENOMEM, EDEVICE (also: context poisoned earlier).  Thread-safe. */
gale_status gale_submit(gale_ctx *ctx, const int32_t *cluster_ids, int32_t n, uint32_t rel_mask,
                        uint64_t *ticket_out);

/* Build into device memory only (no copy to the host), asynchronously on the
 * context stream, in the given form: the kernel launch a leader issues for its
 * batch, without the transfer back (Section 4.5; Section 4.6 for the kernels).
 * Returns a ticket whose blocks are read with gale_block_device after
 * gale_poll reports it ready.  DIRECT mode only (ESTATE otherwise); other
 * errors as gale_submit. */
gale_status gale_build(gale_ctx *ctx, const int32_t *cluster_ids, int32_t n, uint32_t rel_mask,
                       int32_t form, uint64_t *ticket_out);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): gale_build's
 * BATCHED build of rel_mask for the n distinct clusters cluster_ids[0..n),
 * into the caller's device buffer dev_out (out_words int32 words, 256-byte
 * aligned), allocating no device memory.  Every other device buffer of the
 * build (work list and queue words, block headers, the global path's
 * workspace) lives in a static array of GALE_STATIC_SCRATCH_BYTES per GPU,
 * set up by gale_create; a request that needs more (about 64 bytes per
 * cluster plus one workspace slice of its largest global-path cluster) is
 * EINVAL.  Calls on one GPU share that array: the library runs them one at a
 * time in a process, and it keeps the last call's contents.
 *   block_words (host, n + 1 int64, caller memory) receives the word offset
 *   of cluster_ids[i]'s block in dev_out and, at [n], the words needed; it is
 *   filled before anything is built.  With dev_out NULL or out_words below
 *   block_words[n] the call returns ENOMEM and builds nothing (a size query).
 * A block is laid out as an 8-word header {status, nV, nT, nnzVT, nnzVV,
 * nnzTT, cap_vv, cap_tt}, then, each starting on a 32-word boundary, for the
 * relations in rel_mask: VT|VV row ids [nV]; VT offsets [nV + 1] and entries
 * [nnzVT]; TT row ids [nT], offsets [nT + 1] and entries [cap_tt]; VV offsets
 * [nV + 1] and entries [cap_vv]; the contents equal gale_build's blocks.
 * The build runs on the context stream and the call returns when it is done
 * (synchronous).  When a block exceeds its capacity bound (non-manifold
 * faces), the call returns ENOMEM with block_words holding the layout with
 * that block's exact size, which the context remembers: call again with a
 * buffer that large.  DIRECT mode, VT|VV|TT.  Errors: EINVAL (as gale_build, a repeated
 * cluster id, NULL block_words, scratch too small), ENOMEM (as above),
 * ESTATE (no mesh, SERVE mode), EDEVICE. */
#define GALE_STATIC_SCRATCH_BYTES (64ll << 20)
gale_status gale_build_static(gale_ctx *ctx, const int32_t *cluster_ids, int32_t n, uint32_t rel_mask,
                              int32_t *dev_out, int64_t out_words, int64_t *block_words);

/* Choose how batched work runs by measurement: the analogue of the paper's
 * study of threads per segment, threads per block and blocks per request
 * (Appendix A; the kernel's block and thread parameters, Section 4.5).
 * Each candidate value of gale_config.launch_classes (0, 2, 4, 6) builds the
 * clusters ids[0..n) with rel_mask in the BATCHED form, device only, once to
 * warm up and then `reps` times; the one with the shortest mean kernel time
 * is kept for the context's later batched work.  When the request then runs
 * both LDS-path classes and the global path, the share of the CUs the global
 * launch takes (1, 0.8, 0.65, 0.5) is chosen the same way
 * (gale_stats.global_cu_share).  The choice is written to cfg.tune_table_path
 * when one was given (keyed by the mesh's nv, nt and nclusters).  DIRECT mode
 * with a mesh loaded; no other call may use the context meanwhile.
 * chosen_out (may be NULL) receives the chosen value, ms_out (may be NULL; 4
 * doubles) the mean milliseconds of each candidate in the order above.
 * Errors: EINVAL, ESTATE, EDEVICE as gale_build; ENOENT when the tune table
 * cannot be written. */
gale_status gale_autotune(gale_ctx *ctx, const int32_t *cluster_ids, int32_t n, uint32_t rel_mask, int32_t reps,
                          int32_t *chosen_out, double *ms_out);

/* hipGraph-captured submit for a request built again and again (the same
 * clusters and relations, e.g. every step of an iterative analysis); the
 * leader's batched launch of Section 4.5 replayed from a HIP graph.
 * gale_graph_create lays the request's blocks out in one device buffer, copies
 * its work list to the device and captures its launches (queue reset and the
 * persistent kernels of every workgroup shape) in a HIP graph; DIRECT mode.
 * gale_graph_launch replays the graph on the context stream and returns a
 * ticket read with gale_poll and gale_block_device and freed with
 * gale_release; all tickets of one graph share its buffer, so a ticket's
 * blocks are valid until the next gale_graph_launch of the same graph.
 * gale_graph_destroy waits for the context stream and frees the graph and its
 * buffer; it returns ESTATE, and frees nothing, while a ticket of the graph is
 * not released.  Errors: EINVAL, ESTATE, ENOENT (unknown graph), ENOMEM,
 * EDEVICE. */
gale_status gale_graph_create(gale_ctx *ctx, const int32_t *cluster_ids, int32_t n, uint32_t rel_mask,
                              uint64_t *graph_out);
gale_status gale_graph_launch(gale_ctx *ctx, uint64_t graph, uint64_t *ticket_out);
gale_status gale_graph_destroy(gale_ctx *ctx, uint64_t graph);

/* Wait up to timeout_ns (0 = just test, <0 = forever) for the ticket: the
 * consumer waiting on its semaphore until the leader has the relation ready
 * (Section 4.2).  OK = ready; EAGAIN = not yet; ENOENT = unknown ticket; the
 * request's own error (ENOMEM, EDEVICE, ESTATE after gale_destroy began)
 * otherwise.  Thread-safe. */
gale_status gale_poll(gale_ctx *ctx, uint64_t ticket, int64_t timeout_ns);

/* Host view of one block of a ready ticket made with gale_submit: the
 * relation in the form the consumer reads, already in original ids (the
 * paper's local-to-global mapping after the transfer, Section 4.5).  *out
 * points into library-owned pinned host memory valid until
 * gale_release(ticket).  Errors: EINVAL (rel not one bit, NULL), EAGAIN (not
 * ready), ENOENT (cluster or relation not in the ticket), ESTATE (ticket made
 * with gale_build), the request's own error. */
gale_status gale_block(gale_ctx *ctx, uint64_t ticket, int32_t cluster_id, uint32_t rel, gale_csr *out);

/* Device view of one block of a ready ticket made with gale_build or
 * gale_graph_launch (the relation array in GPU memory, Section 4.5).  The
 * pointers are device memory owned by the library, valid until
 * gale_release(ticket).  DIRECT mode.  Errors as gale_block. */
gale_status gale_block_device(gale_ctx *ctx, uint64_t ticket, int32_t cluster_id, uint32_t rel, gale_csr *out);

/* Release a ticket: its views become invalid and its memory is reused, as the
 * paper reuses its preallocated per-consumer memory (Section 4.5).  Waits for
 * the ticket's work if it is still running.  Errors: ENOENT (unknown or
 * already released). */
gale_status gale_release(gale_ctx *ctx, uint64_t ticket);

/* Counters and latency figures of the context, including the paper's
 * waiting-time breakdown per request (Section 5.3) and the queue depth seen
 * when requests are admitted (Section 4.5 reports its mean and spread).
 * Named gale_get_stats because the struct typedef takes the name gale_stats
 * in C.  *out is caller memory, filled completely.  Errors: EINVAL. */
gale_status gale_get_stats(gale_ctx *ctx, gale_stats *out);

/* Set the latency, stage and cache statistics back to zero (between benchmark
 * phases; Section 5.3 measures each run separately).  Errors: EINVAL. */
gale_status gale_reset_stats(gale_ctx *ctx);

/* The hipStream_t the context launches DIRECT-mode work on (the borrowed one,
 * or the library's); NULL for a NULL context.  Borrowed by the caller. */
void *gale_stream(gale_ctx *ctx);

/* Sizes of cluster `cluster` of the loaded mesh (see gale_cluster_info):
 * what the initialization step prepared for that segment (Section 4.3).
 * *out is caller memory.  Errors: EINVAL (NULL, cluster out of range),
 * ESTATE (no mesh loaded).  Thread-safe. */
gale_status gale_get_cluster_info(gale_ctx *ctx, int32_t cluster, gale_cluster_info *out);

/* The edge and triangle lists of the loaded mesh (gale_config.simplex_lists),
 * as the initialization step enumerates them (Section 4.3): edge i is
 * (e[2i], e[2i+1]) and triangle i is (f[3i], f[3i+1], f[3i+2]), each with
 * ascending original vertex ids; the edges internal to cluster k are ids
 * ie[k] .. ie[k+1]-1 and its triangles if_[k] .. if_[k+1]-1 (the interval
 * arrays I_E, I_F).  Numbering: for each cluster in turn, its tetrahedra
 * (those with a vertex in it) in ascending id, each tetrahedron's vertex
 * pairs (triples) in lexicographic order of its ascending vertices; an edge
 * (triangle) internal to the cluster takes the next id when first met.  This
 * is the reading of Section 4.3 under which the example of Section 4.4 holds
 * (I_E = 0, 9, 12; f5 = v0 v3 v4; FE(f5) = e2, e6, e9).  The pointers are
 * library-owned host memory valid until gale_destroy.  Errors: EINVAL (NULL),
 * ESTATE (no mesh, or loaded without simplex_lists). */
typedef struct {
    int64_t ne, nf;
    int32_t ncl, pad;
    const int32_t *e, *f;
    const int64_t *ie, *if_;
} gale_simplices;
gale_status gale_get_simplices(gale_ctx *ctx, gale_simplices *out);

/* Text of a status code (static storage). */
const char *gale_strerror(gale_status s);
/* Detail of the last error raised on the calling thread ("" if none); valid
 * until the thread's next failing call. */
const char *gale_last_error(void);

/* Drain in-flight work, fail pending and waiting requests with ESTATE, wait
 * until no other thread is inside gale_poll / gale_release on this context,
 * and free everything the context owns (the end of the paper's producer
 * threads, Section 4.2).  Borrowed streams and arenas are not freed. */
void gale_destroy(gale_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif /* GALE_H */
