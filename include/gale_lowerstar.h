/* gale_lowerstar.h -- a CPU consumer of the relation blocks: critical-point
 * classification of a piecewise-linear scalar field by lower and upper links.
 *
 * The paper's Critical Points workload (Section 5.1) is a consumer of this
 * kind: it walks the mesh vertices and reads VV and VT to find minima, maxima
 * and saddles of a scalar field.  This function runs on the host, on blocks
 * returned by gale_block, and is used by the serving workload (many consumer
 * threads requesting clusters and classifying their vertices).
 *
 * For a vertex v, order vertices by (f, original id) (ties broken by id, so
 * the order is total).  The link of v has as vertices VV(v) and as edges the
 * pairs of other vertices of each tetrahedron of VT(v).  Its lower (upper)
 * part is induced by the link vertices below (above) v.  With c- and c+ the
 * numbers of connected components of the lower and upper parts:
 *   GALE_CP_MINIMUM  c- == 0
 *   GALE_CP_MAXIMUM  c+ == 0 (and c- > 0)
 *   GALE_CP_SADDLE   otherwise, when c- > 1 or c+ > 1
 *   GALE_CP_REGULAR  otherwise (c- == c+ == 1)
 * An isolated vertex (empty link) is a minimum.
 */
#ifndef GALE_LOWERSTAR_H
#define GALE_LOWERSTAR_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GALE_CP_REGULAR 0
#define GALE_CP_MINIMUM 1
#define GALE_CP_MAXIMUM 2
#define GALE_CP_SADDLE  3

/* Classify every row of one cluster.
 *   nrows, row_ids          rows of the cluster's VT and VV blocks (same rows)
 *   vt_off[nrows+1], vt_ent VT block: original tetrahedron ids per row
 *   vv_off[nrows+1], vv_ent VV block: original vertex ids per row, ascending
 *   tets[nt*4]              the mesh (host memory), to read each tetrahedron's vertices
 *   nt, field[nv], nv       the scalar field, one float per vertex
 *   labels[nrows]           out: GALE_CP_* per row
 * All pointers are host memory owned by the caller; nothing is kept.
 * Returns 0, or -1 (GALE_EINVAL) on a NULL pointer, an id out of range, or a
 * VT entry whose tetrahedron does not contain the row vertex.  Thread-safe. */
int32_t gale_lowerstar_classify(int32_t nrows, const int32_t *row_ids, const int32_t *vt_off,
                                const int32_t *vt_ent, const int32_t *vv_off, const int32_t *vv_ent,
                                const int32_t *tets, int64_t nt, const float *field, int32_t nv,
                                int32_t *labels);

/* The consumer workload, run by native threads against a context (either
 * mode): each thread draws k from Zipf(zipf_s) truncated to {1..64} after every
 * access; k = 1 takes the next cluster from a shared cursor over
 * cluster_order, k >= 2 re-accesses the thread's (k-1)-th most recent cluster
 * (the next new one while fewer are recent).  An access is gale_submit of one
 * cluster with rel_mask (which must include VT and VV), gale_poll,
 * gale_block of VT and VV, gale_lowerstar_classify, gale_release.  The first
 * labels of a cluster are kept (as a 64-bit hash of row ids and labels);
 * every later access must reproduce them.  Latency = submit -> poll ready,
 * per access.  This mirrors the paper's consumer threads, which request
 * relations for the segment they move to and wait for them (Sections 4.4, 5.1). */
typedef struct {
    int32_t        threads;        /* consumer threads, >= 1 */
    int32_t        n_order;        /* clusters in cluster_order */
    const int32_t *cluster_order;  /* the cursor's order (e.g. Morton order of the clusters) */
    uint32_t       rel_mask;       /* relations requested per access (VT and VV at least) */
    int32_t        pad;
    uint64_t       seed;
    double         zipf_s;         /* Zipf exponent, e.g. 1.1 */
    const int32_t *tets;           /* nt*4, host */
    int64_t        nt;
    const float   *field;          /* nv, host */
    int32_t        nv;
    int32_t        pad2;
} gale_consumer_cfg;

typedef struct {
    uint64_t accesses, reaccesses, mismatches, errors;
    uint64_t clusters;             /* distinct clusters classified */
    uint64_t minima, maxima, saddles, regular;  /* labels at each cluster's first access */
    double   wall_s;
    double   lat_p50_us, lat_p99_us, lat_mean_us, lat_max_us;
    int32_t  first_error;          /* gale status of the first failed call, 0 if none */
    int32_t  pad;
} gale_consumer_result;

/* Run the workload to the end of the cursor; blocks until every thread has
 * finished.  ctx must have a mesh loaded and be usable from many threads
 * (GALE_MODE_SERVE, or DIRECT).  Returns GALE_OK (per-access failures are
 * counted in out->errors) or GALE_EINVAL for a bad argument. */
int32_t gale_consumer_run(struct gale_ctx *ctx, const gale_consumer_cfg *cfg, gale_consumer_result *out);

#ifdef __cplusplus
}
#endif

#endif /* GALE_LOWERSTAR_H */
