/* gale_gradient.h -- a second CPU consumer of the relation blocks: the
 * discrete gradient of a scalar field (the paper's DiscreteGradient workload,
 * Section 5.1: for every vertex, the simplices of its lower star are paired,
 * the vertex with an edge, remaining edges with triangles, and so on; it reads
 * the coboundary relations VE, VF and VT, and the boundary relations EV, FV,
 * FE, TV, TF, which the consumer takes from the edge and triangle lists and
 * the mesh itself, Section 4.4).
 *
 * The pairing is the lower-star construction of Robins, Wood and Sheppard
 * (IEEE TPAMI 2011, ProcessLowerStars):
 *   - vertices are ordered by (f, original id);
 *   - the lower star of v holds the simplices containing v whose other
 *     vertices are all below v;
 *   - a simplex's key is its vertices' (f, id) sorted from the highest down,
 *     compared lexicographically, a proper prefix first;
 *   - an empty lower star leaves v critical; otherwise v is paired with its
 *     smallest edge, the other edges wait in queue zero, and simplices with
 *     exactly one unclassified facet in the lower star go to queue one; both
 *     queues pop the smallest key: from queue one a simplex with no
 *     unclassified facet moves to queue zero, otherwise it is paired with that
 *     facet; from queue zero a simplex is critical; after each step the
 *     cofaces of what was classified that now have exactly one unclassified
 *     facet join queue one.
 * Simplex ids are edge and triangle ids of gale_get_simplices and the mesh's
 * tetrahedron ids.
 */
#ifndef GALE_GRADIENT_H
#define GALE_GRADIENT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* The gradient of the lower stars of one cluster's vertices.
 *   nrows, row_ids        the cluster's vertices (rows of its VE, VF, VT blocks)
 *   ve_off, ve_ent        VE block (edge ids per row)
 *   vf_off, vf_ent        VF block (triangle ids per row)
 *   vt_off, vt_ent        VT block (tetrahedron ids per row)
 *   edges[2 ne], faces[3 nf]  the edge and triangle lists (ascending vertex ids)
 *   tets[4 nt], field[nv]     the mesh and its scalar field
 *   rec[3 cap_rec]        out: records {dim, lower id, upper id}: a pair of a
 *                         dim-simplex with a (dim+1)-simplex, or upper = -1
 *                         for a critical dim-simplex; in row order, each row's
 *                         records in the order the construction makes them
 *   n_rec                 out: records written
 * Every simplex of the rows' lower stars appears in exactly one record;
 * nrows + (entries of VE, VF, VT) records always suffice.  Host memory owned
 * by the caller; nothing is kept.  Returns 0, or -1 (GALE_EINVAL) on a NULL
 * pointer, an id out of range, a block entry that does not contain its row
 * vertex, or too small a record array.  Thread-safe. */
int32_t gale_gradient_cluster(int32_t nrows, const int32_t *row_ids, const int32_t *ve_off, const int32_t *ve_ent,
                              const int32_t *vf_off, const int32_t *vf_ent, const int32_t *vt_off,
                              const int32_t *vt_ent, const int32_t *edges, int64_t ne, const int32_t *faces,
                              int64_t nf, const int32_t *tets, int64_t nt, const float *field, int32_t nv,
                              int32_t *rec, int64_t cap_rec, int64_t *n_rec);

/* The DiscreteGradient workload with native consumer threads: each thread
 * takes the next cluster from a shared cursor over cluster_order, requests
 * VE, VF and VT for it (gale_submit on a DIRECT-mode context loaded with
 * gale_config.simplex_lists: the request is built on the GPU and copied back
 * before the call returns), reads the blocks, computes the cluster's gradient
 * and releases the ticket.  The paper runs this workload with one queue per
 * relation (Section 5.1); here one request carries the three relations. */
typedef struct {
    int32_t        threads;        /* consumer threads, >= 1 */
    int32_t        n_order;        /* clusters in cluster_order */
    const int32_t *cluster_order;
    const int32_t *tets;           /* nt*4, host */
    int64_t        nt;
    const float   *field;          /* nv, host */
    int32_t        nv;
    int32_t        pad;
} gale_gradient_cfg;

typedef struct {
    uint64_t clusters, errors;
    uint64_t critical[4];          /* critical simplices by dimension */
    uint64_t pairs[3];             /* pairs by the lower simplex's dimension (vertex-edge, edge-triangle,
                                      triangle-tetrahedron) */
    double   wall_s;
    double   lat_p50_us, lat_p99_us, lat_mean_us, lat_max_us;  /* per request: submit -> blocks ready */
    double   request_s_max;        /* per thread, the summed request time, maximum over threads */
    double   compute_s_max;        /* per thread, the summed gradient time, maximum over threads */
    int32_t  first_error;          /* gale status of the first failed call, 0 if none */
    int32_t  pad;
} gale_gradient_result;

/* Run the workload over cluster_order; blocks until every thread has
 * finished.  Returns GALE_OK (per-request failures are counted in
 * out->errors), GALE_EINVAL for a bad argument, GALE_ESTATE for a context
 * that is not in DIRECT mode or was loaded without simplex_lists. */
int32_t gale_gradient_run(struct gale_ctx *ctx, const gale_gradient_cfg *cfg, gale_gradient_result *out);

#ifdef __cplusplus
}
#endif

#endif /* GALE_GRADIENT_H */
