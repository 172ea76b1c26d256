/*
 * CPU oracle for localized VT / VV / TT relation blocks.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this file's library.  It shares no
 * code, header, table or helper with the GPU library; it is written from the
 * definitions in the paper, not from the GPU algorithm.
 *
 * What it computes (paper, Section 2.2 "Topological Relations" and Table 1;
 * Section 4.3 "Input data" for the segment rule):
 *   - VT(v): the tetrahedra whose four vertices include v (coboundary
 *     relation of a vertex).
 *   - VV(v): the vertices that share an edge with v.  In a tetrahedral mesh
 *     every pair of vertices of a tetrahedron is an edge, so VV(v) is the union
 *     of the vertex sets of the tetrahedra in VT(v), minus v itself (Fig. 1
 *     lists VV(v0) = [v1, v2, v3] without v0).
 *   - TT(t): the tetrahedra that share a triangle (a 2-face) with t: for each
 *     face {a,b,c} of t, VT(a) n VT(b) n VT(c) minus t.
 *   - A segment (cluster) C owns as VT/VV rows the vertices v with S[v] = C.
 *   - A tetrahedron is internal to exactly one segment (Section 4.3: the
 *     segment of its lowest-index vertex).  Cluster ids here are in spatial
 *     order and vertex ids are arbitrary, so the rule is read as: the owner of
 *     t is the smallest cluster id among its four vertices.  Under the paper's
 *     segment-contiguous vertex numbering both readings give the same owner.
 *     A cluster's TT rows are its internal tetrahedra.
 *   - Rows are listed in ascending original id; every list is in ascending
 *     original id with duplicates removed (set semantics).
 *
 * Steps (each a plain definition, no blocking or reordering):
 *   O0 validate input; O1 global VT by counting sort over tetrahedra in
 *   ascending id (so every VT list is ascending); O2 VT/VV rows per cluster;
 *   O3 TT rows per cluster by the owner rule; O4 emit (row ids, offsets from 0,
 *   entries) in original ids.
 *
 * Edges and triangles (oracle_enumerate; Section 4.3 "Initialization", read
 * through the worked example of Section 4.4): the lists E and F number every
 * edge and triangle of the mesh, each stored as its ascending vertex tuple.
 * For each cluster k in turn, the cluster's tetrahedra (those with a vertex
 * in k) are visited in ascending id; each tetrahedron's edges (triangles) are
 * taken as the pairs (triples) of its ascending vertices in lexicographic
 * order, and an edge internal to k (smallest cluster among its vertices = k)
 * that is not listed yet is appended.  I_E[k] is the first id of cluster k's
 * edges (the interval array of Section 4.3).  With this order the example of
 * Section 4.4 comes out as printed (12 edges, I_E = 0, 9, 12; f5 = v0 v3 v4 and
 * FE(f5) = e2, e6, e9), which a plain lexicographic sort would not give.
 * The further coboundary relations (Section 2.2, Table 1) per cluster k:
 *   - VE(v), VF(v): ids of the edges / triangles containing v, rows = the
 *     vertices of k;
 *   - EF(e), ET(e): ids of the triangles / tetrahedra containing e, rows = the
 *     edges internal to k in id order (row ids are edge ids);
 *   - FT(f): the tetrahedra containing f, rows = the triangles internal to k.
 *
 * Planted mistakes: oracle_set_mutation() switches on one deliberately wrong
 * variant so the tests can show that their pins catch it.  Mutation 0 (the
 * default) is the oracle proper.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_EINVAL (-1)
#define ORC_ENOMEM (-2)

#define REL_VT 1
#define REL_VV 2
#define REL_TT 4
#define REL_VE 8
#define REL_VF 16
#define REL_EF 32
#define REL_ET 64
#define REL_FT 128

/* One block's arrays (rows, offsets, entries) and their capacities.  A
 * context is read-only while blocks are built, so threads that each own a
 * buffer may build blocks of one context at the same time. */
typedef struct {
    int64_t nrows, nnz;
    int32_t *rows, *off, *ent;
    int64_t cap_rows, cap_ent;
} oracle_buf;

typedef struct {
    int32_t nv;
    int64_t nt;
    int32_t ncl;
    int32_t *tv;        /* nt*4, copy of input */
    int32_t *cl;        /* nv, copy of input */
    int64_t *vt_off;    /* nv+1 */
    int32_t *vt;        /* 4*nt, tetrahedron ids, each list ascending */
    int32_t *owner;     /* nt */
    int64_t *vrow_off;  /* ncl+1 */
    int32_t *vrows;     /* nv: vertices grouped by cluster, ascending id */
    int64_t *trow_off;  /* ncl+1 */
    int32_t *trows;     /* nt: tetrahedra grouped by owner, ascending id */
    int mutation;
    int owner_mut;      /* mutation the owner table was built under */
    oracle_buf b;       /* the block last built by oracle_block */
    /* edges and triangles (oracle_enumerate): E[i] = (ea[i], eb[i]) with
     * ea < eb, F[i] = (fa, fb, fc) ascending; cluster k's internal ones are
     * ids [ie[k], ie[k+1]) and [if_[k], if_[k+1]).  Lookup lists: for each
     * vertex a, the edges / triangles whose smallest vertex is a, with ids. */
    int enumerated;
    int64_t ne, nf;
    int32_t *ea, *eb, *fa, *fb, *fc;
    int64_t *ie, *if_;
    int64_t *el_off, *fl_off;  /* nv+1: list capacity of each vertex */
    int32_t *el_n, *fl_n;      /* nv: list length */
    int32_t *el_b, *fl_b, *fl_c;
    int64_t *el_id, *fl_id;
} oracle_ctx;

static int cmp_i32(const void *a, const void *b) {
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

/* sort ascending and drop repeats; returns the new length */
static int64_t sort_unique(int32_t *a, int64_t n) {
    if (n <= 1) return n;
    qsort(a, (size_t)n, sizeof(int32_t), cmp_i32);
    int64_t w = 1;
    for (int64_t i = 1; i < n; ++i)
        if (a[i] != a[w - 1]) a[w++] = a[i];
    return w;
}

void oracle_destroy(oracle_ctx *c) {
    if (!c) return;
    free(c->tv); free(c->cl); free(c->vt_off); free(c->vt); free(c->owner);
    free(c->vrow_off); free(c->vrows); free(c->trow_off); free(c->trows);
    free(c->b.rows); free(c->b.off); free(c->b.ent);
    free(c->ea); free(c->eb); free(c->fa); free(c->fb); free(c->fc); free(c->ie); free(c->if_);
    free(c->el_off); free(c->fl_off); free(c->el_n); free(c->fl_n); free(c->el_b); free(c->fl_b);
    free(c->fl_c); free(c->el_id); free(c->fl_id);
    free(c);
}

void oracle_set_mutation(oracle_ctx *c, int m) { c->mutation = m; }

/* O0: every vertex id in range, four distinct vertices per tetrahedron, every
 * cluster id in [0, ncl), ncl >= 1. */
int oracle_validate(int32_t nv, int64_t nt, const int32_t *tv, const int32_t *cl, int32_t ncl) {
    if (nv < 0 || nt < 0 || ncl <= 0) return ORC_EINVAL;
    if (nt > 0x7fffffffLL) return ORC_EINVAL;
    for (int64_t t = 0; t < nt; ++t) {
        const int32_t *q = tv + 4 * t;
        for (int i = 0; i < 4; ++i) {
            if (q[i] < 0 || q[i] >= nv) return ORC_EINVAL;
            for (int j = 0; j < i; ++j)
                if (q[i] == q[j]) return ORC_EINVAL;
        }
    }
    for (int32_t v = 0; v < nv; ++v)
        if (cl[v] < 0 || cl[v] >= ncl) return ORC_EINVAL;
    return ORC_OK;
}

int oracle_create(int32_t nv, int64_t nt, const int32_t *tv, const int32_t *cl, int32_t ncl,
                  oracle_ctx **out) {
    *out = NULL;
    int st = oracle_validate(nv, nt, tv, cl, ncl);
    if (st) return st;
    oracle_ctx *c = (oracle_ctx *)calloc(1, sizeof(oracle_ctx));
    if (!c) return ORC_ENOMEM;
    c->nv = nv; c->nt = nt; c->ncl = ncl;
    c->tv = (int32_t *)malloc(sizeof(int32_t) * (size_t)(4 * nt + 1));
    c->cl = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nv + 1));
    c->vt_off = (int64_t *)calloc((size_t)nv + 1, sizeof(int64_t));
    c->vt = (int32_t *)malloc(sizeof(int32_t) * (size_t)(4 * nt + 1));
    c->owner = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nt + 1));
    c->vrow_off = (int64_t *)calloc((size_t)ncl + 1, sizeof(int64_t));
    c->vrows = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nv + 1));
    c->trow_off = (int64_t *)calloc((size_t)ncl + 1, sizeof(int64_t));
    c->trows = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nt + 1));
    if (!c->tv || !c->cl || !c->vt_off || !c->vt || !c->owner || !c->vrow_off || !c->vrows ||
        !c->trow_off || !c->trows) {
        oracle_destroy(c);
        return ORC_ENOMEM;
    }
    memcpy(c->tv, tv, sizeof(int32_t) * (size_t)(4 * nt));
    memcpy(c->cl, cl, sizeof(int32_t) * (size_t)nv);

    /* O1: global VT.  Count the occurrences of each vertex, exclusive prefix
     * sum, then fill while visiting tetrahedra in ascending id. */
    for (int64_t i = 0; i < 4 * nt; ++i) c->vt_off[c->tv[i] + 1]++;
    for (int32_t v = 0; v < nv; ++v) c->vt_off[v + 1] += c->vt_off[v];
    {
        int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nv + 1));
        if (!fill) { oracle_destroy(c); return ORC_ENOMEM; }
        memcpy(fill, c->vt_off, sizeof(int64_t) * (size_t)(nv + 1));
        for (int64_t t = 0; t < nt; ++t)
            for (int i = 0; i < 4; ++i) c->vt[fill[c->tv[4 * t + i]]++] = (int32_t)t;
        free(fill);
    }

    /* owner(t): smallest cluster id among the four vertices (Section 4.3). */
    for (int64_t t = 0; t < nt; ++t) {
        int32_t o = c->cl[c->tv[4 * t]];
        for (int i = 1; i < 4; ++i) {
            int32_t k = c->cl[c->tv[4 * t + i]];
            if (c->mutation == 3 ? (k > o) : (k < o)) o = k;
        }
        c->owner[t] = o;
    }

    /* O2/O3 row sets: vertices by cluster, tetrahedra by owner, each in
     * ascending id (counting sort over ascending ids). */
    for (int32_t v = 0; v < nv; ++v) c->vrow_off[c->cl[v] + 1]++;
    for (int32_t k = 0; k < ncl; ++k) c->vrow_off[k + 1] += c->vrow_off[k];
    for (int64_t t = 0; t < nt; ++t) c->trow_off[c->owner[t] + 1]++;
    for (int32_t k = 0; k < ncl; ++k) c->trow_off[k + 1] += c->trow_off[k];
    {
        int64_t *fv = (int64_t *)malloc(sizeof(int64_t) * (size_t)(ncl + 1));
        int64_t *ft = (int64_t *)malloc(sizeof(int64_t) * (size_t)(ncl + 1));
        if (!fv || !ft) { free(fv); free(ft); oracle_destroy(c); return ORC_ENOMEM; }
        memcpy(fv, c->vrow_off, sizeof(int64_t) * (size_t)(ncl + 1));
        memcpy(ft, c->trow_off, sizeof(int64_t) * (size_t)(ncl + 1));
        for (int32_t v = 0; v < nv; ++v) c->vrows[fv[c->cl[v]]++] = v;
        for (int64_t t = 0; t < nt; ++t) c->trows[ft[c->owner[t]]++] = (int32_t)t;
        free(fv); free(ft);
    }
    *out = c;
    return ORC_OK;
}

/* Recompute the owner table if the mutation that changes it is switched on
 * after creation (tests switch mutations on an existing context). */
static void refresh_rows(oracle_ctx *c) {
    for (int64_t t = 0; t < c->nt; ++t) {
        int32_t o = c->cl[c->tv[4 * t]];
        for (int i = 1; i < 4; ++i) {
            int32_t k = c->cl[c->tv[4 * t + i]];
            if (c->mutation == 3 ? (k > o) : (k < o)) o = k;
        }
        c->owner[t] = o;
    }
    memset(c->trow_off, 0, sizeof(int64_t) * (size_t)(c->ncl + 1));
    for (int64_t t = 0; t < c->nt; ++t) c->trow_off[c->owner[t] + 1]++;
    for (int32_t k = 0; k < c->ncl; ++k) c->trow_off[k + 1] += c->trow_off[k];
    int64_t *ft = (int64_t *)malloc(sizeof(int64_t) * (size_t)(c->ncl + 1));
    memcpy(ft, c->trow_off, sizeof(int64_t) * (size_t)(c->ncl + 1));
    for (int64_t t = 0; t < c->nt; ++t) c->trows[ft[c->owner[t]]++] = (int32_t)t;
    free(ft);
    c->owner_mut = c->mutation;
}

/* ---------------------------------------------------------------------------
 * Edges and triangles
 * ------------------------------------------------------------------------ */

/* owner of a simplex: the smallest cluster id among its n vertices (the
 * largest under planted mistake 3) */
static int32_t simplex_owner(const oracle_ctx *c, const int32_t *q, int n) {
    int32_t o = c->cl[q[0]];
    for (int i = 1; i < n; ++i) {
        int32_t k = c->cl[q[i]];
        if (c->mutation == 3 ? (k > o) : (k < o)) o = k;
    }
    return o;
}

/* id of edge {a < b}, or -1 */
static int64_t edge_id(const oracle_ctx *c, int32_t a, int32_t b) {
    const int64_t o = c->el_off[a];
    for (int32_t i = 0; i < c->el_n[a]; ++i)
        if (c->el_b[o + i] == b) return c->el_id[o + i];
    return -1;
}

/* id of triangle {a < b < c3}, or -1 */
static int64_t face_id(const oracle_ctx *c, int32_t a, int32_t b, int32_t c3) {
    const int64_t o = c->fl_off[a];
    for (int32_t i = 0; i < c->fl_n[a]; ++i)
        if (c->fl_b[o + i] == b && c->fl_c[o + i] == c3) return c->fl_id[o + i];
    return -1;
}

static void sort4(int32_t *q) {
    for (int i = 1; i < 4; ++i)
        for (int j = i; j > 0 && q[j - 1] > q[j]; --j) {
            int32_t x = q[j]; q[j] = q[j - 1]; q[j - 1] = x;
        }
}

/* the tetrahedra with a vertex in cluster k, ascending id; returns the count
 * (out holds at least the sum of the rows' VT degrees) */
static int64_t star_of(const oracle_ctx *c, int32_t k, int32_t *out) {
    int64_t n = 0;
    for (int64_t r = c->vrow_off[k]; r < c->vrow_off[k + 1]; ++r) {
        int32_t v = c->vrows[r];
        for (int64_t i = c->vt_off[v]; i < c->vt_off[v + 1]; ++i) out[n++] = c->vt[i];
    }
    return sort_unique(out, n);
}

/* planted mistake 10: a cluster's edges and triangles in ascending vertex
 * tuples instead of discovery order (ids in the lookup lists rewritten) */
static int cmp_pair(const void *x, const void *y) {
    const int64_t *p = (const int64_t *)x, *q = (const int64_t *)y;
    return (p[0] > q[0]) - (p[0] < q[0]);
}
static void relist_sorted(oracle_ctx *c, int64_t e0, int64_t e1, int64_t f0, int64_t f1) {
    int64_t n = e1 - e0 > f1 - f0 ? e1 - e0 : f1 - f0;
    int64_t *key = (int64_t *)malloc(sizeof(int64_t) * 2 * (size_t)(n + 1));
    int32_t *t0 = (int32_t *)malloc(sizeof(int32_t) * 3 * (size_t)(n + 1));
    for (int64_t i = e0; i < e1; ++i) {
        key[2 * (i - e0)] = ((int64_t)c->ea[i] << 31) | c->eb[i];
        key[2 * (i - e0) + 1] = i;
    }
    qsort(key, (size_t)(e1 - e0), 2 * sizeof(int64_t), cmp_pair);
    for (int64_t i = 0; i < e1 - e0; ++i) { t0[2 * i] = c->ea[key[2 * i + 1]]; t0[2 * i + 1] = c->eb[key[2 * i + 1]]; }
    for (int64_t i = 0; i < e1 - e0; ++i) {
        c->ea[e0 + i] = t0[2 * i]; c->eb[e0 + i] = t0[2 * i + 1];
        const int64_t o = c->el_off[c->ea[e0 + i]];
        for (int32_t j = 0; j < c->el_n[c->ea[e0 + i]]; ++j)
            if (c->el_b[o + j] == c->eb[e0 + i]) c->el_id[o + j] = e0 + i;
    }
    (void)f0; (void)f1;
    free(key); free(t0);
}

/* Number the edges and triangles (see the header).  Idempotent. */
int oracle_enumerate(oracle_ctx *c) {
    if (c->enumerated) return ORC_OK;
    const int32_t nv = c->nv, ncl = c->ncl;
    const int64_t nt = c->nt;
    c->el_off = (int64_t *)calloc((size_t)nv + 1, sizeof(int64_t));
    c->fl_off = (int64_t *)calloc((size_t)nv + 1, sizeof(int64_t));
    c->el_n = (int32_t *)calloc((size_t)nv + 1, sizeof(int32_t));
    c->fl_n = (int32_t *)calloc((size_t)nv + 1, sizeof(int32_t));
    c->ie = (int64_t *)calloc((size_t)ncl + 1, sizeof(int64_t));
    c->if_ = (int64_t *)calloc((size_t)ncl + 1, sizeof(int64_t));
    if (!c->el_off || !c->fl_off || !c->el_n || !c->fl_n || !c->ie || !c->if_) return ORC_ENOMEM;
    /* a tetrahedron containing a has at most three edges and three triangles
     * whose smallest vertex is a */
    for (int32_t v = 0; v < nv; ++v) {
        const int64_t d = c->vt_off[v + 1] - c->vt_off[v];
        c->el_off[v + 1] = c->el_off[v] + 3 * d;
        c->fl_off[v + 1] = c->fl_off[v] + 3 * d;
    }
    const size_t cap = (size_t)c->el_off[nv] + 1;
    c->el_b = (int32_t *)malloc(sizeof(int32_t) * cap);
    c->el_id = (int64_t *)malloc(sizeof(int64_t) * cap);
    c->fl_b = (int32_t *)malloc(sizeof(int32_t) * cap);
    c->fl_c = (int32_t *)malloc(sizeof(int32_t) * cap);
    c->fl_id = (int64_t *)malloc(sizeof(int64_t) * cap);
    c->ea = (int32_t *)malloc(sizeof(int32_t) * (size_t)(6 * nt + 1));
    c->eb = (int32_t *)malloc(sizeof(int32_t) * (size_t)(6 * nt + 1));
    c->fa = (int32_t *)malloc(sizeof(int32_t) * (size_t)(4 * nt + 1));
    c->fb = (int32_t *)malloc(sizeof(int32_t) * (size_t)(4 * nt + 1));
    c->fc = (int32_t *)malloc(sizeof(int32_t) * (size_t)(4 * nt + 1));
    int32_t *star = (int32_t *)malloc(sizeof(int32_t) * (size_t)(4 * nt + 1));
    if (!c->el_b || !c->el_id || !c->fl_b || !c->fl_c || !c->fl_id || !c->ea || !c->eb || !c->fa || !c->fb ||
        !c->fc || !star) {
        free(star);
        return ORC_ENOMEM;
    }
    static const int P2[6][2] = {{0, 1}, {0, 2}, {0, 3}, {1, 2}, {1, 3}, {2, 3}};
    static const int P3[4][3] = {{0, 1, 2}, {0, 1, 3}, {0, 2, 3}, {1, 2, 3}};
    int64_t ne = 0, nf = 0;
    for (int32_t k = 0; k < ncl; ++k) {
        c->ie[k] = ne;
        c->if_[k] = nf;
        const int64_t ns = star_of(c, k, star);
        for (int64_t i = 0; i < ns; ++i) {
            int32_t s[4];
            memcpy(s, c->tv + 4 * (int64_t)star[i], sizeof(s));
            sort4(s);
            for (int j = 0; j < 6; ++j) {
                int32_t q[2] = {s[P2[j][0]], s[P2[j][1]]};
                if (simplex_owner(c, q, 2) != k || edge_id(c, q[0], q[1]) >= 0) continue;
                c->ea[ne] = q[0];
                c->eb[ne] = q[1];
                const int64_t o = c->el_off[q[0]] + c->el_n[q[0]]++;
                c->el_b[o] = q[1];
                c->el_id[o] = ne++;
            }
            for (int j = 0; j < 4; ++j) {
                int32_t q[3] = {s[P3[j][0]], s[P3[j][1]], s[P3[j][2]]};
                if (simplex_owner(c, q, 3) != k || face_id(c, q[0], q[1], q[2]) >= 0) continue;
                c->fa[nf] = q[0];
                c->fb[nf] = q[1];
                c->fc[nf] = q[2];
                const int64_t o = c->fl_off[q[0]] + c->fl_n[q[0]]++;
                c->fl_b[o] = q[1];
                c->fl_c[o] = q[2];
                c->fl_id[o] = nf++;
            }
        }
        if (c->mutation == 10) relist_sorted(c, c->ie[k], ne, c->if_[k], nf);
    }
    c->ie[ncl] = ne;
    c->if_[ncl] = nf;
    c->ne = ne;
    c->nf = nf;
    free(star);
    c->enumerated = 1;
    return ORC_OK;
}

int64_t oracle_num_edges(const oracle_ctx *c) { return c->enumerated ? c->ne : -1; }
int64_t oracle_num_faces(const oracle_ctx *c) { return c->enumerated ? c->nf : -1; }

/* copy E (2 per edge), F (3 per triangle) and the interval arrays out */
void oracle_simplices(const oracle_ctx *c, int32_t *e, int64_t *ie, int32_t *f, int64_t *if_) {
    for (int64_t i = 0; i < c->ne; ++i) { e[2 * i] = c->ea[i]; e[2 * i + 1] = c->eb[i]; }
    for (int64_t i = 0; i < c->nf; ++i) { f[3 * i] = c->fa[i]; f[3 * i + 1] = c->fb[i]; f[3 * i + 2] = c->fc[i]; }
    memcpy(ie, c->ie, sizeof(int64_t) * (size_t)(c->ncl + 1));
    memcpy(if_, c->if_, sizeof(int64_t) * (size_t)(c->ncl + 1));
}

/* number of elements common to two ascending lists, written to out */
static int64_t intersect2(const int32_t *a, int64_t na, const int32_t *b, int64_t nb, int32_t *out) {
    int64_t i = 0, j = 0, w = 0;
    while (i < na && j < nb) {
        if (a[i] == b[j]) { out[w++] = a[i]; ++i; ++j; }
        else if (a[i] < b[j]) ++i;
        else ++j;
    }
    return w;
}

static int reserve(oracle_buf *b, int64_t rows, int64_t ent);
static int64_t intersect3(const int32_t *a, int64_t na, const int32_t *b, int64_t nb,
                          const int32_t *c3, int64_t nc, int32_t *out);

/* VE / VF / EF / ET / FT block of cluster k into b (the context must be
 * enumerated) */
static int cobound_block(const oracle_ctx *c, oracle_buf *b, int32_t k, int32_t rel, int64_t *nrows,
                         int64_t *nnz) {
    if (!c->enumerated) return ORC_EINVAL;
    int64_t n, cap = 0;
    if (rel == REL_VE || rel == REL_VF) {
        n = c->vrow_off[k + 1] - c->vrow_off[k];
        for (int64_t r = 0; r < n; ++r) {
            const int32_t v = c->vrows[c->vrow_off[k] + r];
            cap += 3 * (c->vt_off[v + 1] - c->vt_off[v]);
        }
    } else {
        const int64_t *iv = rel == REL_FT ? c->if_ : c->ie;
        n = iv[k + 1] - iv[k];
        for (int64_t r = 0; r < n; ++r) {
            const int64_t id = iv[k] + r;
            const int32_t a = rel == REL_FT ? c->fa[id] : c->ea[id];
            const int64_t d = c->vt_off[a + 1] - c->vt_off[a];
            cap += (rel == REL_EF ? 2 : 1) * d;
        }
    }
    if (reserve(b, n, cap + 1)) return ORC_ENOMEM;
    int64_t w = 0;
    b->off[0] = 0;
    for (int64_t r = 0; r < n; ++r) {
        const int64_t s0 = w;
        if (rel == REL_VE || rel == REL_VF) {
            const int32_t v = c->vrows[c->vrow_off[k] + r];
            b->rows[r] = v;
            for (int64_t i = c->vt_off[v]; i < c->vt_off[v + 1]; ++i) {
                const int32_t *q = c->tv + 4 * (int64_t)c->vt[i];
                int32_t o[3];
                int m = 0;
                for (int j = 0; j < 4; ++j)
                    if (q[j] != v) o[m++] = q[j];
                if (rel == REL_VE) {
                    for (int j = 0; j < 3; ++j)
                        b->ent[w++] = (int32_t)edge_id(c, v < o[j] ? v : o[j], v < o[j] ? o[j] : v);
                } else {
                    const int nfc = c->mutation == 12 ? 2 : 3;
                    for (int j = 0; j < nfc; ++j) {
                        /* the triangle of v and the two other vertices but o[j] */
                        int32_t f[3] = {v, o[(j + 1) % 3], o[(j + 2) % 3]};
                        for (int x = 1; x < 3; ++x)
                            for (int y = x; y > 0 && f[y - 1] > f[y]; --y) {
                                int32_t z = f[y]; f[y] = f[y - 1]; f[y - 1] = z;
                            }
                        b->ent[w++] = (int32_t)face_id(c, f[0], f[1], f[2]);
                    }
                }
            }
        } else if (rel == REL_EF || rel == REL_ET) {
            const int64_t id = c->ie[k] + r;
            const int32_t a = c->ea[id], e2 = c->eb[id];
            b->rows[r] = (int32_t)id;
            const int32_t *la = c->vt + c->vt_off[a];
            const int32_t *lb = c->vt + c->vt_off[e2];
            const int64_t na = c->vt_off[a + 1] - c->vt_off[a], nb = c->vt_off[e2 + 1] - c->vt_off[e2];
            int64_t got = c->mutation == 13 ? (memcpy(b->ent + w, la, sizeof(int32_t) * (size_t)na), na)
                                             : intersect2(la, na, lb, nb, b->ent + w);
            if (rel == REL_ET) {
                w += got;
            } else {
                /* the two triangles of each such tetrahedron that contain the edge */
                int32_t *tl = (int32_t *)malloc(sizeof(int32_t) * (size_t)(got + 1));
                memcpy(tl, b->ent + w, sizeof(int32_t) * (size_t)got);
                for (int64_t i = 0; i < got; ++i) {
                    const int32_t *q = c->tv + 4 * (int64_t)tl[i];
                    for (int j = 0; j < 4; ++j) {
                        if (q[j] == a || q[j] == e2) continue;
                        int32_t f[3] = {a, e2, q[j]};
                        for (int x = 1; x < 3; ++x)
                            for (int y = x; y > 0 && f[y - 1] > f[y]; --y) {
                                int32_t z = f[y]; f[y] = f[y - 1]; f[y - 1] = z;
                            }
                        b->ent[w++] = (int32_t)face_id(c, f[0], f[1], f[2]);
                    }
                }
                free(tl);
            }
        } else {
            const int64_t id = c->if_[k] + r;
            const int32_t a = c->fa[id], b2 = c->fb[id], c3 = c->fc[id];
            b->rows[r] = (int32_t)id;
            w += intersect3(c->vt + c->vt_off[a], c->vt_off[a + 1] - c->vt_off[a], c->vt + c->vt_off[b2],
                            c->vt_off[b2 + 1] - c->vt_off[b2], c->vt + c->vt_off[c3],
                            c->vt_off[c3 + 1] - c->vt_off[c3], b->ent + w);
        }
        w = s0 + sort_unique(b->ent + s0, w - s0);
        b->off[r + 1] = (int32_t)w;
    }
    *nrows = n;
    *nnz = w;
    b->nrows = n;
    b->nnz = w;
    return ORC_OK;
}

static int reserve(oracle_buf *b, int64_t rows, int64_t ent) {
    if (rows + 1 > b->cap_rows) {
        free(b->rows); free(b->off);
        b->cap_rows = rows + 1;
        b->rows = (int32_t *)malloc(sizeof(int32_t) * (size_t)b->cap_rows);
        b->off = (int32_t *)malloc(sizeof(int32_t) * (size_t)(b->cap_rows + 1));
        if (!b->rows || !b->off) return ORC_ENOMEM;
    }
    if (ent > b->cap_ent) {
        free(b->ent);
        b->cap_ent = ent + ent / 2 + 16;
        b->ent = (int32_t *)malloc(sizeof(int32_t) * (size_t)b->cap_ent);
        if (!b->ent) return ORC_ENOMEM;
    }
    return ORC_OK;
}

/* number of elements common to three ascending lists, written to out */
static int64_t intersect3(const int32_t *a, int64_t na, const int32_t *b, int64_t nb,
                          const int32_t *c3, int64_t nc, int32_t *out) {
    int64_t i = 0, j = 0, k = 0, w = 0;
    while (i < na && j < nb && k < nc) {
        int32_t x = a[i], y = b[j], z = c3[k];
        if (x == y && y == z) { out[w++] = x; ++i; ++j; ++k; continue; }
        int32_t m = x > y ? x : y;
        m = m > z ? m : z;
        if (x < m) ++i;
        if (y < m) ++j;
        if (z < m) ++k;
    }
    return w;
}

/* O2-O4: build the block (cluster k, one relation) into buffer b.  Returns
 * status; *nrows / *nnz receive the sizes.  Reads the context only. */
int oracle_block_into(const oracle_ctx *c, oracle_buf *b, int32_t k, int32_t rel, int64_t *nrows, int64_t *nnz) {
    if (k < 0 || k >= c->ncl) return ORC_EINVAL;
    if (rel == REL_VE || rel == REL_VF || rel == REL_EF || rel == REL_ET || rel == REL_FT)
        return cobound_block(c, b, k, rel, nrows, nnz);
    if (rel != REL_VT && rel != REL_VV && rel != REL_TT) return ORC_EINVAL;
    if ((c->mutation == 3) != (c->owner_mut == 3)) return ORC_EINVAL;  /* owner table of another mutation */
    if (rel == REL_VT || rel == REL_VV) {
        const int32_t *rows = c->vrows + c->vrow_off[k];
        int64_t n = c->vrow_off[k + 1] - c->vrow_off[k];
        int64_t cap = 0;
        for (int64_t r = 0; r < n; ++r) {
            int32_t v = rows[r];
            int64_t deg = c->vt_off[v + 1] - c->vt_off[v];
            cap += rel == REL_VT ? deg : 4 * deg;
        }
        if (reserve(b, n, cap + 1)) return ORC_ENOMEM;
        int64_t w = 0;
        b->off[0] = 0;
        for (int64_t r = 0; r < n; ++r) {
            int32_t v = rows[c->mutation == 7 ? n - 1 - r : r];
            b->rows[r] = v;
            const int32_t *lst = c->vt + c->vt_off[v];
            int64_t deg = c->vt_off[v + 1] - c->vt_off[v];
            if (rel == REL_VT) {
                if (c->mutation == 8 && deg > 0) deg -= 1;
                for (int64_t i = 0; i < deg; ++i)
                    b->ent[w + i] = lst[c->mutation == 4 ? deg - 1 - i : i];
                w += deg;
            } else {
                int64_t s = w;
                int64_t use = (c->mutation == 6 && deg > 0) ? 1 : deg;
                for (int64_t i = 0; i < use; ++i) {
                    const int32_t *q = c->tv + 4 * (int64_t)lst[i];
                    for (int j = 0; j < 4; ++j)
                        if (q[j] != v || c->mutation == 1) b->ent[w++] = q[j];
                }
                w = s + sort_unique(b->ent + s, w - s);
            }
            b->off[r + 1] = (int32_t)w;
        }
        *nrows = n;
        *nnz = w;
    } else {
        const int32_t *rows = c->trows + c->trow_off[k];
        int64_t n = c->trow_off[k + 1] - c->trow_off[k];
        /* capacity: the neighbours found through one face lie in VT of the
         * face's first vertex, so four times the largest degree bounds a row */
        int64_t cap = 0;
        for (int64_t r = 0; r < n; ++r) {
            const int32_t *q = c->tv + 4 * (int64_t)rows[r];
            int64_t mx = 0;
            for (int j = 0; j < 4; ++j) {
                int64_t d = c->vt_off[q[j] + 1] - c->vt_off[q[j]];
                if (d > mx) mx = d;
            }
            cap += 4 * mx;
        }
        if (reserve(b, n, cap + 1)) return ORC_ENOMEM;
        int64_t w = 0;
        b->off[0] = 0;
        for (int64_t r = 0; r < n; ++r) {
            int32_t t = rows[r];
            b->rows[r] = t;
            const int32_t *q = c->tv + 4 * (int64_t)t;
            int64_t s = w;
            int nfaces = c->mutation == 9 ? 3 : 4;
            for (int omit = 0; omit < nfaces; ++omit) {
                int32_t f[3];
                int m = 0;
                for (int j = 0; j < 4; ++j)
                    if (j != omit) f[m++] = q[j];
                const int32_t *la = c->vt + c->vt_off[f[0]];
                const int32_t *lb = c->vt + c->vt_off[f[1]];
                const int32_t *lc = c->vt + c->vt_off[f[2]];
                int64_t na = c->vt_off[f[0] + 1] - c->vt_off[f[0]];
                int64_t nb = c->vt_off[f[1] + 1] - c->vt_off[f[1]];
                int64_t nc = c->vt_off[f[2] + 1] - c->vt_off[f[2]];
                int64_t got;
                if (c->mutation == 5) /* wrong: adjacency through an edge */
                    got = intersect3(la, na, lb, nb, lb, nb, b->ent + w);
                else
                    got = intersect3(la, na, lb, nb, lc, nc, b->ent + w);
                int64_t keep = 0;
                for (int64_t i = 0; i < got; ++i)
                    if (b->ent[w + i] != t || c->mutation == 2) b->ent[w + keep++] = b->ent[w + i];
                w += keep;
            }
            w = s + sort_unique(b->ent + s, w - s);
            b->off[r + 1] = (int32_t)w;
        }
        *nrows = n;
        *nnz = w;
    }
    b->nrows = *nrows;
    b->nnz = *nnz;
    return ORC_OK;
}

/* The same into the context's own buffer (one caller at a time); switches
 * the owner table when the owner mutation was turned on or off. */
int oracle_block(oracle_ctx *c, int32_t k, int32_t rel, int64_t *nrows, int64_t *nnz) {
    if ((c->mutation == 3) != (c->owner_mut == 3)) refresh_rows(c);
    return oracle_block_into(c, &c->b, k, rel, nrows, nnz);
}

/* copy a buffer's block out: rows[nrows], offsets[nrows+1], entries[nnz] */
void oracle_buf_copy(const oracle_buf *b, int32_t *rows, int32_t *offsets, int32_t *entries) {
    if (b->nrows) memcpy(rows, b->rows, sizeof(int32_t) * (size_t)b->nrows);
    memcpy(offsets, b->off, sizeof(int32_t) * (size_t)(b->nrows + 1));
    if (b->nnz) memcpy(entries, b->ent, sizeof(int32_t) * (size_t)b->nnz);
}

/* copy the last block of oracle_block out */
void oracle_block_copy(const oracle_ctx *c, int32_t *rows, int32_t *offsets, int32_t *entries) {
    oracle_buf_copy(&c->b, rows, offsets, entries);
}

oracle_buf *oracle_buf_new(void) { return (oracle_buf *)calloc(1, sizeof(oracle_buf)); }

void oracle_buf_free(oracle_buf *b) {
    if (!b) return;
    free(b->rows); free(b->off); free(b->ent);
    free(b);
}

/* accessors used by the tests */
int32_t oracle_owner(oracle_ctx *c, int64_t t) {
    if ((c->mutation == 3) != (c->owner_mut == 3)) refresh_rows(c);
    return c->owner[t];
}
int64_t oracle_vt_degree(const oracle_ctx *c, int32_t v) { return c->vt_off[v + 1] - c->vt_off[v]; }
