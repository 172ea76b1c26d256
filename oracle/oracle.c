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
