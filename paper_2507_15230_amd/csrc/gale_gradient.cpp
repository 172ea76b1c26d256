// gale_gradient.cpp -- host consumer: discrete gradient of a scalar field
// from a cluster's VE, VF and VT blocks (include/gale_gradient.h).
//
// Per vertex v the lower star is gathered from the blocks (an edge of VE(v),
// a triangle of VF(v), a tetrahedron of VT(v) whose other vertices all lie
// below v), each simplex with its key (vertex orders from the highest down).
// Facets within the lower star are found through the other vertices: the
// edge {v, a} by a, the triangle {v, a, b} by (a, b).  The two queues are
// binary heaps of lower-star indices ordered by key; a simplex classified
// while it waits in a queue is skipped when it comes up.
#include <stdint.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cstring>
#include <functional>
#include <mutex>
#include <queue>
#include <thread>
#include <vector>

#include "../../include/gale.h"
#include "../../include/gale_gradient.h"

namespace {

struct Ord {
    float f;
    int32_t id;
};
inline bool ord_less(const Ord &a, const Ord &b) { return a.f < b.f || (a.f == b.f && a.id < b.id); }

struct Cell {
    int dim;          // 1 edge, 2 triangle, 3 tetrahedron
    int32_t id;
    int32_t oth[3];   // the other vertices (not v), ascending by order
    int n;            // how many: dim
    Ord key[4];       // v first, then the others from the highest down
    int nk;
    int state;        // 0 unclassified, 1 classified
    int facet[3], nf; // lower-star facets (indices), those containing v
    std::vector<int> cof;
};

// lexicographic key order, a proper prefix first
inline bool key_less(const Cell &a, const Cell &b) {
    const int n = std::min(a.nk, b.nk);
    for (int i = 0; i < n; ++i) {
        if (ord_less(a.key[i], b.key[i])) return true;
        if (ord_less(b.key[i], a.key[i])) return false;
    }
    return a.nk < b.nk;
}

struct Gradient {
    const int32_t *edges, *faces, *tets;
    int64_t ne, nf, nt;
    const float *field;
    int32_t nv;
    std::vector<Cell> cells;
    std::vector<int32_t> rec;

    Ord ord(int32_t x) const { return Ord{field[x], x}; }

    // lower star of v from its block rows; false on an inconsistent entry
    bool gather(int32_t v, const int32_t *ve, int32_t nve, const int32_t *vf, int32_t nvf, const int32_t *vt,
                int32_t nvt) {
        cells.clear();
        const Ord ov = ord(v);
        auto add = [&](int dim, int32_t id, int32_t *o, int n) -> bool {
            for (int i = 0; i < n; ++i) {
                if (o[i] < 0 || o[i] >= nv) return false;
                if (!ord_less(ord(o[i]), ov)) return true;  // not in the lower star
            }
            Cell c;
            c.dim = dim;
            c.id = id;
            c.n = n;
            // the others from the highest down
            std::sort(o, o + n, [&](int32_t a, int32_t b) { return ord_less(ord(b), ord(a)); });
            for (int i = 0; i < n; ++i) c.oth[i] = o[i];
            c.key[0] = ov;
            for (int i = 0; i < n; ++i) c.key[1 + i] = ord(o[i]);
            c.nk = n + 1;
            c.state = 0;
            c.nf = 0;
            cells.push_back(std::move(c));
            return true;
        };
        for (int32_t i = 0; i < nve; ++i) {
            const int32_t e = ve[i];
            if (e < 0 || e >= ne) return false;
            const int32_t a = edges[2 * (int64_t)e], b = edges[2 * (int64_t)e + 1];
            if (a != v && b != v) return false;
            int32_t o[1] = {a == v ? b : a};
            if (!add(1, e, o, 1)) return false;
        }
        for (int32_t i = 0; i < nvf; ++i) {
            const int32_t f = vf[i];
            if (f < 0 || f >= nf) return false;
            int32_t o[3], m = 0;
            bool has = false;
            for (int j = 0; j < 3; ++j) {
                const int32_t x = faces[3 * (int64_t)f + j];
                if (x == v) has = true;
                else if (m < 2) o[m++] = x;
            }
            if (!has || m != 2) return false;
            if (!add(2, f, o, 2)) return false;
        }
        for (int32_t i = 0; i < nvt; ++i) {
            const int32_t t = vt[i];
            if (t < 0 || t >= nt) return false;
            int32_t o[3], m = 0;
            bool has = false;
            for (int j = 0; j < 4; ++j) {
                const int32_t x = tets[4 * (int64_t)t + j];
                if (x == v) has = true;
                else if (m < 3) o[m++] = x;
            }
            if (!has || m != 3) return false;
            if (!add(3, t, o, 3)) return false;
        }
        // facets in the lower star: drop one of the other vertices
        const int nc = (int)cells.size();
        for (int i = 0; i < nc; ++i) {
            Cell &c = cells[i];
            if (c.dim == 1) continue;
            for (int drop = 0; drop < c.n; ++drop) {
                int32_t want[2];
                int m = 0;
                for (int j = 0; j < c.n; ++j)
                    if (j != drop) want[m++] = c.oth[j];
                for (int k = 0; k < nc; ++k) {
                    const Cell &d = cells[k];
                    if (d.dim != c.dim - 1) continue;
                    bool same = true;
                    for (int j = 0; j < m && same; ++j) same = d.oth[j] == want[j];
                    if (same) {
                        c.facet[c.nf++] = k;
                        cells[k].cof.push_back(i);
                        break;
                    }
                }
            }
        }
        return true;
    }

    int unclassified_facets(const Cell &c, int *which) const {
        int n = 0;
        for (int j = 0; j < c.nf; ++j)
            if (cells[c.facet[j]].state == 0) {
                ++n;
                *which = c.facet[j];
            }
        return n;
    }

    void emit(int dim, int32_t lo, int32_t up) {
        rec.push_back(dim);
        rec.push_back(lo);
        rec.push_back(up);
    }

    void process(int32_t v) {
        const int nc = (int)cells.size();
        int delta = -1;
        for (int i = 0; i < nc; ++i)
            if (cells[i].dim == 1 && (delta < 0 || key_less(cells[i], cells[delta]))) delta = i;
        if (delta < 0) {
            emit(0, v, -1);
            return;
        }
        emit(0, v, cells[delta].id);
        cells[delta].state = 1;
        auto greater = [&](int a, int b) { return key_less(cells[b], cells[a]); };
        std::priority_queue<int, std::vector<int>, decltype(greater)> pq0(greater), pq1(greater);
        for (int i = 0; i < nc; ++i)
            if (cells[i].dim == 1 && i != delta) pq0.push(i);
        auto push_ready_cofaces = [&](int s) {
            for (int b : cells[s].cof) {
                int w;
                if (cells[b].state == 0 && unclassified_facets(cells[b], &w) == 1) pq1.push(b);
            }
        };
        push_ready_cofaces(delta);
        while (!pq1.empty() || !pq0.empty()) {
            while (!pq1.empty()) {
                const int a = pq1.top();
                pq1.pop();
                if (cells[a].state) continue;
                int face = -1;
                if (unclassified_facets(cells[a], &face) == 0) {
                    pq0.push(a);
                    continue;
                }
                emit(cells[face].dim, cells[face].id, cells[a].id);
                cells[face].state = 1;
                cells[a].state = 1;
                push_ready_cofaces(a);
                push_ready_cofaces(face);
            }
            while (!pq0.empty()) {
                const int g = pq0.top();
                pq0.pop();
                if (cells[g].state) continue;
                emit(cells[g].dim, cells[g].id, -1);
                cells[g].state = 1;
                push_ready_cofaces(g);
                break;
            }
        }
    }
};

}  // namespace

extern "C" int32_t gale_gradient_cluster(int32_t nrows, const int32_t *row_ids, const int32_t *ve_off,
                                         const int32_t *ve_ent, const int32_t *vf_off, const int32_t *vf_ent,
                                         const int32_t *vt_off, const int32_t *vt_ent, const int32_t *edges,
                                         int64_t ne, const int32_t *faces, int64_t nf, const int32_t *tets,
                                         int64_t nt, const float *field, int32_t nv, int32_t *rec, int64_t cap_rec,
                                         int64_t *n_rec) {
    if (nrows < 0 || !n_rec) return -1;
    *n_rec = 0;
    if (nrows == 0) return 0;
    if (!row_ids || !ve_off || !vf_off || !vt_off || !edges || !faces || !tets || !field || !rec) return -1;
    Gradient g{edges, faces, tets, ne, nf, nt, field, nv, {}, {}};
    for (int32_t r = 0; r < nrows; ++r) {
        const int32_t v = row_ids[r];
        if (v < 0 || v >= nv) return -1;
        if (!g.gather(v, ve_ent + ve_off[r], ve_off[r + 1] - ve_off[r], vf_ent + vf_off[r],
                      vf_off[r + 1] - vf_off[r], vt_ent + vt_off[r], vt_off[r + 1] - vt_off[r]))
            return -1;
        g.process(v);
    }
    const int64_t n = (int64_t)g.rec.size() / 3;
    if (n > cap_rec) return -1;
    std::memcpy(rec, g.rec.data(), g.rec.size() * sizeof(int32_t));
    *n_rec = n;
    return 0;
}

extern "C" int32_t gale_gradient_run(gale_ctx *ctx, const gale_gradient_cfg *cfg, gale_gradient_result *out) {
    if (!ctx || !cfg || !out || cfg->threads < 1 || cfg->n_order < 0 || (cfg->n_order > 0 && !cfg->cluster_order) ||
        !cfg->tets || !cfg->field)
        return GALE_EINVAL;
    std::memset(out, 0, sizeof(*out));
    gale_simplices sx;
    if (gale_get_simplices(ctx, &sx) != GALE_OK) return GALE_ESTATE;
    const uint32_t mask = GALE_REL_VT | GALE_REL_VE | GALE_REL_VF;
    std::atomic<int32_t> cursor{0};
    std::mutex mu;
    std::vector<double> lat;
    double req_max = 0.0, comp_max = 0.0;
    using Clock = std::chrono::steady_clock;
    const auto t_start = Clock::now();
    auto worker = [&]() {
        std::vector<double> my_lat;
        uint64_t crit[4] = {0, 0, 0, 0}, pairs[3] = {0, 0, 0}, clusters = 0, errors = 0;
        int32_t first_error = 0;
        double req_s = 0.0, comp_s = 0.0;
        std::vector<int32_t> rec;
        while (true) {
            const int32_t i = cursor.fetch_add(1);
            if (i >= cfg->n_order) break;
            const int32_t k = cfg->cluster_order[i];
            const auto t0 = Clock::now();
            uint64_t tk = 0;
            gale_status s = gale_submit(ctx, &k, 1, mask, &tk);
            gale_csr ve, vf, vt;
            if (s == GALE_OK) s = gale_poll(ctx, tk, -1);
            if (s == GALE_OK) s = gale_block(ctx, tk, k, GALE_REL_VE, &ve);
            if (s == GALE_OK) s = gale_block(ctx, tk, k, GALE_REL_VF, &vf);
            if (s == GALE_OK) s = gale_block(ctx, tk, k, GALE_REL_VT, &vt);
            const auto t1 = Clock::now();
            if (s == GALE_OK) {
                my_lat.push_back(std::chrono::duration<double, std::micro>(t1 - t0).count());
                req_s += std::chrono::duration<double>(t1 - t0).count();
                rec.resize(3 * (size_t)(ve.nrows + ve.nnz + vf.nnz + vt.nnz));
                int64_t nrec = 0;
                const int32_t st = gale_gradient_cluster(
                    ve.nrows, ve.row_ids, ve.offsets, ve.entries, vf.offsets, vf.entries, vt.offsets, vt.entries,
                    sx.e, sx.ne, sx.f, sx.nf, cfg->tets, cfg->nt, cfg->field, cfg->nv, rec.data(),
                    (int64_t)rec.size() / 3, &nrec);
                comp_s += std::chrono::duration<double>(Clock::now() - t1).count();
                if (st != 0) {
                    s = GALE_EINVAL;
                } else {
                    for (int64_t j = 0; j < nrec; ++j) {
                        const int32_t d = rec[3 * j], up = rec[3 * j + 2];
                        if (up < 0) crit[d & 3]++;
                        else pairs[d < 3 ? d : 2]++;
                    }
                    ++clusters;
                }
            }
            if (tk) (void)gale_release(ctx, tk);
            if (s != GALE_OK) {
                ++errors;
                if (!first_error) first_error = s;
            }
        }
        std::lock_guard<std::mutex> g(mu);
        for (int d = 0; d < 4; ++d) out->critical[d] += crit[d];
        for (int d = 0; d < 3; ++d) out->pairs[d] += pairs[d];
        out->clusters += clusters;
        out->errors += errors;
        if (!out->first_error) out->first_error = first_error;
        lat.insert(lat.end(), my_lat.begin(), my_lat.end());
        req_max = std::max(req_max, req_s);
        comp_max = std::max(comp_max, comp_s);
    };
    std::vector<std::thread> th;
    for (int i = 0; i < cfg->threads; ++i) th.emplace_back(worker);
    for (auto &t : th) t.join();
    out->wall_s = std::chrono::duration<double>(Clock::now() - t_start).count();
    out->request_s_max = req_max;
    out->compute_s_max = comp_max;
    if (!lat.empty()) {
        std::sort(lat.begin(), lat.end());
        auto pct = [&](double p) { return lat[std::min(lat.size() - 1, (size_t)(p * (double)(lat.size() - 1) + 0.5))]; };
        out->lat_p50_us = pct(0.50);
        out->lat_p99_us = pct(0.99);
        double sum = 0.0;
        for (double x : lat) sum += x;
        out->lat_mean_us = sum / (double)lat.size();
        out->lat_max_us = lat.back();
    }
    return GALE_OK;
}
