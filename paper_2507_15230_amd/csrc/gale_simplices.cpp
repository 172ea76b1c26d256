// gale_simplices.cpp -- the edge and triangle lists of the initialization
// step (paper, Section 4.3: E, F and their interval arrays I_E, I_F are
// enumerated on the CPU when an algorithm needs edge or triangle relations).
//
// Numbering: for each cluster k, its star tetrahedra are visited in ascending
// id; a tetrahedron's edges (triangles) are the pairs (triples) of its
// ascending vertices in lexicographic order; an edge internal to k (the
// smallest cluster among its vertices is k) gets the next id of k's interval
// the first time it is met.  This is the order under which the worked example
// of Section 4.4 comes out as printed.  Clusters are independent here (an
// edge is internal to exactly one), so they are enumerated in parallel from
// the per-cluster streams, then placed by the prefix sums of their counts.
//
// For the GPU the lists are indexed by each simplex's smallest vertex: for
// vertex a, the edges {a < b} as (b, id) sorted by b, and the triangles
// {a < b < c} as (b, c, id) sorted by (b, c).
#include <algorithm>
#include <atomic>
#include <cstring>
#include <thread>
#include <vector>

#include "gale_host.h"

namespace gale {

namespace {

int nthreads() {
    unsigned n = std::thread::hardware_concurrency();
    if (n == 0) n = 4;
    return (int)std::min<unsigned>(n, 32);
}

template <class F>
void run_threads(F f) {
    const int P = nthreads();
    std::vector<std::thread> th;
    for (int i = 0; i < P; ++i) th.emplace_back(f, i);
    for (auto &t : th) t.join();
}

// stream tetrahedron i of cluster m as four local ids (ascending)
inline void local_tet(const HostStreams &hs, const ClusterMeta &m, int64_t i, int32_t *l) {
    const uint8_t *tb = hs.tets.data() + m.tb_off;
    if (m.flags & kMetaWide) {
        std::memcpy(l, tb + 16 * i, 16);
    } else {
        uint16_t q[4];
        std::memcpy(q, tb + 8 * i, 8);
        for (int j = 0; j < 4; ++j) l[j] = q[j];
    }
}

constexpr int kPairs[6][2] = {{0, 1}, {0, 2}, {0, 3}, {1, 2}, {1, 3}, {2, 3}};
constexpr int kTriples[4][3] = {{0, 1, 2}, {0, 1, 3}, {0, 2, 3}, {1, 2, 3}};

}  // namespace

gale_status enumerate_simplices(const HostStreams &hs, HostSimplices &out, std::string &err) {
    const int32_t ncl = hs.ncl, nv = hs.nv;
    std::vector<std::vector<int32_t>> edges(ncl), faces(ncl);  // original ids, 2 / 3 per simplex, in id order
    std::vector<int64_t> et_inst(ncl, 0), ft_inst(ncl, 0);
    std::atomic<int32_t> next{0};
    run_threads([&](int) {
        std::vector<std::pair<uint64_t, int64_t>> ek;              // (local pair key, first visit)
        std::vector<std::pair<std::pair<uint64_t, uint32_t>, int64_t>> fk;
        std::vector<int64_t> order;
        while (true) {
            const int32_t k = next.fetch_add(1);
            if (k >= ncl) break;
            const ClusterMeta &m = hs.meta[k];
            const int32_t *lv = hs.lverts.data() + m.lv_off;
            const int32_t *id = hs.tid.data() + m.tet_off;
            // the star in ascending tetrahedron id: merge of the internal part
            // [0, nT) and the rest [nT, ns), each ascending
            order.clear();
            int64_t i = 0, j = m.nT;
            while (i < m.nT || j < m.ns) {
                const bool take_i = j >= m.ns || (i < m.nT && (id[i] & 0x7fffffff) < (id[j] & 0x7fffffff));
                order.push_back(take_i ? i++ : j++);
            }
            ek.clear();
            fk.clear();
            int64_t seq = 0, ne_inst = 0, nf_inst = 0;
            for (int64_t p : order) {
                int32_t l[4];
                local_tet(hs, m, p, l);
                bool low[4], row[4];
                for (int q = 0; q < 4; ++q) {
                    low[q] = (lv[l[q]] & 0x40000000) != 0;
                    row[q] = lv[l[q]] < 0;
                }
                for (int q = 0; q < 6; ++q, ++seq) {
                    const int a = kPairs[q][0], b = kPairs[q][1];
                    if (low[a] || low[b] || !(row[a] || row[b])) continue;
                    ek.emplace_back(((uint64_t)(uint32_t)l[a] << 32) | (uint32_t)l[b], seq);
                    ++ne_inst;
                }
                for (int q = 0; q < 4; ++q, ++seq) {
                    const int a = kTriples[q][0], b = kTriples[q][1], c = kTriples[q][2];
                    if (low[a] || low[b] || low[c] || !(row[a] || row[b] || row[c])) continue;
                    fk.push_back({{((uint64_t)(uint32_t)l[a] << 32) | (uint32_t)l[b], (uint32_t)l[c]}, seq});
                    ++nf_inst;
                }
            }
            et_inst[k] = ne_inst;
            ft_inst[k] = nf_inst;
            // first visit of each distinct simplex, then visit order
            std::sort(ek.begin(), ek.end());
            ek.erase(std::unique(ek.begin(), ek.end(), [](const auto &x, const auto &y) { return x.first == y.first; }),
                     ek.end());
            std::sort(ek.begin(), ek.end(), [](const auto &x, const auto &y) { return x.second < y.second; });
            std::sort(fk.begin(), fk.end());
            fk.erase(std::unique(fk.begin(), fk.end(), [](const auto &x, const auto &y) { return x.first == y.first; }),
                     fk.end());
            std::sort(fk.begin(), fk.end(), [](const auto &x, const auto &y) { return x.second < y.second; });
            auto orig = [&](uint32_t l) { return lv[l] & 0x3fffffff; };
            auto &E = edges[k];
            E.resize(2 * ek.size());
            for (size_t q = 0; q < ek.size(); ++q) {
                E[2 * q] = orig((uint32_t)(ek[q].first >> 32));
                E[2 * q + 1] = orig((uint32_t)ek[q].first);
            }
            auto &F = faces[k];
            F.resize(3 * fk.size());
            for (size_t q = 0; q < fk.size(); ++q) {
                F[3 * q] = orig((uint32_t)(fk[q].first.first >> 32));
                F[3 * q + 1] = orig((uint32_t)fk[q].first.first);
                F[3 * q + 2] = orig(fk[q].first.second);
            }
        }
    });
    out.ie.assign(ncl + 1, 0);
    out.if_.assign(ncl + 1, 0);
    for (int32_t k = 0; k < ncl; ++k) {
        out.ie[k + 1] = out.ie[k] + (int64_t)edges[k].size() / 2;
        out.if_[k + 1] = out.if_[k] + (int64_t)faces[k].size() / 3;
    }
    const int64_t ne = out.ie[ncl], nf = out.if_[ncl];
    if (ne > 0x7fffffffLL || nf > 0x7fffffffLL) {
        err = "more than 2^31 edges or triangles";
        return GALE_EINVAL;
    }
    out.e.resize(2 * ne);
    out.f.resize(3 * nf);
    out.ext.assign(ncl, ExtMeta{});
    for (int32_t k = 0; k < ncl; ++k) {
        ExtMeta &x = out.ext[k];
        x.e0 = (int32_t)out.ie[k];
        x.ne = (int32_t)(out.ie[k + 1] - out.ie[k]);
        x.f0 = (int32_t)out.if_[k];
        x.nf = (int32_t)(out.if_[k + 1] - out.if_[k]);
        if (et_inst[k] > 0x3fffffffLL || ft_inst[k] > 0x3fffffffLL) {
            err = "a cluster has more than 2^30 edge or triangle incidences";
            return GALE_EINVAL;
        }
        x.et_inst = (int32_t)et_inst[k];
        x.ft_inst = (int32_t)ft_inst[k];
    }
    next = 0;
    run_threads([&](int) {
        while (true) {
            const int32_t k = next.fetch_add(1);
            if (k >= ncl) break;
            std::copy(edges[k].begin(), edges[k].end(), out.e.begin() + 2 * out.ie[k]);
            std::copy(faces[k].begin(), faces[k].end(), out.f.begin() + 3 * out.if_[k]);
            std::vector<int32_t>().swap(edges[k]);
            std::vector<int32_t>().swap(faces[k]);
        }
    });
    // index by smallest vertex
    out.eoff.assign((size_t)nv + 1, 0);
    out.foff.assign((size_t)nv + 1, 0);
    for (int64_t i = 0; i < ne; ++i) out.eoff[out.e[2 * i] + 1]++;
    for (int64_t i = 0; i < nf; ++i) out.foff[out.f[3 * i] + 1]++;
    for (int32_t v = 0; v < nv; ++v) {
        out.eoff[v + 1] += out.eoff[v];
        out.foff[v + 1] += out.foff[v];
    }
    out.eidx.resize(2 * ne);
    out.fidx.resize(4 * nf);
    {
        std::vector<int32_t> fe(out.eoff.begin(), out.eoff.end() - 1), ff(out.foff.begin(), out.foff.end() - 1);
        for (int64_t i = 0; i < ne; ++i) {
            const int32_t w = fe[out.e[2 * i]]++;
            out.eidx[2 * (int64_t)w] = out.e[2 * i + 1];
            out.eidx[2 * (int64_t)w + 1] = (int32_t)i;
        }
        for (int64_t i = 0; i < nf; ++i) {
            const int32_t w = ff[out.f[3 * i]]++;
            out.fidx[4 * (int64_t)w] = out.f[3 * i + 1];
            out.fidx[4 * (int64_t)w + 1] = out.f[3 * i + 2];
            out.fidx[4 * (int64_t)w + 2] = (int32_t)i;
            out.fidx[4 * (int64_t)w + 3] = 0;
        }
    }
    std::atomic<int64_t> nextv{0};
    run_threads([&](int) {
        while (true) {
            const int64_t v0 = nextv.fetch_add(4096);
            if (v0 >= nv) break;
            for (int64_t v = v0; v < std::min<int64_t>(nv, v0 + 4096); ++v) {
                auto *e2 = reinterpret_cast<std::pair<int32_t, int32_t> *>(out.eidx.data()) + out.eoff[v];
                std::sort(e2, e2 + (out.eoff[v + 1] - out.eoff[v]));
                struct F4 {
                    int32_t b, c, id, pad;
                };
                auto *f4 = reinterpret_cast<F4 *>(out.fidx.data()) + out.foff[v];
                std::sort(f4, f4 + (out.foff[v + 1] - out.foff[v]),
                          [](const F4 &x, const F4 &y) { return x.b != y.b ? x.b < y.b : x.c < y.c; });
            }
        }
    });
    return GALE_OK;
}

}  // namespace gale
