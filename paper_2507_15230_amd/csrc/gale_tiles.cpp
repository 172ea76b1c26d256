// gale_tiles.cpp -- tiles of large clusters for the batched form.
//
// A cluster whose working set is far larger than a workgroup's LDS would run
// on the global-memory path, several times slower per vertex than the LDS
// path.  In the batched form such a cluster is built as tiles instead: its
// vertices are split into groups of about `tile_vt` VT entries, each group
// (a tile) is treated as a cluster of its own by the stream preparation and
// the kernels, and a stitch pass assembles the cluster's block from its
// tiles' blocks.
//
// Tiles are pseudo-clusters numbered in cluster order (the tiles of cluster
// C take consecutive ids), so the smallest pseudo-cluster among a
// tetrahedron's vertices lies in its owner cluster: a tetrahedron internal to
// C is a TT row of exactly one tile of C, and the tile's halo (computed by the
// same rule as a cluster's) holds the neighbours its rows need.  The block of
// C then has as rows the union of its tiles' rows (vertices, and internal
// tetrahedra), each row's list unchanged; the stitch places every row by its
// id (vmap, tmap below).
//
// Vertices are assigned to tiles in breadth-first order over the cluster's
// own edges (restarting at the smallest unassigned id for a disconnected
// part), cut where the running VT count passes a multiple of the tile size,
// so that a tile is a few connected layers rather than scattered vertices.
#include <algorithm>
#include <atomic>
#include <thread>
#include <vector>

#include "gale_host.h"

namespace gale {

namespace {
int nthreads_tiles() {
    unsigned n = std::thread::hardware_concurrency();
    if (n == 0) n = 4;
    return (int)std::min<unsigned>(n, 32);
}
}  // namespace

gale_status plan_tiles(int32_t nv, int64_t nt, const int32_t *tv, const int32_t *cl, int32_t ncl,
                       const std::vector<ClusterMeta> &meta, int64_t tile_vt, TilePlan &tp) {
    tp = TilePlan{};
    tp.tile_first.assign(ncl, -1);
    tp.tile_count.assign(ncl, 0);
    if (tile_vt <= 0) return GALE_OK;
    std::vector<int32_t> big;
    for (int32_t k = 0; k < ncl; ++k)
        if ((int64_t)meta[k].nnzVT > tile_vt && meta[k].nV > 1) big.push_back(k);
    if (big.empty()) return GALE_OK;
    // vertices of each cluster (ascending id) and each vertex's tetrahedra
    std::vector<int64_t> voff(ncl + 1, 0), toff(nv + 1, 0);
    for (int32_t v = 0; v < nv; ++v) voff[cl[v] + 1]++;
    for (int32_t k = 0; k < ncl; ++k) voff[k + 1] += voff[k];
    std::vector<int32_t> verts(nv);
    {
        std::vector<int64_t> f(voff.begin(), voff.end() - 1);
        for (int32_t v = 0; v < nv; ++v) verts[f[cl[v]]++] = v;
    }
    std::vector<char> in_big(ncl, 0);
    for (int32_t k : big) in_big[k] = 1;
    // each big-cluster vertex's tetrahedra: counts by atomic increments, a
    // parallel fill, then each list sorted
    const int P = nthreads_tiles();
    auto par = [&](int64_t n, auto f) {
        std::vector<std::thread> ts;
        const int64_t chunk = (n + P - 1) / P;
        for (int i = 0; i < P; ++i) {
            const int64_t b = i * chunk, e = std::min<int64_t>(n, b + chunk);
            if (b < e) ts.emplace_back(f, b, e);
        }
        for (auto &t : ts) t.join();
    };
    par(4 * nt, [&](int64_t b, int64_t e) {
        for (int64_t i = b; i < e; ++i)
            if (in_big[cl[tv[i]]]) __atomic_fetch_add(&toff[tv[i] + 1], 1, __ATOMIC_RELAXED);
    });
    for (int32_t v = 0; v < nv; ++v) toff[v + 1] += toff[v];
    std::vector<int32_t> vt(toff[nv]);
    {
        std::vector<int64_t> f(toff.begin(), toff.end() - 1);
        par(nt, [&](int64_t b, int64_t e) {
            for (int64_t t = b; t < e; ++t)
                for (int j = 0; j < 4; ++j) {
                    const int32_t v = tv[4 * t + j];
                    if (in_big[cl[v]]) vt[__atomic_fetch_add(&f[v], 1, __ATOMIC_RELAXED)] = (int32_t)t;
                }
        });
        // ascending lists: the same tiles whatever order the threads filled them in
        par(nv, [&](int64_t b, int64_t e) {
            for (int64_t v = b; v < e; ++v) std::sort(vt.begin() + toff[v], vt.begin() + toff[v + 1]);
        });
    }
    // breadth-first order and tile of every vertex of the big clusters
    std::vector<int32_t> tile_of(nv, -1), ntile_of(ncl, 0);
    std::atomic<size_t> next{0};
    std::vector<std::thread> th;
    for (int i = 0; i < nthreads_tiles(); ++i) {
        th.emplace_back([&] {
            std::vector<int32_t> order, queue;
            std::vector<char> seen;
            while (true) {
                const size_t bi = next.fetch_add(1);
                if (bi >= big.size()) break;
                const int32_t k = big[bi];
                const int64_t v0 = voff[k], v1 = voff[k + 1];
                const int64_t n = v1 - v0;
                const int64_t K = std::min<int64_t>((meta[k].nnzVT + tile_vt - 1) / tile_vt, kMaxTilesPerCluster);
                const double target = (double)meta[k].nnzVT / (double)K;
                // vertex -> index within the cluster (verts is ascending)
                auto index_of = [&](int32_t v) -> int64_t {
                    return std::lower_bound(verts.begin() + v0, verts.begin() + v1, v) - (verts.begin() + v0);
                };
                seen.assign(n, 0);
                order.clear();
                for (int64_t s = 0; s < n; ++s) {
                    if (seen[s]) continue;
                    seen[s] = 1;
                    queue.assign(1, verts[v0 + s]);
                    for (size_t q = 0; q < queue.size(); ++q) {
                        const int32_t v = queue[q];
                        order.push_back(v);
                        for (int64_t e = toff[v]; e < toff[v + 1]; ++e) {
                            const int32_t *tt = tv + 4 * (int64_t)vt[e];
                            for (int j = 0; j < 4; ++j) {
                                const int32_t u = tt[j];
                                if (cl[u] != k) continue;
                                const int64_t iu = index_of(u);
                                if (!seen[iu]) {
                                    seen[iu] = 1;
                                    queue.push_back(u);
                                }
                            }
                        }
                    }
                }
                double run = 0.0;
                int32_t last = 0;
                for (int32_t v : order) {
                    int32_t t = (int32_t)(run / target);
                    t = std::min<int32_t>(t, (int32_t)K - 1);
                    tile_of[v] = t;
                    last = std::max(last, t);
                    run += (double)(toff[v + 1] - toff[v]);
                }
                ntile_of[k] = last + 1;
            }
        });
    }
    for (auto &t : th) t.join();
    // pseudo-cluster ids in cluster order; the tiles of a cluster consecutive
    std::vector<int32_t> pfirst(ncl);
    int32_t np = 0, nti = 0;
    for (int32_t k = 0; k < ncl; ++k) {
        pfirst[k] = np;
        if (in_big[k]) {
            tp.tile_first[k] = nti;
            tp.tile_count[k] = ntile_of[k];
            for (int32_t j = 0; j < ntile_of[k]; ++j) tp.pseudo_of_tile.push_back(np + j);
            np += ntile_of[k];
            nti += ntile_of[k];
        } else {
            np += 1;
        }
    }
    tp.npseudo = np;
    tp.ntiles = nti;
    tp.pseudo.resize(nv);
    for (int32_t v = 0; v < nv; ++v) tp.pseudo[v] = pfirst[cl[v]] + (in_big[cl[v]] ? tile_of[v] : 0);
    tp.keep.assign(np, 0);
    for (int32_t p : tp.pseudo_of_tile) tp.keep[p] = 1;
    return GALE_OK;
}

// Stitch maps from the tiles' streams: for every tiled cluster, its vertices
// and its internal tetrahedra in ascending id, each with (tile, row index in
// the tile's block).
void stitch_maps(const TilePlan &tp, const HostStreams &ts, int32_t ncl, std::vector<StitchMeta> &sm,
                 std::vector<int32_t> &maps) {
    sm.assign(ncl, StitchMeta{});
    maps.clear();
    struct Row {
        int32_t id, tile, local;
    };
    std::vector<Row> rows;
    for (int32_t k = 0; k < ncl; ++k) {
        if (tp.tile_count[k] == 0) continue;
        StitchMeta &s = sm[k];
        s.tile_first = tp.tile_first[k];
        s.ntiles = tp.tile_count[k];
        // vertices
        rows.clear();
        for (int32_t j = 0; j < s.ntiles; ++j) {
            const ClusterMeta &m = ts.meta[tp.pseudo_of_tile[s.tile_first + j]];
            int32_t l = 0;
            for (int32_t i = 0; i < m.L; ++i) {
                const int32_t w = ts.lverts[m.lv_off + i];
                if (w < 0) rows.push_back({w & 0x3fffffff, j, l++});
            }
        }
        std::sort(rows.begin(), rows.end(), [](const Row &a, const Row &b) { return a.id < b.id; });
        s.vmap_off = (int64_t)maps.size();
        s.nv = (int32_t)rows.size();
        for (const Row &r : rows) {
            maps.push_back(r.tile);
            maps.push_back(r.local);
        }
        // internal tetrahedra: the first nT stream entries of each tile
        rows.clear();
        for (int32_t j = 0; j < s.ntiles; ++j) {
            const ClusterMeta &m = ts.meta[tp.pseudo_of_tile[s.tile_first + j]];
            for (int32_t i = 0; i < m.nT; ++i) rows.push_back({ts.tid[m.tet_off + i] & 0x7fffffff, j, i});
        }
        std::sort(rows.begin(), rows.end(), [](const Row &a, const Row &b) { return a.id < b.id; });
        s.tmap_off = (int64_t)maps.size();
        s.nt = (int32_t)rows.size();
        for (const Row &r : rows) {
            maps.push_back(r.tile);
            maps.push_back(r.local);
        }
    }
}

}  // namespace gale
