// gale_load.cpp -- host preparation of the per-cluster streams.
//
// The paper's initialization (Section 4.3) runs on the CPU: it builds, per
// segment, the list of external tetrahedra and the interval arrays, and copies
// them to GPU memory.  This is the same step for the per-cluster layout in
// gale_layout.h:
//   1. validate T and S;
//   2. owner(t) = smallest cluster id among t's vertices (internal rule);
//   3. star(C) = tetrahedra with a vertex in C, in ascending id (a stable
//      counting sort by cluster over ascending tetrahedron ids);
//   4. halo(C): a tetrahedron internal to C whose vertices include exactly one
//      vertex of C has an opposite triangle with no vertex in C; the other
//      tetrahedra on that triangle may lie outside star(C).  They are found by
//      intersecting the (ascending) global VT lists of the triangle's vertices
//      and appended as the halo, so that TT rows are complete;
//   5. local vertex table = sorted distinct vertices of star, halo and C;
//      stream tetrahedra are re-expressed in local ids, each tetrahedron's
//      four ids ascending, in the order: internal tetrahedra (the TT rows),
//      the rest of star(C), the halo, each part in ascending tetrahedron id.
// Everything here is integer bookkeeping; no relation entry is produced.
#include <algorithm>
#include <atomic>
#include <cstdint>
#include <cstring>
#include <string>
#include <thread>
#include <vector>

#include "gale_host.h"

namespace gale {

namespace {

int num_threads() {
    unsigned n = std::thread::hardware_concurrency();
    if (n == 0) n = 4;
    return (int)std::min<unsigned>(n, 32);
}

template <class F>
void parallel_for(int64_t n, F f) {
    const int P = num_threads();
    if (n <= 4096 || P == 1) {
        f(0, n, 0);
        return;
    }
    std::vector<std::thread> th;
    const int64_t chunk = (n + P - 1) / P;
    for (int i = 0; i < P; ++i) {
        const int64_t b = i * chunk, e = std::min<int64_t>(n, b + chunk);
        if (b >= e) break;
        th.emplace_back(f, b, e, i);
    }
    for (auto &t : th) t.join();
}

}  // namespace

gale_status prepare_streams(int32_t nv, int64_t nt, const int32_t *tv, const int32_t *cl, int32_t ncl,
                            HostStreams &out, std::string &err, const std::vector<char> *keep) {
    if (nv < 0 || nt < 0 || ncl <= 0) {
        err = "nv, nt must be >= 0 and nclusters >= 1";
        return GALE_EINVAL;
    }
    if (nt > 0x3fffffffLL) {
        err = "more than 2^30 tetrahedra";
        return GALE_EINVAL;
    }
    if ((int64_t)nv > 0x40000000LL) {
        err = "more than 2^30 vertices";
        return GALE_EINVAL;
    }
    if (nt > 0 && !tv) {
        err = "tv is NULL";
        return GALE_EINVAL;
    }
    if (nv > 0 && !cl) {
        err = "cluster_of_vertex is NULL";
        return GALE_EINVAL;
    }
    // 1. validate
    std::atomic<int64_t> bad_t{-1};
    parallel_for(nt, [&](int64_t b, int64_t e, int) {
        for (int64_t t = b; t < e; ++t) {
            const int32_t *q = tv + 4 * t;
            bool ok = true;
            for (int i = 0; i < 4 && ok; ++i) {
                if (q[i] < 0 || q[i] >= nv) ok = false;
                for (int j = 0; j < i && ok; ++j)
                    if (q[i] == q[j]) ok = false;
            }
            if (!ok) {
                int64_t expect = -1;
                bad_t.compare_exchange_strong(expect, t);
                return;
            }
        }
    });
    if (bad_t.load() >= 0) {
        err = "tetrahedron " + std::to_string(bad_t.load()) + " has a vertex id out of range or a repeated vertex";
        return GALE_EINVAL;
    }
    for (int32_t v = 0; v < nv; ++v) {
        if (cl[v] < 0 || cl[v] >= ncl) {
            err = "vertex " + std::to_string(v) + " has cluster id out of range";
            return GALE_EINVAL;
        }
    }

    // rows of every cluster: vertices in ascending id
    std::vector<int64_t> voff(ncl + 1, 0);
    for (int32_t v = 0; v < nv; ++v) voff[cl[v] + 1]++;
    for (int32_t k = 0; k < ncl; ++k) voff[k + 1] += voff[k];
    std::vector<int32_t> vrows(nv);
    {
        std::vector<int64_t> f(voff.begin(), voff.end() - 1);
        for (int32_t v = 0; v < nv; ++v) vrows[f[cl[v]]++] = v;
    }

    // 2. owner and distinct clusters per tetrahedron
    std::vector<int32_t> owner(nt);
    parallel_for(nt, [&](int64_t b, int64_t e, int) {
        for (int64_t t = b; t < e; ++t) {
            const int32_t *q = tv + 4 * t;
            int32_t o = cl[q[0]];
            for (int i = 1; i < 4; ++i) o = std::min(o, cl[q[i]]);
            owner[t] = o;
        }
    });

    // 3. star(C): stable counting sort by cluster over ascending tetrahedron ids,
    // per-thread counts so the fill stays in id order.
    const int P = num_threads();
    const int64_t chunk = (nt + P - 1) / std::max(P, 1);
    std::vector<std::vector<int64_t>> cnt(P, std::vector<int64_t>(ncl, 0));
    auto distinct = [&](int64_t t, int32_t *c4) -> int {
        const int32_t *q = tv + 4 * t;
        int n = 0;
        for (int i = 0; i < 4; ++i) {
            const int32_t k = cl[q[i]];
            bool seen = false;
            for (int j = 0; j < n; ++j) seen |= c4[j] == k;
            if (!seen) c4[n++] = k;
        }
        return n;
    };
    {
        std::vector<std::thread> th;
        for (int i = 0; i < P; ++i) {
            th.emplace_back([&, i] {
                const int64_t b = i * chunk, e = std::min<int64_t>(nt, b + chunk);
                int32_t c4[4];
                for (int64_t t = b; t < e; ++t) {
                    const int n = distinct(t, c4);
                    for (int j = 0; j < n; ++j) cnt[i][c4[j]]++;
                }
            });
        }
        for (auto &t : th) t.join();
    }
    std::vector<int64_t> soff(ncl + 1, 0);
    for (int32_t k = 0; k < ncl; ++k) {
        int64_t s = 0;
        for (int i = 0; i < P; ++i) s += cnt[i][k];
        soff[k + 1] = soff[k] + s;
    }
    std::vector<int32_t> star(soff[ncl]);
    {
        // start position of (thread i, cluster k)
        for (int32_t k = 0; k < ncl; ++k) {
            int64_t pos = soff[k];
            for (int i = 0; i < P; ++i) {
                const int64_t c = cnt[i][k];
                cnt[i][k] = pos;
                pos += c;
            }
        }
        std::vector<std::thread> th;
        for (int i = 0; i < P; ++i) {
            th.emplace_back([&, i] {
                const int64_t b = i * chunk, e = std::min<int64_t>(nt, b + chunk);
                int32_t c4[4];
                for (int64_t t = b; t < e; ++t) {
                    const int n = distinct(t, c4);
                    for (int j = 0; j < n; ++j) star[cnt[i][c4[j]]++] = (int32_t)t;
                }
            });
        }
        for (auto &t : th) t.join();
    }
    cnt.clear();
    cnt.shrink_to_fit();

    // 4. halo.  Global VT (lists ascending) for the triangles that need it:
    // counts by atomic increments, then each list filled and sorted.
    std::vector<int64_t> vtoff(nv + 1, 0);
    parallel_for(nt, [&](int64_t b, int64_t e, int) {
        for (int64_t i = 4 * b; i < 4 * e; ++i) __atomic_fetch_add(&vtoff[tv[i] + 1], 1, __ATOMIC_RELAXED);
    });
    for (int32_t v = 0; v < nv; ++v) vtoff[v + 1] += vtoff[v];
    std::vector<int32_t> vt(4 * nt);
    {
        std::vector<int64_t> f(vtoff.begin(), vtoff.end() - 1);
        parallel_for(nt, [&](int64_t b, int64_t e, int) {
            for (int64_t t = b; t < e; ++t)
                for (int i = 0; i < 4; ++i) vt[__atomic_fetch_add(&f[tv[4 * t + i]], 1, __ATOMIC_RELAXED)] = (int32_t)t;
        });
        parallel_for(nv, [&](int64_t b, int64_t e, int) {
            for (int64_t v = b; v < e; ++v) std::sort(vt.begin() + vtoff[v], vt.begin() + vtoff[v + 1]);
        });
    }
    std::vector<std::vector<std::pair<int32_t, int32_t>>> halo_parts(P);
    {
        std::vector<std::thread> th;
        for (int i = 0; i < P; ++i) {
            th.emplace_back([&, i] {
                const int64_t b = i * chunk, e = std::min<int64_t>(nt, b + chunk);
                auto &outp = halo_parts[i];
                for (int64_t t = b; t < e; ++t) {
                    const int32_t *q = tv + 4 * t;
                    const int32_t o = owner[t];
                    int inC = 0, only = -1;
                    for (int j = 0; j < 4; ++j)
                        if (cl[q[j]] == o) { ++inC; only = j; }
                    if (inC != 1) continue;
                    int32_t f[3];
                    int m = 0;
                    for (int j = 0; j < 4; ++j)
                        if (j != only) f[m++] = q[j];
                    const int32_t *la = vt.data() + vtoff[f[0]], *lb = vt.data() + vtoff[f[1]],
                                  *lc = vt.data() + vtoff[f[2]];
                    const int64_t na = vtoff[f[0] + 1] - vtoff[f[0]], nb = vtoff[f[1] + 1] - vtoff[f[1]],
                                  nc = vtoff[f[2] + 1] - vtoff[f[2]];
                    int64_t x = 0, y = 0, z = 0;
                    while (x < na && y < nb && z < nc) {
                        const int32_t A = la[x], Bv = lb[y], Cv = lc[z];
                        if (A == Bv && Bv == Cv) {
                            if (A != (int32_t)t) {
                                const int32_t *qq = tv + 4 * (int64_t)A;
                                bool touches = false;
                                for (int j = 0; j < 4; ++j) touches |= cl[qq[j]] == o;
                                if (!touches) outp.emplace_back(o, A);
                            }
                            ++x; ++y; ++z;
                            continue;
                        }
                        const int32_t mx = std::max(A, std::max(Bv, Cv));
                        if (A < mx) ++x;
                        if (Bv < mx) ++y;
                        if (Cv < mx) ++z;
                    }
                }
            });
        }
        for (auto &t : th) t.join();
    }
    vt.clear();
    vt.shrink_to_fit();
    vtoff.clear();
    vtoff.shrink_to_fit();
    std::vector<std::pair<int32_t, int32_t>> halo;
    {
        size_t tot = 0;
        for (auto &h : halo_parts) tot += h.size();
        halo.reserve(tot);
        for (auto &h : halo_parts) {
            halo.insert(halo.end(), h.begin(), h.end());
            h.clear();
            h.shrink_to_fit();
        }
        std::sort(halo.begin(), halo.end());
        halo.erase(std::unique(halo.begin(), halo.end()), halo.end());
    }
    std::vector<int64_t> hoff(ncl + 1, 0);
    for (auto &p : halo) hoff[p.first + 1]++;
    for (int32_t k = 0; k < ncl; ++k) hoff[k + 1] += hoff[k];

    // 5. local tables and encoded streams, per cluster.  Each thread keeps
    // two arrays over all vertices: the last cluster that met the vertex
    // (distinct vertices without sorting the star's four-per-tetrahedron
    // list) and the vertex's local id in the cluster it works on.
    out.meta.assign(ncl, ClusterMeta{});
    std::vector<std::vector<int32_t>> ltab(ncl);
    std::atomic<int32_t> next{0};
    std::atomic<int> too_big{0};
    // row index of every vertex within its cluster (rank by ascending id)
    std::vector<int32_t> rowof(nv);
    parallel_for(ncl, [&](int64_t b, int64_t e, int) {
        for (int64_t k = b; k < e; ++k)
            for (int64_t s2 = voff[k]; s2 < voff[k + 1]; ++s2) rowof[vrows[s2]] = (int32_t)(s2 - voff[k]);
    });
    {
        std::vector<std::thread> th;
        for (int i = 0; i < P; ++i) {
            th.emplace_back([&] {
                std::vector<int32_t> stamp(nv, -1);
                std::vector<int32_t> deg;
                while (true) {
                    const int32_t k = next.fetch_add(1);
                    if (k >= ncl) break;
                    if (keep && !(*keep)[k]) continue;  // streams of this cluster not wanted
                    auto &tab = ltab[k];
                    const int64_t s0 = soff[k], s1 = soff[k + 1];
                    const int64_t h0 = hoff[k], h1 = hoff[k + 1];
                    tab.clear();
                    auto add = [&](int32_t v) {
                        if (stamp[v] != k) {
                            stamp[v] = k;
                            tab.push_back(v);
                        }
                    };
                    for (int64_t s2 = s0; s2 < s1; ++s2)
                        for (int j = 0; j < 4; ++j) add(tv[4 * (int64_t)star[s2] + j]);
                    for (int64_t s2 = h0; s2 < h1; ++s2)
                        for (int j = 0; j < 4; ++j) add(tv[4 * (int64_t)halo[s2].second + j]);
                    for (int64_t s2 = voff[k]; s2 < voff[k + 1]; ++s2) add(vrows[s2]);
                    std::sort(tab.begin(), tab.end());
                    tab.shrink_to_fit();
                    ClusterMeta &m = out.meta[k];
                    m.ns = (int32_t)(s1 - s0);
                    m.nh = (int32_t)(h1 - h0);
                    m.L = (int32_t)tab.size();
                    m.nV = (int32_t)(voff[k + 1] - voff[k]);
                    if ((int64_t)tab.size() > 0x7fffffffLL) too_big = 1;
                    int64_t nnz = 0, nT = 0;
                    deg.assign(m.nV, 0);
                    for (int64_t s2 = s0; s2 < s1; ++s2) {
                        const int32_t t = star[s2];
                        if (owner[t] == k) ++nT;
                        for (int j = 0; j < 4; ++j) {
                            const int32_t v = tv[4 * (int64_t)t + j];
                            if (cl[v] == k) {
                                ++nnz;
                                deg[rowof[v]]++;
                            }
                        }
                    }
                    if (nnz > 0x7fffffffLL) too_big = 1;
                    m.nnzVT = (int32_t)nnz;
                    m.nT = (int32_t)nT;
                    int64_t capvv = 0;
                    for (int32_t r = 0; r < m.nV; ++r) {
                        const int64_t d = deg[r];
                        int64_t c = std::min<int64_t>(d + 2, 3 * d);
                        c = std::min<int64_t>(c, (int64_t)m.L - 1);
                        capvv += std::max<int64_t>(c, 0);
                    }
                    if (capvv > 0x7fffffffLL) too_big = 1;
                    m.cap_vv = (int32_t)capvv;
                }
            });
        }
        for (auto &t : th) t.join();
    }
    if (too_big.load()) {
        err = "a cluster exceeds the 2^31 entries limit of one block";
        return GALE_EINVAL;
    }
    int64_t tetn = 0, lvn = 0, tbn = 0;
    for (int32_t k = 0; k < ncl; ++k) {
        ClusterMeta &m = out.meta[k];
        const int64_t ntot = (int64_t)m.ns + m.nh;
        m.flags = m.L > 65535 ? kMetaWide : 0;
        m.tet_off = tetn;
        m.lv_off = lvn;
        m.tb_off = tbn;
        tetn += ntot;
        lvn += m.L;
        tbn += (ntot * ((m.flags & kMetaWide) ? 16 : 8) + 15) / 16 * 16;
    }
    out.tets.assign((size_t)tbn, 0);
    out.tid.assign((size_t)tetn, 0);
    out.lverts.assign((size_t)lvn, 0);
    next = 0;
    {
        std::vector<std::thread> th;
        for (int i = 0; i < P; ++i) {
            th.emplace_back([&] {
                std::vector<int32_t> lid(nv, 0);  // local id of a vertex in the current cluster
                while (true) {
                    const int32_t k = next.fetch_add(1);
                    if (k >= ncl) break;
                    if (keep && !(*keep)[k]) continue;
                    const auto &tab = ltab[k];
                    const ClusterMeta &m = out.meta[k];
                    for (int32_t l = 0; l < m.L; ++l) lid[tab[l]] = l;
                    for (int32_t l = 0; l < m.L; ++l) {
                        const int32_t v = tab[l];
                        const uint32_t row = cl[v] == k ? 0x80000000u : 0u;
                        const uint32_t lower = cl[v] < k ? 0x40000000u : 0u;
                        out.lverts[m.lv_off + l] = (int32_t)((uint32_t)v | row | lower);
                    }
                    auto local = [&](int32_t v) -> int32_t { return lid[v]; };
                    const bool wide = (m.flags & kMetaWide) != 0;
                    uint8_t *tb = out.tets.data() + m.tb_off;
                    auto put = [&](int64_t i, int32_t t) {
                        int32_t l[4];
                        for (int j = 0; j < 4; ++j) l[j] = local(tv[4 * (int64_t)t + j]);
                        std::sort(l, l + 4);
                        for (int j = 0; j < 4; ++j) {
                            if (wide) {
                                std::memcpy(tb + 16 * i + 4 * j, &l[j], 4);
                            } else {
                                const uint16_t l16 = (uint16_t)l[j];
                                std::memcpy(tb + 8 * i + 2 * j, &l16, 2);
                            }
                        }
                    };
                    int64_t p = m.tet_off, i = 0;
                    for (int pass = 0; pass < 2; ++pass) {  // internal first, then the rest of the star
                        for (int64_t s = soff[k]; s < soff[k + 1]; ++s) {
                            const int32_t t = star[s];
                            const bool in = owner[t] == k;
                            if (in != (pass == 0)) continue;
                            put(i, t);
                            out.tid[p] = in ? (int32_t)((uint32_t)t | 0x80000000u) : t;
                            ++p;
                            ++i;
                        }
                    }
                    for (int64_t s = hoff[k]; s < hoff[k + 1]; ++s, ++p, ++i) {
                        const int32_t t = halo[s].second;
                        put(i, t);
                        out.tid[p] = t;
                    }
                }
            });
        }
        for (auto &t : th) t.join();
    }
    out.nv = nv;
    out.nt = nt;
    out.ncl = ncl;
    return GALE_OK;
}

}  // namespace gale
