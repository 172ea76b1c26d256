// gale_lowerstar.cpp -- host consumer: critical-point classification of a
// scalar field from a cluster's VT and VV blocks (include/gale_lowerstar.h).
#include <stdint.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "../../include/gale_lowerstar.h"

namespace {

// (f, id) order: true when a is below b
inline bool below(const float *f, int32_t a, int32_t b) { return f[a] < f[b] || (f[a] == f[b] && a < b); }

struct Dsu {
    std::vector<int32_t> p;
    void reset(int n) {
        p.resize(n);
        for (int i = 0; i < n; ++i) p[i] = i;
    }
    int32_t find(int32_t x) {
        while (p[x] != x) {
            p[x] = p[p[x]];
            x = p[x];
        }
        return x;
    }
    void unite(int32_t a, int32_t b) {
        a = find(a);
        b = find(b);
        if (a != b) p[a < b ? b : a] = a < b ? a : b;
    }
};

}  // namespace

extern "C" int32_t gale_lowerstar_classify(int32_t nrows, const int32_t *row_ids, const int32_t *vt_off,
                                           const int32_t *vt_ent, const int32_t *vv_off, const int32_t *vv_ent,
                                           const int32_t *tets, int64_t nt, const float *field, int32_t nv,
                                           int32_t *labels) {
    if (nrows < 0) return -1;
    if (nrows > 0 && (!row_ids || !vt_off || !vv_off || !labels || !tets || !field)) return -1;
    Dsu dsu;
    std::vector<uint8_t> side;
    for (int32_t r = 0; r < nrows; ++r) {
        const int32_t v = row_ids[r];
        if (v < 0 || v >= nv) return -1;
        const int32_t *nb = vv_ent + vv_off[r];
        const int32_t nl = vv_off[r + 1] - vv_off[r];
        // link vertices: VV(v), ascending; side 1 = below v, 2 = above
        side.assign(nl, 0);
        int lower = 0, upper = 0;
        for (int32_t i = 0; i < nl; ++i) {
            if (nb[i] < 0 || nb[i] >= nv) return -1;
            const bool lo = below(field, nb[i], v);
            side[i] = lo ? 1 : 2;
            lower += lo;
            upper += !lo;
        }
        auto index_of = [&](int32_t u) -> int32_t {
            const int32_t *it = std::lower_bound(nb, nb + nl, u);
            return (it != nb + nl && *it == u) ? (int32_t)(it - nb) : -1;
        };
        // link edges: the other three vertices of each tetrahedron around v
        dsu.reset(nl);
        for (int32_t j = vt_off[r]; j < vt_off[r + 1]; ++j) {
            const int64_t t = vt_ent[j];
            if (t < 0 || t >= nt) return -1;
            int32_t o[3], k = 0;
            bool has_v = false;
            for (int c = 0; c < 4; ++c) {
                const int32_t u = tets[4 * t + c];
                if (u == v) {
                    has_v = true;
                } else if (k < 3) {
                    o[k++] = index_of(u);
                }
            }
            if (!has_v || k != 3 || o[0] < 0 || o[1] < 0 || o[2] < 0) return -1;
            for (int a = 0; a < 3; ++a)
                for (int b = a + 1; b < 3; ++b)
                    if (side[o[a]] == side[o[b]]) dsu.unite(o[a], o[b]);
        }
        int cl = 0, cu = 0;
        for (int32_t i = 0; i < nl; ++i) {
            if (dsu.find(i) != i) continue;
            if (side[i] == 1) ++cl;
            else ++cu;
        }
        int32_t lab;
        if (lower == 0) lab = GALE_CP_MINIMUM;
        else if (upper == 0) lab = GALE_CP_MAXIMUM;
        else if (cl > 1 || cu > 1) lab = GALE_CP_SADDLE;
        else lab = GALE_CP_REGULAR;
        labels[r] = lab;
    }
    return 0;
}

// ---------------------------------------------------------------------------
// native consumer workload
// ---------------------------------------------------------------------------
#include <atomic>
#include <chrono>
#include <deque>
#include <mutex>
#include <thread>
#include <unordered_map>

#include "../../include/gale.h"

namespace {

// splitmix64 (Steele, Lea, Flood 2014): per-thread uniform doubles
struct Rng {
    uint64_t s;
    uint64_t next() {
        uint64_t z = (s += 0x9E3779B97F4A7C15ull);
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        return z ^ (z >> 31);
    }
    double uniform() { return (double)(next() >> 11) * (1.0 / 9007199254740992.0); }
};

uint64_t fnv1a(uint64_t h, const void *p, size_t n) {
    const unsigned char *b = (const unsigned char *)p;
    for (size_t i = 0; i < n; ++i) {
        h ^= b[i];
        h *= 0x100000001B3ull;
    }
    return h;
}

}  // namespace

extern "C" int32_t gale_consumer_run(gale_ctx *ctx, const gale_consumer_cfg *cfg, gale_consumer_result *out) {
    if (!ctx || !cfg || !out || cfg->threads < 1 || cfg->n_order < 0 || (cfg->n_order > 0 && !cfg->cluster_order) ||
        !cfg->tets || !cfg->field || (cfg->rel_mask & 3u) != 3u)
        return GALE_EINVAL;
    std::memset(out, 0, sizeof(*out));
    const int kmax = 64;
    std::vector<double> cdf(kmax);
    {
        double tot = 0.0;
        for (int k = 1; k <= kmax; ++k) tot += 1.0 / std::pow((double)k, cfg->zipf_s);
        double acc = 0.0;
        for (int k = 1; k <= kmax; ++k) {
            acc += 1.0 / std::pow((double)k, cfg->zipf_s);
            cdf[k - 1] = acc / tot;
        }
    }
    std::atomic<int32_t> cursor{0};
    std::mutex mu;
    std::unordered_map<int32_t, uint64_t> first;
    std::vector<std::vector<double>> lat(cfg->threads);
    std::atomic<int32_t> first_error{0};
    uint64_t acc_all = 0, re_all = 0, mis_all = 0, err_all = 0;
    uint64_t cp_all[4] = {0, 0, 0, 0};

    auto worker = [&](int tid) {
        Rng rng{cfg->seed * 0x100000001B3ull + (uint64_t)tid * 0x9E3779B97F4A7C15ull + 1};
        std::deque<int32_t> recent;
        std::vector<int32_t> labels;
        uint64_t acc = 0, re = 0, mis = 0, err = 0;
        uint64_t cp[4] = {0, 0, 0, 0};
        while (true) {
            const double u = rng.uniform();
            int k = (int)(std::upper_bound(cdf.begin(), cdf.end(), u) - cdf.begin()) + 1;
            if (k > kmax) k = kmax;
            int32_t c;
            if (k >= 2 && (int)recent.size() >= k - 1) {
                c = recent[recent.size() - (size_t)(k - 1)];
                ++re;
            } else {
                const int32_t i = cursor.fetch_add(1);
                if (i >= cfg->n_order) break;
                c = cfg->cluster_order[i];
            }
            const auto t0 = std::chrono::steady_clock::now();
            uint64_t tk = 0;
            gale_status s = gale_submit(ctx, &c, 1, cfg->rel_mask, &tk);
            while (s == GALE_EAGAIN) {  // serving queue full: retry shortly
                std::this_thread::sleep_for(std::chrono::microseconds(20));
                s = gale_submit(ctx, &c, 1, cfg->rel_mask, &tk);
            }
            if (s == GALE_OK) s = gale_poll(ctx, tk, -1);
            const auto t1 = std::chrono::steady_clock::now();
            gale_csr vt{}, vv{};
            if (s == GALE_OK) s = gale_block(ctx, tk, c, GALE_REL_VT, &vt);
            if (s == GALE_OK) s = gale_block(ctx, tk, c, GALE_REL_VV, &vv);
            if (s == GALE_OK) {
                labels.resize((size_t)vt.nrows);
                const int32_t cs = gale_lowerstar_classify(vt.nrows, vt.row_ids, vt.offsets, vt.entries, vv.offsets,
                                                           vv.entries, cfg->tets, cfg->nt, cfg->field, cfg->nv,
                                                           labels.data());
                if (cs != 0) s = GALE_EINVAL;
            }
            if (s == GALE_OK) {
                lat[tid].push_back(std::chrono::duration<double, std::micro>(t1 - t0).count());
                uint64_t h = fnv1a(0xCBF29CE484222325ull, vt.row_ids, (size_t)vt.nrows * 4);
                h = fnv1a(h, labels.data(), labels.size() * 4);
                bool fresh = false;
                {
                    std::lock_guard<std::mutex> g(mu);
                    auto it = first.find(c);
                    if (it == first.end()) {
                        first.emplace(c, h);
                        fresh = true;
                    } else if (it->second != h) {
                        ++mis;
                    }
                }
                if (fresh)
                    for (int32_t l : labels) cp[l & 3]++;
                ++acc;
            } else {
                ++err;
                int32_t z = 0;
                first_error.compare_exchange_strong(z, s);
            }
            if (tk) (void)gale_release(ctx, tk);
            recent.push_back(c);
            if (recent.size() > (size_t)kmax) recent.pop_front();
        }
        std::lock_guard<std::mutex> g(mu);
        acc_all += acc;
        re_all += re;
        mis_all += mis;
        err_all += err;
        for (int i = 0; i < 4; ++i) cp_all[i] += cp[i];
    };
    const auto w0 = std::chrono::steady_clock::now();
    std::vector<std::thread> th;
    for (int i = 0; i < cfg->threads; ++i) th.emplace_back(worker, i);
    for (auto &t : th) t.join();
    out->wall_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - w0).count();
    std::vector<double> all;
    for (auto &v : lat) all.insert(all.end(), v.begin(), v.end());
    std::sort(all.begin(), all.end());
    auto pct = [&](double q) -> double {
        if (all.empty()) return 0.0;
        const size_t i = (size_t)std::min<double>((double)all.size() - 1, std::floor(q * (double)(all.size() - 1) + 0.5));
        return all[i];
    };
    out->accesses = acc_all;
    out->reaccesses = re_all;
    out->mismatches = mis_all;
    out->errors = err_all;
    out->clusters = first.size();
    out->regular = cp_all[GALE_CP_REGULAR];
    out->minima = cp_all[GALE_CP_MINIMUM];
    out->maxima = cp_all[GALE_CP_MAXIMUM];
    out->saddles = cp_all[GALE_CP_SADDLE];
    out->lat_p50_us = pct(0.50);
    out->lat_p99_us = pct(0.99);
    double sum = 0.0;
    for (double x : all) sum += x;
    out->lat_mean_us = all.empty() ? 0.0 : sum / (double)all.size();
    out->lat_max_us = all.empty() ? 0.0 : all.back();
    out->first_error = first_error.load();
    return GALE_OK;
}
