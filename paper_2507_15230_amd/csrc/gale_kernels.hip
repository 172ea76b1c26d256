// gale_kernels.hip -- per-cluster VT / VV / TT builders for gfx950.
//
// One workgroup builds every requested relation of one cluster (the paper
// assigns one GPU block per segment, Section 4.6).  The cluster's stream of
// star and halo tetrahedra is read from HBM once and, when the working set
// fits, staged in LDS as 4 x uint16 local vertex ids; all later passes read it
// from LDS.  Working arrays live in LDS (fast path) or, for clusters too large
// for the LDS budget, in a per-workgroup slice of global memory (same
// algorithm, 32-bit types).
//
// All three relations are read from one structure built first: the local VT
// relation of every vertex of the cluster's local table (count per vertex with
// LDS atomics, inclusive scan, scatter of stream positions with atomic
// decrements).  No global atomics are used (the paper's VT kernel is limited
// by atomics on one vertex, Appendix A.1).
//
// VT (Section 4.6: iterate the segment's tetrahedra, take the vertices in the
// segment, relate them): a row's list, sorted; stream order is tetrahedron id
// order, so the sorted positions are the canonical row.
//
// VV (Algorithm 1: for each tetrahedron and each of its vertices in the
// segment, relate the other three, without duplicates): a wave takes one row
// at a time and sets bits in its own LDS bitmap over the local vertex table;
// the table is in original id order, so reading the set bits in word order
// yields the row sorted and duplicate-free.  This replaces the paper's
// fixed-width -1 initialised matrix and atomicPush (Algorithm 2), whose output
// order depends on thread arrival.  Counts first, then emission, so offsets
// are known before any entry is written.
//
// TT (two tetrahedra are adjacent iff they share a triangle, Section 2.2):
// every tetrahedron holding face {a,b,c} of an internal tetrahedron is in the
// local VT lists of a, b and c.  The four faces of t = (x,y,z,w) hold either
// edge xy or edge zw, so a thread scans one list per edge, keeps the
// tetrahedra holding the edge and assigns them to faces by the two other
// vertices.  More than four raw neighbours (a face shared by three or more
// tetrahedra) switches the cluster to exhaustive pairing.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <type_traits>

#include "gale_layout.h"

namespace gale {

constexpr int32_t kIdMask = 0x7fffffff;

#ifdef GALE_PHASE_TIMING
__device__ unsigned long long g_phase_cycles[32];
#define PHASE_MARK(k)                                                              \
    do {                                                                           \
        __syncthreads();                                                           \
        if (threadIdx.x == 0) {                                                    \
            const unsigned long long now = __builtin_amdgcn_s_memtime();          \
            atomicAdd(&g_phase_cycles[(k)], now - phase_t0);                       \
            phase_t0 = now;                                                        \
        }                                                                          \
    } while (0)
#else
#define PHASE_MARK(k) \
    do {              \
    } while (0)
#endif

// ---------------------------------------------------------------------------
// workgroup exclusive scan (wave64 shuffles + one LDS word per wave)
// ---------------------------------------------------------------------------
template <int B>
__device__ __forceinline__ int block_excl_scan(int v, int &total) {
    __shared__ int s_wave[B / 64 + 1];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    int x = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        int y = __shfl_up(x, d, 64);
        if (lane >= d) x += y;
    }
    if (lane == 63) s_wave[wid] = x;
    __syncthreads();
    if (threadIdx.x == 0) {
        int s = 0;
        for (int w = 0; w < B / 64; ++w) {
            int t = s_wave[w];
            s_wave[w] = s;
            s += t;
        }
        s_wave[B / 64] = s;
    }
    __syncthreads();
    const int res = x - v + s_wave[wid];
    total = s_wave[B / 64];
    __syncthreads();
    return res;
}

// ---------------------------------------------------------------------------
// faces
// ---------------------------------------------------------------------------
__device__ __forceinline__ void cswap(int &x, int &y) {
    int lo = min(x, y), hi = max(x, y);
    x = lo;
    y = hi;
}

__device__ __forceinline__ int shared_vertices(int4 t, int4 u) {
    int c = 0;
    c += (t.x == u.x) | (t.x == u.y) | (t.x == u.z) | (t.x == u.w);
    c += (t.y == u.x) | (t.y == u.y) | (t.y == u.z) | (t.y == u.w);
    c += (t.z == u.x) | (t.z == u.y) | (t.z == u.z) | (t.z == u.w);
    c += (t.w == u.x) | (t.w == u.y) | (t.w == u.z) | (t.w == u.w);
    return c;
}

// ---------------------------------------------------------------------------
// small helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ void wave_fence() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

__device__ __forceinline__ int wave_sum(int x) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) x += __shfl_xor(x, d, 64);
    return x;
}

__device__ __forceinline__ int wave_excl_scan(int v, int &total) {
    const int lane = threadIdx.x & 63;
    int x = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const int y = __shfl_up(x, d, 64);
        if (lane >= d) x += y;
    }
    total = __shfl(x, 63, 64);
    return x - v;
}

__device__ __forceinline__ bool has_vertex(int4 t, int u) {
    return t.x == u || t.y == u || t.z == u || t.w == u;
}

__device__ __forceinline__ void cswap_u(uint32_t &x, uint32_t &y) {
    const uint32_t lo = min(x, y), hi = max(x, y);
    x = lo;
    y = hi;
}

// Sort a[0..n) ascending in place; n <= 32 through a register bitonic network,
// longer runs by insertion.
template <typename T>
__device__ __forceinline__ void sort_run(T *a, int n) {
    if (n <= 1) return;
    if (n <= 32) {
        uint32_t v[32];
#pragma unroll
        for (int i = 0; i < 32; ++i) v[i] = i < n ? (uint32_t)a[i] : 0xFFFFFFFFu;
#pragma unroll
        for (int k = 2; k <= 32; k <<= 1) {
#pragma unroll
            for (int j = k >> 1; j > 0; j >>= 1) {
#pragma unroll
                for (int i = 0; i < 32; ++i) {
                    const int l = i ^ j;
                    if (l > i) {
                        if ((i & k) == 0)
                            cswap_u(v[i], v[l]);
                        else
                            cswap_u(v[l], v[i]);
                    }
                }
            }
        }
#pragma unroll
        for (int i = 0; i < 32; ++i)
            if (i < n) a[i] = (T)v[i];
        return;
    }
    for (int i = 1; i < n; ++i) {
        const T x = a[i];
        int j = i - 1;
        while (j >= 0 && a[j] > x) {
            a[j + 1] = a[j];
            --j;
        }
        a[j + 1] = x;
    }
}

// ---------------------------------------------------------------------------
// one cluster
// ---------------------------------------------------------------------------
// The local VT relation of every vertex in the cluster's local table is built
// first (count, scan, scatter of stream positions); it is the one structure
// the three relations are read from:
//   VT  a row's list, sorted (stream order is tetrahedron id order);
//   VV  the union of the vertices of a row's tetrahedra, through a bitmap over
//       the local table, which is in original id order;
//   TT  the tetrahedra sharing a face of an internal tetrahedron all lie in
//       the list of each of the face's vertices: scan the shortest one.
template <int B, bool kL>
__device__ void build_cluster(const KArgs &a, const WorkItem &it, const ClusterMeta &m, const Plan &pl,
                              char *smem, char *ws) {
    using PosT = typename std::conditional<kL, uint16_t, int32_t>::type;
    using LidT = typename std::conditional<kL, uint16_t, int32_t>::type;
    constexpr int NW = B / 64;

    __shared__ int s_status;
    __shared__ int s_fail;
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int ns = m.ns, nh = m.nh, ntot = ns + nh, nT = m.nT, L = m.L, nV = m.nV;
    const uint32_t mask = it.mask;
    const char *tb = a.s.tets + m.tb_off;
    const bool wide = (m.flags & kMetaWide) != 0;
    const int32_t *idg = a.s.tid + m.tet_off;
    const int32_t *lvg = a.s.lverts + m.lv_off;
    int32_t *blk = a.out + it.out_word;
    const BlockLayout lay = block_layout(mask, nV, nT, m.nnzVT, it.cap_vv, it.cap_tt);
    char *base = kL ? smem : ws;

    ushort4 *lt = reinterpret_cast<ushort4 *>(smem + pl.lt);
    unsigned long long *ib = reinterpret_cast<unsigned long long *>(base + pl.ib);
    int32_t *ibp = reinterpret_cast<int32_t *>(base + pl.ibp);
    int32_t *cnt = reinterpret_cast<int32_t *>(base + pl.cnt);
    PosT *lvt = reinterpret_cast<PosT *>(base + pl.lvt);
    LidT *rowl = reinterpret_cast<LidT *>(base + pl.rowl);
    uint32_t *wbm = reinterpret_cast<uint32_t *>(base + pl.wbm);

    if (tid == 0) {
        s_status = 0;
        s_fail = 0;
    }
#ifdef GALE_PHASE_TIMING
    unsigned long long phase_t0 = __builtin_amdgcn_s_memtime();
#endif

    auto tet = [&](int p) -> int4 {
        if constexpr (kL) {
            const ushort4 q = lt[p];
            return make_int4(q.x, q.y, q.z, q.w);
        } else {
            if (wide) return reinterpret_cast<const int4 *>(tb)[p];
            const ushort4 q = reinterpret_cast<const ushort4 *>(tb)[p];
            return make_int4(q.x, q.y, q.z, q.w);
        }
    };
    auto internal = [&](int p) -> bool { return p < ns && ((ib[p >> 6] >> (p & 63)) & 1ull); };

    // ---- stage the stream in LDS; zero the local VT counters --------------
    if constexpr (kL) {
        // the LDS path only takes 4 x uint16 streams; copy 16 B (two tetrahedra)
        // per load, the stream and lt both padded to 16 B
        constexpr int U = 8;
        const int nq = (ntot + 1) >> 1;
        const uint4 *src = reinterpret_cast<const uint4 *>(tb);
        uint4 *dst = reinterpret_cast<uint4 *>(lt);
        for (int i0 = 0; i0 < nq; i0 += B * U) {
            uint4 t[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int i = i0 + u * B + tid;
                t[u] = i < nq ? src[i] : make_uint4(0u, 0u, 0u, 0u);
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int i = i0 + u * B + tid;
                if (i < nq) dst[i] = t[u];
            }
        }
    }
    if (mask & kRelTT) {
        const int nwords = (ns + 63) >> 6;
        for (int w = wave; w < nwords; w += NW) {
            const int p = w * 64 + lane;
            const bool f = p < ns && idg[p] < 0;
            const unsigned long long bits = __ballot(f);
            if (lane == 0) ib[w] = bits;
        }
    }
    for (int v = tid; v <= L; v += B) cnt[v] = 0;

    // rows: local id of each row, row ids of the block
    if (mask & (kRelVT | kRelVV)) {
        int carry = 0;
        for (int i0 = 0; i0 < L; i0 += B) {
            const int i = i0 + tid;
            const int32_t lv = i < L ? lvg[i] : 0;
            const int f = (i < L && lv < 0) ? 1 : 0;
            int tot;
            const int ex = block_excl_scan<B>(f, tot);
            if (f) {
                const int r = carry + ex;
                if (r < nV) {
                    rowl[r] = (LidT)i;
                    blk[lay.vrows + r] = lv & kIdMask;
                }
            }
            carry += tot;
        }
        if (tid == 0 && carry != nV) s_status |= kStInconsistent;
    }
    __syncthreads();
    if (mask & kRelTT) {
        // internal tetrahedra before each flag word: TT row index of a tetrahedron
        const int nwords = (ns + 63) >> 6;
        int carry = 0;
        for (int w0 = 0; w0 < nwords; w0 += B) {
            const int w = w0 + tid;
            const int x = w < nwords ? __popcll(ib[w]) : 0;
            int tot;
            const int ex = block_excl_scan<B>(x, tot);
            if (w < nwords) ibp[w] = carry + ex;
            carry += tot;
        }
        if (tid == 0 && carry != nT) s_status |= kStInconsistent;
    }
    PHASE_MARK(0);

    // ---- local VT over every local vertex ---------------------------------
    for (int p = tid; p < ntot; p += B) {
        const int4 t = tet(p);
        atomicAdd(&cnt[t.x], 1);
        atomicAdd(&cnt[t.y], 1);
        atomicAdd(&cnt[t.z], 1);
        atomicAdd(&cnt[t.w], 1);
    }
    __syncthreads();
    PHASE_MARK(1);
    {
        int carry = 0;
        for (int v0 = 0; v0 < L; v0 += B) {
            const int v = v0 + tid;
            const int x = v < L ? cnt[v] : 0;
            int tot;
            const int ex = block_excl_scan<B>(x, tot);
            if (v < L) cnt[v] = carry + ex + x;  // end of the list
            carry += tot;
        }
        if (tid == 0) {
            cnt[L] = carry;
            if (carry != 4 * ntot) s_status |= kStInconsistent;
        }
    }
    __syncthreads();
    PHASE_MARK(2);
    for (int p = tid; p < ntot; p += B) {
        const int4 t = tet(p);
        lvt[atomicSub(&cnt[t.x], 1) - 1] = (PosT)p;
        lvt[atomicSub(&cnt[t.y], 1) - 1] = (PosT)p;
        lvt[atomicSub(&cnt[t.z], 1) - 1] = (PosT)p;
        lvt[atomicSub(&cnt[t.w], 1) - 1] = (PosT)p;
    }
    __syncthreads();  // cnt[v] = start of v's list, cnt[v+1] = its end
    PHASE_MARK(3);

    // ---- VT ----------------------------------------------------------------
    if (mask & kRelVT) {
        for (int r = tid; r < nV; r += B) {
            const int u = rowl[r];
            const int s0 = cnt[u];
            sort_run(lvt + s0, cnt[u + 1] - s0);
        }
        __syncthreads();
        PHASE_MARK(4);
        int carry = 0;
        for (int r0 = 0; r0 < nV; r0 += B) {
            const int r = r0 + tid;
            int u = 0, s0 = 0, n = 0;
            if (r < nV) {
                u = rowl[r];
                s0 = cnt[u];
                n = cnt[u + 1] - s0;
            }
            int tot;
            const int ex = block_excl_scan<B>(n, tot);
            if (r < nV) {
                const int o = carry + ex;
                if (o + n <= m.nnzVT) {
                    blk[lay.vt_off + r] = o;
                    int j = 0;
                    for (; j + 4 <= n; j += 4) {
                        const int32_t a0 = idg[lvt[s0 + j]], a1 = idg[lvt[s0 + j + 1]];
                        const int32_t a2 = idg[lvt[s0 + j + 2]], a3 = idg[lvt[s0 + j + 3]];
                        blk[lay.vt_ent + o + j] = a0 & kIdMask;
                        blk[lay.vt_ent + o + j + 1] = a1 & kIdMask;
                        blk[lay.vt_ent + o + j + 2] = a2 & kIdMask;
                        blk[lay.vt_ent + o + j + 3] = a3 & kIdMask;
                    }
                    for (; j < n; ++j) blk[lay.vt_ent + o + j] = idg[lvt[s0 + j]] & kIdMask;
                }
            }
            carry += tot;
        }
        if (tid == 0) {
            blk[lay.vt_off + nV] = carry;
            if (carry != m.nnzVT) s_status |= kStInconsistent;
        }
        __syncthreads();
        PHASE_MARK(5);
    }

    // ---- VV: one row at a time per group of B/32 lanes, bitmap over the local table
    if (mask & kRelVV) {
        constexpr int NG = 32;
        constexpr int G = B / NG;
        const int W = pl.W;
        const int grp = tid / G, gl = tid % G;
        uint32_t *wb = wbm + (int64_t)grp * W;
        const int cap = it.cap_vv;
        for (int w = gl; w < W; w += G) wb[w] = 0u;
        wave_fence();
        auto set_row_bits = [&](int self, int s0, int e0) {
            for (int i = s0 + gl; i < e0; i += G) {
                const int4 t = tet(lvt[i]);
                if (t.x != self) atomicOr(&wb[t.x >> 5], 1u << (t.x & 31));
                if (t.y != self) atomicOr(&wb[t.y >> 5], 1u << (t.y & 31));
                if (t.z != self) atomicOr(&wb[t.z >> 5], 1u << (t.z & 31));
                if (t.w != self) atomicOr(&wb[t.w >> 5], 1u << (t.w & 31));
            }
            wave_fence();
        };
        // pass 1: counts
        for (int r = grp; r < nV; r += NG) {
            const int u = rowl[r];
            set_row_bits(u, cnt[u], cnt[u + 1]);
            int c = 0;
            for (int w = gl; w < W; w += G) {
                c += __popc(wb[w]);
                wb[w] = 0u;
            }
#pragma unroll
            for (int d = G / 2; d >= 1; d >>= 1) c += __shfl_xor(c, d, G);
            if (gl == 0) blk[lay.vv_off + r] = c;  // the count, turned into the offset below
            wave_fence();
        }
        __syncthreads();
        PHASE_MARK(6);
        int carry = 0;
        for (int r0 = 0; r0 < nV; r0 += B) {
            const int r = r0 + tid;
            const int x = r < nV ? blk[lay.vv_off + r] : 0;
            int tot;
            const int ex = block_excl_scan<B>(x, tot);
            if (r < nV) blk[lay.vv_off + r] = carry + ex;
            carry += tot;
        }
        if (tid == 0) {
            blk[lay.vv_off + nV] = carry;
            blk[4] = carry;
            if (carry > cap) s_status |= kStVVOverflow;
        }
        __syncthreads();
        // pass 2: emit local ids in word order (ascending original id) ...
        if (carry <= cap) {
            for (int r = grp; r < nV; r += NG) {
                const int u = rowl[r];
                set_row_bits(u, cnt[u], cnt[u + 1]);
                int o = blk[lay.vv_off + r];
                for (int w0 = 0; w0 < W; w0 += G) {
                    const int w = w0 + gl;
                    uint32_t bits = 0u;
                    if (w < W) {
                        bits = wb[w];
                        wb[w] = 0u;
                    }
                    const int n = __popc(bits);
                    int x = n;
#pragma unroll
                    for (int d = 1; d < G; d <<= 1) {
                        const int y = __shfl_up(x, d, G);
                        if (gl >= d) x += y;
                    }
                    const int tot = __shfl(x, G - 1, G);
                    int pos = o + x - n;
                    while (bits) {
                        const int b = __ffs(bits) - 1;
                        bits &= bits - 1u;
                        blk[lay.vv_ent + pos] = w * 32 + b;
                        ++pos;
                    }
                    o += tot;
                }
                wave_fence();
            }
            __syncthreads();
            // ... then map local ids to original ids in one flat pass
            constexpr int U = 4;
            for (int e0 = 0; e0 < carry; e0 += B * U) {
                int32_t l[U];
#pragma unroll
                for (int uu = 0; uu < U; ++uu) {
                    const int e = e0 + uu * B + tid;
                    l[uu] = e < carry ? blk[lay.vv_ent + e] : 0;
                }
#pragma unroll
                for (int uu = 0; uu < U; ++uu) l[uu] = lvg[l[uu]];
#pragma unroll
                for (int uu = 0; uu < U; ++uu) {
                    const int e = e0 + uu * B + tid;
                    if (e < carry) blk[lay.vv_ent + e] = l[uu] & kIdMask;
                }
            }
        }
        __syncthreads();
        PHASE_MARK(7);
    }

    // ---- TT ----------------------------------------------------------------
    // Every internal tetrahedron finds its neighbours independently and writes
    // them, sorted, into its own provisional window of four entries (row r at
    // 4r; the capacity is at least 4 per row) with the count in tt_off[r]; one
    // scan then gives the offsets and the rows are moved down in place.
    if (mask & kRelTT) {
        const int cap = it.cap_tt;
        const bool room = cap >= 4 * nT;  // the host always sizes TT for at least 4 per row
        for (int p = tid; p < ns && room; p += B) {
            if (!internal(p)) continue;
            const int row = ibp[p >> 6] + __popcll(ib[p >> 6] & ((1ull << (p & 63)) - 1ull));
            int q0 = -1, q1 = -1, q2 = -1, q3 = -1;
            int raw = 0;
            {
                const int4 t = tet(p);
                // Faces omitting t.z or t.w both hold the edge (t.x, t.y); faces
                // omitting t.x or t.y both hold (t.z, t.w).  The tetrahedra
                // around an edge are the entries of one endpoint's list that hold
                // the other endpoint: scan the shorter list of each edge, keep
                // those, and sort them to faces by the remaining two vertices.
                const int sx = cnt[t.x], ex = cnt[t.x + 1], sy = cnt[t.y], ey = cnt[t.y + 1];
                const int sz = cnt[t.z], ez = cnt[t.z + 1], sw = cnt[t.w], ew = cnt[t.w + 1];
                // branch-free selects keep the four slots in registers
                auto record = [&](int q) {
                    q0 = raw == 0 ? q : q0;
                    q1 = raw == 1 ? q : q1;
                    q2 = raw == 2 ? q : q2;
                    q3 = raw == 3 ? q : q3;
                    ++raw;
                };
                auto edge = [&](int st, int en, int other, int f0, int f1) {
                    auto visit = [&](int q, int4 tq) {
                        if (q != p && has_vertex(tq, other)) {
                            if (has_vertex(tq, f0)) record(q);
                            if (has_vertex(tq, f1)) record(q);
                        }
                    };
                    int i = st;
                    for (; i + 4 <= en; i += 4) {
                        const int qa = lvt[i], qb = lvt[i + 1], qc = lvt[i + 2], qd = lvt[i + 3];
                        const int4 ta = tet(qa), tb2 = tet(qb), tc = tet(qc), td = tet(qd);
                        visit(qa, ta);
                        visit(qb, tb2);
                        visit(qc, tc);
                        visit(qd, td);
                    }
                    for (; i < en; ++i) {
                        const int q = lvt[i];
                        visit(q, tet(q));
                    }
                };
                if (ex - sx <= ey - sy) edge(sx, ex, t.y, t.z, t.w);
                else edge(sy, ey, t.x, t.z, t.w);
                if (ez - sz <= ew - sw) edge(sz, ez, t.w, t.x, t.y);
                else edge(sw, ew, t.z, t.x, t.y);
                if (raw > 4) s_fail = 1;  // a face shared by three or more tetrahedra: exhaustive path
            }
            int n0 = q0 >= 0 ? idg[q0] & kIdMask : 0x7fffffff;
            int n1 = q1 >= 0 ? idg[q1] & kIdMask : 0x7fffffff;
            int n2 = q2 >= 0 ? idg[q2] & kIdMask : 0x7fffffff;
            int n3 = q3 >= 0 ? idg[q3] & kIdMask : 0x7fffffff;
            cswap(n0, n1); cswap(n2, n3); cswap(n0, n2); cswap(n1, n3); cswap(n1, n2);
            // a duplicated tetrahedron is reached through several faces: list it once
            if (n3 == n2) n3 = 0x7fffffff;
            if (n2 == n1) { n2 = n3; n3 = 0x7fffffff; }
            if (n1 == n0) { n1 = n2; n2 = n3; n3 = 0x7fffffff; }
            const int c = (n0 != 0x7fffffff) + (n1 != 0x7fffffff) + (n2 != 0x7fffffff) + (n3 != 0x7fffffff);
            if (row < nT && room) {
                blk[lay.trows + row] = idg[p] & kIdMask;
                blk[lay.tt_off + row] = c;
                int32_t *w = blk + lay.tt_ent + 4 * (int64_t)row;
                if (c > 0) w[0] = n0;
                if (c > 1) w[1] = n1;
                if (c > 2) w[2] = n2;
                if (c > 3) w[3] = n3;
            }
        }
        __syncthreads();
        int rcarry = nT, ecarry = 0;
        const bool exhaustive = s_fail || !room;
        if (!exhaustive) {
            for (int r0 = 0; r0 < nT; r0 += B) {
                const int r = r0 + tid;
                int c = 0, e0 = 0, e1 = 0, e2 = 0, e3 = 0;
                if (r < nT) {
                    c = blk[lay.tt_off + r];
                    const int32_t *w = blk + lay.tt_ent + 4 * (int64_t)r;
                    if (c > 0) e0 = w[0];
                    if (c > 1) e1 = w[1];
                    if (c > 2) e2 = w[2];
                    if (c > 3) e3 = w[3];
                }
                int tot;
                const int ex = block_excl_scan<B>(c, tot);  // its barriers order every read before the writes
                if (r < nT) {
                    const int o = ecarry + ex;
                    blk[lay.tt_off + r] = o;
                    int32_t *w = blk + lay.tt_ent + o;
                    if (c > 0) w[0] = e0;
                    if (c > 1) w[1] = e1;
                    if (c > 2) w[2] = e2;
                    if (c > 3) w[3] = e3;
                }
                ecarry += tot;
            }
        }
        __syncthreads();
        PHASE_MARK(8);
        if (exhaustive) {
            // exhaustive pairing, rows rebuilt from scratch (non-manifold faces)
            if (tid == 0) s_status |= kStTTFallback;
            rcarry = 0;
            ecarry = 0;
            for (int p0 = 0; p0 < ns; p0 += B) {
                const int p = p0 + tid;
                const bool in = internal(p);
                int c = 0;
                int4 t = make_int4(0, 0, 0, 0);
                if (in) {
                    t = tet(p);
                    for (int q = 0; q < ntot; ++q)
                        if (q != p && shared_vertices(t, tet(q)) >= 3) ++c;
                }
                int rtot, etot;
                const int rex = block_excl_scan<B>(in ? 1 : 0, rtot);
                const int eex = block_excl_scan<B>(c, etot);
                if (in) {
                    const int row = rcarry + rex;
                    int pos = ecarry + eex;
                    if (row < nT) {
                        blk[lay.trows + row] = idg[p] & kIdMask;
                        blk[lay.tt_off + row] = pos;
                    }
                    const int start = pos;
                    for (int q = 0; q < ntot; ++q) {
                        if (q != p && shared_vertices(t, tet(q)) >= 3) {
                            if (pos < cap) blk[lay.tt_ent + pos] = idg[q] & kIdMask;
                            ++pos;
                        }
                    }
                    // the star part and the halo part are each ascending; sort the row
                    const int end = min(pos, cap);
                    for (int i = start + 1; i < end; ++i) {
                        const int32_t x = blk[lay.tt_ent + i];
                        int j = i - 1;
                        while (j >= start && blk[lay.tt_ent + j] > x) {
                            blk[lay.tt_ent + j + 1] = blk[lay.tt_ent + j];
                            --j;
                        }
                        blk[lay.tt_ent + j + 1] = x;
                    }
                }
                rcarry += rtot;
                ecarry += etot;
            }
        }
        if (tid == 0) {
            blk[lay.tt_off + (rcarry <= nT ? rcarry : nT)] = ecarry;
            blk[5] = ecarry;
            if (rcarry != nT) s_status |= kStInconsistent;
            if (ecarry > cap) s_status |= kStTTOverflow;
        }
        PHASE_MARK(9);
    }
    __syncthreads();

    // ---- header --------------------------------------------------------
    if (tid == 0) {
        int32_t h[8];
        h[0] = s_status;
        h[1] = nV;
        h[2] = nT;
        h[3] = m.nnzVT;
        h[4] = (mask & kRelVV) ? blk[4] : 0;
        h[5] = (mask & kRelTT) ? blk[5] : 0;
        h[6] = it.cap_vv;
        h[7] = it.cap_tt;
        for (int i = 0; i < 8; ++i) blk[i] = h[i];
        if (a.hdr)
            for (int i = 0; i < 8; ++i) a.hdr[(int64_t)it.hdr_index * 8 + i] = h[i];
    }
    __syncthreads();
}

// One work item on the LDS path (kL) or the global-workspace path.  The host
// sorts items by path with the same plan functions; an item that does not
// fit what it was sent to is reported in its header and skipped.
template <int B, bool kL>
__device__ void process_item(const KArgs &a, const WorkItem &it, char *smem, char *ws) {
    const ClusterMeta m = a.s.meta[it.cluster];
    const Plan lp = lds_plan(m, it.mask, a.lds_budget, B);
    const bool ok = kL ? (lp.ok != 0) : (ws != nullptr);
    if (!ok) {
        if (threadIdx.x == 0) {
            int32_t *blk = a.out + it.out_word;
            blk[0] = kStInconsistent;
            if (a.hdr) a.hdr[(int64_t)it.hdr_index * 8] = kStInconsistent;
        }
        __syncthreads();
        return;
    }
    if constexpr (kL) {
        build_cluster<B, true>(a, it, m, lp, smem, ws);
    } else {
        const Plan gp = ws_plan(m, it.mask, B);
        build_cluster<B, false>(a, it, m, gp, smem, ws);
    }
}

// One work item per workgroup: item blockIdx.x.  Used for the per-cluster
// (plain) form, one launch per (cluster, relation).
template <int B, bool kL>
__global__ __launch_bounds__(B) void gale_items_kernel(KArgs a) {
    extern __shared__ __attribute__((aligned(16))) char smem[];
    const int i = blockIdx.x;
    if (i >= a.nitems) return;
    char *ws = a.ws ? a.ws + (int64_t)blockIdx.x * a.ws_stride : nullptr;
    process_item<B, kL>(a, a.items[i], smem, ws);
}

// Persistent form: each workgroup takes the next item from the device work
// queue until the list is exhausted (every workgroup reaches the exit test).
template <int B, bool kL>
__global__ __launch_bounds__(B) void gale_persistent_kernel(KArgs a) {
    extern __shared__ __attribute__((aligned(16))) char smem[];
    __shared__ int s_idx;
    char *ws = a.ws ? a.ws + (int64_t)blockIdx.x * a.ws_stride : nullptr;
    while (true) {
        if (threadIdx.x == 0) s_idx = atomicAdd(a.queue, 1);
        __syncthreads();
        const int idx = s_idx;
        __syncthreads();
        if (idx >= a.nitems) break;
        process_item<B, kL>(a, a.items[idx], smem, ws);
    }
}

// ---------------------------------------------------------------------------
// host-side launch wrappers
// ---------------------------------------------------------------------------
template <bool kL>
static hipError_t launch_items_t(const KArgs &a, int block_threads, int grid, size_t lds, hipStream_t st) {
    if (block_threads == 1024) {
        hipLaunchKernelGGL((gale_items_kernel<1024, kL>), dim3(grid), dim3(1024), lds, st, a);
    } else if (block_threads == 512) {
        hipLaunchKernelGGL((gale_items_kernel<512, kL>), dim3(grid), dim3(512), lds, st, a);
    } else {
        hipLaunchKernelGGL((gale_items_kernel<256, kL>), dim3(grid), dim3(256), lds, st, a);
    }
    return hipGetLastError();
}

template <bool kL>
static hipError_t launch_persistent_t(const KArgs &a, int block_threads, int grid, size_t lds, hipStream_t st) {
    if (block_threads == 1024) {
        hipLaunchKernelGGL((gale_persistent_kernel<1024, kL>), dim3(grid), dim3(1024), lds, st, a);
    } else if (block_threads == 512) {
        hipLaunchKernelGGL((gale_persistent_kernel<512, kL>), dim3(grid), dim3(512), lds, st, a);
    } else {
        hipLaunchKernelGGL((gale_persistent_kernel<256, kL>), dim3(grid), dim3(256), lds, st, a);
    }
    return hipGetLastError();
}

hipError_t launch_items(const KArgs &a, bool lds_path, int block_threads, int grid, size_t lds, hipStream_t st) {
    return lds_path ? launch_items_t<true>(a, block_threads, grid, lds, st)
                    : launch_items_t<false>(a, block_threads, grid, 0, st);
}

hipError_t launch_persistent(const KArgs &a, bool lds_path, int block_threads, int grid, size_t lds,
                             hipStream_t st) {
    return lds_path ? launch_persistent_t<true>(a, block_threads, grid, lds, st)
                    : launch_persistent_t<false>(a, block_threads, grid, 0, st);
}

hipError_t set_lds_limits(size_t lds) {
    const void *fns[] = {
        (const void *)gale_items_kernel<256, true>,       (const void *)gale_items_kernel<512, true>,
        (const void *)gale_items_kernel<1024, true>,      (const void *)gale_persistent_kernel<256, true>,
        (const void *)gale_persistent_kernel<512, true>,  (const void *)gale_persistent_kernel<1024, true>,
    };
    for (const void *f : fns) {
        const hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

#ifdef GALE_PHASE_TIMING
extern "C" int gale_debug_phase_cycles(unsigned long long *out, int reset) {
    hipError_t e = hipMemcpyFromSymbol(out, HIP_SYMBOL(g_phase_cycles), sizeof(g_phase_cycles));
    if (reset) {
        unsigned long long z[32] = {0};
        hipMemcpyToSymbol(HIP_SYMBOL(g_phase_cycles), z, sizeof(z));
    }
    return (int)e;
}
#endif

hipError_t persistent_occupancy(int block_threads, bool lds_path, size_t lds, int *blocks_per_cu) {
    if (lds_path) {
        if (block_threads == 1024)
            return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, gale_persistent_kernel<1024, true>, 1024, lds);
        if (block_threads == 512)
            return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, gale_persistent_kernel<512, true>, 512, lds);
        return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, gale_persistent_kernel<256, true>, 256, lds);
    }
    if (block_threads == 1024)
        return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, gale_persistent_kernel<1024, false>, 1024, 0);
    if (block_threads == 512)
        return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, gale_persistent_kernel<512, false>, 512, 0);
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, gale_persistent_kernel<256, false>, 256, 0);
}

}  // namespace gale
