// gale_kernels.hip -- per-cluster VT / VV / TT builders for gfx950.
//
// One workgroup builds every requested relation of one cluster (the paper
// assigns one GPU block per segment, Section 4.6); a persistent launch takes
// clusters from a device queue.  The working arrays of a cluster live in one
// of three places, chosen per cluster by the host with the plan functions of
// gale_layout.h:
//   LDS path     everything in LDS, the stream staged there as 4 x uint16
//                local vertex ids; 16-bit ids, positions and cells;
//   hybrid path  (global path, LDS plan too large) the face table, lower-
//                cluster bits, row index, row ids, VT counts and VV bitmaps
//                in LDS, the partner cells and local VT lists in a
//                per-workgroup slice of global memory, the stream read from
//                global memory;
//   global path  every array in the workspace slice (32-bit types).
//
// VT and VV are read from one structure: the local VT relation of every row
// of the cluster (count per vertex with LDS atomics, scan, scatter with
// atomic decrements).  No global atomics on the VT counts (the paper's VT
// kernel is limited by atomics on one vertex, Appendix A.1).
//
// VT (Section 4.6: iterate the segment's tetrahedra, take the vertices in the
// segment, relate them): a row's list sorted by original tetrahedron id, by
// register sorting networks (a thread per row up to 32 entries, a wave per
// row beyond).
//
// VV (Algorithm 1: for each tetrahedron and each of its vertices in the
// segment, relate the other three, without duplicates): a group of 8, 16 or 32
// lanes takes one row at a time and sets bits in its own LDS bitmap over the
// local vertex table; the table is in original id order, so reading the set
// bits in word order yields the row sorted and duplicate-free.  This replaces
// the paper's fixed-width -1 initialised matrix and atomicPush (Algorithm 2),
// whose output order depends on thread arrival.  Counts first, then emission,
// so offsets are known before any entry is written.
//
// TT (two tetrahedra are adjacent iff they share a triangle, Section 2.2):
// a hash table keyed by the triangle (its three local ids, sorted).
// Internal tetrahedra insert their four faces; the second to insert a face
// pairs the two and writes each into the other's partner cell for that face.
// The remaining stream tetrahedra then look their faces up and write
// themselves into the internal partner's cell.  A face met a third time
// (non-manifold) switches the cluster to chain pairing: the table is built
// again with each face's internal tetrahedra linked through their partner
// cells, and every row takes the whole chain of each of its faces (linear in
// the stream and the entries).  When the table is smaller than the faces, the
// faces are split by hash into passes.  TT runs before the local VT is built
// and shares its LDS region.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <type_traits>

#include "gale_devutil.h"
#include "gale_layout.h"

namespace gale {

constexpr int32_t kIdMask = 0x7fffffff;   // tetrahedron id (bit 31: internal)
constexpr int32_t kVidMask = 0x3fffffff;  // vertex id (bit 31: row, bit 30: lower cluster)

#ifdef GALE_PHASE_TIMING
__device__ unsigned long long g_phase_cycles[48];
// wave-level event counters (phase-timing builds only): slot k += 1 once per
// wave that reaches the mark with at least one active lane
#define WAVE_COUNT(k)                                                                      \
    do {                                                                                   \
        const unsigned long long act_ = __ballot(1);                                       \
        if ((int)(threadIdx.x & 63) == __ffsll((long long)act_) - 1)                       \
            atomicAdd(&g_phase_cycles[(k)], 1ull);                                         \
    } while (0)
#define PHASE_MARK(k)                                                              \
    do {                                                                           \
        __syncthreads();                                                           \
        if (threadIdx.x == 0) {                                                    \
            const unsigned long long now = __builtin_amdgcn_s_memtime();          \
            atomicAdd(&g_phase_cycles[(k) + (kL ? 0 : kH ? 32 : 16)], now - phase_t0); \
            if ((k) == 0) atomicAdd(&g_phase_cycles[(kL ? 0 : kH ? 32 : 16) + 15], 1ull); \
            phase_t0 = now;                                                        \
        }                                                                          \
    } while (0)
#else
#define WAVE_COUNT(k) \
    do {              \
    } while (0)
#define PHASE_MARK(k) \
    do {              \
    } while (0)
#endif

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
// one cluster
// ---------------------------------------------------------------------------
// Cells of the face table and of the partner windows.  A cell holds 0
// (empty) or a stream position + 1, and changes once.  LDS cells are uint16
// (a stream on the LDS path has at most 65535 tetrahedra), accessed through
// the 32-bit word holding two of them; global cells are uint32.
//   read     the cell and the word holding it;
//   try_set  an empty cell, by compare-and-swap of its word against the word
//            read (fails when the word changed: read again);
//   mark     a partner cell by atomic OR; true when it already held another
//            tetrahedron, which means a third tetrahedron on one face (the
//            windows are then discarded, so what the OR leaves does not
//            matter).  The same pair can be marked twice: a face of t is found
//            through t's record of another face, and later t finds its partner
//            through one of the partner's records; that is not a conflict.
template <bool kL>
struct Cells;
template <>
struct Cells<true> {
    using T = uint16_t;
    __device__ static uint32_t *word(T *a, uint32_t i) { return reinterpret_cast<uint32_t *>(a) + (i >> 1); }
    __device__ static uint32_t read(T *a, uint32_t i, uint32_t &w) {
        w = __atomic_load_n(word(a, i), __ATOMIC_RELAXED);
        return (w >> ((i & 1) * 16)) & 0xFFFFu;
    }
    __device__ static bool try_set(T *a, uint32_t i, uint32_t w, uint32_t v) {
        return atomicCAS(word(a, i), w, w | (v << ((i & 1) * 16))) == w;
    }
    __device__ static bool mark(T *a, uint32_t i, uint32_t v) {
        const int sh = (i & 1) * 16;
        const uint32_t old = (atomicOr(word(a, i), v << sh) >> sh) & 0xFFFFu;
        return old != 0u && old != v;
    }
    __device__ static void mark_issue(T *a, uint32_t i, uint32_t v, uint32_t &w) {
        w = atomicOr(word(a, i), v << ((i & 1) * 16));
    }
    __device__ static bool mark_bad(uint32_t i, uint32_t v, uint32_t w) {
        const uint32_t old = (w >> ((i & 1) * 16)) & 0xFFFFu;
        return old != 0u && old != v;
    }
    __device__ static uint32_t get(const T *a, uint32_t i) { return a[i]; }
};
template <>
struct Cells<false> {
    using T = uint32_t;
    __device__ static uint32_t read(T *a, uint32_t i, uint32_t &w) {
        w = __atomic_load_n(a + i, __ATOMIC_RELAXED);
        return w;
    }
    __device__ static bool try_set(T *a, uint32_t i, uint32_t w, uint32_t v) { return atomicCAS(a + i, w, v) == w; }
    __device__ static bool mark(T *a, uint32_t i, uint32_t v) {
        const uint32_t old = atomicOr(a + i, v);
        return old != 0u && old != v;
    }
    __device__ static void mark_issue(T *a, uint32_t i, uint32_t v, uint32_t &w) { w = atomicOr(a + i, v); }
    __device__ static bool mark_bad(uint32_t, uint32_t v, uint32_t w) { return w != 0u && w != v; }
    __device__ static uint32_t get(const T *a, uint32_t i) { return a[i]; }
};

// Hash of a triangle given by its sorted local ids: a multiply-add chain
// followed by the "lowbias32" integer finaliser (C. Wellons, 2018).
__device__ __forceinline__ uint32_t face_hash(int a, int b, int c) {
    uint32_t h = (uint32_t)a * 0x9E3779B1u + (uint32_t)b;
    h = h * 0x85EBCA77u + (uint32_t)c;
    h ^= h >> 16;
    h *= 0x7feb352du;
    h ^= h >> 15;
    h *= 0x846ca68bu;
    h ^= h >> 16;
    return h;
}

// Face k of a tetrahedron with ascending ids s omits s[k].
__device__ __forceinline__ void face_of(int4 s, int k, int &a, int &b, int &c) {
    a = k == 0 ? s.y : s.x;
    b = k <= 1 ? s.z : s.y;
    c = k == 3 ? s.z : s.w;
}

// Which face of the tetrahedron s (ascending ids) is {a < b < c}; -1 if none.
__device__ __forceinline__ int face_index(int4 s, int a, int b, int c) {
    const int k = s.x != a ? 0 : s.y != b ? 1 : s.z != c ? 2 : 3;
    int fa, fb, fc;
    face_of(s, k, fa, fb, fc);
    return (fa == a && fb == b && fc == c) ? k : -1;
}

// Build the requested relations of one cluster.  TT first, from the internal
// tetrahedra staged in LDS and a face table; then, for VT / VV, the local VT
// relation of every vertex in the cluster's local table (count, scan, scatter
// of stream positions), from which
//   VT  a row's list, ordered by original tetrahedron id;
//   VV  the union of the vertices of a row's tetrahedra, through a bitmap over
//       the local table, which is in original id order.
template <int B, bool kL, bool kH>
__device__ __attribute__((always_inline)) void build_cluster(const KArgs &a, const WorkItem &it, const ClusterMeta &m, const Plan &pl,
                              char *smem, char *ws) {
    using PosT = typename std::conditional<kL, uint16_t, int32_t>::type;
    using LidT = typename std::conditional<kL || kH, uint16_t, int32_t>::type;

    __shared__ int s_status;
    __shared__ int s_fail;
    __shared__ int s_full;
    int sp = 0;  // block scan buffer parity
    const int tid = threadIdx.x;
    const int ns = m.ns, nh = m.nh, ntot = ns + nh, nT = m.nT, L = m.L, nV = m.nV;
    const uint32_t mask = it.mask;
    const char *tb = a.s.tets + m.tb_off;
    const bool wide = (m.flags & kMetaWide) != 0;
    const int32_t *idg = a.s.tid + m.tet_off;
    const int32_t *lvg = a.s.lverts + m.lv_off;
    int32_t *blk = a.out + it.out_word;
    const BlockLayout lay = block_layout(mask, nV, nT, m.nnzVT, it.cap_vv, it.cap_tt);
    char *base = kL ? smem : ws;
    // the most used arrays: in LDS on the LDS path and on the hybrid global path
    char *hot = (kL || kH) ? smem : ws;
    ushort4 *lt = reinterpret_cast<ushort4 *>(smem + pl.lt);

    if (tid == 0) {
        s_status = 0;
        s_fail = 0;
        s_full = 0;
    }
#ifdef GALE_PHASE_TIMING
    unsigned long long phase_t0 = __builtin_amdgcn_s_memtime();
#endif

    // a stream tetrahedron from global memory / from wherever it is staged
    auto tet_global = [&](int p) -> int4 {
        if (wide) return reinterpret_cast<const int4 *>(tb)[p];
        const ushort4 q = reinterpret_cast<const ushort4 *>(tb)[p];
        return make_int4(q.x, q.y, q.z, q.w);
    };
    auto tet = [&](int p) -> int4 {
        if constexpr (kL) {
            const ushort4 q = lt[p];
            return make_int4(q.x, q.y, q.z, q.w);
        } else {
            return tet_global(p);
        }
    };
    // copy stream tetrahedra [t0, t1) to LDS, 16 B (two tetrahedra) per load;
    // the stream and lt are both padded to 16 B
    auto stage = [&](int t0, int t1) {
        if constexpr (kL) {
            constexpr int U = 8;
            const int q0 = t0 >> 1, q1 = (t1 + 1) >> 1;
            const uint4 *src = reinterpret_cast<const uint4 *>(tb);
            uint4 *dst = reinterpret_cast<uint4 *>(lt);
            for (int i0 = q0; i0 < q1; i0 += B * U) {
                uint4 t[U];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int i = i0 + u * B + tid;
                    t[u] = i < q1 ? src[i] : make_uint4(0u, 0u, 0u, 0u);
                }
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int i = i0 + u * B + tid;
                    if (i < q1) dst[i] = t[u];
                }
            }
        }
    };

    const bool want_v = (mask & (kRelVT | kRelVV)) != 0;
    stage(0, (mask & kRelTT) ? nT : (want_v ? ns : 0));
    __syncthreads();
    PHASE_MARK(0);

    // ---- TT ----------------------------------------------------------------
    // Internal tetrahedra (stream positions 0..nT-1, the rows) enter their four
    // faces in the table; the second to reach a face marks the partner cell of
    // the holder and its own.  Then every other stream tetrahedron looks its
    // faces up and marks the holder's cell.  A mark that finds its cell set
    // means a third tetrahedron on one face: chain pairing instead.
    if (mask & kRelTT) {
        using CL = Cells<kL>;
        using CT = typename CL::T;
        CT *win = reinterpret_cast<CT *>(base + pl.win);
        CT *ht = reinterpret_cast<CT *>(hot + pl.ht);
        uint32_t *win32 = reinterpret_cast<uint32_t *>(win);
        uint32_t *ht32 = reinterpret_cast<uint32_t *>(ht);
        const int H = pl.H;
        // probe positions: cells, or on the LDS path words of two cells
        const int Hp = kL ? H / 2 : H;
        const int cap = it.cap_tt;
        const int win_words = kL ? 2 * nT : (kH ? 8 * nT : 4 * nT);  // 4 cells per row
        const int ht_words = kL ? H / 2 : (kH ? 2 * H : H);
        // hybrid path: 64-bit cells that hold the face itself, so that a probe
        // step never reads the holder from global memory:
        //   bits 0..16 stream position + 1, 17..18 the holder's face index,
        //   19..63 the face's sorted local ids (15 bits each)
        unsigned long long *ht64 = reinterpret_cast<unsigned long long *>(hot + pl.ht);
        // hybrid path: 64-bit partner cells that a mark adds (position + 1) +
        // 2^32 to, without waiting for the old value; a cell marked once holds
        // its partner below bit 32, a high half above 1 means a third
        // tetrahedron on the face (seen when the rows are read)
        unsigned long long *win64 = reinterpret_cast<unsigned long long *>(base + pl.win);

        using Ins = std::integral_constant<bool, true>;
        using Look = std::integral_constant<bool, false>;

        // lower-cluster vertices: a face holding one is no face of a TT row
        uint32_t *lowb = reinterpret_cast<uint32_t *>(hot + pl.lowb);
        {
            const int lane = tid & 63, nwords = (L + 31) >> 5;
            for (int w0 = (tid >> 6) * 2; w0 < nwords; w0 += (B / 64) * 2) {
                const int i = w0 * 32 + lane;
                const unsigned long long bits = __ballot(i < L && (lvg[i] & 0x40000000));
                if (lane == 0) {
                    lowb[w0] = (uint32_t)bits;
                    if (w0 + 1 < nwords) lowb[w0 + 1] = (uint32_t)(bits >> 32);
                }
            }
        }
        __syncthreads();
        auto is_low = [&](int v) -> uint32_t { return (lowb[v >> 5] >> (v & 31)) & 1u; };

        // Each lane takes stream positions p0 + tid, p0 + tid + B, ... below
        // p1.  The four faces of its tetrahedron are hashed together; then the
        // lane works through the faces to visit (those of this pass; for
        // lookups, those with no vertex in a lower cluster) one probe step
        // (linear probing) per iteration, going on to its next face as soon as
        // one is done, so the wave waits for the lane with the most steps over
        // four faces rather than for the longest chain of each face in turn.
        // kIns: enter the faces (internal tetrahedra) or only look them up.
        auto stream_faces = [&](auto ins_tag, int p0, int p1, int pass, int P) {
            constexpr bool kIns = decltype(ins_tag)::value;
            for (int p = p0 + tid; p < p1; p += B) {
                int4 s;
                uint32_t todo;
                if constexpr (kIns) {
                    s = tet(p);
                    todo = 0xFu;
                } else {
                    s = tet_global(p);
                    // one lower vertex: only the face without it; two or more: none
                    const uint32_t lm = is_low(s.x) | is_low(s.y) << 1 | is_low(s.z) << 2 | is_low(s.w) << 3;
                    todo = lm == 0u ? 0xFu : (__popc(lm) > 1 ? 0u : lm);
                }
                // the faces to visit (this pass's; for lookups, those with no
                // vertex of a lower cluster), moved to the front of a queue of
                // (face index, current cell); the lane works on the head and
                // shifts the queue when it is done with that face
                int q0k = 0, q1k = 0, q2k = 0, q3k = 0;
                uint32_t q0i = 0u, q1i = 0u, q2i = 0u, q3i = 0u;
                int nq = 0;
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    int a0, b0, c0;
                    face_of(s, k, a0, b0, c0);
                    const uint32_t h = face_hash(a0, b0, c0);
                    const bool take =
                        ((todo >> k) & 1u) && (P <= 1 || (int)(((h & 0xFFFFu) * (uint32_t)P) >> 16) == pass);
                    const uint32_t i = (uint32_t)(((unsigned long long)h * (uint32_t)Hp) >> 32);
                    if (take && nq == 0) { q0k = k; q0i = i; }
                    if (take && nq == 1) { q1k = k; q1i = i; }
                    if (take && nq == 2) { q2k = k; q2i = i; }
                    if (take && nq == 3) { q3k = k; q3i = i; }
                    nq += take ? 1 : 0;
                }
                int fa = 0, fb = 0, fc = 0;
                if (nq > 0) face_of(s, q0k, fa, fb, fc);
                int left = 2 * Hp + 2;  // a failed swap reads its cell again; each cell changes once
                while (nq > 0) {
                    const int k = q0k;
                    uint32_t &idx = q0i;
                    bool stop;
                    if constexpr (kH) {
                        const unsigned long long key = (unsigned long long)fa | (unsigned long long)fb << 15 |
                                                       (unsigned long long)fc << 30;
                        const unsigned long long w = __atomic_load_n(ht64 + idx, __ATOMIC_RELAXED);
                        const bool used = w != 0ull;
                        const uint32_t c = (uint32_t)(w & 0x1FFFFull);
                        const int q = (int)c - 1;
                        const bool hit = used && (w >> 19) == key && q != p;
                        stop = hit || (!used && !kIns);
                        if (kIns && !used) {
                            const unsigned long long mine = (unsigned long long)(p + 1) |
                                                            (unsigned long long)k << 17 | key << 19;
                            stop = atomicCAS(ht64 + idx, 0ull, mine) == 0ull;
                        }
                        if (hit) {
                            const int kq = (int)((w >> 17) & 3ull);
                            (void)atomicAdd(win64 + 4 * (uint32_t)q + kq, (1ull << 32) | (unsigned long long)(p + 1));
                            if (kIns) (void)atomicAdd(win64 + 4 * (uint32_t)p + k, (1ull << 32) | (unsigned long long)c);
                        }
                        if (used && !hit) idx = idx + 1 == (uint32_t)H ? 0u : idx + 1;
                    } else if constexpr (kL) {
                        // LDS cells in pairs: a probe step reads the 32-bit
                        // word of two cells and looks at both, the low one
                        // first; an insert takes the first empty one, so an
                        // empty low cell means that the face is not there
                        uint32_t *wp = ht32 + idx;
                        const uint32_t w = __atomic_load_n(wp, __ATOMIC_RELAXED);
                        const uint32_t c0 = w & 0xFFFFu, c1 = w >> 16;
                        const int q0 = c0 == 0u ? 0 : (int)c0 - 1, q1 = c1 == 0u ? 0 : (int)c1 - 1;
                        // the holders' faces that are {fa, fb, fc}, if any (a
                        // tetrahedron meets its own earlier faces: skip them)
                        const int k0 = face_index(tet(q0), fa, fb, fc), k1 = face_index(tet(q1), fa, fb, fc);
                        const bool h0 = c0 != 0u && q0 != p && k0 >= 0;
                        const bool hit = h0 || (c1 != 0u && q1 != p && k1 >= 0);
                        const bool room = c0 == 0u || c1 == 0u;
                        stop = hit || (room && !kIns);
                        if (kIns && !hit && room) {
                            const uint32_t v = (uint32_t)p + 1u;
                            stop = atomicCAS(wp, w, c0 == 0u ? (w | v) : (w | (v << 16))) == w;  // else: read again
                        }
                        if (hit) {
                            const uint32_t c = h0 ? c0 : c1;
                            const int q = h0 ? q0 : q1, kq = h0 ? k0 : k1;
                            // both marks issued before either old value is looked at
                            uint32_t o1, o2 = 0u;
                            const uint32_t v1 = (uint32_t)p + 1u, i1 = 4 * (uint32_t)q + kq, i2 = 4 * (uint32_t)p + k;
                            CL::mark_issue(win, i1, v1, o1);
                            if (kIns) CL::mark_issue(win, i2, c, o2);
                            bool bad = CL::mark_bad(i1, v1, o1);
                            if (kIns) bad |= CL::mark_bad(i2, c, o2);
                            if (bad) s_fail = 1;
                        }
                        if (!hit && !room) idx = idx + 1 == (uint32_t)Hp ? 0u : idx + 1;
                    } else {
                        uint32_t w;
                        const uint32_t c = CL::read(ht, idx, w);
                        const int q = c == 0u ? 0 : (int)c - 1;
                        // the holder's face that is {fa, fb, fc}, if any (a tetrahedron
                        // meets its own earlier faces on the way: skip them)
                        const int kq = face_index(tet(q), fa, fb, fc);
                        const bool hit = c != 0u && q != p && kq >= 0;
                        stop = hit || (c == 0u && !kIns);
                        if (kIns && c == 0u) stop = CL::try_set(ht, idx, w, (uint32_t)p + 1u);
                        if (hit) {
                            // both marks issued before either old value is looked at
                            uint32_t o1, o2 = 0u;
                            const uint32_t v1 = (uint32_t)p + 1u, i1 = 4 * (uint32_t)q + kq, i2 = 4 * (uint32_t)p + k;
                            CL::mark_issue(win, i1, v1, o1);
                            if (kIns) CL::mark_issue(win, i2, c, o2);
                            bool bad = CL::mark_bad(i1, v1, o1);
                            if (kIns) bad |= CL::mark_bad(i2, c, o2);
                            if (bad) s_fail = 1;
                        }
                        if (c != 0u && !hit) idx = idx + 1 == (uint32_t)H ? 0u : idx + 1;
                    }
                    if (--left == 0 && !stop) {
                        if (kIns) s_full = 1;
                        stop = true;
                    }
                    if (stop) {
                        q0k = q1k; q0i = q1i;
                        q1k = q2k; q1i = q2i;
                        q2k = q3k; q2i = q3i;
                        --nq;
                        left = 2 * Hp + 2;
                        if (nq > 0) face_of(s, q0k, fa, fb, fc);
                    }
                }
            }
        };

        int P = pl.P;
        while (true) {
            for (int i = tid; i < win_words; i += B) win32[i] = 0u;
            for (int pass = 0; pass < P; ++pass) {
                for (int i = tid; i < ht_words; i += B) ht32[i] = 0u;
                __syncthreads();
                stream_faces(Ins{}, 0, nT, pass, P);
                __syncthreads();
                PHASE_MARK(7);
                if (s_full) break;
                stream_faces(Look{}, nT, ntot, pass, P);
                __syncthreads();
                PHASE_MARK(8);
            }
            const int full = s_full, fail = s_fail;
            __syncthreads();
            if (!full || fail) break;
            // a pass overfilled the table: twice the passes, from the start
            P *= 2;
            if (tid == 0) s_full = 0;
            if (P > kMaxFacePasses) {
                if (tid == 0) s_fail = 2;  // only exhaustive pairing is left
                break;
            }
        }
        __syncthreads();
        PHASE_MARK(1);
        // tetrahedron ids: from a copy over the face table when it fits (LDS)
        int32_t *idl = reinterpret_cast<int32_t *>(ht);
        const int64_t ht_bytes = (int64_t)(kH ? 8 : sizeof(CT)) * H;
        const bool ids_lds = (kL || kH) && ht_bytes >= 4 * (int64_t)ntot;
        if (ids_lds) {
            for (int i = tid; i < ntot; i += B) idl[i] = idg[i];
            __syncthreads();
        }
        auto id_of = [&](int p) -> int32_t { return ids_lds ? idl[p] : idg[p]; };
        int ecarry = 0;
        if (s_fail == 0) {
            // partners mapped to original ids, sorted; a repeated tetrahedron
            // reached through several faces is listed once
            for (int r0 = 0; r0 < nT; r0 += B) {
                const int r = r0 + tid;
                int n0 = 0x7fffffff, n1 = 0x7fffffff, n2 = 0x7fffffff, n3 = 0x7fffffff;
                int c = 0;
                if (r < nT) {
                    uint32_t w0, w1, w2, w3;
                    if constexpr (kH) {
                        unsigned long long x[4];
#pragma unroll
                        for (int j = 0; j < 4; ++j)
                            x[j] = __hip_atomic_load(win64 + 4 * r + j, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        const bool twice = (x[0] >> 32) > 1 || (x[1] >> 32) > 1 || (x[2] >> 32) > 1 || (x[3] >> 32) > 1;
                        if (twice) s_fail = 1;  // the rows are built again by chain pairing
                        w0 = twice ? 0u : (uint32_t)x[0];
                        w1 = twice ? 0u : (uint32_t)x[1];
                        w2 = twice ? 0u : (uint32_t)x[2];
                        w3 = twice ? 0u : (uint32_t)x[3];
                    } else if constexpr (kL) {
                        // the row's four 16-bit cells in one 8-byte read
                        const uint2 q = reinterpret_cast<const uint2 *>(win)[r];
                        w0 = q.x & 0xFFFFu;
                        w1 = q.x >> 16;
                        w2 = q.y & 0xFFFFu;
                        w3 = q.y >> 16;
                    } else {
                        w0 = CL::get(win, 4 * r);
                        w1 = CL::get(win, 4 * r + 1);
                        w2 = CL::get(win, 4 * r + 2);
                        w3 = CL::get(win, 4 * r + 3);
                    }
                    if (w0 != 0u) n0 = id_of(w0 - 1) & kIdMask;
                    if (w1 != 0u) n1 = id_of(w1 - 1) & kIdMask;
                    if (w2 != 0u) n2 = id_of(w2 - 1) & kIdMask;
                    if (w3 != 0u) n3 = id_of(w3 - 1) & kIdMask;
                    cswap(n0, n1); cswap(n2, n3); cswap(n0, n2); cswap(n1, n3); cswap(n1, n2);
                    if (n3 == n2) n3 = 0x7fffffff;
                    if (n2 == n1) { n2 = n3; n3 = 0x7fffffff; }
                    if (n1 == n0) { n1 = n2; n2 = n3; n3 = 0x7fffffff; }
                    c = (n0 != 0x7fffffff) + (n1 != 0x7fffffff) + (n2 != 0x7fffffff) + (n3 != 0x7fffffff);
                }
                int tot;
                const int ex = block_excl_scan<B>(c, tot, sp);
                if (r < nT) {
                    const int32_t id = id_of(r);
                    if (id >= 0) s_status |= kStInconsistent;  // position r must be internal
                    const int o = ecarry + ex;
                    blk[lay.trows + r] = id & kIdMask;
                    blk[lay.tt_off + r] = o;
                    if (o + c <= cap) {
                        int32_t *w = blk + lay.tt_ent + o;
                        if (c > 0) w[0] = n0;
                        if (c > 1) w[1] = n1;
                        if (c > 2) w[2] = n2;
                        if (c > 3) w[3] = n3;
                    }
                }
                ecarry += tot;
            }
        }
        __syncthreads();
        // Chain pairing, when a face has more than two tetrahedra (or the
        // partner cells saw a third one): the face table is built again, the
        // internal tetrahedra on one face forming a chain through their
        // partner cells (the holder's cell points to the latest to arrive,
        // which points to the one before, ...).  Every internal tetrahedron
        // then takes as partners the whole chain of each of its faces, and
        // every other stream tetrahedron is a partner of every tetrahedron on
        // the chains of its faces, so the work is the stream's faces plus the
        // entries.  A count sweep, a scan of the counts to each row's end, a
        // scatter sweep that counts each row down to its start, and a sort of
        // each row.  A tetrahedron with the same four vertices as the row's
        // shares all four faces with it and is taken through face 0 only.
        bool paired = s_fail == 0;
        if (!paired && s_fail == 1) {
            if (tid == 0) atomicOr(&s_status, kStTTFallback);
            int32_t *rc = blk + lay.tt_off;  // per-row counts, then each row's end, then its start
            int32_t *ent = blk + lay.tt_ent;
            // chain cells: the next internal tetrahedron on the face (position + 1), 0 at the end
            // (global cells are read past the L1 cache: other waves change them by atomics)
            auto link_get = [&](uint32_t i) -> uint32_t {
                if constexpr (kH)
                    return (uint32_t)__hip_atomic_load(win64 + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                else if constexpr (kL)
                    return CL::get(win, i);
                else
                    return __hip_atomic_load(win32 + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            };
            auto rc_get = [&](int r) -> int { return __hip_atomic_load(rc + r, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); };
            auto link_exch = [&](uint32_t i, uint32_t v) -> uint32_t {
                if constexpr (kH) {
                    return (uint32_t)atomicExch(win64 + i, (unsigned long long)v);
                } else if constexpr (kL) {
                    uint32_t *wp = CL::word(win, i);
                    const int sh = (i & 1) * 16;
                    uint32_t w = __atomic_load_n(wp, __ATOMIC_RELAXED);
                    while (true) {
                        const uint32_t o = atomicCAS(wp, w, (w & ~(0xFFFFu << sh)) | (v << sh));
                        if (o == w) return (w >> sh) & 0xFFFFu;
                        w = o;
                    }
                } else {
                    return atomicExch(win32 + i, v);
                }
            };
            // a tetrahedron's own cell, empty before and written once
            auto link_set = [&](uint32_t i, uint32_t v) {
                if constexpr (kH) win64[i] = v;
                else if constexpr (kL) atomicOr(CL::word(win, i), v << ((i & 1) * 16));
                else win32[i] = v;
            };
            // the holder of face {fa, fb, fc} (hash h) and its face index;
            // with ins, position p enters it as holder when the face is not
            // in the table yet.  -1: not in the table, or (ins) table full.
            auto find = [&](bool ins, int p, int k, int fa, int fb, int fc, uint32_t h, int &kh) -> int {
                uint32_t idx = (uint32_t)(((unsigned long long)h * (uint32_t)H) >> 32);
                for (int left = H; left > 0;) {
                    if constexpr (kH) {
                        const unsigned long long key = (unsigned long long)fa | (unsigned long long)fb << 15 |
                                                       (unsigned long long)fc << 30;
                        const unsigned long long w = __atomic_load_n(ht64 + idx, __ATOMIC_RELAXED);
                        if (w == 0ull) {
                            if (!ins) return -1;
                            const unsigned long long mine = (unsigned long long)(p + 1) |
                                                            (unsigned long long)k << 17 | key << 19;
                            if (atomicCAS(ht64 + idx, 0ull, mine) == 0ull) {
                                kh = k;
                                return p;
                            }
                            continue;  // the cell was taken: read it again
                        }
                        if ((w >> 19) == key) {
                            kh = (int)((w >> 17) & 3ull);
                            return (int)(w & 0x1FFFFull) - 1;
                        }
                    } else {
                        uint32_t w;
                        const uint32_t c = CL::read(ht, idx, w);
                        if (c == 0u) {
                            if (!ins) return -1;
                            if (CL::try_set(ht, idx, w, (uint32_t)p + 1u)) {
                                kh = k;
                                return p;
                            }
                            continue;  // the cell's word changed: read it again
                        }
                        const int q = (int)c - 1;
                        const int kq = q < nT ? face_index(tet(q), fa, fb, fc) : -1;
                        if (kq >= 0) {
                            kh = kq;
                            return q;
                        }
                    }
                    idx = idx + 1 == (uint32_t)H ? 0u : idx + 1;
                    --left;
                }
                if (ins) s_full = 1;
                return -1;
            };
            // every internal tetrahedron on the chain of face {fa, fb, fc} from its holder
            auto walk = [&](int u, int ku, int fa, int fb, int fc, auto &&f) {
                for (int n = 0; n <= nT; ++n) {
                    f(u);
                    const uint32_t nx = link_get(4u * (uint32_t)u + (uint32_t)ku);
                    if (nx == 0u) return;
                    u = (int)nx - 1;
                    ku = u < nT ? face_index(tet(u), fa, fb, fc) : -1;
                    if (ku < 0) break;
                }
                atomicOr(&s_status, kStInconsistent);
            };
            auto emit = [&](bool scatter, int r, int u) {
                if (!scatter) {
                    atomicAdd(rc + r, 1);
                } else {
                    const int slot = atomicSub(rc + r, 1) - 1;
                    if (slot >= 0 && slot < cap) ent[slot] = idg[u] & kIdMask;
                }
            };
            auto in_pass = [&](uint32_t h, int pass, int Pc) {
                return Pc <= 1 || (int)(((h & 0xFFFFu) * (uint32_t)Pc) >> 16) == pass;
            };
            auto sweep = [&](bool scatter, int Pc) {
                for (int i = tid; i < win_words; i += B) win32[i] = 0u;
                for (int pass = 0; pass < Pc; ++pass) {
                    for (int i = tid; i < ht_words; i += B) ht32[i] = 0u;
                    __syncthreads();
                    for (int p = tid; p < nT; p += B) {
                        const int4 s = tet(p);
                        for (int k = 0; k < 4; ++k) {
                            int fa, fb, fc;
                            face_of(s, k, fa, fb, fc);
                            const uint32_t h = face_hash(fa, fb, fc);
                            if (!in_pass(h, pass, Pc)) continue;
                            int kh = 0;
                            const int q = find(true, p, k, fa, fb, fc, h, kh);
                            if (q >= 0 && q != p)
                                link_set(4u * (uint32_t)p + k, link_exch(4u * (uint32_t)q + kh, (uint32_t)p + 1u));
                        }
                    }
                    __syncthreads();
                    if (s_full) break;
                    for (int p = tid; p < nT; p += B) {
                        const int4 s = tet(p);
                        for (int k = 0; k < 4; ++k) {
                            int fa, fb, fc;
                            face_of(s, k, fa, fb, fc);
                            const uint32_t h = face_hash(fa, fb, fc);
                            if (!in_pass(h, pass, Pc)) continue;
                            int kh = 0;
                            const int q = find(false, p, k, fa, fb, fc, h, kh);
                            if (q < 0) {
                                atomicOr(&s_status, kStInconsistent);
                                continue;
                            }
                            walk(q, kh, fa, fb, fc, [&](int u) {
                                if (u != p && (k == 0 || shared_vertices(s, tet(u)) < 4)) emit(scatter, p, u);
                            });
                        }
                    }
                    for (int p = nT + tid; p < ntot; p += B) {
                        const int4 s = tet_global(p);
                        const uint32_t lm = is_low(s.x) | is_low(s.y) << 1 | is_low(s.z) << 2 | is_low(s.w) << 3;
                        const uint32_t todo = lm == 0u ? 0xFu : (__popc(lm) > 1 ? 0u : lm);
                        for (int k = 0; k < 4; ++k) {
                            if (!((todo >> k) & 1u)) continue;
                            int fa, fb, fc;
                            face_of(s, k, fa, fb, fc);
                            const uint32_t h = face_hash(fa, fb, fc);
                            if (!in_pass(h, pass, Pc)) continue;
                            int kh = 0;
                            const int q = find(false, p, k, fa, fb, fc, h, kh);
                            if (q >= 0) walk(q, kh, fa, fb, fc, [&](int u) { emit(scatter, u, p); });
                        }
                    }
                    __syncthreads();
                }
            };
            int Pc = P;
            while (Pc <= kMaxFacePasses) {
                for (int i = tid; i < nT; i += B) rc[i] = 0;
                if (tid == 0) s_full = 0;
                __syncthreads();
                sweep(false, Pc);
                __syncthreads();
                if (!s_full) {
                    paired = true;
                    break;
                }
                Pc *= 2;
            }
            if (paired) {
                ecarry = 0;
                for (int r0 = 0; r0 < nT; r0 += B) {
                    const int r = r0 + tid;
                    const int c = r < nT ? rc_get(r) : 0;
                    int tot;
                    const int ex = block_excl_scan<B>(c, tot, sp);
                    if (r < nT) rc[r] = ecarry + ex + c;
                    ecarry += tot;
                }
                __syncthreads();
                sweep(true, Pc);
                __syncthreads();
                if (tid == 0 && s_full) atomicOr(&s_status, kStInconsistent);
                for (int r = tid; r < nT; r += B) {
                    const int32_t id = idg[r];
                    if (id >= 0) atomicOr(&s_status, kStInconsistent);  // position r must be internal
                    blk[lay.trows + r] = id & kIdMask;
                    const int st = min(max(rc_get(r), 0), cap);
                    const int en = max(min(r + 1 < nT ? rc_get(r + 1) : ecarry, cap), st);
                    for (int i = st + 1; i < en; ++i) {
                        const int32_t x = ent[i];
                        int j = i - 1;
                        while (j >= st && ent[j] > x) {
                            ent[j + 1] = ent[j];
                            --j;
                        }
                        ent[j + 1] = x;
                    }
                }
            }
            __syncthreads();
        }
        if (!paired) {
            // exhaustive pairing (a face table that stays full); rows are positions 0..nT-1
            ecarry = 0;
            if (tid == 0) atomicOr(&s_status, kStTTFallback);
            auto tet_any = [&](int q) -> int4 { return q < nT ? tet(q) : tet_global(q); };
            for (int r0 = 0; r0 < nT; r0 += B) {
                const int r = r0 + tid;
                int c = 0;
                int4 t = make_int4(0, 0, 0, 0);
                if (r < nT) {
                    t = tet(r);
                    for (int q = 0; q < ntot; ++q)
                        if (q != r && shared_vertices(t, tet_any(q)) >= 3) ++c;
                }
                int etot;
                const int eex = block_excl_scan<B>(c, etot, sp);
                if (r < nT) {
                    int pos = ecarry + eex;
                    blk[lay.trows + r] = idg[r] & kIdMask;
                    blk[lay.tt_off + r] = pos;
                    const int start = pos;
                    for (int q = 0; q < ntot; ++q) {
                        if (q != r && shared_vertices(t, tet_any(q)) >= 3) {
                            if (pos < cap) blk[lay.tt_ent + pos] = idg[q] & kIdMask;
                            ++pos;
                        }
                    }
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
                ecarry += etot;
            }
        }
        if (tid == 0) {
            blk[lay.tt_off + nT] = ecarry;
            blk[5] = ecarry;
            if (ecarry > cap) s_status |= kStTTOverflow;
        }
        __syncthreads();
        PHASE_MARK(2);
        if (want_v) {
            stage(nT, ns);
            __syncthreads();
        }
    }

    if (want_v) {
        LidT *rix = reinterpret_cast<LidT *>(hot + pl.rix);
        LidT *rowl = reinterpret_cast<LidT *>(hot + pl.rowl);
        int32_t *cnt = reinterpret_cast<int32_t *>(hot + pl.cnt);
        PosT *lvt = reinterpret_cast<PosT *>(base + pl.lvt);
        ushort4 *lv4 = reinterpret_cast<ushort4 *>(ws + (kH ? pl.lv4 : 0));  // hybrid path only
        uint32_t *wbm = reinterpret_cast<uint32_t *>(hot + pl.wbm);
        constexpr LidT kNoRow = (LidT)-1;

        // rows: row index of each local vertex, local id of each row, row ids
        {
            int carry = 0;
            for (int i0 = 0; i0 < L; i0 += B) {
                const int i = i0 + tid;
                const int32_t lv = i < L ? lvg[i] : 0;
                const int f = (i < L && lv < 0) ? 1 : 0;
                int tot;
                const int ex = block_excl_scan<B>(f, tot, sp);
                if (i < L) {
                    const int r = carry + ex;
                    const bool row = f && r < nV;
                    rix[i] = row ? (LidT)r : kNoRow;
                    if (row) {
                        rowl[r] = (LidT)i;
                        blk[lay.vrows + r] = lv & kVidMask;
                    }
                }
                carry += tot;
            }
            if (tid == 0 && carry != nV) s_status |= kStInconsistent;
        }
        for (int r = tid; r <= nV; r += B) cnt[r] = 0;
        __syncthreads();

        // ---- local VT of the rows (the star holds every tetrahedron of a row)
        for (int p = tid; p < ns; p += B) {
            const int4 t = tet(p);
            const LidT r0 = rix[t.x], r1 = rix[t.y], r2 = rix[t.z], r3 = rix[t.w];
            if (r0 != kNoRow) atomicAdd(&cnt[r0], 1);
            if (r1 != kNoRow) atomicAdd(&cnt[r1], 1);
            if (r2 != kNoRow) atomicAdd(&cnt[r2], 1);
            if (r3 != kNoRow) atomicAdd(&cnt[r3], 1);
        }
        __syncthreads();
        {
            int carry = 0;
            for (int r0 = 0; r0 < nV; r0 += B) {
                const int r = r0 + tid;
                const int x = r < nV ? cnt[r] : 0;
                int tot;
                const int ex = block_excl_scan<B>(x, tot, sp);
                if (r < nV) cnt[r] = carry + ex + x;  // end of the list
                carry += tot;
            }
            if (tid == 0) {
                cnt[nV] = carry;
                if (carry != m.nnzVT) s_status |= kStInconsistent;
            }
        }
        __syncthreads();
        const bool vt_ok = cnt[nV] == m.nnzVT;  // else the lists would not fit
        if (vt_ok) {
            for (int p = tid; p < ns; p += B) {
                const int4 t = tet(p);
                const LidT r0 = rix[t.x], r1 = rix[t.y], r2 = rix[t.z], r3 = rix[t.w];
                if constexpr (kH) {
                    // the entry's tetrahedron id (VT) and local ids (VV)
                    const int32_t id = idg[p] & kIdMask;
                    const ushort4 t4 = make_ushort4((uint16_t)t.x, (uint16_t)t.y, (uint16_t)t.z, (uint16_t)t.w);
                    auto put = [&](LidT r) {
                        const int j = atomicSub(&cnt[r], 1) - 1;
                        lvt[j] = id;
                        lv4[j] = t4;
                    };
                    if (r0 != kNoRow) put(r0);
                    if (r1 != kNoRow) put(r1);
                    if (r2 != kNoRow) put(r2);
                    if (r3 != kNoRow) put(r3);
                } else {
                    if (r0 != kNoRow) lvt[atomicSub(&cnt[r0], 1) - 1] = (PosT)p;
                    if (r1 != kNoRow) lvt[atomicSub(&cnt[r1], 1) - 1] = (PosT)p;
                    if (r2 != kNoRow) lvt[atomicSub(&cnt[r2], 1) - 1] = (PosT)p;
                    if (r3 != kNoRow) lvt[atomicSub(&cnt[r3], 1) - 1] = (PosT)p;
                }
            }
        }
        __syncthreads();  // cnt[r] = start of row r's list, cnt[r+1] = its end
        PHASE_MARK(3);
        // ---- VV: one row per group of G lanes (8, 16 or 32), in rounds of B/G
        // rows.  The group marks the row's neighbours in its bitmap over the
        // local table; each lane takes a run of consecutive words (into
        // registers when they are few) and counts their bits; the round's
        // counts give every row its offset after one barrier; the row is then
        // emitted in word order, which is original id order.
        if ((mask & kRelVV) && vt_ok) {
            __shared__ int s_vc[2][B / 8];
            const int W = pl.W;
            // original ids of the local table: an LDS copy on the LDS path and,
            // when it fits, on the hybrid path
            const bool lvl_on = kL || (kH && pl.lvl >= 0);
            int32_t *lvl = reinterpret_cast<int32_t *>(hot + (pl.lvl > 0 ? pl.lvl : 0));
            const int cap = it.cap_vv;
            const int Wg = (int)vv_group_words(W);  // a group's bitmap, then its summary
            for (int i = tid; i < (B / pl.G) * Wg; i += B) wbm[i] = 0u;
            if (lvl_on)
                for (int i = tid; i < L; i += B) lvl[i] = lvg[i] & kVidMask;
            __syncthreads();
            auto orig = [&](int l) -> int32_t { return lvl_on ? lvl[l] : (lvg[l] & kVidMask); };
            int base_off = 0;
            auto rows_by = [&](auto gtag) {
                constexpr int G = decltype(gtag)::value;
                constexpr int NG = B / G;
                constexpr int KMAX = 8;  // bitmap words a lane keeps in registers
                const int grp = tid / G, gl = tid % G;
                uint32_t *wb = wbm + (int64_t)grp * Wg;
                uint32_t *sb = wb + W;  // bit b of sb[s]: word 32 s + b has a bit set
                const int K = (W + G - 1) / G;  // words per lane
                const int wbeg = gl * K, wend = min(W, wbeg + K);
                const bool in_regs = K <= KMAX;
                // larger bitmaps: a lane takes a run of summary words (32 bitmap
                // words each) and visits only the words marked in them
                const int SW = (W + 31) / 32, SK = (SW + G - 1) / G;
                const int sbeg = gl * SK, send = min(SW, sbeg + SK);
                auto mark = [&](int v) {
                    atomicOr(&wb[v >> 5], 1u << (v & 31));
                    if (!in_regs) atomicOr(&sb[v >> 10], 1u << ((v >> 5) & 31));
                };
                // the row vertex is one of each tetrahedron's four ascending
                // ids: the other three by selects, then marked
                auto mark_others = [&](int4 t, int self) {
                    const bool sx = t.x == self, sy = t.y == self;
                    mark(sx ? t.y : t.x);
                    mark((sx || sy) ? t.z : t.y);
                    mark(t.w == self ? t.z : t.w);
                };
                auto entry_tet = [&](int i) -> int4 {
                    if constexpr (kH) {
                        const ushort4 q = lv4[i];
                        return make_int4(q.x, q.y, q.z, q.w);
                    } else {
                        return tet(lvt[i]);
                    }
                };
                int par = 0;
                for (int r0 = 0; r0 < nV; r0 += NG) {
                    const int r = r0 + grp;
                    if (r < nV) {
                        const int self = rowl[r];
                        const int e1 = cnt[r + 1];
                        int i = cnt[r] + gl;
                        // two entries per step, their reads overlapped
                        for (; i + G < e1; i += 2 * G) {
                            const int4 t0 = entry_tet(i), t1 = entry_tet(i + G);
                            mark_others(t0, self);
                            mark_others(t1, self);
                        }
                        if (i < e1) mark_others(entry_tet(i), self);
                    }
                    wave_fence();
                    // this lane's run of words: into registers (and cleared), counted
                    uint32_t wv[KMAX];
                    int n = 0;
                    if (in_regs) {
#pragma unroll
                        for (int j = 0; j < KMAX; ++j) {
                            const int w = wbeg + j;
                            wv[j] = w < wend ? wb[w] : 0u;
                            n += __popc(wv[j]);
                        }
#pragma unroll
                        for (int j = 0; j < KMAX; ++j)
                            if (wv[j]) wb[wbeg + j] = 0u;
                    } else {
                        for (int s = sbeg; s < send; ++s) {
                            uint32_t sbits = sb[s];
                            while (sbits) {
                                const int b = __ffs(sbits) - 1;
                                sbits &= sbits - 1u;
                                n += __popc(wb[s * 32 + b]);
                            }
                        }
                    }
                    int c = n;
#pragma unroll
                    for (int d = G / 2; d >= 1; d >>= 1) c += lane_xor(c, d);
                    if (gl == 0) s_vc[par][grp] = c;
                    __syncthreads();
                    // this round's offsets: base + counts of the groups before.
                    // Every wave scans the NG counts itself, one or two per lane.
                    constexpr int E = NG > 64 ? 2 : 1;
                    const int lane = tid & 63;
                    const int a0 = lane * E < NG ? s_vc[par][lane * E] : 0;
                    const int a1 = (E == 2 && lane * E + 1 < NG) ? s_vc[par][lane * E + 1] : 0;
                    const int lsum = a0 + a1;
                    const int incl = wave_incl_sum(lsum);
                    const int src = grp / E;
                    int x = __shfl(incl - lsum, src, 64);
                    if (E == 2) {
                        const int f = __shfl(a0, src, 64);
                        if (grp & 1) x += f;
                    }
                    const int round_total = __shfl(incl, 63, 64);
                    const int o_row = base_off + x;
                    par ^= 1;
                    // each lane's place in its row: the counts of the group's
                    // lanes before it (every lane here, so DPP row shifts serve
                    // groups within one 16-lane row)
                    int y = n;
#pragma unroll
                    for (int d = 1; d < G; d <<= 1) {
                        int z;
                        if constexpr (G <= 16) {
                            z = d == 1 ? __builtin_amdgcn_update_dpp(0, y, 0x111, 0xF, 0xF, false)
                              : d == 2 ? __builtin_amdgcn_update_dpp(0, y, 0x112, 0xF, 0xF, false)
                              : d == 4 ? __builtin_amdgcn_update_dpp(0, y, 0x114, 0xF, 0xF, false)
                                       : __builtin_amdgcn_update_dpp(0, y, 0x118, 0xF, 0xF, false);
                        } else {
                            z = __shfl_up(y, d, G);
                        }
                        if (gl >= d) y += z;
                    }
                    if (r < nV) {
                        if (gl == 0) blk[lay.vv_off + r] = o_row;
                        const bool fits = o_row + c <= cap;
                        int pos = o_row + y - n;
                        if (in_regs) {
#pragma unroll
                            for (int j = 0; j < KMAX; ++j) {
                                uint32_t bits = fits ? wv[j] : 0u;
                                while (bits) {
                                    const int b = __ffs(bits) - 1;
                                    bits &= bits - 1u;
                                    blk[lay.vv_ent + pos] = orig((wbeg + j) * 32 + b);
                                    ++pos;
                                }
                            }
                        } else {
                            // the same run of summary words as counted, in word order
                            for (int s = sbeg; s < send; ++s) {
                                uint32_t sbits = sb[s];
                                if (!sbits) continue;
                                sb[s] = 0u;
                                while (sbits) {
                                    const int w = s * 32 + __ffs(sbits) - 1;
                                    sbits &= sbits - 1u;
                                    uint32_t bits = wb[w];
                                    wb[w] = 0u;
                                    if (fits) {
                                        while (bits) {
                                            const int b = __ffs(bits) - 1;
                                            bits &= bits - 1u;
                                            blk[lay.vv_ent + pos] = orig(w * 32 + b);
                                            ++pos;
                                        }
                                    }
                                }
                            }
                        }
                    }
                    base_off += round_total;
                }
            };
            if (pl.G == 8) rows_by(std::integral_constant<int, 8>{});
            else if (pl.G == 16) rows_by(std::integral_constant<int, 16>{});
            else rows_by(std::integral_constant<int, 32>{});
            if (tid == 0) {
                blk[lay.vv_off + nV] = base_off;
                blk[4] = base_off;
                if (base_off > cap) s_status |= kStVVOverflow;
            }
            __syncthreads();
            PHASE_MARK(5);
        }

        // ---- VT: a row's tetrahedra by original id; the offsets are the lists'.
        // LDS path: rows sorted by their threads into a buffer over the star
        // tetrahedra's region (no longer needed), then copied out in order.
        if ((mask & kRelVT) && vt_ok) {
            int32_t *buf = reinterpret_cast<int32_t *>(smem + pl.lt);
            const int bcap = kL ? (int)((pl.rix - pl.lt) / 4) : 0;
            // a local VT entry's tetrahedron id (the hybrid path stored it;
            // the LDS path reads an LDS copy of the star's ids when the
            // space after the V arrays holds one)
            int32_t *ids_l = reinterpret_cast<int32_t *>(smem + pl.wbm);
            const bool ids_lds = kL && (int64_t)a.lds_budget - pl.wbm >= 4 * (int64_t)ns;
            if (ids_lds) {
                for (int i = tid; i < ns; i += B) ids_l[i] = idg[i] & kIdMask;
                __syncthreads();
            }
            auto vt_key = [&](int e) -> int32_t {
                if constexpr (kH) return lvt[e];
                else return ids_lds ? ids_l[lvt[e]] : (idg[lvt[e]] & kIdMask);
            };
            // rows of at most 32 entries: one thread each, in registers, with
            // a network of 8, 16 or 32 for the wave's longest such row; longer
            // rows: the wave of the row's thread, after its short rows
            auto sort_short = [&](auto ntag, int r, int32_t *dst) {
                constexpr int N = decltype(ntag)::value;
                const int s0 = cnt[r], n = cnt[r + 1] - s0;
                uint32_t v[N];
#pragma unroll
                for (int i = 0; i < N; ++i)
                    v[i] = i < n ? (uint32_t)vt_key(s0 + i) : 0xFFFFFFFFu;
                sort_regs<N>(v);
#pragma unroll
                for (int i = 0; i < N; ++i)
                    if (i < n) dst[i] = (int32_t)v[i];
            };
            // rows [rb, rb + B) with row rb + tid for this thread; dst_of(r)
            // is where row r's sorted list goes
            auto sort_rows = [&](int rb, int re, auto dst_of) {
                const int r = rb + tid;
                const int n = r < re ? cnt[r + 1] - cnt[r] : -1;
                const bool shrt = n >= 0 && n <= 32, lng = n > 32;
                const unsigned long long over16 = __ballot(shrt && n > 16), over8 = __ballot(shrt && n > 8);
                if (shrt) {
                    if (over16)
                        sort_short(std::integral_constant<int, 32>{}, r, dst_of(r));
                    else if (over8)
                        sort_short(std::integral_constant<int, 16>{}, r, dst_of(r));
                    else
                        sort_short(std::integral_constant<int, 8>{}, r, dst_of(r));
                }
                unsigned long long bal = __ballot(lng);
                while (bal) {
                    const int rr = rb + (tid & ~63) + __ffsll((long long)bal) - 1;
                    bal &= bal - 1;
                    const int s0 = cnt[rr];
                    wave_sort(
                        cnt[rr + 1] - s0, [&](int i) { return vt_key(s0 + i); }, dst_of(rr));
                }
            };
            for (int r = tid; r < nV; r += B) blk[lay.vt_off + r] = cnt[r];
            if (tid == 0) blk[lay.vt_off + nV] = cnt[nV];
            if constexpr (!kL) {
                for (int rb = 0; rb < nV; rb += B)
                    sort_rows(rb, nV, [&](int r) { return blk + lay.vt_ent + cnt[r]; });
                __syncthreads();
            } else {
                int r0 = 0;
                while (r0 < nV) {
                    // rows [r0, r1): at most B of them, their entries within the buffer
                    int lo = r0, hi = min(nV, r0 + B);
                    while (lo < hi) {
                        const int mid = (lo + hi + 1) >> 1;
                        if (cnt[mid] - cnt[r0] <= bcap) lo = mid;
                        else hi = mid - 1;
                    }
                    const int e0 = cnt[r0];
                    if (lo == r0) {
                        // row r0 alone exceeds the buffer: sorted straight into the block
                        sort_rows(r0, r0 + 1, [&](int r) { return blk + lay.vt_ent + cnt[r]; });
                        __syncthreads();
                        r0 += 1;
                        continue;
                    }
                    const int r1 = lo;
                    sort_rows(r0, r1, [&](int r) { return buf + (cnt[r] - e0); });
                    __syncthreads();
                    const int ne = cnt[r1] - e0;
                    for (int e = tid; e < ne; e += B) blk[lay.vt_ent + e0 + e] = buf[e];
                    __syncthreads();
                    r0 = r1;
                }
            }
            PHASE_MARK(4);
        }
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
__device__ __attribute__((always_inline)) void process_item(const KArgs &a, const WorkItem &it, char *smem, char *ws) {
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
        build_cluster<B, true, false>(a, it, m, lp, smem, ws);
    } else {
        const Plan hp = hyb_plan(m, it.mask, a.lds_budget, B);
        if (hp.ok) {
            build_cluster<B, false, true>(a, it, m, hp, smem, ws);
        } else {
            const Plan gp = ws_plan(m, it.mask, B);
            build_cluster<B, false, false>(a, it, m, gp, smem, ws);
        }
    }
}

// One work item per workgroup: item blockIdx.x.  Used for the per-cluster
// (plain) form, one launch per (cluster, relation).
template <int B, bool kL>
__global__ __launch_bounds__(B, 4) void gale_items_kernel(KArgs a) {
    extern __shared__ __attribute__((aligned(16))) char smem[];
    const int i = blockIdx.x;
    if (i >= a.nitems) return;
    char *ws = a.ws ? a.ws + (int64_t)blockIdx.x * a.ws_stride : nullptr;
    process_item<B, kL>(a, a.items[i], smem, ws);
}

// Persistent form: each workgroup takes the next item from the device work
// queue until the list is exhausted (every workgroup reaches the exit test).
template <int B, bool kL>
__global__ __launch_bounds__(B, 4) void gale_persistent_kernel(KArgs a) {
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

// Zero n words (queue words of a captured batch: a kernel node instead of a
// memset node, so graph replays start from zero).
__global__ __launch_bounds__(64) void gale_zero_kernel(int32_t *p, int n) {
    const int i = threadIdx.x;
    if (i < n) p[i] = 0;
}

// ---------------------------------------------------------------------------
// host-side launch wrappers
// ---------------------------------------------------------------------------
hipError_t launch_zero(int32_t *p, int n, hipStream_t st) {
    (void)hipGetLastError();
    hipLaunchKernelGGL(gale_zero_kernel, dim3(1), dim3(64), 0, st, p, n);
    return hipGetLastError();
}

template <bool kL>
static hipError_t launch_items_t(const KArgs &a, int block_threads, int grid, size_t lds, hipStream_t st) {
    (void)hipGetLastError();  // the launch status below is this launch's, not an earlier call's
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
    (void)hipGetLastError();  // the launch status below is this launch's, not an earlier call's
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
                    : launch_items_t<false>(a, block_threads, grid, lds, st);
}

hipError_t launch_persistent(const KArgs &a, bool lds_path, int block_threads, int grid, size_t lds,
                             hipStream_t st) {
    return lds_path ? launch_persistent_t<true>(a, block_threads, grid, lds, st)
                    : launch_persistent_t<false>(a, block_threads, grid, lds, st);
}

// every builder kernel takes dynamic LDS (the global path for its hybrid form)
static const void *const kLdsKernels[] = {
    (const void *)gale_items_kernel<256, true>,       (const void *)gale_items_kernel<512, true>,
    (const void *)gale_items_kernel<1024, true>,      (const void *)gale_persistent_kernel<256, true>,
    (const void *)gale_persistent_kernel<512, true>,  (const void *)gale_persistent_kernel<1024, true>,
    (const void *)gale_items_kernel<256, false>,      (const void *)gale_items_kernel<512, false>,
    (const void *)gale_items_kernel<1024, false>,     (const void *)gale_persistent_kernel<256, false>,
    (const void *)gale_persistent_kernel<512, false>, (const void *)gale_persistent_kernel<1024, false>,
};

hipError_t static_lds_bytes(int64_t *bytes) {
    int64_t mx = 0;
    for (const void *f : kLdsKernels) {
        hipFuncAttributes at;
        const hipError_t e = hipFuncGetAttributes(&at, f);
        if (e != hipSuccess) return e;
        mx = at.sharedSizeBytes > (size_t)mx ? (int64_t)at.sharedSizeBytes : mx;
    }
    *bytes = mx;
    return hipSuccess;
}

hipError_t set_lds_limits(size_t lds) {
    for (const void *f : kLdsKernels) {
        const hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

#ifdef GALE_PHASE_TIMING
extern "C" int gale_debug_phase_cycles(unsigned long long *out, int reset) {
    hipError_t e = hipMemcpyFromSymbol(out, HIP_SYMBOL(g_phase_cycles), sizeof(g_phase_cycles));
    if (reset) {
        unsigned long long z[48] = {0};
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
        return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, gale_persistent_kernel<1024, false>, 1024, lds);
    if (block_threads == 512)
        return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, gale_persistent_kernel<512, false>, 512, lds);
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, gale_persistent_kernel<256, false>, 256, lds);
}

}  // namespace gale
