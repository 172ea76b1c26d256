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
// VT (paper Section 4.6: iterate the segment's tetrahedra, take the vertices
// that belong to the segment, relate them): count per row with LDS atomics,
// inclusive scan, scatter stream positions with atomic decrements, then sort
// each row's positions.  Stream order is ascending tetrahedron id, so sorted
// positions are the canonical VT row.  No global atomics (the paper's VT
// kernel is limited by atomics on one vertex, Appendix A.1).
//
// VV (Algorithm 1: for each tetrahedron and each of its vertices in the
// segment, relate the other three vertices, without duplicates): per pass of
// rc rows, each row owns an LDS bitmap over the local vertex table; the table
// is sorted by original id, so reading the set bits in order yields the row
// already sorted and duplicate-free.  Replaces the paper's fixed-width -1
// initialised relation matrix and atomicPush (Algorithm 2), whose output order
// depends on thread arrival.
//
// TT (two tetrahedra are adjacent iff they share a triangle, Section 2.2): the
// faces of the tetrahedra internal to the cluster go into an LDS hash table
// keyed by their sorted local vertex ids (each slot holds up to two face
// references); the faces of the other stream tetrahedra (external star and
// halo) are then looked up and attached as the second sharer.  A face met a
// third time (non-manifold) or a full table switches the cluster to an
// exhaustive O(rows x stream) pairing.
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
struct Face {
    int a, b, c;  // ascending local ids
};

__device__ __forceinline__ bool operator==(const Face &x, const Face &y) {
    return x.a == y.a && x.b == y.b && x.c == y.c;
}

__device__ __forceinline__ void cswap(int &x, int &y) {
    int lo = min(x, y), hi = max(x, y);
    x = lo;
    y = hi;
}

// face k of t is t without its k-th vertex
__device__ __forceinline__ Face face_of(int4 t, int k) {
    int a, b, c;
    if (k == 0) { a = t.y; b = t.z; c = t.w; }
    else if (k == 1) { a = t.x; b = t.z; c = t.w; }
    else if (k == 2) { a = t.x; b = t.y; c = t.w; }
    else { a = t.x; b = t.y; c = t.z; }
    cswap(a, b);
    cswap(b, c);
    cswap(a, b);
    return Face{a, b, c};
}

__device__ __forceinline__ uint32_t face_hash(const Face &f) {
    uint32_t h = (uint32_t)f.a * 0x9E3779B1u ^ (uint32_t)f.b * 0x85EBCA77u ^ (uint32_t)f.c * 0xC2B2AE3Du;
    h ^= h >> 15;
    h *= 0x2C1B3C6Du;
    h ^= h >> 12;
    h *= 0x297A2D39u;
    h ^= h >> 15;
    return h;
}

__device__ __forceinline__ uint32_t fast_range(uint32_t h, uint32_t n) {
    return (uint32_t)(((uint64_t)h * (uint64_t)n) >> 32);
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
template <int B, bool kL>
__device__ void build_cluster(const KArgs &a, const WorkItem &it, const ClusterMeta &m, const Plan &pl,
                              char *smem, char *ws) {
    using PosT = typename std::conditional<kL, uint16_t, int32_t>::type;
    using RowT = typename std::conditional<kL, int16_t, int32_t>::type;
    using SlotT = typename std::conditional<kL, uint32_t, unsigned long long>::type;
    constexpr int kRefBits = kL ? 16 : 32;
    constexpr SlotT kRefMask = kL ? (SlotT)0xFFFFu : (SlotT)0xFFFFFFFFull;
    constexpr SlotT kEmpty = kL ? (SlotT)0xFFFFFFFFu : (SlotT)0xFFFFFFFFFFFFFFFFull;

    __shared__ int s_status;
    const int tid = threadIdx.x;
    const int ns = m.ns, nh = m.nh, ntot = ns + nh, nT = m.nT, L = m.L, nV = m.nV;
    const uint32_t mask = it.mask;
    const int4 *tg = a.s.tets + m.tet_off;
    const int32_t *idg = a.s.tid + m.tet_off;
    const int32_t *lvg = a.s.lverts + m.lv_off;
    int32_t *blk = a.out + it.out_word;
    const BlockLayout lay = block_layout(mask, nV, nT, m.nnzVT, it.cap_vv, it.cap_tt);
    char *base = kL ? smem : ws;

    ushort4 *lt = reinterpret_cast<ushort4 *>(smem + pl.tets);
    unsigned long long *ib = reinterpret_cast<unsigned long long *>(smem + pl.ibits);

    if (tid == 0) s_status = 0;
#ifdef GALE_PHASE_TIMING
    unsigned long long phase_t0 = __builtin_amdgcn_s_memtime();
#endif

    auto tet = [&](int p) -> int4 {
        if constexpr (kL) {
            ushort4 q = lt[p];
            return make_int4(q.x, q.y, q.z, q.w);
        } else {
            return tg[p];
        }
    };
    auto internal = [&](int p) -> bool {
        if constexpr (kL) {
            return p < ns && ((ib[p >> 6] >> (p & 63)) & 1ull);
        } else {
            return p < ns && idg[p] < 0;
        }
    };

    // ---- stage the stream in LDS ---------------------------------------
    if constexpr (kL) {
        for (int p = tid; p < ntot; p += B) {
            int4 t = tg[p];
            lt[p] = make_ushort4((unsigned short)t.x, (unsigned short)t.y, (unsigned short)t.z,
                                 (unsigned short)t.w);
        }
        if (mask & kRelTT) {
            const int lane = tid & 63, wid = tid >> 6;
            const int nwords = (ns + 63) >> 6;
            for (int w = wid; w < nwords; w += B / 64) {
                const int p = w * 64 + lane;
                const bool f = p < ns && idg[p] < 0;
                const unsigned long long bits = __ballot(f);
                if (lane == 0) ib[w] = bits;
            }
        }
    }
    __syncthreads();
    PHASE_MARK(0);

#ifdef GALE_DEBUG_CHECKS
    auto check_lt = [&](int bit) {
        if constexpr (kL) {
            for (int p = tid; p < ntot; p += B) {
                int4 t = tg[p];
                ushort4 q = lt[p];
                if (q.x != (unsigned short)t.x || q.y != (unsigned short)t.y || q.z != (unsigned short)t.z ||
                    q.w != (unsigned short)t.w)
                    atomicOr(&s_status, bit);
            }
        }
        __syncthreads();
    };
    check_lt(1 << 16);
#endif
    // ---- VT / VV ---------------------------------------------------------
    if (mask & (kRelVT | kRelVV)) {
        RowT *rowOf = reinterpret_cast<RowT *>(base + pl.rowof);
        int32_t *cnt = reinterpret_cast<int32_t *>(base + pl.cnt);
        PosT *lst = reinterpret_cast<PosT *>(base + pl.lst);

        // local vertex -> row index; row ids
        int carry = 0;
        for (int i0 = 0; i0 < L; i0 += B) {
            const int i = i0 + tid;
            const int32_t lv = i < L ? lvg[i] : 0;
            const int f = (i < L && lv < 0) ? 1 : 0;
            int tot;
            const int ex = block_excl_scan<B>(f, tot);
            if (i < L) {
                const int r = carry + ex;
                // rows past nV would mean inconsistent metadata: drop them (flagged below)
                rowOf[i] = (f && r < nV) ? (RowT)r : (RowT)-1;
                if (f && r < nV) blk[lay.vrows + r] = lv & kIdMask;
            }
            carry += tot;
        }
        if (tid == 0 && carry != nV) s_status |= kStInconsistent;
        for (int r = tid; r <= nV; r += B) cnt[r] = 0;
        __syncthreads();
        PHASE_MARK(1);

        // count
        for (int p = tid; p < ns; p += B) {
            const int4 t = tet(p);
            const int r0 = rowOf[t.x], r1 = rowOf[t.y], r2 = rowOf[t.z], r3 = rowOf[t.w];
            if (r0 >= 0) atomicAdd(&cnt[r0], 1);
            if (r1 >= 0) atomicAdd(&cnt[r1], 1);
            if (r2 >= 0) atomicAdd(&cnt[r2], 1);
            if (r3 >= 0) atomicAdd(&cnt[r3], 1);
        }
        __syncthreads();

        PHASE_MARK(2);
        // inclusive scan: cnt[r] = end of row r
        carry = 0;
        for (int r0 = 0; r0 < nV; r0 += B) {
            const int r = r0 + tid;
            const int v = r < nV ? cnt[r] : 0;
            int tot;
            const int ex = block_excl_scan<B>(v, tot);
            if (r < nV) cnt[r] = carry + ex + v;
            carry += tot;
        }
        const int nnz = carry;
        const bool vt_ok = nnz == m.nnzVT;
        if (tid == 0) {
            cnt[nV] = nnz;
            if (!vt_ok) s_status |= kStInconsistent;
        }
        __syncthreads();

        PHASE_MARK(3);
        // scatter stream positions; afterwards cnt[r] = start of row r
        if (vt_ok) {
            for (int p = tid; p < ns; p += B) {
                const int4 t = tet(p);
                const int r0 = rowOf[t.x], r1 = rowOf[t.y], r2 = rowOf[t.z], r3 = rowOf[t.w];
                if (r0 >= 0) lst[atomicSub(&cnt[r0], 1) - 1] = (PosT)p;
                if (r1 >= 0) lst[atomicSub(&cnt[r1], 1) - 1] = (PosT)p;
                if (r2 >= 0) lst[atomicSub(&cnt[r2], 1) - 1] = (PosT)p;
                if (r3 >= 0) lst[atomicSub(&cnt[r3], 1) - 1] = (PosT)p;
            }
        }
        __syncthreads();

        PHASE_MARK(4);
        if (vt_ok) {
            // sort each row's positions (rows are short; insertion sort)
            for (int r = tid; r < nV; r += B) {
                const int s = cnt[r], e = cnt[r + 1];
                for (int i = s + 1; i < e; ++i) {
                    const PosT x = lst[i];
                    int j = i - 1;
                    while (j >= s && lst[j] > x) {
                        lst[j + 1] = lst[j];
                        --j;
                    }
                    lst[j + 1] = x;
                }
            }
        }
        __syncthreads();

        PHASE_MARK(5);
        if ((mask & kRelVT) && vt_ok) {
            for (int r = tid; r <= nV; r += B) blk[lay.vt_off + r] = cnt[r];
            for (int e = tid; e < nnz; e += B) blk[lay.vt_ent + e] = idg[lst[e]] & kIdMask;
        }

        PHASE_MARK(6);
        if ((mask & kRelVV) && vt_ok) {
            uint32_t *bm = reinterpret_cast<uint32_t *>(base + pl.bm);
            const int rc = pl.rc, W = pl.W, Wp = pl.Wp;
            const int cap = it.cap_vv;
            int vcarry = 0;
            for (int r0 = 0; r0 < nV; r0 += rc) {
                const int nr = min(rc, nV - r0);
                for (int w = tid; w < nr * Wp; w += B) bm[w] = 0u;
                __syncthreads();
                int c = 0;
                if (tid < nr) {
                    const int r = r0 + tid;
                    uint32_t *row = bm + (int64_t)tid * Wp;
                    const int s = cnt[r], e = cnt[r + 1];
                    for (int i = s; i < e; ++i) {
                        const int4 t = tet(lst[i]);
                        if (rowOf[t.x] != r) row[t.x >> 5] |= 1u << (t.x & 31);
                        if (rowOf[t.y] != r) row[t.y >> 5] |= 1u << (t.y & 31);
                        if (rowOf[t.z] != r) row[t.z >> 5] |= 1u << (t.z & 31);
                        if (rowOf[t.w] != r) row[t.w >> 5] |= 1u << (t.w & 31);
                    }
                    for (int w = 0; w < W; ++w) c += __popc(row[w]);
                }
                int tot;
                const int ex = block_excl_scan<B>(c, tot);
                if (tid < nr) {
                    const int r = r0 + tid;
                    int pos = vcarry + ex;
                    blk[lay.vv_off + r] = pos;
                    const uint32_t *row = bm + (int64_t)tid * Wp;
                    for (int w = 0; w < W; ++w) {
                        uint32_t bits = row[w];
                        while (bits) {
                            const int b = __ffs(bits) - 1;
                            bits &= bits - 1u;
                            if (pos < cap) blk[lay.vv_ent + pos] = lvg[w * 32 + b] & kIdMask;
                            ++pos;
                        }
                    }
                }
                vcarry += tot;
                __syncthreads();
            }
            if (tid == 0) {
                blk[lay.vv_off + nV] = vcarry;
                blk[4] = vcarry;
                if (vcarry > cap) s_status |= kStVVOverflow;
            }
        }
        __syncthreads();
        PHASE_MARK(7);
    }

#ifdef GALE_DEBUG_CHECKS
    check_lt(1 << 17);
#endif
    // ---- TT --------------------------------------------------------------
    if (mask & kRelTT) {
        SlotT *ht = reinterpret_cast<SlotT *>(base + pl.ht);
        const uint32_t H = (uint32_t)pl.H;
        const int cap = it.cap_tt;
        __shared__ int s_fail;
        if (tid == 0) s_fail = 0;
        for (uint32_t i = tid; i < H; i += B) ht[i] = kEmpty;
        __syncthreads();

        auto face_of_ref = [&](uint32_t ref) -> Face { return face_of(tet((int)(ref >> 2)), (int)(ref & 3u)); };

        // attach ref as the second sharer of slot s whose first sharer has the same face
        auto attach = [&](uint32_t s, SlotT cur, uint32_t ref) {
            const SlotT first = cur & kRefMask;
            while (true) {
                if (((cur >> kRefBits) & kRefMask) != kRefMask) {
                    s_fail = 1;  // third sharer: non-manifold face
                    return;
                }
                const SlotT want = ((SlotT)ref << kRefBits) | first;
                const SlotT got = atomicCAS(&ht[s], cur, want);
                if (got == cur) return;
                cur = got;
            }
        };

        // faces of internal tetrahedra
        if (H > 0) {
            for (int p = tid; p < ns; p += B) {
                if (!internal(p)) continue;
                const int4 t = tet(p);
                for (int k = 0; k < 4; ++k) {
                    const Face f = face_of(t, k);
                    const uint32_t ref = (uint32_t)p * 4u + (uint32_t)k;
                    uint32_t s = fast_range(face_hash(f), H);
                    bool done = false;
                    for (uint32_t n = 0; n < H && !done; ++n) {
                        const SlotT cur = atomicCAS(&ht[s], kEmpty, ((SlotT)kRefMask << kRefBits) | (SlotT)ref);
                        if (cur == kEmpty) {
                            done = true;
                        } else if (face_of_ref((uint32_t)(cur & kRefMask)) == f) {
                            attach(s, cur, ref);
                            done = true;
                        } else {
                            s = (s + 1 == H) ? 0 : s + 1;
                        }
                    }
                    if (!done) s_fail = 1;  // table full
                }
            }
        }
        __syncthreads();

        PHASE_MARK(8);
        // faces of the other stream tetrahedra: attach where an internal face matches
        if (H > 0) {
            for (int p = tid; p < ntot; p += B) {
                if (internal(p)) continue;
                const int4 t = tet(p);
                for (int k = 0; k < 4; ++k) {
                    const Face f = face_of(t, k);
                    const uint32_t ref = (uint32_t)p * 4u + (uint32_t)k;
                    uint32_t s = fast_range(face_hash(f), H);
                    for (uint32_t n = 0; n < H; ++n) {
                        const SlotT cur = __atomic_load_n(&ht[s], __ATOMIC_RELAXED);
                        if (cur == kEmpty) break;
                        if (face_of_ref((uint32_t)(cur & kRefMask)) == f) {
                            attach(s, cur, ref);
                            break;
                        }
                        s = (s + 1 == H) ? 0 : s + 1;
                    }
                }
            }
        }
        __syncthreads();
#ifdef GALE_DEBUG_CHECKS
        check_lt(1 << 18);
#endif
        PHASE_MARK(9);
        const bool fallback = s_fail != 0;
        if (tid == 0 && fallback) s_status |= kStTTFallback;

        int rcarry = 0, ecarry = 0;
        for (int p0 = 0; p0 < ns; p0 += B) {
            const int p = p0 + tid;
            const bool in = internal(p);
            int n0 = 0x7fffffff, n1 = 0x7fffffff, n2 = 0x7fffffff, n3 = 0x7fffffff;
            int c = 0;
            if (in && !fallback) {
                const int4 t = tet(p);
                int nb[4];
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    nb[k] = 0x7fffffff;
                    const Face f = face_of(t, k);
                    const uint32_t myref = (uint32_t)p * 4u + (uint32_t)k;
                    uint32_t s = fast_range(face_hash(f), H);
                    for (uint32_t n = 0; n < H; ++n) {
                        const SlotT cur = ht[s];
                        if (cur == kEmpty) break;
                        const uint32_t first = (uint32_t)(cur & kRefMask);
                        const uint32_t second = (uint32_t)((cur >> kRefBits) & kRefMask);
                        if (first == myref) {
                            if (second != (uint32_t)kRefMask) nb[k] = idg[second >> 2] & kIdMask;
                            break;
                        }
                        if (face_of_ref(first) == f) {
                            nb[k] = idg[first >> 2] & kIdMask;
                            break;
                        }
                        s = (s + 1 == H) ? 0 : s + 1;
                    }
                }
                n0 = nb[0]; n1 = nb[1]; n2 = nb[2]; n3 = nb[3];
                cswap(n0, n1); cswap(n2, n3); cswap(n0, n2); cswap(n1, n3); cswap(n1, n2);
                // drop repeats (a duplicated tetrahedron shares several faces) and missing
                if (n3 == n2) n3 = 0x7fffffff;
                if (n2 == n1) { n2 = n3; n3 = 0x7fffffff; }
                if (n1 == n0) { n1 = n2; n2 = n3; n3 = 0x7fffffff; }
                c = (n0 != 0x7fffffff) + (n1 != 0x7fffffff) + (n2 != 0x7fffffff) + (n3 != 0x7fffffff);
            } else if (in) {
                const int4 t = tet(p);
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
                if (!fallback) {
                    if (c > 0 && pos + 0 < cap) blk[lay.tt_ent + pos + 0] = n0;
                    if (c > 1 && pos + 1 < cap) blk[lay.tt_ent + pos + 1] = n1;
                    if (c > 2 && pos + 2 < cap) blk[lay.tt_ent + pos + 2] = n2;
                    if (c > 3 && pos + 3 < cap) blk[lay.tt_ent + pos + 3] = n3;
                } else {
                    const int4 t = tet(p);
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
            }
            rcarry += rtot;
            ecarry += etot;
        }
        if (tid == 0) {
            blk[lay.tt_off + (rcarry <= nT ? rcarry : nT)] = ecarry;
            blk[5] = ecarry;
            if (rcarry != nT) s_status |= kStInconsistent;
            if (ecarry > cap) s_status |= kStTTOverflow;
        }
        PHASE_MARK(10);
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
#ifdef GALE_DEBUG_CHECKS
        h[6] = (int32_t)pl.ht | (kL ? (1 << 30) : 0);
        h[7] = (int32_t)pl.rowof;
#endif
        for (int i = 0; i < 8; ++i) blk[i] = h[i];
        if (a.hdr)
            for (int i = 0; i < 8; ++i) a.hdr[(int64_t)it.hdr_index * 8 + i] = h[i];
    }
    __syncthreads();
}

template <int B>
__device__ void process_item(const KArgs &a, const WorkItem &it, char *smem, char *ws) {
    const ClusterMeta m = a.s.meta[it.cluster];
    const Plan lp = lds_plan(m, it.mask, a.lds_budget, B);
    if (lp.ok) {
        build_cluster<B, true>(a, it, m, lp, smem, ws);
    } else if (ws == nullptr) {
        // the host sizes the workspace from the same plan; without it, report and skip
        if (threadIdx.x == 0) {
            int32_t *blk = a.out + it.out_word;
            blk[0] = kStInconsistent;
            if (a.hdr) a.hdr[(int64_t)it.hdr_index * 8] = kStInconsistent;
        }
        __syncthreads();
    } else {
        const Plan gp = ws_plan(m, it.mask, B);
        build_cluster<B, false>(a, it, m, gp, smem, ws);
    }
}

// One work item per workgroup: item blockIdx.x.  Used for the per-cluster
// (plain) form, one launch per (cluster, relation).
template <int B>
__global__ __launch_bounds__(B) void gale_items_kernel(KArgs a) {
    extern __shared__ __attribute__((aligned(16))) char smem[];
    const int i = blockIdx.x;
    if (i >= a.nitems) return;
    char *ws = a.ws ? a.ws + (int64_t)blockIdx.x * a.ws_stride : nullptr;
    process_item<B>(a, a.items[i], smem, ws);
}

// Persistent form: each workgroup takes the next item from the device work
// queue until the list is exhausted (every workgroup reaches the exit test).
template <int B>
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
        process_item<B>(a, a.items[idx], smem, ws);
    }
}

// ---------------------------------------------------------------------------
// host-side launch wrappers
// ---------------------------------------------------------------------------
hipError_t launch_items(const KArgs &a, int block_threads, int grid, size_t lds, hipStream_t st) {
    if (block_threads == 1024) {
        hipLaunchKernelGGL(gale_items_kernel<1024>, dim3(grid), dim3(1024), lds, st, a);
    } else if (block_threads == 512) {
        hipLaunchKernelGGL(gale_items_kernel<512>, dim3(grid), dim3(512), lds, st, a);
    } else {
        hipLaunchKernelGGL(gale_items_kernel<256>, dim3(grid), dim3(256), lds, st, a);
    }
    return hipGetLastError();
}

hipError_t launch_persistent(const KArgs &a, int block_threads, int grid, size_t lds, hipStream_t st) {
    if (block_threads == 1024) {
        hipLaunchKernelGGL(gale_persistent_kernel<1024>, dim3(grid), dim3(1024), lds, st, a);
    } else if (block_threads == 512) {
        hipLaunchKernelGGL(gale_persistent_kernel<512>, dim3(grid), dim3(512), lds, st, a);
    } else {
        hipLaunchKernelGGL(gale_persistent_kernel<256>, dim3(grid), dim3(256), lds, st, a);
    }
    return hipGetLastError();
}

hipError_t set_lds_limits(size_t lds) {
    hipError_t e;
    e = hipFuncSetAttribute((const void *)gale_items_kernel<256>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    e = hipFuncSetAttribute((const void *)gale_items_kernel<512>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    e = hipFuncSetAttribute((const void *)gale_persistent_kernel<256>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    e = hipFuncSetAttribute((const void *)gale_items_kernel<1024>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    e = hipFuncSetAttribute((const void *)gale_persistent_kernel<1024>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    return hipFuncSetAttribute((const void *)gale_persistent_kernel<512>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
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

hipError_t persistent_occupancy(int block_threads, size_t lds, int *blocks_per_cu) {
    if (block_threads == 1024)
        return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, gale_persistent_kernel<1024>, 1024, lds);
    if (block_threads == 512)
        return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, gale_persistent_kernel<512>, 512, lds);
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, gale_persistent_kernel<256>, 256, lds);
}

}  // namespace gale
