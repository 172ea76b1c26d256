// gale_cobound.hip -- per-cluster VE / VF / EF / ET / FT builders for gfx950.
//
// The coboundary relations of edges and triangles (paper, Section 2.2,
// Table 1): VE(v) and VF(v) the edges and triangles containing a vertex of
// the cluster, EF(e) and ET(e) the triangles and tetrahedra containing an
// edge internal to the cluster, FT(f) the tetrahedra containing an internal
// triangle.  Every simplex containing such a row contains a vertex of the
// cluster, so the cluster's star holds all of them; as in Section 4.6 the
// kernel iterates the star's tetrahedra, takes the vertex combinations each
// relation needs and relates them, here as (row, entry id) incidences:
//   count the incidences of every row (LDS-free atomics in the workgroup's
//   workspace slice), scan, scatter the entry ids, then sort each row and drop
//   repeats (a triangle through a vertex is met from both its tetrahedra),
//   scan the distinct counts and write the CSR block.
// Edge and triangle ids come from the lists of the initialization step
// (Section 4.3), looked up by binary search in the list of the simplex's
// smallest vertex.  One workgroup per (cluster, relation mask), taken from a
// device queue by a persistent launch.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gale_devutil.h"
#include "gale_host.h"
#include "gale_layout.h"

namespace gale {

namespace {

constexpr int32_t kVidMask = 0x3fffffff;

__device__ __forceinline__ int32_t edge_id(const Simplices &s, int32_t u, int32_t v) {
    int lo = s.eoff[u], hi = s.eoff[u + 1];
    const int end = hi;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (s.eidx[2 * mid] < v) lo = mid + 1;
        else hi = mid;
    }
    return (lo < end && s.eidx[2 * lo] == v) ? s.eidx[2 * lo + 1] : -1;
}

__device__ __forceinline__ int32_t face_id(const Simplices &s, int32_t a, int32_t b, int32_t c) {
    int lo = s.foff[a], hi = s.foff[a + 1];
    const int end = hi;
    const int4 *f = reinterpret_cast<const int4 *>(s.fidx);
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        const int4 q = f[mid];
        if (q.x < b || (q.x == b && q.y < c)) lo = mid + 1;
        else hi = mid;
    }
    if (lo < end) {
        const int4 q = f[lo];
        if (q.x == b && q.y == c) return q.z;
    }
    return -1;
}

constexpr int kPair[6][2] = {{0, 1}, {0, 2}, {0, 3}, {1, 2}, {1, 3}, {2, 3}};

// One wave sorts n keys that may repeat (n wave-uniform): the bitonic
// networks up to 256, beyond that each key goes to its stable rank (smaller
// keys, plus equal keys earlier in the list).
template <class F>
__device__ __forceinline__ void wave_sort_rep(int n, const F &key, int32_t *dst) {
    if (n <= 256) {
        wave_sort(n, key, dst);
        return;
    }
    const int lane = threadIdx.x & 63;
    for (int i0 = 0; i0 < n; i0 += 64) {
        const int i = i0 + lane;
        const uint32_t x = i < n ? (uint32_t)key(i) : 0xFFFFFFFFu;
        int rk = 0;
        for (int j = 0; j < n; ++j) {
            const uint32_t y = (uint32_t)key(j);
            rk += (y < x) | ((y == x) & (j < i));
        }
        if (i < n) dst[rk] = (int32_t)x;
    }
}

// Workspace words of one work item: row index and row vertex of every local
// vertex, counts and fill pointers per row, two incidence arrays.
__host__ __device__ __forceinline__ void ext_ws_words(const ClusterMeta &m, const ExtMeta &x, uint32_t mask,
                                                      int64_t &R, int64_t &I, int64_t &total) {
    R = 0;
    I = 0;
    for (int r = 0; r < 5; ++r) {
        if (!(mask & (kRelVE << r))) continue;
        R = ext_nrows(r, m, x) > R ? ext_nrows(r, m, x) : R;
        I = ext_cap(r, m, x) > I ? ext_cap(r, m, x) : I;
    }
    total = (int64_t)m.L + m.nV + 2 * (R + 1) + 2 * I + 16;
}

template <int B>
__device__ __attribute__((always_inline)) void ext_item(const KArgs &a, const WorkItem &it, int32_t *ws) {
    __shared__ int s_status;
    int sp = 0;
    const int tid = threadIdx.x, lane = tid & 63;
    const ClusterMeta m = a.s.meta[it.cluster];
    const ExtMeta x = a.x.ext[it.cluster];
    const uint32_t mask = it.mask;
    const ExtLayout lay = ext_layout(mask, m, x);
    int32_t *blk = a.out + it.out_word;
    const char *tb = a.s.tets + m.tb_off;
    const bool wide = (m.flags & kMetaWide) != 0;
    const int32_t *idg = a.s.tid + m.tet_off;
    const int32_t *lvg = a.s.lverts + m.lv_off;
    int64_t R, I, W;
    ext_ws_words(m, x, mask, R, I, W);
    int32_t *rix = ws;
    int32_t *rowl = rix + m.L;
    int32_t *cnt = rowl + m.nV;
    int32_t *fill = cnt + (R + 1);
    int32_t *keys = fill + (R + 1);
    int32_t *keys2 = keys + I;
    if (tid == 0) s_status = 0;

    // rows of VE / VF: the cluster's vertices in local (= original id) order
    if (mask & (kRelVE | kRelVF)) {
        int carry = 0;
        for (int i0 = 0; i0 < m.L; i0 += B) {
            const int i = i0 + tid;
            const int f = (i < m.L && lvg[i] < 0) ? 1 : 0;
            int tot;
            const int ex = block_excl_scan<B>(f, tot, sp);
            if (i < m.L) {
                rix[i] = f ? carry + ex : -1;
                if (f && carry + ex < m.nV) rowl[carry + ex] = i;
            }
            carry += tot;
        }
        if (tid == 0 && carry != m.nV) atomicOr(&s_status, kStInconsistent);
    }
    __syncthreads();

    auto tet = [&](int p, int32_t *l) {
        if (wide) {
            const int4 q = reinterpret_cast<const int4 *>(tb)[p];
            l[0] = q.x, l[1] = q.y, l[2] = q.z, l[3] = q.w;
        } else {
            const ushort4 q = reinterpret_cast<const ushort4 *>(tb)[p];
            l[0] = q.x, l[1] = q.y, l[2] = q.z, l[3] = q.w;
        }
    };

    for (int r = 0; r < 5; ++r) {
        if (!(mask & (kRelVE << r))) continue;
        const int nr = lay.nrows[r], cap = lay.cap[r];
        for (int i = tid; i <= nr; i += B) cnt[i] = 0;
        __syncthreads();
        // The incidences of tetrahedron p for relation r: emit(row, id) for
        // each; with keyed = false the ids are not looked up (counting pass,
        // VE / VF, whose rows need no lookup).
        auto incidences = [&](int p, bool keyed, auto emit) {
            int32_t l[4], o[4];
            bool row[4], low[4];
            tet(p, l);
            for (int q = 0; q < 4; ++q) {
                const int32_t w = lvg[l[q]];
                o[q] = w & kVidMask;
                row[q] = w < 0;
                low[q] = (w & 0x40000000) != 0;
            }
            const int32_t tid_p = idg[p] & 0x7fffffff;
            if (r == 0) {  // VE: the three edges at each row vertex
                for (int q = 0; q < 4; ++q) {
                    if (!row[q]) continue;
                    const int rr = rix[l[q]];
                    if (rr < 0 || rr >= m.nV) {
                        atomicOr(&s_status, kStInconsistent);
                        continue;
                    }
                    for (int q2 = 0; q2 < 4; ++q2) {
                        if (q2 == q) continue;
                        emit(rr, keyed ? edge_id(a.x, o[q < q2 ? q : q2], o[q < q2 ? q2 : q]) : 0);
                    }
                }
            } else if (r == 1) {  // VF: the three triangles at each row vertex
                for (int q = 0; q < 4; ++q) {
                    if (!row[q]) continue;
                    const int rr = rix[l[q]];
                    if (rr < 0 || rr >= m.nV) {
                        atomicOr(&s_status, kStInconsistent);
                        continue;
                    }
                    for (int j = 0; j < 4; ++j) {
                        if (j == q) continue;  // the triangle without vertex j
                        const int i0 = j == 0 ? 1 : 0, i1 = j <= 1 ? 2 : 1, i2 = j == 3 ? 2 : 3;
                        emit(rr, keyed ? face_id(a.x, o[i0], o[i1], o[i2]) : 0);
                    }
                }
            } else if (r <= 3) {  // EF / ET: the internal edges of the tetrahedron
                for (int q = 0; q < 6; ++q) {
                    const int qa = kPair[q][0], qb = kPair[q][1];
                    if (low[qa] || low[qb] || !(row[qa] || row[qb])) continue;
                    const int32_t e = edge_id(a.x, o[qa], o[qb]);
                    const int rr = e - x.e0;
                    if (e < 0 || rr < 0 || rr >= x.ne) {
                        atomicOr(&s_status, kStInconsistent);
                        continue;
                    }
                    if (r == 3) {
                        emit(rr, tid_p);
                    } else {
                        for (int qc = 0; qc < 4; ++qc) {
                            if (qc == qa || qc == qb) continue;
                            // ascending: the three indices in order
                            const int i0 = qc < qa ? qc : qa;
                            const int i2 = qc > qb ? qc : qb;
                            const int i1 = qa + qb + qc - i0 - i2;
                            emit(rr, keyed ? face_id(a.x, o[i0], o[i1], o[i2]) : 0);
                        }
                    }
                }
            } else {  // FT: the internal triangles of the tetrahedron
                for (int j = 0; j < 4; ++j) {
                    const int i0 = j == 0 ? 1 : 0, i1 = j <= 1 ? 2 : 1, i2 = j == 3 ? 2 : 3;
                    if (low[i0] || low[i1] || low[i2] || !(row[i0] || row[i1] || row[i2])) continue;
                    const int32_t f = face_id(a.x, o[i0], o[i1], o[i2]);
                    const int rr = f - x.f0;
                    if (f < 0 || rr < 0 || rr >= x.nf) {
                        atomicOr(&s_status, kStInconsistent);
                        continue;
                    }
                    emit(rr, tid_p);
                }
            }
        };
        for (int p = tid; p < m.ns; p += B)
            incidences(p, false, [&](int rr, int32_t) { atomicAdd(&cnt[rr], 1); });
        __syncthreads();
        {
            int carry = 0;
            for (int r0 = 0; r0 < nr; r0 += B) {
                const int rr = r0 + tid;
                const int v = rr < nr ? cnt[rr] : 0;
                int tot;
                const int ex = block_excl_scan<B>(v, tot, sp);
                if (rr < nr) {
                    cnt[rr] = carry + ex;
                    fill[rr] = carry + ex;
                }
                carry += tot;
            }
            if (tid == 0) {
                cnt[nr] = carry;
                if (carry > cap) atomicOr(&s_status, kStInconsistent);
            }
        }
        __syncthreads();
        if (cnt[nr] > cap) break;  // reported; never write past the capacity
        for (int p = tid; p < m.ns; p += B)
            incidences(p, true, [&](int rr, int32_t id) { keys[atomicAdd(&fill[rr], 1)] = id; });
        __syncthreads();
        // each row sorted into keys2 at its start, repeats dropped; the
        // distinct count replaces the fill pointer
        for (int rb = 0; rb < nr; rb += B) {
            const int rr = rb + tid;
            const int n = rr < nr ? cnt[rr + 1] - cnt[rr] : -1;
            const bool shrt = n >= 0 && n <= 32, lng = n > 32;
            const unsigned long long o16 = __ballot(shrt && n > 16), o8 = __ballot(shrt && n > 8),
                                     o4 = __ballot(shrt && n > 4);
            auto short_row = [&](auto ntag) {
                constexpr int N = decltype(ntag)::value;
                const int s0 = cnt[rr];
                uint32_t v[N];
#pragma unroll
                for (int i = 0; i < N; ++i) v[i] = i < n ? (uint32_t)keys[s0 + i] : 0xFFFFFFFFu;
                sort_regs<N>(v);
                int u = 0;
                uint32_t prev = 0xFFFFFFFFu;
#pragma unroll
                for (int i = 0; i < N; ++i) {
                    if (i < n && v[i] != prev) {
                        keys2[s0 + u] = (int32_t)v[i];
                        ++u;
                    }
                    prev = v[i];
                }
                fill[rr] = u;
            };
            if (shrt) {
                if (o16) short_row(std::integral_constant<int, 32>{});
                else if (o8) short_row(std::integral_constant<int, 16>{});
                else if (o4) short_row(std::integral_constant<int, 8>{});
                else short_row(std::integral_constant<int, 4>{});
            }
            unsigned long long bal = __ballot(lng);
            while (bal) {
                const int r2 = rb + (tid & ~63) + __ffsll((long long)bal) - 1;
                bal &= bal - 1;
                const int s0 = cnt[r2], n2 = cnt[r2 + 1] - s0;
                wave_sort_rep(n2, [&](int i) { return keys[s0 + i]; }, keys2 + s0);
                __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
                __builtin_amdgcn_wave_barrier();
                // drop repeats in place (a value is kept when it differs from
                // the one before it; writes never pass the chunk being read)
                int u = 0, prev = -1;
                for (int i0 = 0; i0 < n2; i0 += 64) {
                    const int i = i0 + lane;
                    const int v = i < n2 ? keys2[s0 + i] : -1;
                    int before = __shfl_up(v, 1, 64);
                    if (lane == 0) before = prev;
                    const bool keep = i < n2 && v != before;
                    const unsigned long long km = __ballot(keep);
                    const int rank = __popcll(km & ((1ull << lane) - 1ull));
                    if (keep) keys2[s0 + u + rank] = v;
                    prev = __shfl(v, 63, 64);
                    u += __popcll(km);
                }
                if (lane == 0) fill[r2] = u;
                __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
                __builtin_amdgcn_wave_barrier();
            }
        }
        __syncthreads();
        {
            int carry = 0;
            for (int r0 = 0; r0 < nr; r0 += B) {
                const int rr = r0 + tid;
                const int u = rr < nr ? fill[rr] : 0;
                int tot;
                const int ex = block_excl_scan<B>(u, tot, sp);
                if (rr < nr) {
                    const int o = carry + ex;
                    blk[lay.off[r] + rr] = o;
                    blk[lay.rows[r] + rr] = r <= 1 ? (lvg[rowl[rr]] & kVidMask) : (r <= 3 ? x.e0 + rr : x.f0 + rr);
                    const int s0 = cnt[rr];
                    for (int j = 0; j < u; ++j) blk[lay.ent[r] + o + j] = keys2[s0 + j];
                }
                carry += tot;
            }
            if (tid == 0) {
                blk[lay.off[r] + nr] = carry;
                blk[1 + r] = carry;
            }
        }
        __syncthreads();
    }
    __syncthreads();
    if (tid == 0) {
        int32_t h[8];
        h[0] = s_status;
        for (int r = 0; r < 5; ++r) h[1 + r] = (mask & (kRelVE << r)) ? blk[1 + r] : 0;
        h[6] = h[7] = 0;
        for (int i = 0; i < 8; ++i) blk[i] = h[i];
        if (a.hdr)
            for (int i = 0; i < 8; ++i) a.hdr[(int64_t)it.hdr_index * 8 + i] = h[i];
    }
    __syncthreads();
}

template <int B>
__global__ __launch_bounds__(B) void gale_ext_kernel(KArgs a) {
    __shared__ int s_idx;
    int32_t *ws = reinterpret_cast<int32_t *>(a.ws + (int64_t)blockIdx.x * a.ws_stride);
    while (true) {
        if (threadIdx.x == 0) s_idx = atomicAdd(a.queue, 1);
        __syncthreads();
        const int idx = s_idx;
        __syncthreads();
        if (idx >= a.nitems) break;
        ext_item<B>(a, a.items[idx], ws);
    }
}

}  // namespace

int64_t ext_workspace_bytes(const ClusterMeta &m, const ExtMeta &x, uint32_t mask) {
    int64_t R, I, W;
    ext_ws_words(m, x, mask, R, I, W);
    return (W * 4 + 255) / 256 * 256;
}

hipError_t launch_ext(const KArgs &a, int grid, hipStream_t st) {
    (void)hipGetLastError();
    hipLaunchKernelGGL((gale_ext_kernel<kExtThreads>), dim3(grid), dim3(kExtThreads), 0, st, a);
    return hipGetLastError();
}

}  // namespace gale
