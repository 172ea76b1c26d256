// gale_stitch.hip -- assemble a tiled cluster's block from its tiles' blocks.
//
// Every row of the cluster (a vertex for VT / VV, an internal tetrahedron for
// TT) is a row of exactly one tile, with the same list there; the maps give,
// for the cluster's rows in ascending id, the tile and the row's index in the
// tile's block.  One workgroup per tiled cluster: row ids copied through the
// maps, each relation's row lengths scanned into the cluster's offsets, the
// lists copied; the relations of a cluster are separate items, so several
// workgroups share a cluster.  The header is the tiles' status bits and
// summed counts; a
// tile that exceeded a capacity bound makes the cluster report it (the host
// then builds the whole cluster again with exact capacities).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gale_devutil.h"
#include "gale_host.h"
#include "gale_layout.h"

namespace gale {

namespace {

constexpr int kMaxTiles = kMaxTilesPerCluster;

template <int B>
__device__ __attribute__((always_inline)) void stitch_item(const SArgs &a, const StitchItem &it) {
    __shared__ int s_status, s_nvv, s_ntt, s_nvt;
    __shared__ int64_t s_base[kMaxTiles];
    __shared__ BlockLayout s_lay[kMaxTiles];
    // a chunk's rows: where each list starts in the tile block, and where
    // it goes in the chunk's run of entries
    __shared__ int64_t s_src[B];
    __shared__ int s_pre[B];
    int sp = 0;
    const int tid = threadIdx.x;
    const ClusterMeta m = a.meta[it.cluster];
    const StitchMeta sm = a.sm[it.cluster];
    // the block's relations, and (bits 8..) the one this item assembles
    const uint32_t mask = it.mask & 0xFFu, only = it.mask >> 8;
    const BlockLayout lay = block_layout(mask, m.nV, m.nT, m.nnzVT, it.cap_vv, it.cap_tt);
    int32_t *blk = a.out + it.out_word;
    if (tid == 0) {
        s_status = (sm.ntiles < 1 || sm.ntiles > kMaxTiles || sm.nv != m.nV || sm.nt != m.nT) ? kStInconsistent : 0;
        s_nvv = s_ntt = s_nvt = 0;
    }
    __syncthreads();
    const int nt_ = sm.ntiles < kMaxTiles ? sm.ntiles : kMaxTiles;
    if (tid < nt_) {
        const WorkItem tw = a.tiles[it.tiles + tid];
        const ClusterMeta tm = a.meta[tw.cluster];
        s_base[tid] = tw.out_word;
        s_lay[tid] = block_layout(mask, tm.nV, tm.nT, tm.nnzVT, tw.cap_vv, tw.cap_tt);
        const int32_t *tb = a.out + tw.out_word;
        atomicOr(&s_status, tb[0]);
        atomicAdd(&s_nvt, tb[3]);
        if (mask & kRelVV) atomicAdd(&s_nvv, tb[4]);
        if (mask & kRelTT) atomicAdd(&s_ntt, tb[5]);
    }
    __syncthreads();
    if (tid == 0) {
        if (s_nvt != m.nnzVT) atomicOr(&s_status, kStInconsistent);
        if ((mask & kRelVV) && s_nvv > it.cap_vv) atomicOr(&s_status, kStVVOverflow);
        if ((mask & kRelTT) && s_ntt > it.cap_tt) atomicOr(&s_status, kStTTOverflow);
    }
    __syncthreads();
    const bool copy = (s_status & (kStInconsistent | kStVVOverflow | kStTTOverflow)) == 0;
    auto tile_block = [&](int j) -> const int32_t * { return a.out + s_base[j]; };

    // one relation: rows n from the map at moff; row ids, offsets and lists
    // from each tile's arrays at (rows_at, off_at, ent_at) of its layout
    auto assemble = [&](int n, int64_t moff, int64_t rows_dst, int64_t off_dst, int64_t ent_dst, bool with_rows,
                        auto rows_at, auto off_at, auto ent_at) {
        int carry = 0;
        for (int r0 = 0; r0 < n; r0 += B) {
            const int r = r0 + tid;
            int j = 0, l = 0, c = 0, s0 = 0;
            if (r < n) {
                j = a.maps[moff + 2 * (int64_t)r];
                l = a.maps[moff + 2 * (int64_t)r + 1];
                if (j < 0 || j >= nt_) j = 0;  // guarded by the consistency check above
                const int32_t *tb = tile_block(j);
                const BlockLayout &tl = s_lay[j];
                s0 = tb[off_at(tl) + l];
                c = tb[off_at(tl) + l + 1] - s0;
            }
            int tot;
            const int ex = block_excl_scan<B>(c, tot, sp);
            if (r < n) {
                const int32_t *tb = tile_block(j);
                const BlockLayout &tl = s_lay[j];
                if (with_rows) blk[rows_dst + r] = tb[rows_at(tl) + l];
                blk[off_dst + r] = carry + ex;
                s_src[tid] = s_base[j] + ent_at(tl) + s0;
            }
            s_pre[tid] = r < n ? ex : tot;
            __syncthreads();
            // the chunk's entries, four consecutive words per thread and
            // consecutive threads on consecutive runs: the row of the first
            // word by binary search over the chunk's starts (the last row
            // starting at or before it; empty rows share their start with
            // the next one, rows past the chunk start at its end), the next
            // three by stepping on; the four reads are in flight together
            int32_t *dst = blk + ent_dst + carry;
            for (int e0 = 4 * tid; e0 < tot; e0 += 4 * B) {
                int lo = 0, hi = B - 1;
                while (lo < hi) {
                    const int mid = (lo + hi + 1) >> 1;
                    if (s_pre[mid] <= e0) lo = mid;
                    else hi = mid - 1;
                }
                int32_t v[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int e = e0 + u;
                    v[u] = 0;
                    if (e < tot) {
                        while (lo + 1 < B && s_pre[lo + 1] <= e) ++lo;
                        v[u] = a.out[s_src[lo] + (e - s_pre[lo])];
                    }
                }
#pragma unroll
                for (int u = 0; u < 4; ++u)
                    if (e0 + u < tot) dst[e0 + u] = v[u];
            }
            __syncthreads();
            carry += tot;
        }
        if (tid == 0) blk[off_dst + n] = carry;
    };

    if (copy) {
        if (mask & (kRelVT | kRelVV)) {
            const bool vt = (mask & kRelVT) != 0;
            if (only & kRelVT)
                assemble(m.nV, sm.vmap_off, lay.vrows, lay.vt_off, lay.vt_ent, true,
                         [](const BlockLayout &t) { return t.vrows; }, [](const BlockLayout &t) { return t.vt_off; },
                         [](const BlockLayout &t) { return t.vt_ent; });
            if (only & kRelVV)
                assemble(m.nV, sm.vmap_off, lay.vrows, lay.vv_off, lay.vv_ent, !vt,
                         [](const BlockLayout &t) { return t.vrows; }, [](const BlockLayout &t) { return t.vv_off; },
                         [](const BlockLayout &t) { return t.vv_ent; });
        }
        if (only & kRelTT)
            assemble(m.nT, sm.tmap_off, lay.trows, lay.tt_off, lay.tt_ent, true,
                     [](const BlockLayout &t) { return t.trows; }, [](const BlockLayout &t) { return t.tt_off; },
                     [](const BlockLayout &t) { return t.tt_ent; });
    }
    __syncthreads();
    // every item of the cluster writes the same header (the tiles' status and sums)
    if (tid == 0) {
        int32_t h[8];
        h[0] = s_status;
        h[1] = m.nV;
        h[2] = m.nT;
        h[3] = m.nnzVT;
        h[4] = (mask & kRelVV) ? s_nvv : 0;
        h[5] = (mask & kRelTT) ? s_ntt : 0;
        h[6] = it.cap_vv;
        h[7] = it.cap_tt;
        for (int i = 0; i < 8; ++i) blk[i] = h[i];
        if (a.hdr)
            for (int i = 0; i < 8; ++i) a.hdr[(int64_t)it.hdr_index * 8 + i] = h[i];
    }
    __syncthreads();
}

template <int B>
__global__ __launch_bounds__(B) void gale_stitch_kernel(SArgs a) {
    __shared__ int s_idx;
    while (true) {
        if (threadIdx.x == 0) s_idx = atomicAdd(a.queue, 1);
        __syncthreads();
        const int idx = s_idx;
        __syncthreads();
        if (idx >= a.nitems) break;
        stitch_item<B>(a, a.items[idx]);
    }
}

}  // namespace

hipError_t launch_stitch(const SArgs &a, int grid, hipStream_t st) {
    (void)hipGetLastError();
    hipLaunchKernelGGL((gale_stitch_kernel<kStitchThreads>), dim3(grid), dim3(kStitchThreads), 0, st, a);
    return hipGetLastError();
}

}  // namespace gale
