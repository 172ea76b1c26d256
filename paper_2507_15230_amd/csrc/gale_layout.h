// gale_layout.h -- data layout shared by the host runtime and the GPU kernels.
//
// Per cluster C the load step leaves in device memory (paper, Section 4.3,
// "Initialization": the per-segment list of internal and external tetrahedra
// and the vertex intervals, here re-expressed per cluster):
//
//   lverts[lv_off .. lv_off+L)   local vertex table: the original ids of every
//                                vertex of star(C), halo(C) and C itself, in
//                                ascending original id; bit 31 set when the
//                                vertex belongs to C (a VT/VV row).
//   tets[tet_off .. +ns+nh)      int4: the four local vertex ids of each stream
//                                tetrahedron; first the ns tetrahedra of
//                                star(C) (at least one vertex in C) in ascending
//                                original id, then the nh halo tetrahedra
//                                (no vertex in C, sharing a triangle with a
//                                tetrahedron internal to C), ascending.
//   tid[tet_off .. +ns+nh)       original tetrahedron id; bit 31 set when the
//                                tetrahedron is internal to C (a TT row).
//
// A block (one cluster, a relation mask) is a run of int32 words:
//   header[8] = {status, nV, nT, nnzVT, nnzVV, nnzTT, cap_vv, cap_tt}
//   then, each array starting on a 32-word boundary, for the bits in the mask:
//   VT|VV: vrows[nV]            row ids (original vertex ids, ascending)
//   VT:    vt_off[nV+1], vt_ent[nnzVT]
//   TT:    trows[nT], tt_off[nT+1], tt_ent[cap_tt]
//   VV:    vv_off[nV+1], vv_ent[cap_vv]
// VV comes last so that the unused tail of its capacity can be given back
// once the exact count is known.
// The capacities of VV and TT are bounds chosen by the host; the kernel writes
// the exact counts to the header and never writes past a capacity (status bit
// set instead, and the host rebuilds that block with exact capacities).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gale {

#define GALE_HD __host__ __device__ __forceinline__

constexpr uint32_t kRelVT = 1u, kRelVV = 2u, kRelTT = 4u;
constexpr int kHeaderWords = 8;
constexpr int kAlignWords = 32;

// header status bits
constexpr int kStVVOverflow = 1;   // VV entries exceed cap_vv
constexpr int kStTTOverflow = 2;   // TT entries exceed cap_tt
constexpr int kStInconsistent = 4; // stream metadata disagrees with what the kernel counted
constexpr int kStTTFallback = 8;   // face table could not pair every face (non-manifold face or full table);
                                   // TT was built by the exhaustive path instead (informational)

struct ClusterMeta {
    int64_t tet_off;  // first stream tetrahedron of the cluster
    int64_t lv_off;   // first local vertex of the cluster
    int32_t ns;       // star(C) tetrahedra
    int32_t nh;       // halo tetrahedra
    int32_t nT;       // tetrahedra internal to C (TT rows)
    int32_t L;        // local vertices
    int32_t nV;       // vertices of C (VT/VV rows)
    int32_t nnzVT;    // sum over rows of |VT(v)|, exact
    int32_t cap_vv;   // default VV capacity: sum over rows of min(deg+2, 3 deg, L-1)
    int32_t pad;
};
static_assert(sizeof(ClusterMeta) == 48, "ClusterMeta layout");

struct WorkItem {
    int64_t out_word;  // block start (words) in the output buffer
    int32_t cluster;
    uint32_t mask;
    int32_t cap_vv;
    int32_t cap_tt;
    int32_t hdr_index; // where the header copy goes in the compact header array
    int32_t pad;
};
static_assert(sizeof(WorkItem) == 32, "WorkItem layout");

struct BlockLayout {
    int64_t vrows, vt_off, vt_ent, vv_off, vv_ent, trows, tt_off, tt_ent;
    int64_t total;  // words
};

struct Streams {
    const int4 *tets;        // 4 local vertex ids per stream tetrahedron
    const int32_t *tid;      // original tetrahedron id | internal << 31
    const int32_t *lverts;   // original vertex id | row << 31
    const ClusterMeta *meta;
};

// Kernel arguments (passed by value).
struct KArgs {
    Streams s;
    int32_t *out;            // output buffer (words)
    int32_t *hdr;            // compact header copies, 8 words per item (may be null)
    const WorkItem *items;
    int32_t nitems;
    int32_t lds_budget;      // dynamic LDS bytes of this launch
    int32_t *queue;          // persistent launch: work cursor, 0 at launch
    char *ws;                // global workspace, one slice per workgroup (may be null)
    int64_t ws_stride;
};

GALE_HD int64_t align_words(int64_t w) { return (w + kAlignWords - 1) / kAlignWords * kAlignWords; }

GALE_HD BlockLayout block_layout(uint32_t mask, int32_t nV, int32_t nT, int32_t nnzVT, int32_t cap_vv,
                                 int32_t cap_tt) {
    BlockLayout b;
    b.vrows = b.vt_off = b.vt_ent = b.vv_off = b.vv_ent = b.trows = b.tt_off = b.tt_ent = -1;
    int64_t w = align_words(kHeaderWords);
    if (mask & (kRelVT | kRelVV)) { b.vrows = w; w = align_words(w + nV); }
    if (mask & kRelVT) {
        b.vt_off = w; w = align_words(w + nV + 1);
        b.vt_ent = w; w = align_words(w + nnzVT);
    }
    if (mask & kRelTT) {
        b.trows = w; w = align_words(w + nT);
        b.tt_off = w; w = align_words(w + nT + 1);
        b.tt_ent = w; w = align_words(w + cap_tt);
    }
    if (mask & kRelVV) {
        b.vv_off = w; w = align_words(w + nV + 1);
        b.vv_ent = w; w = align_words(w + cap_vv);
    }
    b.total = w;
    return b;
}

// Slots of the TT face table: ~3.2 per internal tetrahedron (the unique faces
// of a cluster's internal tetrahedra are ~2.2 per tetrahedron in a manifold
// mesh; at most 4), rounded to 64.
GALE_HD int32_t face_table_slots(int32_t nT) {
    if (nT <= 0) return 0;
    int64_t h = ((int64_t)nT * 16 + 4) / 5;
    return (int32_t)((h + 63) / 64 * 64);
}

// Where each working array lives, as byte offsets from the base of the LDS
// (LDS path) or of the workgroup's global workspace slice (global path).
struct Plan {
    int32_t ok;        // LDS path possible within the budget
    int32_t rc;        // VV rows per bitmap pass
    int32_t W, Wp;     // bitmap words per row, padded to an odd stride
    int32_t H;         // face table slots
    int64_t tets, ibits, rowof, cnt, lst, bm, ht;
    int64_t bytes;
};

GALE_HD int64_t align16(int64_t b) { return (b + 15) / 16 * 16; }

// LDS path: tetrahedra staged as 4 x uint16 local ids (8 B), internal flags as
// bits, rowOf int16, list positions uint16, face table slots 2 x uint16.
// Every field is assigned on every path and ok is decided last (no early
// return), so all callers see the same offsets whatever the mask.
GALE_HD Plan lds_plan(const ClusterMeta &m, uint32_t mask, int64_t budget, int32_t block_threads) {
    Plan p{};
    const int64_t ntot = (int64_t)m.ns + m.nh;
    const bool narrow = m.L <= 65535 && m.nV <= 32767 && ntot <= 16383;
    const bool want_tt = (mask & kRelTT) != 0;
    const bool want_v = (mask & (kRelVT | kRelVV)) != 0;
    const bool want_vv = (mask & kRelVV) != 0;
    p.W = (m.L + 31) / 32;
    p.Wp = p.W | 1;
    p.H = want_tt ? face_table_slots(m.nT) : 0;
    p.tets = 0;
    p.ibits = align16(ntot * 8);
    const int64_t region = p.ibits + (want_tt ? align16((int64_t)((m.ns + 63) / 64) * 8) : 0);
    const int64_t bytesB = want_tt ? align16((int64_t)p.H * 4) : 0;
    const int64_t a_rowof = 0;
    const int64_t a_cnt = a_rowof + align16((int64_t)m.L * 2);
    const int64_t a_lst = a_cnt + align16(((int64_t)m.nV + 1) * 4);
    const int64_t a_bm = a_lst + align16((int64_t)m.nnzVT * 2);
    p.rowof = region + a_rowof;
    p.cnt = region + a_cnt;
    p.lst = region + a_lst;
    p.bm = region + a_bm;
    p.ht = region;
    // VV rows per bitmap pass: the largest of min(nV, block), halved down to
    // 16, whose bitmap fits next to the lists
    int32_t rc = 0;
    bool rc_ok = true;
    if (want_vv) {
        rc = m.nV < block_threads ? m.nV : block_threads;
        rc_ok = rc == 0;
        while (rc > 0) {
            const int64_t need = region + a_bm + align16((int64_t)rc * p.Wp * 4);
            if (need <= budget) {
                rc_ok = true;
                break;
            }
            if (rc <= 16) break;
            rc = rc / 2;
        }
    }
    p.rc = rc;
    const int64_t bytesA = want_v ? a_bm + (want_vv ? align16((int64_t)rc * p.Wp * 4) : 0) : 0;
    p.bytes = region + (bytesA > bytesB ? bytesA : bytesB);
    p.ok = (narrow && rc_ok && p.bytes <= budget) ? 1 : 0;
    return p;
}

// Global path: the same arrays in the workgroup's workspace slice, 32-bit
// types, face table slots 2 x uint32; tetrahedra read from the stream.
GALE_HD Plan ws_plan(const ClusterMeta &m, uint32_t mask, int32_t block_threads) {
    Plan p{};
    p.ok = 1;
    p.W = (m.L + 31) / 32;
    p.Wp = p.W | 1;
    p.H = (mask & kRelTT) ? face_table_slots(m.nT) : 0;
    p.tets = 0;
    p.ibits = 0;
    int64_t bytesA = 0;
    int32_t rc = 0;
    if (mask & (kRelVT | kRelVV)) {
        p.rowof = 0;
        int64_t a = align16((int64_t)m.L * 4);
        p.cnt = a;
        a += align16(((int64_t)m.nV + 1) * 4);
        p.lst = a;
        a += align16((int64_t)m.nnzVT * 4);
        p.bm = a;
        if (mask & kRelVV) {
            rc = m.nV < block_threads ? m.nV : block_threads;
            a += align16((int64_t)rc * p.Wp * 4);
        }
        bytesA = a;
    }
    p.rc = rc;
    p.ht = 0;
    int64_t bytesB = (mask & kRelTT) ? align16((int64_t)p.H * 8) : 0;
    p.bytes = bytesA > bytesB ? bytesA : bytesB;
    return p;
}

}  // namespace gale
