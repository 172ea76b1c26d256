// gale_layout.h -- data layout shared by the host runtime and the GPU kernels.
//
// Per cluster C the load step leaves in device memory (paper, Section 4.3,
// "Initialization": the per-segment list of internal and external tetrahedra
// and the vertex intervals, here re-expressed per cluster):
//
//   lverts[lv_off .. lv_off+L)   local vertex table: the original ids of every
//                                vertex of star(C), halo(C) and C itself, in
//                                ascending original id (ids below 2^30); bit
//                                31 set when the vertex belongs to C (a VT/VV
//                                row), bit 30 when its cluster is below C (no
//                                tetrahedron internal to C has such a vertex).
//   tets (bytes from tb_off)     the four local vertex ids of each stream
//                                tetrahedron, ascending, as 4 x uint16 (8 B)
//                                when the local table has at most 65535
//                                vertices, else as 4 x int32 (16 B, flag bit
//                                0).  Order: first the nT tetrahedra internal
//                                to C (stream position = TT row), then the
//                                rest of star(C) (at least one vertex in C),
//                                then the nh halo tetrahedra (no vertex in C,
//                                sharing a triangle with a tetrahedron
//                                internal to C); each part in ascending
//                                original id.  ns counts the whole star.
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
// the further coboundary relations, built from the edge and triangle lists
constexpr uint32_t kRelVE = 8u, kRelVF = 16u, kRelEF = 32u, kRelET = 64u, kRelFT = 128u;
constexpr uint32_t kRelBase = 7u, kRelExt = 0xF8u;
constexpr int kHeaderWords = 8;
constexpr int kAlignWords = 32;

// header status bits
constexpr int kStVVOverflow = 1;   // VV entries exceed cap_vv
constexpr int kStTTOverflow = 2;   // TT entries exceed cap_tt
constexpr int kStInconsistent = 4; // stream metadata disagrees with what the kernel counted
constexpr int kStTTFallback = 8;   // face table could not pair every face (non-manifold face, or a table
                                   // that stays full); TT was built by chain pairing, or by exhaustive
                                   // pairing for a full table (informational)

struct ClusterMeta {
    int64_t tet_off;  // first stream tetrahedron of the cluster (index into tid)
    int64_t lv_off;   // first local vertex of the cluster
    int64_t tb_off;   // byte offset of the cluster's tetrahedra in the stream (16-aligned)
    int32_t ns;       // star(C) tetrahedra
    int32_t nh;       // halo tetrahedra
    int32_t nT;       // tetrahedra internal to C (TT rows)
    int32_t L;        // local vertices
    int32_t nV;       // vertices of C (VT/VV rows)
    int32_t nnzVT;    // sum over rows of |VT(v)|, exact
    int32_t cap_vv;   // default VV capacity: sum over rows of min(deg+2, 3 deg, L-1)
    int32_t flags;    // bit 0: tetrahedra stored as 4 x int32
    int64_t pad;
};
static_assert(sizeof(ClusterMeta) == 64, "ClusterMeta layout");
constexpr int32_t kMetaWide = 1;

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

// Per cluster, for the edge and triangle relations: the cluster's internal
// edges are ids [e0, e0 + ne), its internal triangles [f0, f0 + nf) (the
// interval arrays I_E, I_F of the initialization step); et_inst and ft_inst
// count the (tetrahedron, internal edge) and (tetrahedron, internal triangle)
// pairs of its star, i.e. the entries of its ET and FT blocks.
struct ExtMeta {
    int32_t e0, ne, f0, nf;
    int32_t et_inst, ft_inst;
    int32_t pad[2];
};
static_assert(sizeof(ExtMeta) == 32, "ExtMeta layout");

// Block of the edge and triangle relations (one cluster, the relations of a
// mask within kRelExt): header[8] = {status, nnz VE, VF, EF, ET, FT, 0, 0},
// then for each relation of the mask in the order VE, VF, EF, ET, FT, each
// array on a 32-word boundary: row ids[nrows], offsets[nrows + 1],
// entries[capacity].  Rows: VE, VF the cluster's vertices (original ids,
// ascending); EF, ET its internal edges (edge ids e0 ..); FT its internal
// triangles (triangle ids f0 ..).  Capacities (bounds the host and kernel
// both derive): VE and VF 3 nnzVT (three per (tetrahedron, row vertex) pair),
// EF 2 et_inst, ET et_inst, FT ft_inst (exact).
struct ExtLayout {
    int64_t rows[5], off[5], ent[5];
    int32_t nrows[5], cap[5];
    int64_t total;  // words
};

GALE_HD int32_t ext_nrows(int r, const ClusterMeta &m, const ExtMeta &x) {
    return r <= 1 ? m.nV : (r <= 3 ? x.ne : x.nf);
}

GALE_HD int32_t ext_cap(int r, const ClusterMeta &m, const ExtMeta &x) {
    return r <= 1 ? 3 * m.nnzVT : (r == 2 ? 2 * x.et_inst : (r == 3 ? x.et_inst : x.ft_inst));
}

struct Streams {
    const char *tets;        // stream tetrahedra (see ClusterMeta::tb_off, flags)
    const int32_t *tid;      // original tetrahedron id | internal << 31
    const int32_t *lverts;   // original vertex id | row << 31
    const ClusterMeta *meta;
};

// A cluster built as tiles (batched form): its tiles are metadata entries
// tile_first .. tile_first + ntiles - 1 past the clusters' own; the map
// array holds, from vmap_off, (tile, row in the tile's block) for each of
// its nv vertices in ascending id, and from tmap_off the same for each of its
// nt internal tetrahedra.
constexpr int kMaxTilesPerCluster = 64;
struct StitchMeta {
    int64_t vmap_off, tmap_off;
    int32_t tile_first, ntiles, nv, nt;
};
static_assert(sizeof(StitchMeta) == 32, "StitchMeta layout");

// One relation of a tiled cluster to assemble: the cluster's block
// (out_word, capacities, header slot), its relation mask (bits 0..7) and the
// relation this item copies (bits 8..15), and the position of its tiles' work
// items in the stitch launch's tile table.
struct StitchItem {
    int64_t out_word;
    int32_t cluster;
    uint32_t mask;
    int32_t cap_vv, cap_tt;
    int32_t hdr_index;
    int32_t tiles;
};
static_assert(sizeof(StitchItem) == 32, "StitchItem layout");

struct SArgs {
    const ClusterMeta *meta;   // clusters, then tiles
    const StitchMeta *sm;      // per cluster
    const int32_t *maps;
    int32_t *out;
    int32_t *hdr;
    const StitchItem *items;
    const WorkItem *tiles;     // the tiles' work items (block positions, capacities)
    int32_t nitems;
    int32_t pad;
    int32_t *queue;
};

// Edge and triangle lists indexed by smallest vertex (original ids): edges
// {a < b} of vertex a at eidx[2 eoff[a] .. 2 eoff[a+1]) as (b, id) sorted by
// b; triangles {a < b < c} at fidx[4 foff[a] ..) as (b, c, id, 0) sorted by
// (b, c).
struct Simplices {
    const ExtMeta *ext;
    const int32_t *eoff, *eidx, *foff, *fidx;
};

// Kernel arguments (passed by value).
struct KArgs {
    Streams s;
    Simplices x;
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

GALE_HD ExtLayout ext_layout(uint32_t mask, const ClusterMeta &m, const ExtMeta &x) {
    ExtLayout b;
    int64_t w = align_words(kHeaderWords);
    for (int r = 0; r < 5; ++r) {
        b.nrows[r] = ext_nrows(r, m, x);
        b.cap[r] = ext_cap(r, m, x);
        b.rows[r] = b.off[r] = b.ent[r] = -1;
        if (!(mask & (kRelVE << r))) continue;
        b.rows[r] = w;
        w = align_words(w + b.nrows[r]);
        b.off[r] = w;
        w = align_words(w + b.nrows[r] + 1);
        b.ent[r] = w;
        w = align_words(w + b.cap[r]);
    }
    b.total = w;
    return b;
}

// Where each working array lives, as byte offsets from the base of the LDS
// (LDS path) or of the workgroup's global workspace slice (global path).
//   lt    stream tetrahedra, 4 x uint16 local ids           (LDS path only)
//         (only the internal ones while TT runs; the rest is staged after)
// TT uses the region after the internal tetrahedra for
//   win   four partner cells per TT row (stream positions, one per face)
//   lowb  one bit per local vertex: its cluster is below C
//   ht    face table: H cells holding the stream position of a tetrahedron
// cells are uint16 in LDS and int32 in the global workspace.  VT / VV use
// the region after the star tetrahedra (in the workspace: from its start) for
//   rix   row index of each local vertex (all ones: not a vertex of the cluster)
//   rowl  local id of each row
//   cnt   local VT offsets of the rows, nV + 1
//   lvt   local VT entries: stream positions, nnzVT
//   wbm   one bitmap over the local vertex table per row group (VV)
//   lvl   the original id of each local vertex (VV, LDS path)
// VT runs last and writes its rows through a buffer over the star
// tetrahedra's region (LDS path); TT reads tetrahedron ids from a copy in the
// face table's region when it fits.
struct Plan {
    int32_t ok;       // LDS path possible within the budget
    int32_t W;        // bitmap words per row
    int32_t H;        // face table cells
    int32_t P;        // face table passes (faces split by hash)
    int32_t G;        // lanes per VV row group (8, 16 or 32)
    int32_t pad;
    int64_t lt, win, lowb, ht, rix, rowl, cnt, lvt, wbm, lvl;
    int64_t lv4;      // hybrid path: the local VT entries' tetrahedra (4 x uint16 each), in the workspace
    int64_t bytes;
    int64_t ws_bytes; // hybrid path: workspace bytes used
};

GALE_HD int64_t align16(int64_t b) { return (b + 15) / 16 * 16; }

// Face table passes: at most this many after doublings (then exhaustive
// pairing, every row against every stream tetrahedron); a plan starts with at
// most kLdsFacePasses (LDS path) or
// kHybFacePasses (hybrid path).
constexpr int kMaxFacePasses = 32;
constexpr int kLdsFacePasses = 8;
constexpr int kHybFacePasses = 12;

// Face table passes for H cells: distinct faces are estimated at 2.5 per TT
// row (a closed region has 2 plus half its boundary) at load 0.7; the kernel
// doubles the count and starts again if a pass fills the table.
GALE_HD int32_t face_passes(int32_t nT, int64_t H) {
    if (H <= 0) return 0;
    const int64_t est = (5 * (int64_t)nT) / 2 + 64;
    const int64_t per = (7 * H) / 10 > 0 ? (7 * H) / 10 : 1;
    const int64_t P = (est + per - 1) / per;
    return (int32_t)(P < 1 ? 1 : P);
}

// Face table cells kept per TT row at most (load about 1/3 on a closed region).
GALE_HD int64_t face_cells_max(int32_t nT) { return 6 * (int64_t)nT + 64; }

// Words of one VV row group: its bitmap over the local table (W words) and a
// summary with one bit per bitmap word.
GALE_HD int64_t vv_group_words(int64_t W) { return W + (W + 31) / 32; }

// VT / VV arrays from byte offset off (cell: bytes of an id or position),
// with one VV bitmap per group of vv_group lanes; returns the end.
GALE_HD int64_t v_arrays(Plan &p, const ClusterMeta &m, uint32_t mask, int64_t off, int cell, int block_threads,
                         int vv_group) {
    const bool v = (mask & (kRelVT | kRelVV)) != 0;
    const bool vv = (mask & kRelVV) != 0;
    const int64_t ngroups = block_threads / vv_group;
    p.G = vv_group;
    p.W = (m.L + 31) / 32;
    p.rix = off;
    off += v ? align16((int64_t)m.L * cell) : 0;
    p.rowl = off;
    off += v ? align16((int64_t)m.nV * cell) : 0;
    p.cnt = off;
    off += v ? align16(((int64_t)m.nV + 1) * 4) : 0;
    p.lvt = off;
    off += v ? align16((int64_t)m.nnzVT * cell) : 0;
    p.wbm = off;
    off += vv ? align16(ngroups * vv_group_words(p.W) * 4) : 0;
    p.lvl = off;
    off += (vv && cell == 2) ? align16((int64_t)m.L * 4) : 0;
    return off;
}

// LDS path: uint16 local ids, positions and cells.  Offsets are assigned on
// every path with no early return (the same offsets for every mask).
GALE_HD Plan lds_plan(const ClusterMeta &m, uint32_t mask, int64_t budget, int32_t block_threads) {
    Plan p{};
    const int64_t ntot = (int64_t)m.ns + m.nh;
    const bool narrow = m.L <= 65535 && ntot <= 65535;
    const bool tt = (mask & kRelTT) != 0;
    const bool v = (mask & (kRelVT | kRelVV)) != 0;
    p.lt = 0;
    // TT: partner cells, then the table takes what is left (an even count)
    p.win = align16((int64_t)m.nT * 8);
    p.lowb = p.win + (tt ? align16((int64_t)m.nT * 4 * 2) : 0);
    p.ht = p.lowb + (tt ? align16((int64_t)((m.L + 31) / 32) * 4) : 0);
    int64_t h = tt ? (budget - p.ht) / 2 : 0;
    const int64_t hmax = face_cells_max(m.nT);
    h = h > hmax ? hmax : h;
    h = h < 0 ? 0 : h & ~(int64_t)1;
    p.H = (int32_t)h;
    p.P = tt ? face_passes(m.nT, h) : 0;
    const int64_t tt_end = p.ht + 2 * h;
    // VT / VV after the star tetrahedra (the halo holds no vertex of C); VV
    // rows by groups of 8 lanes when their bitmaps fit and each lane keeps its
    // run of bitmap words in registers (at most 64 words), else 16, else 32
    const bool g8 = (m.L + 31) / 32 <= 64;
    int64_t v_end = v_arrays(p, m, mask, align16((int64_t)m.ns * 8), 2, block_threads, g8 ? 8 : 16);
    if (v_end > budget && g8) v_end = v_arrays(p, m, mask, align16((int64_t)m.ns * 8), 2, block_threads, 16);
    if (v_end > budget) v_end = v_arrays(p, m, mask, align16((int64_t)m.ns * 8), 2, block_threads, 32);
    p.bytes = tt_end > v_end ? tt_end : v_end;
    const bool tt_ok = !tt || (h >= 64 && p.P <= kLdsFacePasses && tt_end <= budget);
    const bool v_ok = !v || v_end <= budget;
    p.ok = (narrow && tt_ok && v_ok) ? 1 : 0;
    return p;
}

// Global path with its most used arrays in LDS (a workgroup of this path
// fills its compute unit's registers, so its LDS is otherwise idle): the face
// table (64-bit cells holding the face's local ids and a stream position, so at
// most 32767 local vertices and 131070 stream tetrahedra when TT is
// requested) and the lower-cluster bits while TT runs; the row
// index and row local ids (uint16: at most 65535 local vertices), VT counts
// and VV bitmaps while VT / VV run.  The
// partner cells and the local VT lists stay in the workspace slice (win and
// lvt are offsets there, both from its start since TT is finished first),
// and the stream is read from global memory.  The local VT lists hold each
// entry's original tetrahedron id (lvt, for VT) and its four local vertex ids
// (lv4, for VV), written by the scatter, so that VT and VV read them in row
// order instead of gathering through stream positions.  The local vertex
// table's original ids are copied to LDS (lvl) when they fit, else lvl < 0.
// bytes is the LDS used.
GALE_HD Plan hyb_plan(const ClusterMeta &m, uint32_t mask, int64_t budget, int32_t block_threads) {
    Plan p{};
    const bool tt = (mask & kRelTT) != 0;
    const bool v = (mask & (kRelVT | kRelVV)) != 0;
    const bool vv = (mask & kRelVV) != 0;
    p.win = 0;
    p.lvt = 0;
    p.lowb = 0;
    p.ht = tt ? align16((int64_t)((m.L + 31) / 32) * 4) : 0;
    int64_t h = tt ? (budget - p.ht) / 8 : 0;
    const int64_t hmax = face_cells_max(m.nT);
    h = h > hmax ? hmax : h;
    h = h < 0 ? 0 : h;
    p.H = (int32_t)h;
    p.P = tt ? face_passes(m.nT, h) : 0;
    const int64_t tt_end = p.ht + 8 * h;
    p.W = (m.L + 31) / 32;
    p.rix = 0;
    p.rowl = p.rix + (v ? align16((int64_t)m.L * 2) : 0);
    p.cnt = p.rowl + (v ? align16((int64_t)m.nV * 2) : 0);
    p.wbm = p.cnt + (v ? align16(((int64_t)m.nV + 1) * 4) : 0);
    p.G = 16;
    int64_t v_end = p.wbm + (vv ? align16((int64_t)(block_threads / 16) * vv_group_words(p.W) * 4) : 0);
    if (v_end > budget) {
        p.G = 32;
        v_end = p.wbm + (vv ? align16((int64_t)(block_threads / 32) * vv_group_words(p.W) * 4) : 0);
    }
    p.lvl = -1;
    if (vv && v_end + align16((int64_t)m.L * 4) <= budget) {
        p.lvl = v_end;
        v_end += align16((int64_t)m.L * 4);
    }
    p.bytes = tt_end > v_end ? tt_end : v_end;
    p.lv4 = align16((int64_t)m.nnzVT * 4);
    // TT: four 64-bit partner cells per row
    const int64_t ws_tt = tt ? (int64_t)m.nT * 32 : 0;
    const int64_t ws_v = v ? p.lv4 + (int64_t)m.nnzVT * 8 : 0;
    p.ws_bytes = align16(ws_tt > ws_v ? ws_tt : ws_v);
    const bool tt_ok = !tt || (h >= 64 && p.P <= kHybFacePasses && m.L <= 32767 &&
                               (int64_t)m.ns + m.nh < (1 << 17) - 1);
    const bool v_ok = !v || (v_end <= budget && m.L <= 65535);
    p.ok = (tt_ok && v_ok) ? 1 : 0;
    return p;
}

// Global path: the same arrays in the workgroup's workspace slice with 32-bit
// ids, positions and cells; the stream is read from global memory.  TT and
// VT / VV both start at the slice base (TT is finished first).
GALE_HD Plan ws_plan(const ClusterMeta &m, uint32_t mask, int32_t block_threads) {
    Plan p{};
    const bool tt = (mask & kRelTT) != 0;
    p.ok = 1;
    p.lt = 0;
    p.win = 0;
    p.lowb = tt ? align16((int64_t)m.nT * 4 * 4) : 0;
    p.ht = p.lowb + (tt ? align16((int64_t)((m.L + 31) / 32) * 4) : 0);
    const int64_t h = tt ? face_cells_max(m.nT) : 0;
    p.H = (int32_t)h;
    p.P = tt ? 1 : 0;
    const int64_t tt_end = p.ht + 4 * h;
    const int64_t v_end = v_arrays(p, m, mask, 0, 4, block_threads, 32);
    p.bytes = tt_end > v_end ? tt_end : v_end;
    return p;
}

}  // namespace gale
