// gale_host.h -- host-side declarations shared by the runtime sources.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/gale.h"
#include "gale_layout.h"

namespace gale {

// Streams prepared on the host by prepare_streams (see gale_layout.h for the
// meaning of each array).
struct HostStreams {
    int32_t nv = 0, ncl = 0;
    int64_t nt = 0;
    std::vector<ClusterMeta> meta;
    std::vector<uint8_t> tets;    // stream tetrahedra, 4 x uint16 or 4 x int32 local ids
    std::vector<int32_t> tid;     // original id | internal << 31
    std::vector<int32_t> lverts;  // original id | row << 31
};

// Edge and triangle lists of the initialization step (enumerate_simplices):
// e / f hold 2 / 3 original ids per edge / triangle by id; ie / if_ the
// interval arrays; eoff, eidx, foff, fidx the index by smallest vertex (see
// Simplices in gale_layout.h); ext the per-cluster ranges and counts.
struct HostSimplices {
    std::vector<int32_t> e, f;
    std::vector<int64_t> ie, if_;
    std::vector<int32_t> eoff, foff, eidx, fidx;
    std::vector<ExtMeta> ext;
};

gale_status enumerate_simplices(const HostStreams &hs, HostSimplices &out, std::string &err);

// Tiles of large clusters (gale_tiles.cpp): pseudo-cluster of every vertex,
// which pseudo-clusters are tiles, and per cluster its first tile and count.
struct TilePlan {
    int32_t ntiles = 0, npseudo = 0;
    std::vector<int32_t> pseudo;          // nv
    std::vector<char> keep;               // npseudo: a tile
    std::vector<int32_t> tile_first, tile_count;  // ncl
    std::vector<int32_t> pseudo_of_tile;  // ntiles
};
gale_status plan_tiles(int32_t nv, int64_t nt, const int32_t *tv, const int32_t *cl, int32_t ncl,
                       const std::vector<ClusterMeta> &meta, int64_t tile_vt, TilePlan &tp);
void stitch_maps(const TilePlan &tp, const HostStreams &ts, int32_t ncl, std::vector<StitchMeta> &sm,
                 std::vector<int32_t> &maps);

// keep (optional, ncl flags): build the local tables and streams of the
// flagged clusters only; the others get empty streams and zero metadata
gale_status prepare_streams(int32_t nv, int64_t nt, const int32_t *tv, const int32_t *cl, int32_t ncl,
                            HostStreams &out, std::string &err, const std::vector<char> *keep = nullptr);

struct KArgs;
hipError_t launch_items(const KArgs &a, bool lds_path, int block_threads, int grid, size_t lds, hipStream_t st);
hipError_t launch_persistent(const KArgs &a, bool lds_path, int block_threads, int grid, size_t lds,
                             hipStream_t st);
hipError_t set_lds_limits(size_t lds);
hipError_t launch_zero(int32_t *p, int n, hipStream_t st);  // n <= 64
hipError_t static_lds_bytes(int64_t *bytes);  // largest static LDS of the LDS-path kernels
hipError_t persistent_occupancy(int block_threads, bool lds_path, size_t lds, int *blocks_per_cu);
// the edge / triangle relation kernel (persistent over a.items, workspace
// slices of a.ws_stride bytes per workgroup)
hipError_t launch_ext(const KArgs &a, int grid, hipStream_t st);
int64_t ext_workspace_bytes(const ClusterMeta &m, const ExtMeta &x, uint32_t mask);
constexpr int kExtThreads = 512;
// the stitch of tiled clusters (persistent over a.items)
hipError_t launch_stitch(const SArgs &a, int grid, hipStream_t st);
constexpr int kStitchThreads = 256;

}  // namespace gale
