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

gale_status prepare_streams(int32_t nv, int64_t nt, const int32_t *tv, const int32_t *cl, int32_t ncl,
                            HostStreams &out, std::string &err);

struct KArgs;
hipError_t launch_items(const KArgs &a, bool lds_path, int block_threads, int grid, size_t lds, hipStream_t st);
hipError_t launch_persistent(const KArgs &a, bool lds_path, int block_threads, int grid, size_t lds,
                             hipStream_t st);
hipError_t set_lds_limits(size_t lds);
hipError_t launch_zero(int32_t *p, int n, hipStream_t st);  // n <= 64
hipError_t static_lds_bytes(int64_t *bytes);  // largest static LDS of the LDS-path kernels
hipError_t persistent_occupancy(int block_threads, bool lds_path, size_t lds, int *blocks_per_cu);

}  // namespace gale
