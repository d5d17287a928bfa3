// HBM-resident decode tier: arguments and launch entry points (the kernel is
// in ndgsbp_hbm.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ndgsbp_internal.h"

namespace ndgsbp {

// Workspace of one workgroup tile (64 frame slots, slot fastest): float rows
// (ds_start + max_slots) x 64, then message rows (m x D) x 64 of the
// message format. The code's one-lane tables (padded degree D) are used.
struct HbmArgs {
    Problem p;               // tables of the one-lane mapping, buffers, sizes
    const uint32_t* vfirst;  // per visit: 1 if it is its CN's first visit in an iteration
    float* fws;              // float rows of every tile
    void* mws;               // message rows of every tile
    uint64_t fws_tile;       // floats per tile
    uint64_t mws_tile;       // messages per tile
    uint32_t* work;          // this launch's {next frame, finished workgroups}, zero at launch
    int32_t early_stop;
    int32_t packed;
    float ymax, cmin;
};

hipError_t launch_hbm(const HbmArgs& a, MsgKind kind, int D, bool uniform, int blocks, int threads,
                      hipStream_t stream);
hipError_t hbm_occupancy(MsgKind kind, int D, bool uniform, int threads, int* blocks_per_cu);
int hbm_max_threads(int D);
int hbm_slots();

}  // namespace ndgsbp
