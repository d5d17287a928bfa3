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
// With sgn_lds the tile also keeps one 64-bit word per VN in LDS, bit l the
// sign (hard decision) of slot l's posterior; with dslot_lds its delta slots
// live in LDS after those words instead of in the float rows.
struct HbmArgs {
    Problem p;               // tables of the one-lane mapping, buffers, sizes
    const uint32_t* vfirst;  // per visit: 1 if it is its CN's first visit in an iteration
    const uint32_t* vdfirst; // per visit: bit k set if edge k writes its VN's first delta slot
    float* fws;              // float rows of every tile
    void* mws;               // message rows of every tile
    uint64_t fws_tile;       // floats per tile
    uint64_t mws_tile;       // messages per tile
    uint32_t* work;          // this launch's {next frame, finished workgroups}, zero at launch
    int32_t early_stop;
    int32_t packed;
    int32_t sgn_lds;         // nonzero: per-VN sign words in dynamic LDS (hbm_sign_bytes)
    int32_t dslot_lds;       // nonzero (with sgn_lds): delta slots in LDS after them (hbm_slot_bytes)
    int32_t max_slots;       // delta slots of the largest group
    float ymax;
};

// Static LDS of the HBM-tier kernel (slot bookkeeping), bytes, an upper bound.
constexpr size_t kHbmStaticLds = 8192;

hipError_t launch_hbm(const HbmArgs& a, MsgKind kind, int D, bool uniform, int blocks, int threads,
                      hipStream_t stream);
// Resident workgroups per CU with `lds_bytes` of dynamic LDS.
hipError_t hbm_occupancy(MsgKind kind, int D, bool uniform, int threads, size_t lds_bytes, int* blocks_per_cu);
// Dynamic LDS of the sign words of an n-VN code, and of the delta slots of
// a tile whose largest group has max_slots of them.
size_t hbm_sign_bytes(int n);
size_t hbm_slot_bytes(int max_slots);
int hbm_max_threads(int D);
int hbm_slots();

}  // namespace ndgsbp
