// Host-side state of a created code (ldpc_code_t): the device tables of
// both CN-lane mappings, launch choices and the HBM-tier workspace.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <atomic>
#include <mutex>

#include "ndgsbp_internal.h"

namespace ndgsbp {

struct DeviceTables {
    int32_t* vcn = nullptr;
    uint32_t* vfirst = nullptr;    // per visit: 1 if it is its CN's first visit in an iteration
    uint32_t* vdfirst = nullptr;   // per visit (one-lane layout): bit k if edge k writes its VN's first delta slot
    int32_t* visit_ptr = nullptr;  // G + 1
    uint2* fix = nullptr;
    int32_t* fix_ptr = nullptr;    // G + 1
    uint32_t* work = nullptr;      // kWorkRing pairs {next frame, finished workgroups}
};

// The tables that depend on the CN-phase mapping (H lanes per CN visit).
struct Layout {
    bool valid = false;
    int32_t H = 1;          // lanes per CN visit
    int32_t D = 0;          // padded CN degree (kernel variant), a multiple of H
    bool uniform = false;   // every CN has degree exactly D
    uint32_t* vw = nullptr;       // edge half-records
    uint32_t* syn_col = nullptr;  // m * SD
};

}  // namespace ndgsbp

struct ldpc_code {
    int32_t device;
    int32_t m, n;
    int64_t nnz;
    int32_t G;  // groups per iteration
    int32_t R;  // iteration blocks: iteration l uses groups ((l-1) mod R) * G ..
    bool vertical = false;  // VN groups (the vertical schedule)
    int64_t cn_visits;
    int64_t edge_updates;
    int32_t max_cn_degree;
    int32_t max_vn_degree;
    int32_t max_group_visits;
    int32_t max_slots;
    ndgsbp::Layout lay[4];    // lay[H - 1]: tables for H = 1, 2 or 4 lanes per CN visit
    int32_t lanes_for[3];     // chosen H per message format (MsgKind)
    int32_t lanes_default[3];
    size_t max_lds;   // LDS a workgroup may use on the code's device
    int32_t num_cus;  // compute units of the code's device
    int32_t ds_start; // float index of the first delta slot
    std::atomic<uint32_t> next_work{0};  // ring position of the next decode call
    ndgsbp::DeviceTables dev;
    // HBM tier: frame-interleaved workspace, grown on demand and shared by
    // the code's HBM-tier launches, which the library orders on the device
    // (each waits for the event recorded after the previous one)
    std::mutex hbm_mu;
    void* hbm_ws = nullptr;
    size_t hbm_ws_bytes = 0;
    hipEvent_t hbm_last = nullptr;
    bool hbm_used = false;
};

namespace ndgsbp {

// Device memory a caller supplies in place of the code's own work counters
// and HBM-tier workspace: `work` two zeroed words, `hbm` a workspace of
// `hbm_bytes` (the tiles in flight are bounded by it).
struct Scratch {
    uint32_t* work;
    void* hbm;
    size_t hbm_bytes;
};

// ldpc_decode with an optional Scratch (nullptr: the code's own buffers).
int decode_enqueue(ldpc_code* c, const float* llr, int32_t num_frames, int32_t max_iter, uint32_t flags,
                   uint8_t* hard, float* post, int32_t* iters, uint8_t* syn_ok, const Scratch* scratch,
                   void* hip_stream);
// Sets the thread's ldpc_last_error message; returns `code`.
int record_error(int code, const char* msg);
// Once per device, with that device current: locates the device's copy of
// the fixed scratch array of ldpc_decode_noalloc and clears its counters
// (ndgsbp_noalloc.hip).
hipError_t noalloc_setup(int device);

}  // namespace ndgsbp
