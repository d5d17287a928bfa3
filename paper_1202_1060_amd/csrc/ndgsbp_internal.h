// Internal definitions shared by the host side (code tables, C ABI) and the
// gfx950 kernels of the NDGSBP decoder.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ndgsbp.h"

namespace ndgsbp {

// The decoder works in log2-scaled LLR units: x' = x * log2(e). Then
// phi(x) = -ln tanh(x/2) becomes psi(y) = log2((1 + 2^-y) / (1 - 2^-y)) with
// psi(y') = phi(x) * log2(e), so both phi evaluations of eq. (1) map to the
// hardware's base-2 exp/log with no extra scaling. Sums and differences are
// linear and unaffected; posteriors are scaled back by ln 2 on store.
constexpr double kLog2e = 1.4426950408889634;
constexpr double kLn2 = 0.6931471805599453;
// Magnitude clamp of the CN update, in nats: [phi(30), 30] at both phi inputs
// of the sign-magnitude rule (phi(30) = 2 atanh(e^-30), about 1.87e-13). In
// pair form the clamp of the phi sum to [phi(30), 30] is a clamp of the
// output magnitude phi(sum) to [phi(30), 30]; the decoder clamps it to
// [0, 30] (the two lower bounds differ by 1.9e-13 nats, which no FP32 sum
// with a posterior keeps), and the lower clamp of |x| needs no instruction
// in FP32 (cn_core).
constexpr double kXMax = 30.0;

// Table layout (built by ldpc_code_create). H lanes share a CN (1, 2 or 4);
// D is the padded CN degree of the kernel variant (a multiple of H, at least
// the largest degree) and DH = D / H the edges per lane:
//   vcn[j]         CN of visit j (visits of group g: visit_ptr[g] ..
//                  visit_ptr[g+1]); its messages are row vcn[j] of L;
//   vw             per visit j and lane h a half-record of W = 2 DH rounded
//                  up to 4 words, at (j * H + h) * W: word k = 4 x posterior
//                  index edge h*DH + k reads (its VN); word DH + k = 4 x
//                  float index the lane writes after the update: the VN's
//                  posterior when the VN has no other edge in this group,
//                  else a delta slot (index >= ds_start) that the fix-up
//                  pass folds in. Padding edges read and write posterior n,
//                  a scratch posterior nobody else reads; with VN groups
//                  (the vertical schedule) an edge whose VN is outside the
//                  group reads its VN and writes posterior n.
//                  The edge order within a row is chosen per CN for LDS
//                  banks (see edge_order in ndgsbp_host.cpp).
//   fix[q]         fix-up entry of a group: x = VN | count << 16,
//                  y = first delta slot (relative to ds_start); a VN's slots
//                  are consecutive and are added in slot order.
//   syn_col        check c at c * SD (SD = D rounded up to 4): 4 x the VN
//                  ids of the check within its first D entries, padded with
//                  4 x (n + 1) (a posterior fixed at +0, i.e. hard bit 0);
//                  entries D .. SD - 1 are always padding and never read.
// LDS of a workgroup (one frame):
//   floats [0, ds_start + max_slots): posteriors (n + 2, ds_start = n + 2)
//     then delta slots;
//   at l_offset: message rows, row (cn * H + h) of lane h of CN cn holding
//     DH messages (FP32, or 16-bit with DH rounded up to even);
//   at sh_offset (the last 16 bytes of the allocation, the same for every
//     problem of a launch): int frame, int flag[2], int problem.

// One decode problem: a code's tables for one CN-lane mapping and the
// buffers of one call.
struct Problem {
    const int32_t* vcn;
    const uint32_t* vw;
    const int32_t* visit_ptr;
    const uint2* fix;
    const int32_t* fix_ptr;
    const uint32_t* syn_col;
    const float* llr;
    uint8_t* hard;
    float* post;
    int32_t* iters;
    uint8_t* syn_ok;
    int32_t n, m, G;
    int32_t max_iter;
    int32_t first;        // launch-wide index of the problem's first frame
    int32_t num_frames;
    uint32_t ds_start_b;  // byte offset of the first delta slot
    uint32_t pad_b;       // byte offset of the scratch posterior n of padding edges
    int32_t l_offset;     // byte offset of the message rows
    int32_t R;            // iteration blocks of G groups: iteration l uses block (l-1) mod R
};

// Kernel arguments. A launch decodes p0 (table == nullptr) or the nprob
// problems of a device table sorted by `first`, whose frames it numbers
// 0 .. total_frames - 1 in table order.
struct DecodeArgs {
    Problem p0;
    const Problem* table;
    int32_t nprob;
    int32_t total_frames;
    uint32_t* work;       // this launch's {next frame, finished workgroups}, zero at launch
    int32_t early_stop;
    int32_t packed;       // hard decisions packed 8 per byte (LSB first)
    int32_t sh_offset;    // byte offset of the workgroup state (frame, flags, problem)
    float ymax;           // upper clamp of |VN->CN message|, log2 units
};

struct LaunchShape {
    int lanes;       // lanes per CN visit (1, 2 or 4)
    int threads;     // workgroup size
    int blocks;      // persistent workgroups
    size_t lds_bytes;
    bool vertical = false;  // VN groups (the vertical schedule)
};

enum MsgKind { kMsgF32 = 0, kMsgF16 = 1, kMsgBF16 = 2 };

// Launch one decode; implemented next to the kernels.
hipError_t launch_decode(const DecodeArgs& a, MsgKind kind, int dmax, bool uniform, const LaunchShape& shape,
                         hipStream_t stream);
// Resident workgroups per CU of a kernel variant.
// `table`: the batched kernel (problems read from a device table).
// mode: 0 one problem, 1 a batch's problem table, 2 the vertical schedule
hipError_t decode_occupancy(MsgKind kind, int dmax, bool uniform, int lanes, int mode, int threads,
                            size_t lds_bytes, int* blocks_per_cu);
int max_threads_for_degree(int dmax);
// Bytes of the message rows of one CN.
int message_row_bytes(MsgKind kind, int dmax, int lanes);
// Largest CN degree any kernel variant handles.
constexpr int kMaxDegree = 32;
// Work counters per code: decode calls in flight on one code at once, at most.
constexpr int kWorkRing = 1024;

}  // namespace ndgsbp
