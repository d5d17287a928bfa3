// Internal definitions shared by the host side (code tables, C ABI) and the
// gfx950 kernels of the NDGSBP decoder.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "ndgsbp.h"

namespace ndgsbp {

// The decoder works in log2-scaled LLR units: x' = x * log2(e). Then
// phi(x) = -ln tanh(x/2) becomes psi(y) = log2((1 + 2^-y) / (1 - 2^-y)) with
// psi(y') = phi(x) * log2(e), so both phi evaluations of eq. (1) map to the
// hardware's base-2 exp/log with no extra scaling. Sums and differences are
// linear and unaffected; posteriors are scaled back by ln 2 on store.
constexpr double kLog2e = 1.4426950408889634;
constexpr double kLn2 = 0.6931471805599453;
// Magnitude clamp of the CN update, in nats: [phi(30), 30]. phi(30) =
// 2 atanh(e^-30) = 2 e^-30 to double precision.
constexpr double kXMax = 30.0;
constexpr double kXMin = 1.8715245937680347e-13;

// Table layout (built by ldpc_code_create for the code's padded degree D,
// the smallest kernel variant >= the largest CN degree):
//   vcn[j]         CN of visit j (visits of group g: visit_ptr[g] ..
//                  visit_ptr[g+1]); its message row in LDS is vcn[j] * D;
//   vw[j*W .. ]    edge records of visit j, W = 2D rounded up to 4 words:
//                  word k = LDS byte offset of the posterior edge k reads
//                  (its VN), word D + k = LDS byte offset the lane writes
//                  after the update: the VN's posterior when the VN has no
//                  other edge in this group, else a delta slot (offset >=
//                  ds_start_b) that the fix-up pass folds in. Padding edges
//                  (k >= degree) read and write posterior n, a scratch
//                  posterior nobody else reads.
//   fix[q]         fix-up entry of a group: x = VN | count << 16,
//                  y = first delta slot (relative to ds_start); a VN's slots
//                  are consecutive and are added in slot order.
//   syn_col[c*D+k] VN ids of check c for the syndrome, padded with n + 1
//                  (a posterior fixed at 0, i.e. hard bit 0).
// LDS of one frame, in this order: posteriors P[n + 2] (floats) and two
// int flags, delta slots
// (floats, ds_start = first index), messages L[m * D] (FP32 or 16-bit).

struct DeviceTables {
    int32_t* vcn = nullptr;
    uint32_t* vw = nullptr;
    int32_t* visit_ptr = nullptr;  // G + 1
    uint2* fix = nullptr;
    int32_t* fix_ptr = nullptr;    // G + 1
    uint16_t* syn_col = nullptr;   // m * D
};

struct DecodeArgs {
    const int32_t* vcn;
    const uint32_t* vw;
    const int32_t* visit_ptr;
    const uint2* fix;
    const int32_t* fix_ptr;
    const uint16_t* syn_col;
    const float* llr;
    uint8_t* hard;
    float* post;
    int32_t* iters;
    uint8_t* syn_ok;
    int32_t n, m, G;
    int32_t max_iter;
    int32_t early_stop;
    int32_t num_frames;
    int32_t ds_start;   // float index of the first delta slot
    uint32_t ds_start_b;  // the same, in bytes
    uint32_t dummy_b;   // byte offset of the scratch posterior n
    int32_t l_offset;   // byte offset of the message array
    float ymin, ymax;   // clamp bounds in log2 units
};

enum MsgKind { kMsgF32 = 0, kMsgF16 = 1, kMsgBF16 = 2 };

// Launch one decode; implemented next to the kernels.
hipError_t launch_decode(const DecodeArgs& a, MsgKind kind, int dmax, bool uniform, int threads,
                         size_t lds_bytes, hipStream_t stream);
// Largest CN degree any kernel variant handles.
constexpr int kMaxDegree = 32;

}  // namespace ndgsbp

struct ldpc_code {
    int32_t device;
    int32_t m, n;
    int64_t nnz;
    int32_t G;
    int64_t cn_visits;
    int64_t edge_updates;
    int32_t max_cn_degree;
    int32_t max_vn_degree;
    int32_t max_group_visits;
    int32_t max_slots;
    int32_t D;        // padded CN degree of the tables (kernel variant)
    bool uniform;     // every CN has degree exactly D
    size_t max_lds;   // LDS a workgroup may use on the code's device
    ndgsbp::DeviceTables dev;
};
