// Device-side arithmetic of the NDGSBP CN update: message storage formats and
// psi, the log2-unit form of phi(x) = -ln tanh(x/2) (Sec. II-C, eq. (1)).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ndgsbp {
namespace dev {

constexpr float kLog2eF = 1.44269504088896341f;
constexpr float kLn2F = 0.693147180559945309f;

// --- message storage formats -------------------------------------------------

struct MsgF32 {
    using T = float;
    static __device__ __forceinline__ T pack(float x) { return x; }
    static __device__ __forceinline__ float unpack(T v) { return v; }
};

struct MsgF16 {
    using T = _Float16;
    static __device__ __forceinline__ T pack(float x) { return (T)x; }  // round to nearest even
    static __device__ __forceinline__ float unpack(T v) { return (float)v; }
};

struct MsgBF16 {
    using T = uint16_t;
    // round to nearest even; inputs are finite (magnitudes are clamped)
    static __device__ __forceinline__ T pack(float x) {
        const uint32_t u = __float_as_uint(x);
        return (T)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
    }
    static __device__ __forceinline__ float unpack(T v) { return __uint_as_float((uint32_t)v << 16); }
};

// --- psi(y) = log2((1 + 2^-y) / (1 - 2^-y)), the log2-unit form of phi ---------

__device__ __forceinline__ float exp2_hw(float x) { return __builtin_amdgcn_exp2f(x); }
__device__ __forceinline__ float log2_hw(float x) { return __builtin_amdgcn_logf(x); }
__device__ __forceinline__ float rcp_hw(float x) { return __builtin_amdgcn_rcpf(x); }

// Forward use (|VN->CN message| -> summand), from v = 2^-y. Small results
// must keep their relative accuracy (they are summed, and a small sum is
// mapped back to a large message), so for v < kFwdSeriesMax the ratio's
// logarithm is replaced by the odd series 2 atanh(v) / ln 2 =
// (2/ln2)(v + v^3/3 + v^5/5 + v^7/7 + ...), truncated after v^7 (relative
// error < 3e-11 there). Large results only need absolute accuracy: a large
// summand drives the other outputs to ~0.
constexpr float kFwdSeriesMax = 0.0625f;
__device__ __forceinline__ float psi_fwd_series(float v) {
    const float w = v * v;
    const float c1 = 2.0f * kLog2eF, c3 = c1 / 3.0f, c5 = c1 / 5.0f, c7 = c1 / 7.0f;
    return v * fmaf(w, fmaf(w, fmaf(w, c7, c5), c3), c1);
}
__device__ __forceinline__ float psi_fwd_general(float v) { return log2_hw((1.0f + v) * rcp_hw(1.0f - v)); }
__device__ __forceinline__ float psi_fwd(float y) {
    const float v = exp2_hw(-y);
    return v < kFwdSeriesMax ? psi_fwd_series(v) : psi_fwd_general(v);
}

// Inverse use (sum -> |CN->VN message|). A small sum gives a large message,
// whose relative accuracy needs 1 - 2^-y without cancellation: for
// z = y ln 2 < 1/4 (y < kInvSeriesMax) it is taken from the Taylor series of
// 1 - e^-z up to z^6 (relative truncation error < 5e-8), written as a
// polynomial in y; above, 1 - v loses at most ~2.7e-7. A large sum gives a
// small message, where absolute accuracy suffices. The result is >= +0
// (log2 of a ratio >= 1).
constexpr float kInvSeriesMax = (float)(0.25 / 0.6931471805599453);
__device__ __forceinline__ float one_minus_exp2_neg(float y) {
    constexpr double l = 0.6931471805599453;
    constexpr float c1 = (float)l, c2 = (float)(-l * l / 2), c3 = (float)(l * l * l / 6),
                    c4 = (float)(-l * l * l * l / 24), c5 = (float)(l * l * l * l * l / 120),
                    c6 = (float)(-l * l * l * l * l * l / 720);
    float p = fmaf(y, c6, c5);
    p = fmaf(y, p, c4);
    p = fmaf(y, p, c3);
    p = fmaf(y, p, c2);
    p = fmaf(y, p, c1);
    return y * p;
}
__device__ __forceinline__ float psi_inv_from(float v, float den) { return log2_hw((1.0f + v) * rcp_hw(den)); }
__device__ __forceinline__ float psi_inv(float y) {
    const float v = exp2_hw(-y);
    return psi_inv_from(v, y < kInvSeriesMax ? one_minus_exp2_neg(y) : 1.0f - v);
}

// True when the predicate holds on any active lane of the wavefront.
__device__ __forceinline__ bool wave_any(bool p) { return __builtin_amdgcn_ballot_w64(p) != 0; }

__device__ __forceinline__ float clampf(float x, float lo, float hi) { return __builtin_amdgcn_fmed3f(x, lo, hi); }

}  // namespace dev
}  // namespace ndgsbp
