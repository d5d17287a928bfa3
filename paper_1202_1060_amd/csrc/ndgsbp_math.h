// Device-side arithmetic of the NDGSBP CN update (Sec. II-C, eq. (1)):
// message storage formats and the complement-product form of the CN rule.
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

// --- eq. (1) in complement-product form ---------------------------------------
//
// With magnitudes in log2 units (y = |x| log2 e) and v = 2^-y = e^-|x|:
//   tanh(|x|/2) = (1 - v)/(1 + v) = 1 - eps,   eps = 2v/(1 + v) = 2/(1 + 2^y),
// and eq. (1) for the edge to n reads |L_{m->n}| = 2 atanh(u) with
// u = prod_{n' != n} (1 - eps_{n'}). The decoder never forms u: it carries
// c = 1 - u, combining inputs with
//   c (+) eps = 1 - (1 - c)(1 - eps) = c + eps - c*eps,
// which adds non-negative terms when c and eps are small (the reliable,
// large-message case where 1 - u would cancel), and returns
//   |L| (log2 units) = log2((1 + u)/(1 - u)) = log2((2 - c)/c).
// This is the same function as the sign-magnitude phi rule
// phi(sum phi(|x|)), phi(x) = -ln tanh(x/2): sum phi = -ln u.
// Where c is close to 1 (some input unreliable) the result is small and only
// its absolute accuracy matters, which the rounding of c near 1 keeps.

__device__ __forceinline__ float exp2_hw(float x) { return __builtin_amdgcn_exp2f(x); }
__device__ __forceinline__ float log2_hw(float x) { return __builtin_amdgcn_logf(x); }
__device__ __forceinline__ float rcp_hw(float x) { return __builtin_amdgcn_rcpf(x); }

// eps = 1 - tanh(|x|/2) = 2v/(1 + v) = 1/(0.5 + 0.5 * 2^y) for magnitude y
// (log2 units): one exp2, one fused multiply-add, one reciprocal (halving
// 1 + 2^y is exact, so this is 2/(1 + 2^y) with the factor 2 moved inside
// the reciprocal, where it costs nothing); relative error a few ulp for all
// y in the clamp range
__device__ __forceinline__ float eps_from_magnitude(float y) { return rcp_hw(fmaf(0.5f, exp2_hw(y), 0.5f)); }

// 1 - (1 - c)(1 - e) in one add and one fused multiply-add
__device__ __forceinline__ float oplus(float c, float e) { return fmaf(-c, e, c + e); }

// log2((2 - c)/c) = log2(2/c - 1): the message magnitude (log2 units) for
// complement c, as one reciprocal, one fused multiply-add and one log2
__device__ __forceinline__ float magnitude_from_complement(float c) { return log2_hw(fmaf(2.0f, rcp_hw(c), -1.0f)); }

__device__ __forceinline__ float clampf(float x, float lo, float hi) { return __builtin_amdgcn_fmed3f(x, lo, hi); }

}  // namespace dev
}  // namespace ndgsbp
