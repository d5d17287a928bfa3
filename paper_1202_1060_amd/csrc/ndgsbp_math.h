// Device-side arithmetic of the NDGSBP CN update (Sec. II-C, eq. (1)):
// message storage formats and the pair form of the CN rule.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ndgsbp {
namespace dev {

constexpr float kLog2eF = 1.44269504088896341f;
constexpr float kLn2F = 0.693147180559945309f;

// --- message storage formats -------------------------------------------------

// pack: one value; pack2: two values (for FP16 one packed conversion). Both
// round to nearest even.
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef _Float16 f16x2 __attribute__((ext_vector_type(2)));

struct MsgF32 {
    using T = float;
    static __device__ __forceinline__ T pack(float x) { return x; }
    static __device__ __forceinline__ void pack2(float a, float b, T& x, T& y) {
        x = a;
        y = b;
    }
    static __device__ __forceinline__ float unpack(T v) { return v; }
};

struct MsgF16 {
    using T = _Float16;
    static __device__ __forceinline__ T pack(float x) { return (T)x; }
    static __device__ __forceinline__ void pack2(float a, float b, T& x, T& y) {
        const f16x2 h = __builtin_convertvector(f32x2{a, b}, f16x2);
        x = h[0];
        y = h[1];
    }
    static __device__ __forceinline__ float unpack(T v) { return (float)v; }
};

struct MsgBF16 {
    using T = uint16_t;
    // inputs are finite (magnitudes are clamped)
    static __device__ __forceinline__ T pack(float x) {
        const uint32_t u = __float_as_uint(x);
        return (T)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
    }
    static __device__ __forceinline__ void pack2(float a, float b, T& x, T& y) {
        x = pack(a);
        y = pack(b);
    }
    static __device__ __forceinline__ float unpack(T v) { return __uint_as_float((uint32_t)v << 16); }
};

// --- eq. (1) in pair form ------------------------------------------------------
//
// With magnitudes in log2 units (y = |x| log2 e) and v = 2^-y = e^-|x|:
//   tanh(|x|/2) = (1 - v)/(1 + v),
// so for a set of inputs prod tanh(|x_i|/2) = N/D with D = prod (1 + v_i),
// N = prod (1 - v_i), and eq. (1) gives the magnitude
//   |L| = 2 atanh(N/D) = ln((D + N)/(D - N)) nats = log2(T/S) (log2 units)
// with S = D - N, T = D + N. The decoder carries the pair (S, T) up to a
// common positive factor, which the ratio ignores:
//   the empty set is (0, 1); adding an input v maps (S, T) to
//   (S + vT, T + vS); two disjoint sets combine to
//   (Ta Sb + Sa Tb, Ta Tb + Sa Sb).
// Every term is non-negative, so nothing cancels: for reliable inputs S is a
// sum of small positive terms (the case where D - N formed directly would
// cancel), and where some input is unreliable log2 T - log2 S is small and
// only its absolute accuracy counts. This is the same function as the
// sign-magnitude phi rule phi(sum phi(|x|)), phi(x) = -ln tanh(x/2), since
// sum phi = -ln(N/D). Per input one exp2, per output two log2.

struct Pair {
    float s, t;
};

__device__ __forceinline__ float exp2_hw(float x) { return __builtin_amdgcn_exp2f(x); }
__device__ __forceinline__ float log2_hw(float x) { return __builtin_amdgcn_logf(x); }

// v = 2^-y for magnitude y (log2 units)
__device__ __forceinline__ float v_from_magnitude(float y) { return exp2_hw(-y); }

// (S, T) of a set with the input v added: two fused multiply-adds
__device__ __forceinline__ Pair pair_add(Pair a, float v) { return {fmaf(v, a.t, a.s), fmaf(v, a.s, a.t)}; }

// (S, T) of the union of two disjoint sets: two products, two fused multiply-adds
__device__ __forceinline__ Pair pair_mul(Pair a, Pair b) { return {fmaf(a.t, b.s, a.s * b.t), fmaf(a.t, b.t, a.s * b.s)}; }

// |L| = log2(T / S) (log2 units); +inf for S = 0 (no other input, or every
// other input a padding edge), which the caller's clamp turns into its maximum
__device__ __forceinline__ float magnitude_from_pair(Pair e) { return log2_hw(e.t) - log2_hw(e.s); }

__device__ __forceinline__ float clampf(float x, float lo, float hi) { return __builtin_amdgcn_fmed3f(x, lo, hi); }

}  // namespace dev
}  // namespace ndgsbp
