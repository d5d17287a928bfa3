// The CN update of eq. (1) and the add-back values for one lane's edges, in
// registers: shared by the LDS-resident and the HBM-resident kernels, so that
// both run the same operations in the same order.
#pragma once

#include <hip/hip_runtime.h>

#include "ndgsbp_math.h"

namespace ndgsbp {
namespace dev {

// Value of the other lane of a lane pair (lanes 2i and 2i+1), by DPP.
__device__ __forceinline__ uint32_t pair_swap(uint32_t x) {
    return (uint32_t)__builtin_amdgcn_mov_dpp((int)x, 0xB1, 0xF, 0xF, false);  // quad_perm [1,0,3,2]
}
// Value of the lane two places away within a quad (lanes 4i..4i+3), by DPP.
__device__ __forceinline__ uint32_t quad_half_swap(uint32_t x) {
    return (uint32_t)__builtin_amdgcn_mov_dpp((int)x, 0x4E, 0xF, 0xF, false);  // quad_perm [2,3,0,1]
}

// One lane's DH edges of a CN visit (H lanes per CN; with H = 2 the lanes of
// a pair hold the two halves of the row, with H = 4 the lanes of a quad its
// four quarters).
//   pv[k]     posterior of edge k's VN (log2 units; never -0.0)
//   lo[k]     the edge's old CN->VN message (as stored, widened)
//   real[k]   edge k is not padding (ignored when UNI)
// Per edge the lane forms the VN->CN message t = pv - lo (eq. (2), the
// posterior being the total of eq. (3)) and eps = 1 - tanh(|t|/2); the eps of
// the other edges of the CN are combined with (+) (ndgsbp_math.h) by exclusive
// prefix and suffix; with H = 2 the two lanes exchange their partial
// combinations and sign parities by DPP; with H = 4 a lane combines its
// pair partner's partial with the other pair's total (two DPP steps).
// Outputs: st[k] the new message in the storage format, wv[k] = new + t,
// the VN's posterior as this edge alone would leave it. A VN with no other edge in the group takes wv as its
// posterior; for a VN with several, wv - pv is this edge's change (new - old
// up to rounding) and the fix-up adds the changes of all its edges.
template <class M, int DH, bool UNI, int H>
__device__ __forceinline__ void cn_core(const float (&pv)[DH], const float (&lo)[DH], const bool (&real)[DH],
                                        float ymax, float cmin, typename M::T (&st)[DH],
                                        float (&wv)[DH]) {
    float t[DH], e[DH];
    uint32_t tb[DH];
    uint32_t sall = 0;
#pragma unroll
    for (int k = 0; k < DH; ++k) {
        t[k] = pv[k] - lo[k];  // VN->CN message, eq. (2)
        // posteriors never hold -0.0, so the sign bit of t is the sign rule
        tb[k] = __float_as_uint(t[k]);
        // |t| is clamped to [0, ymax]: the lower clamp phi(30) of the rule
        // changes nothing in FP32, where 2^y is 1 for every y below it and
        // eps is 1 either way; the constant 0 keeps the clamp one instruction
        // with a single scalar operand
        e[k] = eps_from_magnitude(clampf(fabsf(t[k]), 0.0f, ymax));
        if (!UNI) {
            e[k] = real[k] ? e[k] : 0.0f;  // 0 is the identity of (+)
            tb[k] = real[k] ? tb[k] : 0u;
        }
        sall ^= tb[k];
    }
    // exclusive combination over N(m) \ n: prefix (+) suffix (+ the partner's)
    float pre[DH], c[DH];
    if (DH > 1) pre[1] = e[0];
#pragma unroll
    for (int k = 2; k < DH; ++k) pre[k] = oplus(pre[k - 1], e[k - 1]);
    float suf;
    if (H == 2) {
        const float mine = DH > 1 ? oplus(pre[DH - 1], e[DH - 1]) : e[0];
        suf = __uint_as_float(pair_swap(__float_as_uint(mine)));
        sall ^= pair_swap(sall);
        c[DH - 1] = DH > 1 ? oplus(pre[DH - 1], suf) : suf;
    } else if (H == 4) {
        const float mine = DH > 1 ? oplus(pre[DH - 1], e[DH - 1]) : e[0];
        const float partner = __uint_as_float(pair_swap(__float_as_uint(mine)));
        const float other_pair = __uint_as_float(quad_half_swap(__float_as_uint(oplus(mine, partner))));
        suf = oplus(partner, other_pair);
        sall ^= pair_swap(sall);
        sall ^= quad_half_swap(sall);
        c[DH - 1] = DH > 1 ? oplus(pre[DH - 1], suf) : suf;
    } else {
        suf = 0.0f;
        c[DH - 1] = DH > 1 ? pre[DH - 1] : 0.0f;
    }
#pragma unroll
    for (int k = DH - 2; k >= 0; --k) {
        suf = (H == 1 && k == DH - 2) ? e[k + 1] : oplus(suf, e[k + 1]);
        c[k] = k == 0 ? suf : oplus(pre[k], suf);
    }
#pragma unroll
    for (int k = 0; k < DH; ++k) {
        const float mag = magnitude_from_complement(clampf(c[k], cmin, 1.0f));
        const uint32_t out = __float_as_uint(mag) | ((sall ^ tb[k]) & 0x80000000u);
        st[k] = M::pack(__uint_as_float(out));
        const float ls = M::unpack(st[k]);
        wv[k] = ls + t[k];
    }
}

}  // namespace dev
}  // namespace ndgsbp
