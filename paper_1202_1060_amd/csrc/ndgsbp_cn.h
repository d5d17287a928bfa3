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

// Both values of a pair from the other lane of a lane pair / two places away.
__device__ __forceinline__ Pair pair_swap_pair(Pair p) {
    return {__uint_as_float(pair_swap(__float_as_uint(p.s))), __uint_as_float(pair_swap(__float_as_uint(p.t)))};
}
__device__ __forceinline__ Pair quad_half_swap_pair(Pair p) {
    return {__uint_as_float(quad_half_swap(__float_as_uint(p.s))),
            __uint_as_float(quad_half_swap(__float_as_uint(p.t)))};
}

// One lane's DH edges of a CN visit (H lanes per CN; with H = 2 the lanes of
// a pair hold the two halves of the row, with H = 4 the lanes of a quad its
// four quarters).
//   pv[k]     posterior of edge k's VN (log2 units; never -0.0)
//   lo[k]     the edge's old CN->VN message (as stored, widened)
//   real[k]   edge k is not padding (ignored when UNI)
// Per edge the lane forms the VN->CN message t = pv - lo (eq. (2), the
// posterior being the total of eq. (3)) and v = 2^-|t|; the inputs of the
// other edges of the CN are combined in pair form (ndgsbp_math.h) by
// exclusive prefix and suffix; with H = 2 the two lanes exchange their
// pairs and sign parities by DPP; with H = 4 a lane combines its pair
// partner's pair with the other pair's total (two DPP steps). A padding
// edge has v = 0, the neutral input.
// Outputs: st[k] the new message in the storage format, wv[k] = new + t,
// the VN's posterior as this edge alone would leave it. A VN with no other
// edge in the group takes wv as its posterior; for a VN with several,
// wv - pv is this edge's change (new - old up to rounding) and the fix-up
// adds the changes of all its edges.
template <class M, int DH, bool UNI, int H>
__device__ __forceinline__ void cn_core(const float (&pv)[DH], const float (&lo)[DH], const bool (&real)[DH],
                                        float ymax, typename M::T (&st)[DH], float (&wv)[DH]) {
    float t[DH], v[DH];
    uint32_t tb[DH];
    uint32_t sall = 0;
#pragma unroll
    for (int k = 0; k < DH; ++k) {
        t[k] = pv[k] - lo[k];  // VN->CN message, eq. (2)
        // posteriors never hold -0.0, so the sign bit of t is the sign rule
        tb[k] = __float_as_uint(t[k]);
        // |t| is clamped to [0, ymax]: the lower clamp phi(30) of the rule
        // changes nothing in FP32, where 2^-y is 1 for every y below it
        v[k] = v_from_magnitude(clampf(fabsf(t[k]), 0.0f, ymax));
        if (!UNI) {
            v[k] = real[k] ? v[k] : 0.0f;  // (1 + 0)/(1 - 0): no effect on the product
            tb[k] = real[k] ? tb[k] : 0u;
        }
        sall ^= tb[k];
    }
    // exclusive prefix within the lane: pre[k] holds inputs 0 .. k-1
    Pair pre[DH];
    pre[0] = {0.0f, 1.0f};
    if (DH > 1) pre[1] = {v[0], 1.0f};
#pragma unroll
    for (int k = 2; k < DH; ++k) pre[k] = pair_add(pre[k - 1], v[k - 1]);
    // suf: the other lanes' inputs, then also this lane's inputs k+1 ..
    Pair suf = {0.0f, 1.0f};
    if (H == 2) {
        const Pair mine = DH > 1 ? pair_add(pre[DH - 1], v[DH - 1]) : Pair{v[0], 1.0f};
        suf = pair_swap_pair(mine);
        sall ^= pair_swap(sall);
    } else if (H == 4) {
        const Pair mine = DH > 1 ? pair_add(pre[DH - 1], v[DH - 1]) : Pair{v[0], 1.0f};
        const Pair partner = pair_swap_pair(mine);
        const Pair other_pair = quad_half_swap_pair(pair_mul(mine, partner));
        suf = pair_mul(partner, other_pair);
        sall ^= pair_swap(sall);
        sall ^= quad_half_swap(sall);
    }
    Pair e[DH];  // per edge: every other input of the CN
#pragma unroll
    for (int k = DH - 1; k >= 0; --k) {
        if (H == 1 && k == DH - 1)
            e[k] = pre[k];  // no input after it, none in other lanes
        else if (k == 0)
            e[k] = suf;
        else if (k == 1)
            e[k] = pair_add(suf, v[0]);  // pre[1] is input 0 alone
        else
            e[k] = pair_mul(pre[k], suf);
        if (k > 0) suf = (H == 1 && k == DH - 1) ? Pair{v[k], 1.0f} : pair_add(suf, v[k]);
    }
    float o[DH];
#pragma unroll
    for (int k = 0; k < DH; ++k) {
        const float mag = clampf(magnitude_from_pair(e[k]), 0.0f, ymax);
        o[k] = __uint_as_float(__float_as_uint(mag) | ((sall ^ tb[k]) & 0x80000000u));
    }
    // stored format, two at a time; the add-back uses the stored value
#pragma unroll
    for (int k = 0; k < DH; k += 2) {
        if (k + 1 < DH)
            M::pack2(o[k], o[k + 1], st[k], st[k + 1]);
        else
            st[k] = M::pack(o[k]);
    }
#pragma unroll
    for (int k = 0; k < DH; ++k) wv[k] = M::unpack(st[k]) + t[k];
}

}  // namespace dev
}  // namespace ndgsbp
