// gfx950 kernel of the NDGSBP decoder for codes whose per-frame state does
// not fit in LDS: frame-interleaved state in HBM (Sec. II-C, Steps 2-4).
//
// A workgroup owns a tile of 64 frame slots, slot l = lane l of every wave.
// Its posteriors, delta slots and CN->VN messages live in a device workspace
// laid out row-major with the 64 slots fastest: float row r (posterior r,
// or delta slot r - ds_start) at fws[r * 64 + l]; message k of CN c at
// mws[(c * D + k) * 64 + l]. A wave processes one CN visit at a time for all
// 64 frames: the visit's edge table is the same for every lane, so it comes
// through scalar loads, and every access to the frame state is one 256-byte
// (FP32) or 128-byte (16-bit) row per instruction, fully coalesced.
//
// Per iteration, for each group g in order: the waves split the group's
// visits (eq. (1) and the add-back, the same arithmetic as the LDS kernel,
// cn_core with one lane per CN row); barrier; fix-up of VNs with several
// edges in the group; barrier. After the last group: per-slot syndrome
// (Step 4); slots whose frame is finished write its outputs, and once enough
// slots are idle they take new frames from the launch's work counter, so the
// tile keeps decoding while frames need different numbers of iterations.
//
// Messages are not cleared when a frame starts: in a frame's first
// iteration, the first visit of each CN uses 0 as the old message (the
// initial value), and every later visit reads what an earlier visit of the
// same iteration wrote (each visit writes all D messages of its CN).
#include <hip/hip_runtime.h>

#include "ndgsbp_cn.h"
#include "ndgsbp_hbm.h"
#include "ndgsbp_internal.h"
#include "ndgsbp_math.h"

namespace ndgsbp {
namespace {

using namespace dev;

constexpr int kSlots = 64;       // frames per workgroup tile (one per lane)
constexpr int kMaxWaves = 16;

typedef const __attribute__((address_space(4))) uint32_t const_u32;
__device__ __forceinline__ uint32_t tbl_u32(const uint32_t* base, uint32_t i) { return ((const_u32*)base)[i]; }
__device__ __forceinline__ int32_t tbl_i32(const int32_t* base, uint32_t i) {
    return (int32_t)((const_u32*)base)[i];
}

// Workgroup-size cap per degree: a lane holds a whole CN row in registers.
template <int D>
struct HbmMaxThreads {
    static constexpr int value = D >= 24 ? 256 : D >= 12 ? 512 : 1024;
};

// Wave 0: takes frames from the launch's work counter for the slots in
// `want` (a lane mask), in lane order; lane l gets *frame (-1 if the launch
// has none left). Returns the slots that got a frame; clears *more once the
// counter has passed the last frame.
__device__ __forceinline__ uint64_t claim_slots(const HbmArgs& a, uint64_t want, int lane, int* frame, int* more) {
    const int cnt = __popcll(want);
    if (cnt == 0) return 0;
    unsigned base = 0;
    if (lane == 0) base = atomicAdd(a.work, (unsigned)cnt);
    base = __shfl(base, 0);
    const bool mine = (want >> lane) & 1ull;
    const unsigned f = base + (unsigned)__popcll(want & ((1ull << lane) - 1ull));
    const bool got = mine && f < (unsigned)a.p.num_frames;
    *frame = got ? (int)f : -1;
    if (lane == 0 && base + (unsigned)cnt >= (unsigned)a.p.num_frames) *more = 0;
    return __ballot(got);
}

// Sign masks (SGN: the tile keeps, per VN, a 64-bit word in LDS whose bit l
// is the sign bit of slot l's posterior, i.e. its hard decision): every
// posterior write updates its VN's word with one ballot, so the syndrome and
// the hard-decision outputs read LDS instead of the workspace.
__device__ __forceinline__ void put_sign(uint64_t* sgn, uint32_t v, float x) {
    const uint64_t m = __ballot(__float_as_uint(x) >> 31);
    if ((threadIdx.x & 63) == 0) sgn[v] = m;
}

template <class M, int D, bool UNI>
__global__ __launch_bounds__(HbmMaxThreads<D>::value) void ndgsbp_hbm_kernel(HbmArgs a) {
    using T = typename M::T;
    constexpr int SD = (D + 3) / 4 * 4;
    constexpr int W = (2 * D + 3) / 4 * 4;  // words per visit record (one lane per CN)
    const Problem& p = a.p;
    const int tid = threadIdx.x, nt = blockDim.x;
    // the wave index is wave-uniform: visit indices built from it stay in
    // scalar registers, so the visit records come through scalar loads
    const int lane = tid & 63, wv = __builtin_amdgcn_readfirstlane(tid >> 6), nw = nt >> 6;
    const bool SGN = a.sgn_lds != 0;
    const bool DL = a.dslot_lds != 0;
    float* fw = a.fws + (size_t)blockIdx.x * a.fws_tile;
    T* mw = reinterpret_cast<T*>(a.mws) + (size_t)blockIdx.x * a.mws_tile;
    extern __shared__ __align__(16) uint64_t sgn[];  // n + 2 words when SGN
    // delta slot s of slot l at dsl[s * 64 + l] when DL (after the sign words)
    float* dsl = reinterpret_cast<float*>(sgn + (SGN ? p.n + 2 : 0));

    __shared__ int s_frame[kSlots];   // frame of each slot, -1: none
    __shared__ int s_next[kSlots];    // frame a slot takes after its outputs are written
    __shared__ int s_used[kSlots];    // iterations run on it
    __shared__ int s_fail[kMaxWaves][kSlots];
    __shared__ unsigned long long s_failm[kMaxWaves];  // SGN: slots a wave saw fail
    __shared__ unsigned long long s_mask[3];  // [0] active, [1] to retire, [2] just filled
    __shared__ unsigned long long s_chk;  // slots that check their syndrome this iteration
    __shared__ int s_more;            // the launch may still have frames

    if (SGN)
        for (int v = tid; v < p.n + 2; v += nt) sgn[v] = 0ull;  // n + 1: syndrome padding, always 0
    if (wv == 0) {
        if (lane == 0) s_more = 1;
        int f = -1;
        const uint64_t got = claim_slots(a, ~0ull, lane, &f, &s_more);
        s_frame[lane] = f;
        s_used[lane] = 0;
        if (lane == 0) {
            s_mask[0] = got;
            s_mask[1] = 0;
            s_mask[2] = got;
        }
    }
    __syncthreads();

    for (;;) {
        // start the frames of newly filled slots: posteriors = channel LLRs
        const uint64_t fill = s_mask[2];
        if (fill) {
            const bool mine = (fill >> lane) & 1ull;
            const int f = s_frame[lane];
            const float* y = p.llr + (size_t)(mine ? f : 0) * p.n;
            if ((p.n & 3) == 0 && ((uintptr_t)p.llr & 15u) == 0) {
                // four consecutive LLRs of the lane's frame per load (rows
                // of n floats are then 16-byte aligned)
                for (int q = wv; q < (p.n >> 2); q += nw) {
                    float4 y4 = make_float4(0.f, 0.f, 0.f, 0.f);
                    if (mine) y4 = reinterpret_cast<const float4*>(y)[q];
                    const float x[4] = {y4.x * kLog2eF + 0.0f, y4.y * kLog2eF + 0.0f, y4.z * kLog2eF + 0.0f,
                                        y4.w * kLog2eF + 0.0f};  // + 0: -0.0 -> +0.0
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const uint32_t v = 4u * (uint32_t)q + (uint32_t)i;
                        if (mine) fw[(size_t)v * kSlots + lane] = x[i];
                        if (SGN) {
                            const uint64_t neg = __ballot(mine && (__float_as_uint(x[i]) >> 31));
                            if (lane == 0) sgn[v] = (sgn[v] & ~fill) | neg;
                        }
                    }
                }
            } else {
                for (int v = wv; v < p.n; v += nw) {
                    const float x = mine ? y[v] * kLog2eF + 0.0f : 0.0f;
                    if (mine) fw[(size_t)v * kSlots + lane] = x;
                    if (SGN) {
                        const uint64_t neg = __ballot(mine && (__float_as_uint(x) >> 31));
                        if (lane == 0) sgn[v] = (sgn[v] & ~fill) | neg;
                    }
                }
            }
            // posterior n: scratch of padding edges; n + 1: 0, syndrome padding
            if (mine && wv == 0) {
                fw[(size_t)p.n * kSlots + lane] = 0.0f;
                fw[(size_t)(p.n + 1) * kSlots + lane] = 0.0f;
            }
        }
        __syncthreads();
        const uint64_t active = s_mask[0];
        if (active == 0) break;
        const bool fresh = s_used[lane] == 0;  // this slot's frame is in its first iteration

        for (int g = 0; g < p.G; ++g) {
            const int j0 = tbl_i32(p.visit_ptr, g), j1 = tbl_i32(p.visit_ptr, g + 1);
            for (int j = j0 + wv; j < j1; j += nw) {
                const int cn = tbl_i32(p.vcn, j);
                const bool zero_old = fresh && tbl_u32(a.vfirst, j);
                const uint32_t dfirst = tbl_u32(a.vdfirst, j);
                float pv[D], lo[D], wvals[D];
                bool real[D];
                T st[D];
                uint32_t pa[D], ta[D];
#pragma unroll
                for (int k = 0; k < D; ++k) {
                    pa[k] = tbl_u32(p.vw, (uint32_t)j * W + k);
                    ta[k] = tbl_u32(p.vw, (uint32_t)j * W + D + k);
                }
                T* row = mw + (size_t)cn * D * kSlots + lane;
#pragma unroll
                for (int k = 0; k < D; ++k) {
                    // byte offset 4r of float row r -> element r * 64; the
                    // message row is loaded for every slot (a fresh slot's
                    // bits are replaced by 0), so that no load waits on a
                    // branch
                    pv[k] = fw[(size_t)pa[k] * (kSlots / 4) + lane];
                    const float old = M::unpack(row[k * kSlots]);
                    lo[k] = zero_old ? 0.0f : old;
                    real[k] = pa[k] != p.pad_b;
                }
                cn_core<M, D, UNI, 1>(pv, lo, real, a.ymax, st, wvals);
#pragma unroll
                for (int k = 0; k < D; ++k) {
                    // a posterior target takes w; a delta slot takes this
                    // edge's change w - P, the VN's first slot P + (w - P),
                    // so that the fix-up only adds its slots in order
                    if (ta[k] >= p.ds_start_b) {
                        const float out = (dfirst >> k) & 1u ? pv[k] + (wvals[k] - pv[k]) : wvals[k] - pv[k];
                        if (DL)
                            dsl[((ta[k] - p.ds_start_b) >> 2) * kSlots + lane] = out;
                        else
                            fw[(size_t)ta[k] * (kSlots / 4) + lane] = out;
                    } else {
                        fw[(size_t)ta[k] * (kSlots / 4) + lane] = wvals[k];
                        if (SGN) put_sign(sgn, ta[k] >> 2, wvals[k]);
                    }
                    row[k * kSlots] = st[k];
                }
            }
            __syncthreads();
            const int q0 = tbl_i32(p.fix_ptr, g), q1 = tbl_i32(p.fix_ptr, g + 1);
            if (q1 > q0) {
                for (int q = q0 + wv; q < q1; q += nw) {
                    const uint32_t x = tbl_u32(reinterpret_cast<const uint32_t*>(p.fix), 2 * q);
                    const uint32_t y = tbl_u32(reinterpret_cast<const uint32_t*>(p.fix), 2 * q + 1);
                    const uint32_t v = x & 0xffffu, c = x >> 16;
                    // P + (w_0 - P) + (w_1 - P) + ..., in slot order
                    float acc;
                    if (DL) {
                        const uint32_t d0 = y * kSlots + lane;
                        acc = dsl[d0];
                        for (uint32_t k = 1; k < c; ++k) acc += dsl[d0 + k * kSlots];
                    } else {
                        const size_t d0 = ((size_t)(p.ds_start_b >> 2) + y) * kSlots + lane;
                        acc = fw[d0];
                        for (uint32_t k = 1; k < c; ++k) acc += fw[d0 + (size_t)k * kSlots];
                    }
                    fw[(size_t)v * kSlots + lane] = acc;
                    if (SGN) put_sign(sgn, v, acc);
                }
                __syncthreads();
            }
        }

        // a4: which slots check their syndrome after this iteration
        if (wv == 0) {
            const bool act = (active >> lane) & 1ull;
            const int used = s_used[lane] + (act ? 1 : 0);
            s_used[lane] = used;
            const bool chk = act && (a.early_stop || used == p.max_iter);
            const uint64_t cm = __ballot(chk);
            if (lane == 0) s_chk = cm;
        }
        __syncthreads();
        const uint64_t need = s_chk;
        if (need) {
            if (SGN) {
                // lane l takes check c = 64 i + l of the wave's rounds; a
                // check's parity word XORs the sign words of its VNs (entries
                // D .. SD - 1 are padding); a wave stops once every checking
                // slot has failed some check
                uint64_t x = 0;
                for (int c0 = 64 * wv; c0 < p.m; c0 += 64 * nw) {
                    const int c = c0 + lane;
                    if (c < p.m) {
                        const uint4* col = reinterpret_cast<const uint4*>(p.syn_col + (size_t)c * SD);
                        uint32_t e[SD];
#pragma unroll
                        for (int q = 0; q < SD / 4; ++q) {
                            const uint4 w4 = col[q];
                            e[4 * q] = w4.x;
                            e[4 * q + 1] = w4.y;
                            e[4 * q + 2] = w4.z;
                            e[4 * q + 3] = w4.w;
                        }
                        uint64_t par = 0;
#pragma unroll
                        for (int k = 0; k < D; ++k) par ^= sgn[e[k] >> 2];
                        x |= par;
                    }
                    uint64_t all = x;
#pragma unroll
                    for (int sh = 1; sh < 64; sh <<= 1) {
                        const uint32_t lo32 = (uint32_t)__shfl_xor((int)(uint32_t)all, sh);
                        const uint32_t hi32 = (uint32_t)__shfl_xor((int)(uint32_t)(all >> 32), sh);
                        all |= ((uint64_t)hi32 << 32) | lo32;
                    }
                    x = all;
                    if ((x & need) == need) break;
                }
                if (lane == 0) s_failm[wv] = x;
            } else {
                // hard decision = sign bit of the posterior (no -0.0 is stored);
                // a wave stops once every checking slot has failed one of its checks
                uint32_t x = 0;
                for (int c = wv; c < p.m; c += nw) {
                    uint32_t par = 0;
                    // entries D .. SD - 1 are padding of every row
#pragma unroll
                    for (int k = 0; k < D; ++k)
                        par ^= __float_as_uint(
                            fw[(size_t)tbl_u32(p.syn_col, (uint32_t)c * SD + k) * (kSlots / 4) + lane]);
                    x |= par;
                    if ((__ballot(x >> 31) & need) == need) break;
                }
                s_fail[wv][lane] = (int)(x >> 31);
            }
        }
        __syncthreads();

        // retire finished frames, refill idle slots
        if (wv == 0) {
            const bool act = (active >> lane) & 1ull;
            int fail = 0;
            if (s_chk) {
                if (SGN) {
                    for (int w = 0; w < nw; ++w) fail |= (int)((s_failm[w] >> lane) & 1ull);
                } else {
                    for (int w = 0; w < nw; ++w) fail |= s_fail[w][lane];
                }
            }
            const int used = s_used[lane];
            const bool chk = act && (a.early_stop || used == p.max_iter);
            const bool done = chk && ((a.early_stop && !fail) || used == p.max_iter);
            if (done) {
                const int f = s_frame[lane];
                p.iters[f] = used;
                if (p.syn_ok) p.syn_ok[f] = fail ? 0 : 1;
            }
            const uint64_t dmask = __ballot(done);
            const uint64_t still = active & ~dmask;
            const uint64_t idle = ~still;
            uint64_t filled = 0;
            int nf = -1;
            // refill once a quarter of the tile is idle, or when it is empty;
            // a retiring slot keeps its frame until its outputs are written
            if (s_more && (__popcll(idle) >= kSlots / 4 || still == 0))
                filled = claim_slots(a, idle, lane, &nf, &s_more);
            s_next[lane] = nf;
            if (lane == 0) {
                s_mask[1] = dmask;
                s_mask[2] = filled;
                s_mask[0] = still | filled;
            }
        }
        __syncthreads();
        // outputs of the retired frames
        const uint64_t retired = s_mask[1];
        if (retired) {
            if (SGN) {
                // hard decisions from the sign words, one frame at a time
                uint64_t ret = retired;
                while (ret) {
                    const int sl = __ffsll((long long)ret) - 1;
                    ret &= ret - 1;
                    const int f = s_frame[sl];
                    if (a.packed) {
                        const int nb = (p.n + 7) >> 3;
                        uint8_t* hd = p.hard + (size_t)f * nb;
                        for (int q = tid; q < nb; q += nt) {
                            uint32_t bits = 0;
#pragma unroll
                            for (int k = 0; k < 8; ++k) {
                                const int v = 8 * q + k;
                                if (v < p.n) bits |= (uint32_t)((sgn[v] >> sl) & 1ull) << k;
                            }
                            hd[q] = (uint8_t)bits;
                        }
                    } else {
                        uint8_t* hd = p.hard + (size_t)f * p.n;
                        for (int v = tid; v < p.n; v += nt) hd[v] = (uint8_t)((sgn[v] >> sl) & 1ull);
                    }
                }
                // posteriors: each row read once, every retiring lane writes its value
                if (p.post) {
                    const bool mine = (retired >> lane) & 1ull;
                    float* po = p.post + (size_t)(mine ? s_frame[lane] : 0) * p.n;
                    for (int v = wv; v < p.n; v += nw) {
                        const float x = fw[(size_t)v * kSlots + lane];
                        if (mine) po[v] = x * kLn2F;
                    }
                }
            } else {
                uint64_t ret = retired;
                while (ret) {
                    const int sl = __ffsll((long long)ret) - 1;
                    ret &= ret - 1;
                    const int f = s_frame[sl];
                    const float* col = fw + sl;
                    float* po = p.post ? p.post + (size_t)f * p.n : nullptr;
                    if (a.packed) {
                        const int nb = (p.n + 7) >> 3;
                        uint8_t* hd = p.hard + (size_t)f * nb;
                        for (int q = tid; q < nb; q += nt) {
                            uint32_t bits = 0;
#pragma unroll
                            for (int k = 0; k < 8; ++k) {
                                const int v = 8 * q + k;
                                if (v < p.n) bits |= (col[(size_t)v * kSlots] < 0.0f ? 1u : 0u) << k;
                            }
                            hd[q] = (uint8_t)bits;
                        }
                        if (po)
                            for (int v = tid; v < p.n; v += nt) po[v] = col[(size_t)v * kSlots] * kLn2F;
                    } else {
                        uint8_t* hd = p.hard + (size_t)f * p.n;
                        for (int v = tid; v < p.n; v += nt) {
                            const float x = col[(size_t)v * kSlots];
                            hd[v] = x < 0.0f ? 1 : 0;
                            if (po) po[v] = x * kLn2F;
                        }
                    }
                }
            }
        }
        __syncthreads();
        if (wv == 0) {
            const bool mine = (s_mask[2] >> lane) & 1ull;
            const bool ret = (s_mask[1] >> lane) & 1ull;
            if (mine) {
                s_frame[lane] = s_next[lane];
                s_used[lane] = 0;
            } else if (ret) {
                s_frame[lane] = -1;
            }
        }
        __syncthreads();
    }

    // the last workgroup out resets the launch's counters for the next launch
    __threadfence();
    if (tid == 0) {
        const unsigned done_wgs = atomicAdd(a.work + 1, 1u);
        if (done_wgs == gridDim.x - 1) {
            atomicExch(a.work, 0u);
            atomicExch(a.work + 1, 0u);
        }
    }
}

template <class M, int D, bool UNI>
hipError_t run_hbm(const HbmArgs& a, int blocks, int threads, hipStream_t s) {
    const void* fn = reinterpret_cast<const void*>(&ndgsbp_hbm_kernel<M, D, UNI>);
    HbmArgs copy = a;
    void* args[] = {&copy};
    const size_t lds = (a.sgn_lds ? hbm_sign_bytes(a.p.n) : 0) + (a.dslot_lds ? hbm_slot_bytes(a.max_slots) : 0);
    if (lds) {
        const hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    return hipLaunchKernel(fn, dim3(blocks), dim3(threads), args, lds, s);
}

template <class M, int D, bool UNI>
hipError_t occ_hbm(int threads, size_t lds, int* out) {
    const void* fn = reinterpret_cast<const void*>(&ndgsbp_hbm_kernel<M, D, UNI>);
    if (lds) {
        const hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(out, fn, threads, lds);
}

template <class M, int D>
hipError_t hbm_by_uniform(bool uni, bool launch, const HbmArgs* a, int blocks, int threads, size_t lds,
                          hipStream_t s, int* out) {
    if (launch) return uni ? run_hbm<M, D, true>(*a, blocks, threads, s) : run_hbm<M, D, false>(*a, blocks, threads, s);
    return uni ? occ_hbm<M, D, true>(threads, lds, out) : occ_hbm<M, D, false>(threads, lds, out);
}

template <class M>
hipError_t hbm_by_degree(int D, bool uni, bool launch, const HbmArgs* a, int blocks, int threads, size_t lds,
                         hipStream_t s, int* out) {
    switch (D) {
        case 4: return hbm_by_uniform<M, 4>(uni, launch, a, blocks, threads, lds, s, out);
        case 6: return hbm_by_uniform<M, 6>(uni, launch, a, blocks, threads, lds, s, out);
        case 7: return hbm_by_uniform<M, 7>(uni, launch, a, blocks, threads, lds, s, out);
        case 8: return hbm_by_uniform<M, 8>(uni, launch, a, blocks, threads, lds, s, out);
        case 10: return hbm_by_uniform<M, 10>(uni, launch, a, blocks, threads, lds, s, out);
        case 12: return hbm_by_uniform<M, 12>(uni, launch, a, blocks, threads, lds, s, out);
        case 16: return hbm_by_uniform<M, 16>(uni, launch, a, blocks, threads, lds, s, out);
        case 24: return hbm_by_uniform<M, 24>(uni, launch, a, blocks, threads, lds, s, out);
        case 32: return hbm_by_uniform<M, 32>(uni, launch, a, blocks, threads, lds, s, out);
        default: return hipErrorInvalidValue;
    }
}

hipError_t hbm_dispatch(MsgKind kind, int D, bool uni, bool launch, const HbmArgs* a, int blocks, int threads,
                        size_t lds, hipStream_t s, int* out) {
    switch (kind) {
        case kMsgF32: return hbm_by_degree<MsgF32>(D, uni, launch, a, blocks, threads, lds, s, out);
        case kMsgF16: return hbm_by_degree<MsgF16>(D, uni, launch, a, blocks, threads, lds, s, out);
        case kMsgBF16: return hbm_by_degree<MsgBF16>(D, uni, launch, a, blocks, threads, lds, s, out);
    }
    return hipErrorInvalidValue;
}

}  // namespace

int hbm_max_threads(int D) { return D >= 24 ? 256 : D >= 12 ? 512 : 1024; }
int hbm_slots() { return kSlots; }

hipError_t launch_hbm(const HbmArgs& a, MsgKind kind, int D, bool uniform, int blocks, int threads,
                      hipStream_t stream) {
    return hbm_dispatch(kind, D, uniform, true, &a, blocks, threads, 0, stream, nullptr);
}

hipError_t hbm_occupancy(MsgKind kind, int D, bool uniform, int threads, size_t lds_bytes, int* blocks_per_cu) {
    return hbm_dispatch(kind, D, uniform, false, nullptr, 0, threads, lds_bytes, nullptr, blocks_per_cu);
}

size_t hbm_sign_bytes(int n) { return (size_t)(n + 2) * 8; }
size_t hbm_slot_bytes(int max_slots) { return (size_t)max_slots * kSlots * 4; }

}  // namespace ndgsbp
