// gfx950 kernel of the NDGSBP decoder (Sec. II-C, Steps 2-4).
//
// Persistent workgroups. Each workgroup holds S frame slots in LDS: a slot's
// posteriors, CN->VN messages and delta slots stay resident for the whole
// decode of its frame. Slots are interleaved element by element, so the S
// lanes that work on the same CN (or VN) of the S frames are neighbours and
// share table loads and LDS bank groups. A slot whose frame is finished
// (zero syndrome with early stop, or I_max reached) writes its outputs and
// takes the next frame from a device-wide counter, so frames of different
// lengths keep every slot busy.
//
// One iteration, all slots in step:
//   for each group g (Step 2):
//     CN phase: one lane per (CN visit, slot). For each edge (m, n) the lane
//       forms the VN->CN message as posterior minus old message (equal to
//       eq. (2) because the posterior is the total of eq. (3)), evaluates
//       eq. (1) in sign-magnitude form with exclusive prefix/suffix sums,
//       stores the new message and adds it back into the posterior: directly
//       when the VN has no other edge in the group, else as a delta;
//     barrier;
//     fix-up (only if the group has VNs with several edges in it): one lane
//       per (VN, slot) adds its deltas in a fixed order; barrier.
//   syndrome of the hard decisions for every slot that needs it (Step 4);
//   barrier; finished slots write outputs and are refilled.
// Every CN update of a group reads posteriors and messages as they stood
// before the group, as eq. (1) prescribes for a group processed in parallel.
#include <hip/hip_runtime.h>

#include "ndgsbp_internal.h"
#include "ndgsbp_math.h"

namespace ndgsbp {
namespace {

using namespace dev;

// The kernels declare no static LDS, so the dynamic allocation starts at LDS
// address 0 and computed byte offsets are LDS addresses (checked per launch).
typedef __attribute__((address_space(3))) float lds_float;
typedef __attribute__((address_space(3))) int lds_int;
__device__ __forceinline__ lds_float& lds_f32(uint32_t byte_off) { return *(lds_float*)(size_t)byte_off; }
__device__ __forceinline__ lds_int& lds_i32(uint32_t byte_off) { return *(lds_int*)(size_t)byte_off; }

// Edge table of one lane's share of a visit in registers: 4 x the posterior
// index each edge reads (its VN) and 4 x the float index each edge writes
// back (the posterior, or a delta slot at index >= ds_start). With H lanes
// per CN, lane h of the CN owns edges h*DH .. h*DH + DH - 1 of the padded row.
template <int DH>
struct VisitRegs {
    static constexpr int kWords = (2 * DH + 3) / 4 * 4;  // half-record stride in words
    int cn;
    uint32_t pa[DH];
    uint32_t ta[DH];
};

template <int DH, int H>
__device__ __forceinline__ void load_visit(const DecodeArgs& a, int j, int h, VisitRegs<DH>& r) {
    constexpr int W = VisitRegs<DH>::kWords;
    r.cn = a.vcn[j];
    const uint4* src = reinterpret_cast<const uint4*>(a.vw) + ((size_t)j * H + h) * (W / 4);
    uint32_t w[W];
#pragma unroll
    for (int q = 0; q < W / 4; ++q) {
        const uint4 x = src[q];
        w[4 * q] = x.x;
        w[4 * q + 1] = x.y;
        w[4 * q + 2] = x.z;
        w[4 * q + 3] = x.w;
    }
#pragma unroll
    for (int k = 0; k < DH; ++k) {
        r.pa[k] = w[k];
        r.ta[k] = w[DH + k];
    }
}

template <int S>
struct Log2 {
    static constexpr uint32_t value = S == 1 ? 0 : S == 2 ? 1 : 2;
};

// Byte offset of float element e of a slot (elements interleaved by slot),
// from e4 = 4e: one shift-or.
template <int S>
__device__ __forceinline__ uint32_t fofs4(uint32_t e4, uint32_t slot4) {
    return (e4 << Log2<S>::value) | slot4;
}
// The same from the element index.
template <int S>
__device__ __forceinline__ uint32_t fofs(uint32_t e, uint32_t slot4) {
    return (e << (2 + Log2<S>::value)) | slot4;
}

// Value of the other lane of a lane pair (lanes 2i and 2i+1), by DPP.
__device__ __forceinline__ uint32_t pair_swap(uint32_t x) {
    return (uint32_t)__builtin_amdgcn_mov_dpp((int)x, 0xB1, 0xF, 0xF, false);  // quad_perm [1,0,3,2]
}

// One lane's share of a CN visit for one slot: eq. (1) for its edges, then
// the add-back. With H = 2 the two lanes of a CN exchange their partial
// magnitude sums and sign parities, so every exclusive sum is the lane's own
// prefix + suffix plus the partner's total (all terms are >= 0: no
// cancellation). UNI: every CN has degree D, so no edge is padding.
template <class M, int D, bool UNI, int S, int H>
__device__ __forceinline__ void cn_visit(const DecodeArgs& a, const VisitRegs<D / H>& r, uint32_t h,
                                         uint32_t slot, uint32_t slot4, typename M::T* __restrict__ L) {
    constexpr int DH = D / H;
    typename M::T* row = L + ((size_t)r.cn * D + h * DH) * S + slot;
    float t[DH], lo[DH], ps[DH];
    uint32_t tb[DH];
    uint32_t sall = 0;
#pragma unroll
    for (int k = 0; k < DH; ++k) {
        lo[k] = M::unpack(row[k * S]);
        t[k] = lds_f32(fofs4<S>(r.pa[k], slot4)) - lo[k];  // VN->CN message, eq. (2)
        // posteriors never hold -0.0, so the sign bit of t is the sign rule
        tb[k] = __float_as_uint(t[k]);
        float p = psi_fwd(clampf(fabsf(t[k]), a.ymin, a.ymax));
        if (!UNI) {
            const bool real = r.pa[k] != 4u * (uint32_t)a.n;
            p = real ? p : 0.0f;
            tb[k] = real ? tb[k] : 0u;
        }
        ps[k] = p;
        sall ^= tb[k];
    }
    float pre[DH];
    pre[0] = 0.0f;
#pragma unroll
    for (int k = 1; k < DH; ++k) pre[k] = pre[k - 1] + ps[k - 1];
    float other = 0.0f;
    if (H == 2) {
        const float mine = pre[DH - 1] + ps[DH - 1];
        other = __uint_as_float(pair_swap(__float_as_uint(mine)));
        sall ^= pair_swap(sall);
    }
    float suf = other;
#pragma unroll
    for (int k = DH - 1; k >= 0; --k) {
        const float s = pre[k] + suf;  // sum over N(m) \ n
        suf += ps[k];
        const float mag = psi_inv(clampf(s, a.ymin, a.ymax));
        const uint32_t out = __float_as_uint(mag) | ((sall ^ tb[k]) & 0x80000000u);
        const typename M::T st = M::pack(__uint_as_float(out));
        row[k * S] = st;
        const float ls = M::unpack(st);
        // posterior add-back (the VN's only edge in this group), or the
        // delta new - old for the fix-up pass
        const bool direct = r.ta[k] < 4u * (uint32_t)a.ds_start;
        lds_f32(fofs4<S>(r.ta[k], slot4)) = ls + (direct ? t[k] : -lo[k]);
    }
}

// Workgroup-size cap per degree variant: wide CNs need more registers per lane.
template <int D>
struct MaxThreads {
    static constexpr int value = D >= 24 ? 256 : 1024;
};

// Takes the next frame index from the launch's work counter (-1: none left).
__device__ __forceinline__ int claim_frame(const DecodeArgs& a) {
    const unsigned t = atomicAdd(a.work, 1u);
    return t < (unsigned)a.num_frames ? (int)t : -1;
}

template <int S>
__device__ __forceinline__ void init_slot(const DecodeArgs& a, int slot, int frame, int tid, int nt) {
    const float* y = a.llr + (size_t)frame * a.n;
    for (int v = tid; v < a.n; v += nt)
        lds_f32(fofs<S>(v, 4u * slot)) = y[v] * kLog2eF + 0.0f;  // + 0 turns -0.0 into +0.0
    // posterior n: scratch of padding edges; n + 1: 0, padding of syndrome rows
    if (tid < 2) lds_f32(fofs<S>(a.n + tid, 4u * slot)) = 0.0f;
}

template <class M, int D, int S>
__device__ __forceinline__ void zero_messages(const DecodeArgs& a, typename M::T* L, int slot, int tid, int nt) {
    for (int e = tid; e < a.m * D; e += nt) L[(size_t)e * S + slot] = M::pack(0.0f);
}

template <int S>
__device__ __forceinline__ void write_outputs(const DecodeArgs& a, int slot, int frame, int used, int fail, int tid,
                                              int nt) {
    uint8_t* hd = a.hard + (size_t)frame * a.n;
    float* po = a.post ? a.post + (size_t)frame * a.n : nullptr;
    for (int v = tid; v < a.n; v += nt) {
        const float x = lds_f32(fofs<S>(v, 4u * slot));
        hd[v] = x < 0.0f ? 1 : 0;
        if (po) po[v] = x * kLn2F;
    }
    if (tid == 0) {
        a.iters[frame] = used;
        if (a.syn_ok) a.syn_ok[frame] = fail ? 0 : 1;
    }
}

template <class M, int D, bool UNI, int S, int H>
__global__ __launch_bounds__(MaxThreads<D>::value) void ndgsbp_kernel(DecodeArgs a) {
    constexpr int DH = D / H;
    constexpr int SD = (D + 3) / 4 * 4;  // syndrome row stride (entries)
    extern __shared__ __align__(16) unsigned char smem[];
    typename M::T* L = reinterpret_cast<typename M::T*>(smem + a.l_offset);
    const int tid = threadIdx.x, nt = blockDim.x;
    // CN phase: this lane is half lh of visit item tid / (H S), slot (tid / H) % S
    const int lh = tid % H, vslot = (tid / H) % S, vitem = tid / (H * S), nvitem = nt / (H * S);
    // other phases: item tid / S of slot tid % S
    const int lslot = tid % S, litem = tid / S, nitem = nt / S;
    const uint32_t vslot4 = 4u * vslot, lslot4 = 4u * lslot;
    // per-slot state in LDS: frame index, and "some check failed" flags
    // alternating by iteration parity
    const uint32_t sh = (uint32_t)a.sh_offset;
    if ((size_t)(__attribute__((address_space(3))) unsigned char*)smem != 0) {
        // dynamic LDS does not start at 0: the byte offsets would be wrong
        if (tid == 0 && a.num_frames > 0) a.iters[0] = -1;
        return;
    }

    if (tid < S) {
        lds_i32(sh + 4u * tid) = claim_frame(a);
        lds_i32(sh + 4u * (S + tid)) = 0;
        lds_i32(sh + 4u * (2 * S + tid)) = 0;
    }
    __syncthreads();
    int frame[S], used[S];
#pragma unroll
    for (int s = 0; s < S; ++s) {
        frame[s] = lds_i32(sh + 4u * s);
        used[s] = 0;
        if (frame[s] >= 0) {
            init_slot<S>(a, s, frame[s], tid, nt);
            zero_messages<M, D, S>(a, L, s, tid, nt);
        }
    }
    // the first visit of every lane is fetched one group ahead
    VisitRegs<DH> nxt;
    bool have_nxt = vitem < a.visit_ptr[1];
    if (have_nxt) load_visit<DH, H>(a, vitem, lh, nxt);
    __syncthreads();

    for (int step = 0;; ++step) {
        bool any_active = false;
#pragma unroll
        for (int s = 0; s < S; ++s) any_active |= frame[s] >= 0;
        if (!any_active) break;
        const bool vmine = frame[vslot] >= 0, mine = frame[lslot] >= 0;
        for (int g = 0; g < a.G; ++g) {
            const VisitRegs<DH> cur = nxt;
            const bool have_cur = have_nxt;
            const int gn = g + 1 == a.G ? 0 : g + 1;
            const int jn = a.visit_ptr[gn] + vitem;
            have_nxt = jn < a.visit_ptr[gn + 1];
            if (have_nxt) load_visit<DH, H>(a, jn, lh, nxt);
            if (have_cur && vmine) cn_visit<M, D, UNI, S, H>(a, cur, lh, vslot, vslot4, L);
            for (int j = a.visit_ptr[g] + vitem + nvitem; j < a.visit_ptr[g + 1]; j += nvitem) {
                VisitRegs<DH> extra;
                load_visit<DH, H>(a, j, lh, extra);
                if (vmine) cn_visit<M, D, UNI, S, H>(a, extra, lh, vslot, vslot4, L);
            }
            __syncthreads();
            const int q0 = a.fix_ptr[g], q1 = a.fix_ptr[g + 1];
            if (q1 > q0) {
                if (mine) {
                    for (int q = q0 + litem; q < q1; q += nitem) {
                        const uint2 e = a.fix[q];
                        const uint32_t v = e.x & 0xffffu, c = e.x >> 16;
                        const uint32_t d0 = (uint32_t)a.ds_start + e.y;
                        float acc = lds_f32(fofs<S>(v, lslot4));
                        for (uint32_t k = 0; k < c; ++k) acc += lds_f32(fofs<S>(d0 + k, lslot4));
                        lds_f32(fofs<S>(v, lslot4)) = acc;
                    }
                }
                __syncthreads();
            }
        }
        // a4: hard decisions (d = 1 iff total < 0) and the syndrome over all checks
        const uint32_t fl = sh + 4u * (S + (step & 1) * S);        // this step's flags
        const uint32_t fo = sh + 4u * (S + ((step + 1) & 1) * S);  // last read before this step
        if (tid < S) lds_i32(fo + 4u * tid) = 0;
        bool need = false;
#pragma unroll
        for (int s = 0; s < S; ++s) {
            if (frame[s] >= 0) {
                used[s] += 1;
                need |= a.early_stop || used[s] == a.max_iter;
            }
        }
        if (!need) continue;
        if (mine && (a.early_stop || used[lslot] == a.max_iter)) {
            // the sign bit of a posterior is its hard decision (no -0.0); a
            // lane stops once any check of its slot has been seen to fail
            for (int c = litem; c < a.m; c += nitem) {
                if (lds_i32(fl + lslot4)) break;
                const uint4* col = reinterpret_cast<const uint4*>(a.syn_col + (size_t)c * SD);
                uint32_t x = 0;
#pragma unroll
                for (int q = 0; q < SD / 4; ++q) {
                    const uint4 w = col[q];
                    x ^= __float_as_uint(lds_f32(fofs4<S>(w.x, lslot4))) ^
                         __float_as_uint(lds_f32(fofs4<S>(w.y, lslot4))) ^
                         __float_as_uint(lds_f32(fofs4<S>(w.z, lslot4))) ^
                         __float_as_uint(lds_f32(fofs4<S>(w.w, lslot4)));
                }
                if (x >> 31) lds_i32(fl + lslot4) = 1;
            }
        }
        __syncthreads();
        // finished slots: outputs, then the next frame
        bool any_done = false;
        bool done[S];
        int fail[S];
#pragma unroll
        for (int s = 0; s < S; ++s) {
            fail[s] = lds_i32(fl + 4u * s);
            done[s] = frame[s] >= 0 && ((a.early_stop && !fail[s]) || used[s] == a.max_iter);
            any_done |= done[s];
        }
        if (!any_done) continue;
#pragma unroll
        for (int s = 0; s < S; ++s) {
            if (done[s]) {
                write_outputs<S>(a, s, frame[s], used[s], fail[s], tid, nt);
                if (tid == 0) lds_i32(sh + 4u * s) = claim_frame(a);
            }
        }
        __syncthreads();
#pragma unroll
        for (int s = 0; s < S; ++s) {
            if (done[s]) {
                frame[s] = lds_i32(sh + 4u * s);
                used[s] = 0;
                if (frame[s] >= 0) {
                    init_slot<S>(a, s, frame[s], tid, nt);
                    zero_messages<M, D, S>(a, L, s, tid, nt);
                }
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

template <class M, int D, bool UNI, int S, int H>
struct LaunchF {
    static hipError_t run(const DecodeArgs* a, const LaunchShape* sh, hipStream_t s) {
        const void* fn = reinterpret_cast<const void*>(&ndgsbp_kernel<M, D, UNI, S, H>);
        hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh->lds_bytes);
        if (e != hipSuccess) return e;
        DecodeArgs copy = *a;
        void* args[] = {&copy};
        return hipLaunchKernel(fn, dim3(sh->blocks), dim3(sh->threads), args, sh->lds_bytes, s);
    }
};

template <class M, int D, bool UNI, int S, int H>
struct OccupancyF {
    static hipError_t run(int threads, size_t lds, int* out) {
        const void* fn = reinterpret_cast<const void*>(&ndgsbp_kernel<M, D, UNI, S, H>);
        hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
        return hipOccupancyMaxActiveBlocksPerMultiprocessor(out, fn, threads, lds);
    }
};

// Calls F<M, D, UNI, S, H>::run(args...) for the runtime variant. Lane
// pairs (H = 2) exist for even padded degrees, single lanes for all.
template <template <class, int, bool, int, int> class F, class M, int D, bool UNI, int S, class... A>
hipError_t by_lanes(int lanes, A... args) {
    if (lanes == 1) return F<M, D, UNI, S, 1>::run(args...);
    if constexpr (D % 2 == 0) {
        if (lanes == 2) return F<M, D, UNI, S, 2>::run(args...);
    }
    return hipErrorInvalidValue;
}

template <template <class, int, bool, int, int> class F, class M, int D, bool UNI, class... A>
hipError_t by_slots(int slots, int lanes, A... args) {
    switch (slots) {
        case 1: return by_lanes<F, M, D, UNI, 1>(lanes, args...);
        case 2: return by_lanes<F, M, D, UNI, 2>(lanes, args...);
        default: return hipErrorInvalidValue;
    }
}

template <template <class, int, bool, int, int> class F, class M, int D, class... A>
hipError_t by_uniform(bool uni, int slots, int lanes, A... args) {
    return uni ? by_slots<F, M, D, true>(slots, lanes, args...) : by_slots<F, M, D, false>(slots, lanes, args...);
}

template <template <class, int, bool, int, int> class F, class M, class... A>
hipError_t by_degree(int dmax, bool uni, int slots, int lanes, A... args) {
    switch (dmax) {
        case 4: return by_uniform<F, M, 4>(uni, slots, lanes, args...);
        case 6: return by_uniform<F, M, 6>(uni, slots, lanes, args...);
        case 7: return by_uniform<F, M, 7>(uni, slots, lanes, args...);
        case 8: return by_uniform<F, M, 8>(uni, slots, lanes, args...);
        case 12: return by_uniform<F, M, 12>(uni, slots, lanes, args...);
        case 16: return by_uniform<F, M, 16>(uni, slots, lanes, args...);
        case 24: return by_uniform<F, M, 24>(uni, slots, lanes, args...);
        case 32: return by_uniform<F, M, 32>(uni, slots, lanes, args...);
        default: return hipErrorInvalidValue;
    }
}

template <template <class, int, bool, int, int> class F, class... A>
hipError_t dispatch(MsgKind kind, int dmax, bool uni, int slots, int lanes, A... args) {
    switch (kind) {
        case kMsgF32: return by_degree<F, MsgF32>(dmax, uni, slots, lanes, args...);
        case kMsgF16: return by_degree<F, MsgF16>(dmax, uni, slots, lanes, args...);
        case kMsgBF16: return by_degree<F, MsgBF16>(dmax, uni, slots, lanes, args...);
    }
    return hipErrorInvalidValue;
}

}  // namespace

int max_threads_for_degree(int dmax) { return dmax >= 24 ? 256 : 1024; }

hipError_t launch_decode(const DecodeArgs& a, MsgKind kind, int dmax, bool uniform, const LaunchShape& shape,
                         hipStream_t stream) {
    return dispatch<LaunchF>(kind, dmax, uniform, shape.slots, shape.lanes, &a, &shape, stream);
}

hipError_t decode_occupancy(MsgKind kind, int dmax, bool uniform, int slots, int lanes, int threads,
                            size_t lds_bytes, int* blocks_per_cu) {
    return dispatch<OccupancyF>(kind, dmax, uniform, slots, lanes, threads, lds_bytes, blocks_per_cu);
}

}  // namespace ndgsbp
