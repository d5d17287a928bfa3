// gfx950 kernels of the NDGSBP decoder: one workgroup decodes one frame with
// the frame's posteriors and CN->VN messages resident in LDS for the whole
// decode (Sec. II-C, Steps 2-4).
//
// Per group (one sub-iteration of Step 2) the workgroup runs
//   CN phase: one lane per CN visit. For each edge (m, n) of the CN the lane
//     forms the VN->CN message as posterior minus old message (which equals
//     eq. (2) because the posterior is the total of eq. (3)), evaluates eq. (1)
//     in sign-magnitude form with exclusive prefix/suffix sums, stores the new
//     message and adds it back into the posterior: directly when the VN has no
//     other edge in this group, else as a delta into an LDS slot;
//   barrier;
//   fix-up phase (only if the group has such VNs): one lane per VN with two
//     or more edges in the group adds its deltas in a fixed order;
//   barrier.
// All CN updates of a group read the posteriors and messages as they stood
// before the group, as eq. (1) prescribes for a group processed in parallel.
// After each iteration the lanes check the syndrome of the hard decisions
// (Step 4) and the workgroup stops early when it is zero (if asked).
#include <hip/hip_runtime.h>

#include "ndgsbp_internal.h"

namespace ndgsbp {
namespace {

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

// Forward use (|VN->CN message| -> summand). Small results must keep their
// relative accuracy (they are summed, and a small sum is mapped back to a
// large message), so for v = 2^-y < 1/16 the ratio's logarithm is replaced by
// the odd series 2 atanh(v) / ln 2 = (2/ln2)(v + v^3/3 + v^5/5 + v^7/7 + ...),
// truncated after v^7 (relative error < 3e-11 there). Large results only need
// absolute accuracy: a large summand drives the other outputs to ~0.
__device__ __forceinline__ float psi_fwd(float y) {
    const float v = exp2_hw(-y);
    const float w = v * v;
    const float c1 = 2.0f * kLog2eF, c3 = c1 / 3.0f, c5 = c1 / 5.0f, c7 = c1 / 7.0f;
    const float ser = v * fmaf(w, fmaf(w, fmaf(w, c7, c5), c3), c1);
    const float gen = log2_hw((1.0f + v) * rcp_hw(1.0f - v));
    return v < 0.0625f ? ser : gen;
}

// Inverse use (sum -> |CN->VN message|). A small sum gives a large message,
// whose relative accuracy needs 1 - 2^-y without cancellation: for
// z = y ln 2 < 1/4 it is taken from the Taylor series of 1 - e^-z up to z^6
// (relative truncation error < 5e-8), written as a polynomial in y; above,
// 1 - v loses at most ~2.7e-7. A large sum gives a small message, where
// absolute accuracy suffices. The result is >= +0 (log2 of a ratio >= 1).
__device__ __forceinline__ float psi_inv(float y) {
    constexpr double l = 0.6931471805599453;
    constexpr float c1 = (float)l, c2 = (float)(-l * l / 2), c3 = (float)(l * l * l / 6),
                    c4 = (float)(-l * l * l * l / 24), c5 = (float)(l * l * l * l * l / 120),
                    c6 = (float)(-l * l * l * l * l * l / 720);
    const float v = exp2_hw(-y);
    float p = fmaf(y, c6, c5);
    p = fmaf(y, p, c4);
    p = fmaf(y, p, c3);
    p = fmaf(y, p, c2);
    p = fmaf(y, p, c1);
    const float den = y < (float)(0.25 / l) ? y * p : 1.0f - v;
    return log2_hw((1.0f + v) * rcp_hw(den));
}

__device__ __forceinline__ float clampf(float x, float lo, float hi) { return __builtin_amdgcn_fmed3f(x, lo, hi); }

// --- one CN visit: eq. (1) for every edge of the CN, then the add-back ---------

// Edge table of one visit, held in registers: LDS byte offsets of the
// posterior each edge reads and of the float each edge writes back.
template <int D>
struct VisitRegs {
    static constexpr int kWords = (2 * D + 3) / 4 * 4;  // record stride in words
    int cn;
    uint32_t pa[D];
    uint32_t ta[D];
};

template <int D>
__device__ __forceinline__ void load_visit(const DecodeArgs& a, int j, VisitRegs<D>& r) {
    constexpr int W = VisitRegs<D>::kWords;
    r.cn = a.vcn[j];
    const uint4* src = reinterpret_cast<const uint4*>(a.vw) + (size_t)j * (W / 4);
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
    for (int k = 0; k < D; ++k) {
        r.pa[k] = w[k];
        r.ta[k] = w[D + k];
    }
}

// A float of this workgroup's LDS at a byte offset. The kernels declare no
// static LDS, so the dynamic allocation starts at LDS address 0 and the
// table's byte offsets are LDS addresses (checked once per launch below).
typedef __attribute__((address_space(3))) float lds_float;
__device__ __forceinline__ lds_float& lds_f32(unsigned char*, uint32_t byte_off) {
    return *(lds_float*)(size_t)byte_off;
}

// UNI: every CN has degree D, so no edge is padding.
template <class M, int D, bool UNI>
__device__ __forceinline__ void cn_visit(const DecodeArgs& a, const VisitRegs<D>& r, unsigned char* __restrict__ smem,
                                         typename M::T* __restrict__ L) {
    typename M::T* row = L + (size_t)r.cn * D;
    float t[D], lo[D], ps[D];
    uint32_t tb[D];
    uint32_t sall = 0;
#pragma unroll
    for (int k = 0; k < D; ++k) {
        lo[k] = M::unpack(row[k]);
        t[k] = lds_f32(smem, r.pa[k]) - lo[k];  // VN->CN message, eq. (2)
        // posteriors never hold -0.0, so the sign bit of t is the sign rule
        tb[k] = __float_as_uint(t[k]);
        float p = psi_fwd(clampf(fabsf(t[k]), a.ymin, a.ymax));
        if (!UNI) {
            const bool real = r.pa[k] != a.dummy_b;
            p = real ? p : 0.0f;
            tb[k] = real ? tb[k] : 0u;
        }
        ps[k] = p;
        sall ^= tb[k];
    }
    float pre[D];
    pre[0] = 0.0f;
#pragma unroll
    for (int k = 1; k < D; ++k) pre[k] = pre[k - 1] + ps[k - 1];
    float suf = 0.0f;
#pragma unroll
    for (int k = D - 1; k >= 0; --k) {
        const float s = pre[k] + suf;  // sum over N(m) \ n
        suf += ps[k];
        const float mag = psi_inv(clampf(s, a.ymin, a.ymax));
        const uint32_t out = __float_as_uint(mag) | ((sall ^ tb[k]) & 0x80000000u);
        const typename M::T st = M::pack(__uint_as_float(out));
        row[k] = st;
        const float ls = M::unpack(st);
        // posterior add-back (the VN's only edge in this group), or the
        // delta new - old for the fix-up pass
        const bool direct = r.ta[k] < a.ds_start_b;
        lds_f32(smem, r.ta[k]) = ls + (direct ? t[k] : -lo[k]);
    }
}

// Workgroup-size cap per degree variant: wide CNs need more registers per lane.
template <int D>
struct MaxThreads {
    static constexpr int value = D >= 24 ? 256 : 1024;
};

template <class M, int D, bool UNI>
__global__ __launch_bounds__(MaxThreads<D>::value) void ndgsbp_lds_kernel(DecodeArgs a) {
    extern __shared__ __align__(16) unsigned char smem[];
    float* S = reinterpret_cast<float*>(smem);  // posteriors, then delta slots (floats)
    typename M::T* L = reinterpret_cast<typename M::T*>(smem + a.l_offset);
    const int f = blockIdx.x;
    const int tid = threadIdx.x, nt = blockDim.x;
    if ((size_t)(__attribute__((address_space(3))) unsigned char*)smem != 0) {
        // dynamic LDS does not start at 0: the byte offsets would be wrong
        if (tid == 0) a.iters[f] = -1;
        return;
    }

    // a0: posteriors start at the channel LLRs (log2 units), messages at 0
    const float* y = a.llr + (size_t)f * a.n;
    for (int v = tid; v < a.n; v += nt) S[v] = y[v] * kLog2eF + 0.0f;  // + 0 turns -0.0 into +0.0
    // S[n]: scratch posterior of padding edges; S[n+1] = 0: padding of the
    // syndrome rows; S[n+2], S[n+3]: "some check failed" flags, alternating
    // by iteration parity
    int* flag = reinterpret_cast<int*>(S + a.n + 2);
    if (tid < 2) {
        S[a.n + tid] = 0.0f;
        flag[tid] = 0;
    }
    for (int e = tid; e < a.m * D; e += nt) L[e] = M::pack(0.0f);

    // the first visit of every lane is fetched one group ahead
    VisitRegs<D> nxt;
    bool have_nxt = tid < a.visit_ptr[1];
    if (have_nxt) load_visit<D>(a, tid, nxt);
    __syncthreads();

    int used = a.max_iter, bad = 1;
    for (int it = 1; it <= a.max_iter; ++it) {
        for (int g = 0; g < a.G; ++g) {
            const VisitRegs<D> cur = nxt;
            const bool have_cur = have_nxt;
            const int gn = g + 1 == a.G ? 0 : g + 1;
            const int jn = a.visit_ptr[gn] + tid;
            have_nxt = jn < a.visit_ptr[gn + 1];
            if (have_nxt) load_visit<D>(a, jn, nxt);
            if (have_cur) cn_visit<M, D, UNI>(a, cur, smem, L);
            for (int j = a.visit_ptr[g] + tid + nt; j < a.visit_ptr[g + 1]; j += nt) {
                VisitRegs<D> extra;
                load_visit<D>(a, j, extra);
                cn_visit<M, D, UNI>(a, extra, smem, L);
            }
            __syncthreads();
            const int q0 = a.fix_ptr[g], q1 = a.fix_ptr[g + 1];
            if (q1 > q0) {
                for (int q = q0 + tid; q < q1; q += nt) {
                    const uint2 e = a.fix[q];
                    const int v = (int)(e.x & 0xffffu), c = (int)(e.x >> 16);
                    const float* dsl = S + a.ds_start + e.y;
                    float acc = S[v];
                    for (int k = 0; k < c; ++k) acc += dsl[k];
                    S[v] = acc;
                }
                __syncthreads();
            }
        }
        // a4: hard decisions (d = 1 iff total < 0) and the syndrome over all checks
        if (a.early_stop || it == a.max_iter) {
            // the other flag was last read before this iteration's first barrier
            if (tid == 0) flag[(it + 1) & 1] = 0;
            int any = 0;
            for (int c = tid; c < a.m; c += nt) {
                const uint16_t* col = a.syn_col + (size_t)c * D;
                int par = 0;
#pragma unroll
                for (int k = 0; k < D; ++k) par ^= (S[col[k]] < 0.0f) ? 1 : 0;
                any |= par;
            }
            if (any) flag[it & 1] = 1;
            __syncthreads();
            bad = flag[it & 1];
            if (a.early_stop && !bad) {
                used = it;
                break;
            }
        }
    }

    // a5: outputs
    uint8_t* hd = a.hard + (size_t)f * a.n;
    float* po = a.post ? a.post + (size_t)f * a.n : nullptr;
    for (int v = tid; v < a.n; v += nt) {
        const float x = S[v];
        hd[v] = x < 0.0f ? 1 : 0;
        if (po) po[v] = x * kLn2F;
    }
    if (tid == 0) {
        a.iters[f] = used;
        if (a.syn_ok) a.syn_ok[f] = bad ? 0 : 1;
    }
}

template <class M, int D, bool UNI>
hipError_t launch_t(const DecodeArgs& a, int threads, size_t lds, hipStream_t s) {
    if (threads > MaxThreads<D>::value) threads = MaxThreads<D>::value;
    const void* fn = reinterpret_cast<const void*>(&ndgsbp_lds_kernel<M, D, UNI>);
    hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    DecodeArgs copy = a;
    void* args[] = {&copy};
    return hipLaunchKernel(fn, dim3(a.num_frames), dim3(threads), args, lds, s);
}

template <class M, int D>
hipError_t launch_u(const DecodeArgs& a, bool uniform, int threads, size_t lds, hipStream_t s) {
    return uniform ? launch_t<M, D, true>(a, threads, lds, s) : launch_t<M, D, false>(a, threads, lds, s);
}

template <class M>
hipError_t launch_m(const DecodeArgs& a, int dmax, bool uniform, int threads, size_t lds, hipStream_t s) {
    switch (dmax) {
        case 4: return launch_u<M, 4>(a, uniform, threads, lds, s);
        case 6: return launch_u<M, 6>(a, uniform, threads, lds, s);
        case 7: return launch_u<M, 7>(a, uniform, threads, lds, s);
        case 8: return launch_u<M, 8>(a, uniform, threads, lds, s);
        case 12: return launch_u<M, 12>(a, uniform, threads, lds, s);
        case 16: return launch_u<M, 16>(a, uniform, threads, lds, s);
        case 24: return launch_u<M, 24>(a, uniform, threads, lds, s);
        case 32: return launch_u<M, 32>(a, uniform, threads, lds, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace

hipError_t launch_decode(const DecodeArgs& a, MsgKind kind, int dmax, bool uniform, int threads,
                         size_t lds_bytes, hipStream_t stream) {
    switch (kind) {
        case kMsgF32: return launch_m<MsgF32>(a, dmax, uniform, threads, lds_bytes, stream);
        case kMsgF16: return launch_m<MsgF16>(a, dmax, uniform, threads, lds_bytes, stream);
        case kMsgBF16: return launch_m<MsgBF16>(a, dmax, uniform, threads, lds_bytes, stream);
    }
    return hipErrorInvalidValue;
}

}  // namespace ndgsbp
