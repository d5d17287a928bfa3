// gfx950 kernel of the NDGSBP decoder (Sec. II-C, Steps 2-4).
//
// Persistent workgroups, one frame at a time per workgroup. A frame's
// posteriors, CN->VN messages and delta slots stay resident in LDS for its
// whole decode. When the frame is finished (zero syndrome with early stop,
// or I_max reached) the workgroup writes its outputs and takes the next frame
// from a device-wide counter, so frames needing different numbers of
// iterations never leave a workgroup idle.
//
// One iteration:
//   for each group g (Step 2):
//     CN phase: H lanes per CN visit (H = 1, 2 or 4). For each edge (m, n) a
//       lane forms the VN->CN message as posterior minus old message (equal to
//       eq. (2) because the posterior is the total of eq. (3)), evaluates
//       eq. (1) in pair form (ndgsbp_math.h) with exclusive prefix/suffix
//       combinations, stores the new message and adds it back
//       into the posterior: directly when the VN has no other edge in the
//       group, else as a delta;
//     barrier;
//     fix-up (only if the group has VNs with several edges in it): one lane
//       per such VN adds its deltas in a fixed order; barrier.
//   syndrome of the hard decisions (Step 4); barrier; if finished: outputs,
//   next frame.
// Every CN update of a group reads posteriors and messages as they stood
// before the group, as eq. (1) prescribes for a group processed in parallel.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "ndgsbp_cn.h"
#include "ndgsbp_internal.h"
#include "ndgsbp_math.h"

namespace ndgsbp {
namespace {

using namespace dev;

// The kernels declare no static LDS, so the dynamic allocation starts at LDS
// address 0 and the tables' byte offsets are LDS addresses (checked per
// launch).
typedef __attribute__((address_space(3))) float lds_float;
typedef __attribute__((address_space(3))) int lds_int;
typedef __attribute__((address_space(3))) uint32_t lds_u32;
__device__ __forceinline__ lds_float& lds_f32(uint32_t byte_off) { return *(lds_float*)(size_t)byte_off; }
__device__ __forceinline__ lds_int& lds_i32(uint32_t byte_off) { return *(lds_int*)(size_t)byte_off; }
// A flag that other lanes set during the same phase, read afresh every time
// (a plain read may be kept in a register across a loop).
__device__ __forceinline__ int lds_flag(uint32_t byte_off) {
    return *(volatile __attribute__((address_space(3))) int*)(size_t)byte_off;
}

// Reads of the code tables, which no kernel writes: through the constant
// address space, so wavefront-uniform indices become scalar loads.
typedef const __attribute__((address_space(4))) int32_t const_i32;
__device__ __forceinline__ int32_t table_i32(const int32_t* base, int i) { return ((const_i32*)base)[i]; }

// Message row of one lane: DH messages of its edges, stored in DP slots
// (DP = DH for FP32; DH rounded up to even for 16-bit formats so that a row
// is a whole number of dwords and moves with vector LDS instructions).
template <class M, int DH>
struct Row {
    using T = typename M::T;
    static constexpr int DP = sizeof(T) == 2 ? (DH + 1) / 2 * 2 : DH;
    static constexpr int kWords = DP * (int)sizeof(T) / 4;
    static constexpr int kBytes = 4 * kWords;
    static __device__ __forceinline__ void load(uint32_t off, float (&x)[DH]) {
        uint32_t w[kWords];
        const lds_u32* p = (const lds_u32*)(size_t)off;
#pragma unroll
        for (int q = 0; q < kWords; ++q) w[q] = p[q];
        if constexpr (sizeof(T) == 4) {
#pragma unroll
            for (int k = 0; k < DH; ++k) x[k] = __uint_as_float(w[k]);
        } else {
#pragma unroll
            for (int k = 0; k < DH; ++k) {
                const uint16_t b = (uint16_t)(w[k / 2] >> (16 * (k % 2)));
                x[k] = M::unpack(__builtin_bit_cast(T, b));
            }
        }
    }
    // the padding slot of an odd 16-bit row is written as +0
    static __device__ __forceinline__ void store(uint32_t off, const T (&st)[DH]) {
        uint32_t w[kWords];
        if constexpr (sizeof(T) == 4) {
#pragma unroll
            for (int k = 0; k < DH; ++k) w[k] = __builtin_bit_cast(uint32_t, st[k]);
        } else {
#pragma unroll
            for (int q = 0; q < kWords; ++q) w[q] = 0;
#pragma unroll
            for (int k = 0; k < DH; ++k)
                w[k / 2] |= (uint32_t)__builtin_bit_cast(uint16_t, st[k]) << (16 * (k % 2));
        }
        lds_u32* p = (lds_u32*)(size_t)off;
#pragma unroll
        for (int q = 0; q < kWords; ++q) p[q] = w[q];
    }
};

// Edge table of one lane's share of a visit in registers: LDS byte offsets of
// the posterior each edge reads (its VN) and of the float each edge writes
// back (the posterior, or a delta slot at offset >= ds_start_b). With H lanes
// per CN, lane h owns edges h*DH .. h*DH + DH - 1 of the padded row.
template <int DH>
struct VisitRegs {
    static constexpr int kWords = (2 * DH + 3) / 4 * 4;  // half-record stride in words
    // the record's spare word (DH odd) holds the message row cn * H + h
    static constexpr bool kRowInRecord = kWords > 2 * DH;
    uint32_t rc;  // that row if kRowInRecord, else the visit's CN
    uint32_t pa[DH];
    uint32_t ta[DH];
};

// Visit records of a group start at the uniform address of visit j0; this
// lane's record is `item` visits further, half h.
template <int DH, int H>
__device__ __forceinline__ void load_visit(const Problem& p, int j0, int item, int h, VisitRegs<DH>& r) {
    constexpr int W = VisitRegs<DH>::kWords;
    const unsigned char* wbase = reinterpret_cast<const unsigned char*>(p.vw) + (size_t)j0 * (H * W * 4);
    const uint4* src = reinterpret_cast<const uint4*>(wbase + (uint32_t)(item * H + h) * (uint32_t)(W * 4));
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
    if constexpr (VisitRegs<DH>::kRowInRecord) {
        r.rc = w[2 * DH];
    } else {
        const unsigned char* cbase = reinterpret_cast<const unsigned char*>(p.vcn) + (size_t)j0 * 4;
        r.rc = (uint32_t) * reinterpret_cast<const int32_t*>(cbase + (uint32_t)item * 4u);
    }
}

// One lane's share of a CN visit: eq. (1) for its edges (cn_core), then
// the add-back into LDS. VERT (the vertical, VN-group schedule): an edge
// whose add-back target is the scratch word (ta = 4n) is an input only, its
// VN being outside the group: its message keeps its old bits.
template <class M, int D, bool UNI, int H, bool VERT, bool LATE = false>
__device__ __forceinline__ void cn_visit(const DecodeArgs& a, const Problem& p, const VisitRegs<D / H>& r,
                                         uint32_t h) {
    constexpr int DH = D / H;
    using R = Row<M, DH>;
    const uint32_t ri = VisitRegs<DH>::kRowInRecord ? r.rc : r.rc * H + h;
    const uint32_t row = (uint32_t)p.l_offset + __umul24(ri, (uint32_t)R::kBytes);
    float pv[DH], lo[DH], wv[DH];
    bool real[DH];
    typename M::T st[DH];
    // the visit's LDS loads issue ahead of other waves' arithmetic, so that
    // more of them are in flight; the arithmetic runs at the base priority,
    // which is raised (LATE) for the visits of a group's later passes: the
    // waves that run them are the ones the group barrier waits for
    __builtin_amdgcn_s_setprio(LATE ? 2 : 1);
    R::load(row, lo);
#pragma unroll
    for (int k = 0; k < DH; ++k) {
        pv[k] = lds_f32(r.pa[k]);
        real[k] = r.pa[k] != p.pad_b;
    }
    __builtin_amdgcn_s_setprio(LATE ? 1 : 0);
    cn_core<M, DH, UNI, H>(pv, lo, real, a.ymax, st, wv);
    if constexpr (VERT) {
#pragma unroll
        for (int k = 0; k < DH; ++k)
            if (r.ta[k] == p.pad_b) st[k] = M::pack(lo[k]);  // exact: lo came from these bits
    }
#pragma unroll
    for (int k = 0; k < DH; ++k) lds_f32(r.ta[k]) = wv[k];
    R::store(row, st);
}

// Fix-up of one VN with c >= 2 edges in the group (a VN with one edge has
// no entry): its posterior P plus the change w - P of each of its edges (w:
// the posterior that edge alone would leave, in its slot), added in slot
// order. The first four slots are loaded together (reads past the VN's
// slots land in the LDS allocation and are unused).
__device__ __forceinline__ void fold_deltas(const Problem& p, uint2 e) {
    const uint32_t v = e.x & 0xffffu, c = e.x >> 16;
    const uint32_t d0 = p.ds_start_b + 4u * e.y;
    const float p0 = lds_f32(4u * v);
    float d[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) d[k] = lds_f32(d0 + 4u * k);
    float acc = p0 + (d[0] - p0);
    acc += d[1] - p0;
#pragma unroll
    for (int k = 2; k < 4; ++k) acc = (uint32_t)k < c ? acc + (d[k] - p0) : acc;
    for (uint32_t k = 4; k < c; ++k) acc += lds_f32(d0 + 4u * k) - p0;
    lds_f32(4u * v) = acc;
}

// Syndrome rows (LDS byte offsets of a check's posteriors, stored padded to
// SD) that a lane keeps in registers for its first K checks tid, tid + nt,
// ...; a check past m reads the constant +0 posterior n + 1 only. Entries
// D .. SD - 1 of every row are padding (no check has more than D entries),
// so they are neither kept nor read.
// K (measured on the n=2304 workload): one check with two lanes per CN, two
// with one, none above degree 8; more registers per lane would cut the
// workgroups resident per CU.
template <int SD, int H>
struct SynChecks {
    static constexpr int value = SD > 8 ? 0 : H >= 2 ? 1 : 2;
};
template <int SD, int D, int K>
struct SynRows {
    uint32_t w[K > 0 ? K : 1][D];
    __device__ __forceinline__ void load(const Problem& p, int tid, int nt) {
#pragma unroll
        for (int j = 0; j < K; ++j) {
            const int c = tid + j * nt;
            if (c < p.m) {
                const uint4* col = reinterpret_cast<const uint4*>(p.syn_col + (size_t)c * SD);
                uint32_t e[SD];
#pragma unroll
                for (int q = 0; q < SD / 4; ++q) {
                    const uint4 x = col[q];
                    e[4 * q] = x.x;
                    e[4 * q + 1] = x.y;
                    e[4 * q + 2] = x.z;
                    e[4 * q + 3] = x.w;
                }
#pragma unroll
                for (int k = 0; k < D; ++k) w[j][k] = e[k];
            } else {
#pragma unroll
                for (int k = 0; k < D; ++k) w[j][k] = 4u * (uint32_t)(p.n + 1);
            }
        }
    }
};

// Workgroup-size cap per degree variant: wide CNs need more registers per lane.
template <int D>
struct MaxThreads {
    static constexpr int value = D >= 24 ? 256 : D >= 16 ? 512 : 1024;
};

// Takes the next frame of the launch from its work counter (thread 0) and
// stores, at the workgroup state, the frame's index within its problem (-1:
// none left) and the problem's index.
__device__ __forceinline__ void claim_frame(const DecodeArgs& a, uint32_t sh) {
    const unsigned t = atomicAdd(a.work, 1u);
    int frame = -1, prob = 0;
    if (t < (unsigned)a.total_frames) {
        frame = (int)t;
        if (a.table) {
            // last problem whose first frame is at or before t
            int lo = 0, hi = a.nprob - 1;
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (a.table[mid].first <= (int)t)
                    lo = mid;
                else
                    hi = mid - 1;
            }
            prob = lo;
            frame = (int)t - a.table[lo].first;
        }
    }
    lds_i32(sh) = frame;
    lds_i32(sh + 12) = prob;
}

// Problem `idx` of the launch; the table is read through the constant
// address space so that the fields land in scalar registers.
static_assert(sizeof(Problem) % 16 == 0, "Problem is read as 16-byte words");
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
struct ProblemWords {
    u32x4 w[sizeof(Problem) / 16];
};
template <bool TABLE>
__device__ __forceinline__ Problem get_problem(const DecodeArgs& a, int idx) {
    typedef const __attribute__((address_space(4))) u32x4 const_u4;
    if constexpr (!TABLE) return a.p0;
    const const_u4* src = (const const_u4*)(a.table + idx);
    ProblemWords pw;
#pragma unroll
    for (int i = 0; i < (int)(sizeof(Problem) / 16); ++i) pw.w[i] = src[i];
    return __builtin_bit_cast(Problem, pw);
}

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x4v __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(3))) f32x4 lds_f32x4;
typedef __attribute__((address_space(3))) u32x4v lds_u32x4;

// A frame's 16-byte words are read and written whole when n is a multiple
// of 4 and the buffer is 16-byte aligned (every frame then is).
__device__ __forceinline__ bool quad_frames(const void* buf, int n) {
    return (n & 3) == 0 && (reinterpret_cast<uintptr_t>(buf) & 15) == 0;
}

// The lane index, opaque to the compiler when OPAQUE, so that the addresses
// of the 16-byte frame-start and output loops are formed where they are
// used instead of being hoisted out of the frame loop, where they would hold
// registers through every CN phase.
template <bool OPAQUE>
__device__ __forceinline__ int fresh_lane(int tid) {
    if constexpr (OPAQUE) asm volatile("" : "+v"(tid));
    return tid;
}

template <class M, int D, int H, bool VEC>
__device__ __forceinline__ void init_frame(const Problem& p, int frame, int tid_, int nt) {
    const int tid = fresh_lane<VEC>(tid_);
    const float* y = p.llr + (size_t)frame * p.n;
    // posteriors in log2 units; + 0 turns -0.0 into +0.0
    if (VEC && quad_frames(p.llr, p.n)) {
        const f32x4* y4 = reinterpret_cast<const f32x4*>(y);
        for (int q = tid; q < (p.n >> 2); q += nt) *(lds_f32x4*)(size_t)(16u * q) = y4[q] * kLog2eF + 0.0f;
    } else {
        for (int v = tid; v < p.n; v += nt) lds_f32(4u * v) = y[v] * kLog2eF + 0.0f;
    }
    // posterior n: scratch of padding edges; n + 1: 0, padding of syndrome rows
    if (tid < 2) lds_f32(4u * (p.n + tid)) = 0.0f;
    // messages start at 0 (every format stores +0 as all-zero bits); the
    // message area starts on 16 bytes and is padded to 16
    if (VEC) {
        const int quads = (p.m * H * Row<M, D / H>::kWords + 3) >> 2;
        for (int q = tid; q < quads; q += nt)
            *(lds_u32x4*)(size_t)((uint32_t)p.l_offset + 16u * q) = u32x4v{0u, 0u, 0u, 0u};
    } else {
        const int words = p.m * H * Row<M, D / H>::kWords;
        for (int q = tid; q < words; q += nt) lds_i32((uint32_t)p.l_offset + 4u * q) = 0;
    }
}

template <bool VEC>
__device__ __forceinline__ void write_outputs(const DecodeArgs& a, const Problem& p, int frame, int used, int fail,
                                              int tid_, int nt) {
    const int tid = fresh_lane<VEC>(tid_);
    float* po = p.post ? p.post + (size_t)frame * p.n : nullptr;
    if (a.packed) {
        // byte q holds d_{8q} .. d_{8q+7}, bit k = d_{8q+k}; bits past n are 0
        const int nb = (p.n + 7) >> 3;
        uint8_t* hd = p.hard + (size_t)frame * nb;
        for (int q = tid; q < nb; q += nt) {
            uint32_t bits = 0;
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                const int v = 8 * q + k;
                if (v < p.n) bits |= (lds_f32(4u * v) < 0.0f ? 1u : 0u) << k;
            }
            hd[q] = (uint8_t)bits;
        }
        if (po)
            for (int v = tid; v < p.n; v += nt) po[v] = lds_f32(4u * v) * kLn2F;
    } else {
        uint8_t* hd = p.hard + (size_t)frame * p.n;
        if (VEC && (p.n & 3) == 0 && (reinterpret_cast<uintptr_t>(p.hard) & 3) == 0 && (!po || quad_frames(p.post, p.n))) {
            // four VNs per lane: one 16-byte LDS read, a 4-byte and a 16-byte store
            for (int q = tid; q < (p.n >> 2); q += nt) {
                const f32x4 x = *(const lds_f32x4*)(size_t)(16u * q);
                const uint32_t bits = (x.x < 0.0f ? 1u : 0u) | (x.y < 0.0f ? 1u << 8 : 0u) |
                                      (x.z < 0.0f ? 1u << 16 : 0u) | (x.w < 0.0f ? 1u << 24 : 0u);
                reinterpret_cast<uint32_t*>(hd)[q] = bits;
                if (po) reinterpret_cast<f32x4*>(po)[q] = x * kLn2F;
            }
        } else {
            for (int v = tid; v < p.n; v += nt) {
                const float x = lds_f32(4u * v);
                hd[v] = x < 0.0f ? 1 : 0;
                if (po) po[v] = x * kLn2F;
            }
        }
    }
    if (tid == 0) {
        p.iters[frame] = used;
        if (p.syn_ok) p.syn_ok[frame] = fail ? 0 : 1;
    }
}

// TABLE: the launch reads its problems from a.table (batched decoding);
// otherwise it decodes a.p0, whose fields stay kernel arguments.
// MODE 0: one problem in the kernel arguments; 1 (TABLE): the problems of a
// batch from a device table; 2 (VERT): one problem whose groups are VN
// groups (the vertical schedule).
template <class M, int D, bool UNI, int H, int MODE>
__global__ __launch_bounds__(MaxThreads<D>::value) void ndgsbp_kernel(DecodeArgs a) {
    constexpr bool TABLE = MODE == 1;
    constexpr bool VERT = MODE == 2;
    constexpr int DH = D / H;
    constexpr int SD = (D + 3) / 4 * 4;  // syndrome row stride (entries)
    constexpr int SYNK = SynChecks<SD, H>::value;
    extern __shared__ __align__(16) unsigned char smem[];
    const int tid = threadIdx.x, nt = blockDim.x;
    // CN phase: this lane is half lh of visit vitem
    const int lh = tid % H, vitem = tid / H, nvitem = nt / H;
    // state in LDS: the frame index, "some check failed" flags alternating
    // by iteration parity, and the problem index
    const uint32_t sh = (uint32_t)a.sh_offset;
    if ((size_t)(__attribute__((address_space(3))) unsigned char*)smem != 0) {
        // dynamic LDS does not start at 0: the byte offsets would be wrong
        if (tid == 0 && a.total_frames > 0) get_problem<TABLE>(a, 0).iters[0] = -1;
        return;
    }

    if (tid == 0) {
        claim_frame(a, sh);
        lds_i32(sh + 4) = 0;
        lds_i32(sh + 8) = 0;
    }
    __syncthreads();
    int frame = __builtin_amdgcn_readfirstlane(lds_i32(sh));
    int pid = TABLE ? __builtin_amdgcn_readfirstlane(lds_i32(sh + 12)) : 0;
    Problem p = get_problem<TABLE>(a, pid);
    int used = 0;
    if (frame >= 0) init_frame<M, D, H, !TABLE>(p, frame, tid, nt);
    // the first visit of every lane is fetched one group ahead, and so are
    // the group's visit and fix-up ranges (carried in scalar registers, so
    // that a group waits on one round of table loads, not three)
    VisitRegs<DH> nxt;
    int jn0 = table_i32(p.visit_ptr, 0), jn1 = table_i32(p.visit_ptr, 1);
    int qn0 = table_i32(p.fix_ptr, 0), qn1 = table_i32(p.fix_ptr, 1);
    bool have_nxt = vitem < jn1 - jn0;
    if (have_nxt) load_visit<DH, H>(p, jn0, vitem, lh, nxt);
    // rows of this lane's first SYNK checks, kept for the whole decode
    SynRows<SD, D, SYNK> srow;
    srow.load(p, tid, nt);
    __syncthreads();

    // first group of this iteration's block (a new grouping every iteration
    // when the code has R > 1 blocks of G groups)
    int gb = 0;
    for (int step = 0; frame >= 0; ++step) {
        const int gb_next = gb + p.G < p.G * p.R ? gb + p.G : 0;
        for (int gi = 0; gi < p.G; ++gi) {
            const int g = gb + gi;
            const VisitRegs<DH> cur = nxt;
            const bool have_cur = have_nxt;
            const int j0 = jn0, j1 = jn1, q0 = qn0, q1 = qn1;
            const int gn = gi + 1 == p.G ? gb_next : g + 1;
            jn0 = table_i32(p.visit_ptr, gn);
            jn1 = table_i32(p.visit_ptr, gn + 1);
            qn0 = table_i32(p.fix_ptr, gn);
            qn1 = table_i32(p.fix_ptr, gn + 1);
            have_nxt = vitem < jn1 - jn0;
            if (have_nxt) load_visit<DH, H>(p, jn0, vitem, lh, nxt);
            // this lane's first fix-up entry of the group, fetched before the CN phase
            const uint2 fix0 = q0 + tid < q1 ? p.fix[q0 + tid] : make_uint2(0u, 0u);
            if (have_cur) cn_visit<M, D, UNI, H, VERT>(a, p, cur, lh);
            for (int item = vitem + nvitem; item < j1 - j0; item += nvitem) {
                VisitRegs<DH> extra;
                load_visit<DH, H>(p, j0, item, lh, extra);
                cn_visit<M, D, UNI, H, VERT, true>(a, p, extra, lh);
            }
            __builtin_amdgcn_s_setprio(0);
            __syncthreads();
            if (q1 > q0) {
                // the waves that fold are the group's critical path (everyone
                // else waits at the barrier): they issue ahead of the other
                // workgroups' CN phases on the same SIMD
                if (q0 + tid < q1) {
                    __builtin_amdgcn_s_setprio(2);
                    fold_deltas(p, fix0);
                }
                for (int q = q0 + tid + nt; q < q1; q += nt) fold_deltas(p, p.fix[q]);
                __syncthreads();
                __builtin_amdgcn_s_setprio(0);
            }
        }
        gb = gb_next;
        // a4: hard decisions (d = 1 iff total < 0) and the syndrome over all checks
        used += 1;
        const uint32_t fl = sh + 4u + 4u * (step & 1);        // this step's flag
        const uint32_t fo = sh + 4u + 4u * ((step + 1) & 1);  // last read before this step
        // cleared every step, so the next step starts from 0 whether or not
        // this one checks (the group barriers order it after the last read)
        if (tid == 0) lds_i32(fo) = 0;
        const bool check = a.early_stop || used == p.max_iter;
        if (!check) continue;
        // the syndrome and a frame change are short phases between barriers:
        // ahead of other workgroups' CN phases too, behind the fold
        __builtin_amdgcn_s_setprio(1);
        // the sign bit of a posterior is its hard decision (no -0.0); a lane
        // stops once any check has been seen to fail
        {
            // the lane's first checks, from rows held in registers
            uint32_t x = 0;
#pragma unroll
            for (int j = 0; j < SYNK; ++j) {
                uint32_t par = 0;
#pragma unroll
                for (int k = 0; k < D; ++k) par ^= __float_as_uint(lds_f32(srow.w[j][k]));
                x |= par;
            }
            if (x >> 31) lds_i32(fl) = 1;
        }
        for (int c = tid + SYNK * nt; c < p.m; c += nt) {
            const uint4* col = reinterpret_cast<const uint4*>(p.syn_col + (size_t)c * SD);
            uint32_t e[SD];
#pragma unroll
            for (int q = 0; q < SD / 4; ++q) {
                const uint4 w = col[q];
                e[4 * q] = w.x;
                e[4 * q + 1] = w.y;
                e[4 * q + 2] = w.z;
                e[4 * q + 3] = w.w;
            }
            // stop once any check of the frame has failed (the row load above
            // is then unused)
            if (lds_flag(fl)) break;
            uint32_t x = 0;
#pragma unroll
            for (int k = 0; k < D; ++k) x ^= __float_as_uint(lds_f32(e[k]));
            if (x >> 31) lds_i32(fl) = 1;
        }
        __syncthreads();
        const int fail = lds_i32(fl);
        if (!((a.early_stop && !fail) || used == p.max_iter)) {
            __builtin_amdgcn_s_setprio(0);
            continue;
        }
        // finished: outputs, then the next frame (of this or another problem)
        write_outputs<!TABLE>(a, p, frame, used, fail, tid, nt);
        if (tid == 0) claim_frame(a, sh);
        __syncthreads();
        frame = __builtin_amdgcn_readfirstlane(lds_i32(sh));
        used = 0;
        if (frame >= 0) {
            // a new frame starts at block 0: the prefetched first group is
            // right unless the block changed or the problem did
            bool reload = gb != 0;
            if constexpr (TABLE) {
                const int np = __builtin_amdgcn_readfirstlane(lds_i32(sh + 12));
                if (np != pid) {
                    pid = np;
                    p = get_problem<TABLE>(a, pid);
                    srow.load(p, tid, nt);
                    reload = true;
                }
            }
            if (reload) {
                jn0 = table_i32(p.visit_ptr, 0);
                jn1 = table_i32(p.visit_ptr, 1);
                qn0 = table_i32(p.fix_ptr, 0);
                qn1 = table_i32(p.fix_ptr, 1);
                have_nxt = vitem < jn1 - jn0;
                if (have_nxt) load_visit<DH, H>(p, jn0, vitem, lh, nxt);
            }
            gb = 0;
            init_frame<M, D, H, !TABLE>(p, frame, tid, nt);
        }
        __syncthreads();
        __builtin_amdgcn_s_setprio(0);
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

// The vertical schedule is built for 32- and 16-bit messages with one or
// two lanes per CN visit.
template <class M, int H>
constexpr bool kVertical = H <= 2 && !std::is_same<M, MsgBF16>::value;

template <class M, int D, bool UNI, int H>
const void* kernel_for(int mode) {
    if (mode == 1) return reinterpret_cast<const void*>(&ndgsbp_kernel<M, D, UNI, H, 1>);
    if (mode == 2) {
        if constexpr (kVertical<M, H>) return reinterpret_cast<const void*>(&ndgsbp_kernel<M, D, UNI, H, 2>);
        return nullptr;
    }
    return reinterpret_cast<const void*>(&ndgsbp_kernel<M, D, UNI, H, 0>);
}

template <class M, int D, bool UNI, int H>
struct LaunchF {
    static hipError_t run(const DecodeArgs* a, const LaunchShape* sh, hipStream_t s) {
        const void* fn = kernel_for<M, D, UNI, H>(a->table ? 1 : sh->vertical ? 2 : 0);
        if (!fn) return hipErrorInvalidValue;
        hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh->lds_bytes);
        if (e != hipSuccess) return e;
        DecodeArgs copy = *a;
        void* args[] = {&copy};
        return hipLaunchKernel(fn, dim3(sh->blocks), dim3(sh->threads), args, sh->lds_bytes, s);
    }
};

template <class M, int D, bool UNI, int H>
struct OccupancyF {
    static hipError_t run(int mode, int threads, size_t lds, int* out) {
        const void* fn = kernel_for<M, D, UNI, H>(mode);
        if (!fn) return hipErrorInvalidValue;
        hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
        return hipOccupancyMaxActiveBlocksPerMultiprocessor(out, fn, threads, lds);
    }
};

// Calls F<M, D, UNI, H>::run(args...) for the runtime variant. Lane pairs
// (H = 2) exist for even padded degrees, single lanes for all.
template <template <class, int, bool, int> class F, class M, int D, bool UNI, class... A>
hipError_t by_lanes(int lanes, A... args) {
    if (lanes == 1) return F<M, D, UNI, 1>::run(args...);
    if constexpr (D % 2 == 0) {
        if (lanes == 2) return F<M, D, UNI, 2>::run(args...);
    }
    if constexpr (D % 4 == 0) {
        if (lanes == 4) return F<M, D, UNI, 4>::run(args...);
    }
    return hipErrorInvalidValue;
}

template <template <class, int, bool, int> class F, class M, int D, class... A>
hipError_t by_uniform(bool uni, int lanes, A... args) {
    return uni ? by_lanes<F, M, D, true>(lanes, args...) : by_lanes<F, M, D, false>(lanes, args...);
}

template <template <class, int, bool, int> class F, class M, class... A>
hipError_t by_degree(int dmax, bool uni, int lanes, A... args) {
    switch (dmax) {
        case 4: return by_uniform<F, M, 4>(uni, lanes, args...);
        case 6: return by_uniform<F, M, 6>(uni, lanes, args...);
        case 7: return by_uniform<F, M, 7>(uni, lanes, args...);
        case 8: return by_uniform<F, M, 8>(uni, lanes, args...);
        case 10: return by_uniform<F, M, 10>(uni, lanes, args...);
        case 12: return by_uniform<F, M, 12>(uni, lanes, args...);
        case 16: return by_uniform<F, M, 16>(uni, lanes, args...);
        case 24: return by_uniform<F, M, 24>(uni, lanes, args...);
        case 32: return by_uniform<F, M, 32>(uni, lanes, args...);
        default: return hipErrorInvalidValue;
    }
}

template <template <class, int, bool, int> class F, class... A>
hipError_t dispatch(MsgKind kind, int dmax, bool uni, int lanes, A... args) {
    switch (kind) {
        case kMsgF32: return by_degree<F, MsgF32>(dmax, uni, lanes, args...);
        case kMsgF16: return by_degree<F, MsgF16>(dmax, uni, lanes, args...);
        case kMsgBF16: return by_degree<F, MsgBF16>(dmax, uni, lanes, args...);
    }
    return hipErrorInvalidValue;
}

}  // namespace

int max_threads_for_degree(int dmax) { return dmax >= 24 ? 256 : dmax >= 16 ? 512 : 1024; }

int message_row_bytes(MsgKind kind, int dmax, int lanes) {
    const int dh = dmax / lanes;
    const int dp = kind == kMsgF32 ? dh : (dh + 1) / 2 * 2;
    return lanes * dp * (kind == kMsgF32 ? 4 : 2);
}

hipError_t launch_decode(const DecodeArgs& a, MsgKind kind, int dmax, bool uniform, const LaunchShape& shape,
                         hipStream_t stream) {
    return dispatch<LaunchF>(kind, dmax, uniform, shape.lanes, &a, &shape, stream);
}

hipError_t decode_occupancy(MsgKind kind, int dmax, bool uniform, int lanes, int mode, int threads,
                            size_t lds_bytes, int* blocks_per_cu) {
    return dispatch<OccupancyF>(kind, dmax, uniform, lanes, mode, threads, lds_bytes, blocks_per_cu);
}

}  // namespace ndgsbp
