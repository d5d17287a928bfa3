// C ABI of the NDGSBP decoder: validation, code tables, launch selection.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "ndgsbp.h"
#include "ndgsbp_internal.h"

using namespace ndgsbp;

namespace {

thread_local std::string g_last_error;

int fail(int code, const std::string& msg) {
    g_last_error = msg;
    return code;
}

int hip_fail(hipError_t e, const char* what) {
    return fail(LDPC_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

size_t align16(size_t x) { return (x + 15) & ~size_t(15); }

// Restores the caller's current device on scope exit.
struct DeviceGuard {
    int prev = -1;
    bool ok = false;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) return;
        if (prev != dev && hipSetDevice(dev) != hipSuccess) return;
        ok = true;
    }
    ~DeviceGuard() {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

template <class T>
hipError_t upload(T** dst, const std::vector<T>& src) {
    *dst = nullptr;
    size_t bytes = std::max<size_t>(sizeof(T), src.size() * sizeof(T));
    hipError_t e = hipMalloc((void**)dst, bytes);
    if (e != hipSuccess) return e;
    if (!src.empty()) e = hipMemcpy(*dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice);
    return e;
}

void free_tables(DeviceTables& t) {
    (void)hipFree(t.vcn);
    (void)hipFree(t.vw);
    (void)hipFree(t.visit_ptr);
    (void)hipFree(t.fix);
    (void)hipFree(t.fix_ptr);
    (void)hipFree(t.syn_col);
    (void)hipFree(t.work);
    t = DeviceTables{};
}

// Expands the grouping into explicit CN lists (validated).
int expand_groups(const ldpc_grouping* g, int m, std::vector<std::vector<int32_t>>& out) {
    if (!g) return fail(LDPC_EINVAL, "grouping is NULL");
    if (g->num_groups < 1) return fail(LDPC_EINVAL, "num_groups must be >= 1");
    out.assign(g->num_groups, {});
    if (g->kind == LDPC_GROUPS_WINDOWS) {
        if (g->overlap < 0) return fail(LDPC_EINVAL, "overlap must be >= 0");
        if (g->num_groups > m) return fail(LDPC_EINVAL, "more windows than CNs");
        const int G = g->num_groups;
        for (int k = 0; k < G; ++k) {
            const int64_t start = (int64_t)k * m / G;
            const int64_t next = (int64_t)(k + 1) * m / G;
            int64_t len;
            if (g->wrap || k < G - 1)
                len = next - start + g->overlap;
            else
                len = m - start;
            if (len > m) return fail(LDPC_EINVAL, "window longer than m (overlap too large)");
            for (int64_t i = 0; i < len; ++i) {
                int64_t c = start + i;
                if (g->wrap)
                    c %= m;
                else if (c >= m)
                    break;
                out[k].push_back((int32_t)c);
            }
        }
    } else if (g->kind == LDPC_GROUPS_EXPLICIT) {
        if (!g->group_ptr || !g->group_cn) return fail(LDPC_EINVAL, "explicit grouping needs group_ptr/group_cn");
        if (g->group_ptr[0] != 0) return fail(LDPC_EINVAL, "group_ptr[0] must be 0");
        for (int k = 0; k < g->num_groups; ++k) {
            if (g->group_ptr[k + 1] < g->group_ptr[k]) return fail(LDPC_EINVAL, "group_ptr not monotone");
            for (int32_t q = g->group_ptr[k]; q < g->group_ptr[k + 1]; ++q) {
                const int32_t c = g->group_cn[q];
                if (c < 0 || c >= m) return fail(LDPC_EINVAL, "group CN out of range");
                out[k].push_back(c);
            }
        }
    } else {
        return fail(LDPC_EINVAL, "unknown grouping kind");
    }
    // no CN twice in a group; every CN in some group
    std::vector<int32_t> stamp(m, -1);
    std::vector<char> covered(m, 0);
    for (size_t k = 0; k < out.size(); ++k) {
        if (out[k].empty()) return fail(LDPC_EINVAL, "empty group");
        for (int32_t c : out[k]) {
            if (stamp[c] == (int32_t)k) return fail(LDPC_EINVAL, "CN repeated within a group");
            stamp[c] = (int32_t)k;
            covered[c] = 1;
        }
    }
    for (int c = 0; c < m; ++c)
        if (!covered[c]) return fail(LDPC_EINVAL, "CN " + std::to_string(c) + " belongs to no group");
    return LDPC_OK;
}

// LDS of a workgroup (layout in ndgsbp_internal.h).
size_t float_bytes(const ldpc_code* c) { return align16((size_t)(c->ds_start + c->max_slots) * 4); }
size_t msg_bytes(const ldpc_code* c, MsgKind kind) {
    return align16((size_t)c->m * message_row_bytes(kind, c->D, c->H));
}
size_t lds_bytes(const ldpc_code* c, MsgKind kind) { return float_bytes(c) + msg_bytes(c, kind) + 16; }

int threads_for(const ldpc_code* c) {
    const int cap = max_threads_for_degree(c->D);
    int t = ((c->H * c->max_group_visits + 63) / 64) * 64;
    return std::max(64, std::min(t, cap));
}

// Padded degree of the kernel variant for h lanes per CN.
int pick_degree(int d, int h) {
    static const int kD1[] = {4, 6, 7, 8, 12, 16, 24, 32};
    static const int kD2[] = {4, 6, 8, 12, 16, 24, 32};
    if (h == 1) {
        for (int x : kD1)
            if (d <= x) return x;
    } else {
        for (int x : kD2)
            if (d <= x) return x;
    }
    return -1;
}

// Lanes per CN visit: the choice that wastes the fewest lane-edge slots in
// the CN phase (idle lanes of the last wave plus padding edges), two lanes
// on a tie. NDGSBP_LANES_PER_CN (1 or 2) overrides.
int pick_lanes(int maxd, int max_visits, int64_t max_edges) {
    const char* env = getenv("NDGSBP_LANES_PER_CN");
    if (env && (atoi(env) == 1 || atoi(env) == 2)) return atoi(env);
    double best_eff = -1.0;
    int best = 1;
    for (int h : {2, 1}) {
        const int D = pick_degree(maxd, h);
        const int lanes = std::min(1024, ((h * max_visits + 63) / 64) * 64);
        const double eff = (double)max_edges / ((double)lanes * (D / h));
        if (eff > best_eff + 1e-9) {
            best_eff = eff;
            best = h;
        }
    }
    return best;
}

}  // namespace

extern "C" {

const char* ldpc_last_error(void) { return g_last_error.c_str(); }

int ldpc_code_create(const ldpc_h_csr* H, const ldpc_grouping* grouping, int32_t device, ldpc_code_t* out) {
    g_last_error.clear();
    if (!out) return fail(LDPC_EINVAL, "out is NULL");
    *out = nullptr;
    if (!H || !H->row_ptr || (!H->col_idx && H->nnz > 0)) return fail(LDPC_EINVAL, "H or its arrays are NULL");
    const int m = H->m, n = H->n;
    if (m < 1 || n < 1) return fail(LDPC_EINVAL, "m and n must be >= 1");
    if (H->nnz < 0 || H->nnz > INT32_MAX) return fail(LDPC_EINVAL, "nnz out of range");
    if (n > 65533) return fail(LDPC_EUNSUPPORTED, "n > 65533 (16-bit VN ids plus two scratch posteriors)");
    if (H->row_ptr[0] != 0 || H->row_ptr[m] != H->nnz) return fail(LDPC_EINVAL, "row_ptr must run 0..nnz");
    std::vector<int32_t> vdeg(n, 0), stamp(n, -1);
    int maxd = 0;
    for (int i = 0; i < m; ++i) {
        const int32_t b = H->row_ptr[i], e = H->row_ptr[i + 1];
        if (e < b) return fail(LDPC_EINVAL, "row_ptr not monotone");
        maxd = std::max(maxd, e - b);
        for (int32_t q = b; q < e; ++q) {
            const int32_t v = H->col_idx[q];
            if (v < 0 || v >= n) return fail(LDPC_EINVAL, "col_idx out of range");
            if (stamp[v] == i) return fail(LDPC_EINVAL, "VN repeated within a row");
            stamp[v] = i;
            vdeg[v]++;
        }
    }
    if (maxd > kMaxDegree) return fail(LDPC_EUNSUPPORTED, "CN degree above 32");
    std::vector<std::vector<int32_t>> groups;
    int rc = expand_groups(grouping, m, groups);
    if (rc) return rc;

    ldpc_code* c = new (std::nothrow) ldpc_code();
    if (!c) return fail(LDPC_ENOMEM, "host allocation failed");
    c->device = device;
    c->m = m;
    c->n = n;
    c->nnz = H->nnz;
    c->G = (int32_t)groups.size();
    c->max_cn_degree = maxd;
    c->max_vn_degree = n ? *std::max_element(vdeg.begin(), vdeg.end()) : 0;

    // lanes per CN and padded degree of the tables and kernel variant
    {
        int max_visits = 0;
        int64_t max_edges = 0;
        for (const auto& grp : groups) {
            int64_t ed = 0;
            for (int32_t cn : grp) ed += H->row_ptr[cn + 1] - H->row_ptr[cn];
            max_visits = std::max<int>(max_visits, (int)grp.size());
            max_edges = std::max(max_edges, ed);
        }
        c->H = pick_lanes(std::max(1, maxd), max_visits, max_edges);
    }
    c->D = pick_degree(std::max(1, maxd), c->H);
    c->uniform = true;
    for (int i = 0; i < m; ++i)
        if (H->row_ptr[i + 1] - H->row_ptr[i] != c->D) c->uniform = false;
    const int D = c->D;
    const int LH = c->H, DH = D / LH;
    const int W = (2 * DH + 3) / 4 * 4;  // words per half-record
    const int SD = (D + 3) / 4 * 4;      // syndrome row stride
    // float index of the first delta slot: right after the posteriors
    // (n real, one scratch for padding edges, one zero for syndrome padding)
    const int32_t ds_start = n + 2;
    c->ds_start = ds_start;

    // visit, edge-word and fix-up tables
    std::vector<int32_t> vcn;
    std::vector<uint32_t> vw;
    std::vector<int32_t> visit_ptr(1, 0), fix_ptr(1, 0);
    std::vector<uint2> fix;
    std::vector<int32_t> cnt(n, 0), first_slot(n, -1), next_fill(n, 0);
    std::vector<int32_t> seen_order;
    c->cn_visits = 0;
    c->edge_updates = 0;
    c->max_group_visits = 0;
    c->max_slots = 0;
    for (const auto& grp : groups) {
        // multiplicity of each VN inside the group
        seen_order.clear();
        for (int32_t cn : grp)
            for (int32_t q = H->row_ptr[cn]; q < H->row_ptr[cn + 1]; ++q) {
                const int32_t v = H->col_idx[q];
                if (cnt[v]++ == 0) seen_order.push_back(v);
            }
        // consecutive delta slots for every VN with two or more edges here,
        // VNs in order of first appearance, edges in visit order
        int32_t slots = 0;
        for (int32_t v : seen_order)
            if (cnt[v] >= 2) {
                first_slot[v] = slots;
                fix.push_back(make_uint2((uint32_t)v | ((uint32_t)cnt[v] << 16), (uint32_t)slots));
                slots += cnt[v];
            }
        if ((int64_t)ds_start + slots > (1 << 20)) {
            delete c;
            return fail(LDPC_EUNSUPPORTED, "too many delta slots in one group");
        }
        for (int32_t cn : grp) {
            const int32_t b = H->row_ptr[cn], d = H->row_ptr[cn + 1] - b;
            vcn.push_back(cn);
            const size_t rec = vw.size();
            vw.resize(rec + (size_t)LH * W, 0u);
            for (int32_t k = 0; k < D; ++k) {
                uint32_t src = 4u * (uint32_t)n, dst = 4u * (uint32_t)n;  // padding edge
                if (k < d) {
                    const int32_t v = H->col_idx[b + k];
                    const int32_t tgt = cnt[v] >= 2 ? ds_start + first_slot[v] + next_fill[v]++ : v;
                    src = 4u * (uint32_t)v;
                    dst = 4u * (uint32_t)tgt;
                }
                const size_t half = rec + (size_t)(k / DH) * W;
                vw[half + k % DH] = src;
                vw[half + DH + k % DH] = dst;
            }
            c->edge_updates += d;
        }
        for (int32_t v : seen_order) {
            cnt[v] = 0;
            first_slot[v] = -1;
            next_fill[v] = 0;
        }
        c->cn_visits += (int64_t)grp.size();
        c->max_group_visits = std::max<int32_t>(c->max_group_visits, (int32_t)grp.size());
        c->max_slots = std::max(c->max_slots, slots);
        visit_ptr.push_back((int32_t)vcn.size());
        fix_ptr.push_back((int32_t)fix.size());
    }
    std::vector<uint32_t> syn_col((size_t)m * SD, 4u * (uint32_t)(n + 1));
    for (int i = 0; i < m; ++i)
        for (int32_t q = H->row_ptr[i]; q < H->row_ptr[i + 1]; ++q)
            syn_col[(size_t)i * SD + (q - H->row_ptr[i])] = 4u * (uint32_t)H->col_idx[q];

    DeviceGuard guard(device);
    if (!guard.ok) {
        delete c;
        return fail(LDPC_EHIP, "cannot select device " + std::to_string(device));
    }
    hipError_t e = hipSuccess;
    if (e == hipSuccess) e = upload(&c->dev.vcn, vcn);
    if (e == hipSuccess) e = upload(&c->dev.vw, vw);
    if (e == hipSuccess) e = upload(&c->dev.visit_ptr, visit_ptr);
    if (e == hipSuccess) e = upload(&c->dev.fix, fix);
    if (e == hipSuccess) e = upload(&c->dev.fix_ptr, fix_ptr);
    if (e == hipSuccess) e = upload(&c->dev.syn_col, syn_col);
    if (e == hipSuccess) e = hipMalloc((void**)&c->dev.work, sizeof(uint32_t) * 2 * kWorkRing);
    if (e == hipSuccess) e = hipMemset(c->dev.work, 0, sizeof(uint32_t) * 2 * kWorkRing);
    if (e == hipSuccess) {
        int v = 0;
        e = hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, device);
        c->max_lds = (size_t)v;
    }
    if (e == hipSuccess) e = hipDeviceGetAttribute(&c->num_cus, hipDeviceAttributeMultiprocessorCount, device);
    if (e != hipSuccess) {
        free_tables(c->dev);
        delete c;
        return e == hipErrorOutOfMemory ? fail(LDPC_ENOMEM, "device allocation failed")
                                        : hip_fail(e, "uploading code tables");
    }
    *out = c;
    return LDPC_OK;
}

int ldpc_code_destroy(ldpc_code_t code) {
    g_last_error.clear();
    if (!code) return LDPC_OK;
    {
        DeviceGuard guard(code->device);
        free_tables(code->dev);
    }
    delete code;
    return LDPC_OK;
}

int ldpc_code_query(ldpc_code_t c, ldpc_code_info* info) {
    g_last_error.clear();
    if (!c || !info) return fail(LDPC_EINVAL, "code or info is NULL");
    info->m = c->m;
    info->n = c->n;
    info->nnz = c->nnz;
    info->num_groups = c->G;
    info->cn_visits = c->cn_visits;
    info->edge_updates = c->edge_updates;
    info->max_cn_degree = c->max_cn_degree;
    info->max_vn_degree = c->max_vn_degree;
    info->device = c->device;
    info->lds_bytes_fp32 = (int64_t)lds_bytes(c, kMsgF32);
    info->lds_bytes_16 = (int64_t)lds_bytes(c, kMsgF16);
    return LDPC_OK;
}

int ldpc_decode(ldpc_code_t c, const float* llr, int32_t num_frames, int32_t max_iter, uint32_t flags,
                uint8_t* hard, float* post, int32_t* iters, uint8_t* syn_ok, void* hip_stream) {
    g_last_error.clear();
    if (!c) return fail(LDPC_EINVAL, "code is NULL");
    if (num_frames < 0) return fail(LDPC_EINVAL, "num_frames < 0");
    if (max_iter < 1) return fail(LDPC_EINVAL, "max_iter < 1");
    const uint32_t known = LDPC_FLAG_EARLY_STOP | LDPC_FLAG_MSG_FP16 | LDPC_FLAG_MSG_BF16;
    if (flags & ~known) return fail(LDPC_EINVAL, "unknown flag bits");
    if ((flags & LDPC_FLAG_MSG_FP16) && (flags & LDPC_FLAG_MSG_BF16))
        return fail(LDPC_EINVAL, "MSG_FP16 and MSG_BF16 are exclusive");
    if (num_frames == 0) return LDPC_OK;
    if (!llr || !hard || !iters) return fail(LDPC_EINVAL, "llr, hard and iters are required");
    const MsgKind kind = (flags & LDPC_FLAG_MSG_FP16) ? kMsgF16 : (flags & LDPC_FLAG_MSG_BF16) ? kMsgBF16 : kMsgF32;

    DeviceGuard guard(c->device);
    if (!guard.ok) return fail(LDPC_EHIP, "cannot select the code's device");
    if (lds_bytes(c, kind) > c->max_lds)
        return fail(LDPC_EUNSUPPORTED, "one frame needs " + std::to_string(lds_bytes(c, kind)) +
                                           " B of LDS, device allows " + std::to_string(c->max_lds));
    LaunchShape shape;
    shape.lanes = c->H;
    shape.threads = threads_for(c);
    shape.lds_bytes = lds_bytes(c, kind);
    int per_cu = 0;
    hipError_t oe = decode_occupancy(kind, c->D, c->uniform, shape.lanes, shape.threads, shape.lds_bytes, &per_cu);
    if (oe != hipSuccess) return hip_fail(oe, "occupancy query");
    if (per_cu < 1) return fail(LDPC_EUNSUPPORTED, "kernel variant cannot be resident");
    shape.blocks = (int)std::min<int64_t>((int64_t)per_cu * c->num_cus, num_frames);

    DecodeArgs a;
    a.vcn = c->dev.vcn;
    a.vw = c->dev.vw;
    a.visit_ptr = c->dev.visit_ptr;
    a.fix = c->dev.fix;
    a.fix_ptr = c->dev.fix_ptr;
    a.syn_col = c->dev.syn_col;
    a.llr = llr;
    a.hard = hard;
    a.post = post;
    a.iters = iters;
    a.syn_ok = syn_ok;
    a.work = c->dev.work + 2 * (c->next_work.fetch_add(1) % kWorkRing);
    a.n = c->n;
    a.m = c->m;
    a.G = c->G;
    a.max_iter = max_iter;
    a.early_stop = (flags & LDPC_FLAG_EARLY_STOP) ? 1 : 0;
    a.num_frames = num_frames;
    a.ds_start_b = 4u * (uint32_t)c->ds_start;
    a.pad_b = 4u * (uint32_t)c->n;
    a.l_offset = (int32_t)float_bytes(c);
    a.sh_offset = (int32_t)(float_bytes(c) + msg_bytes(c, kind));
    a.ymin = (float)(kXMin * kLog2e);
    a.ymax = (float)(kXMax * kLog2e);
    a.cmin = (float)kXMin;
    hipError_t e = launch_decode(a, kind, c->D, c->uniform, shape, (hipStream_t)hip_stream);
    if (e != hipSuccess) return hip_fail(e, "decode launch");
    return LDPC_OK;
}

}  // extern "C"
