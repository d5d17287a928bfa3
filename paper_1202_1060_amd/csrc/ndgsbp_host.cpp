// C ABI of the NDGSBP decoder: validation, code tables, launch selection.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
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

// LDS of one frame: posteriors (n + 2 floats, two flags), delta slots,
// messages (m * D).
size_t p_bytes(const ldpc_code* c) { return align16((size_t)(c->n + 4) * 4); }
size_t ds_bytes(const ldpc_code* c) { return align16((size_t)c->max_slots * 4); }
size_t lds_bytes(const ldpc_code* c, MsgKind kind) {
    const size_t msg = kind == kMsgF32 ? 4 : 2;
    return p_bytes(c) + ds_bytes(c) + align16((size_t)c->m * c->D * msg);
}

int pick_dmax(int d) {
    static const int kDs[] = {4, 6, 7, 8, 12, 16, 24, 32};
    for (int x : kDs)
        if (d <= x) return x;
    return -1;
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

    // padded degree of the tables and kernel variant
    c->D = pick_dmax(std::max(1, maxd));
    c->uniform = true;
    for (int i = 0; i < m; ++i)
        if (H->row_ptr[i + 1] - H->row_ptr[i] != c->D) c->uniform = false;
    const int D = c->D;
    const int W = (2 * D + 3) / 4 * 4;  // words per visit record
    // float index of the first delta slot: right after the posteriors
    const int32_t ds_start = (int32_t)(align16((size_t)(n + 4) * 4) / 4);

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
        if ((int64_t)ds_start + slots > 65535 || (int64_t)ds_start + slots > (1 << 20)) {
            delete c;
            return fail(LDPC_EUNSUPPORTED, "posteriors plus delta slots exceed 16-bit LDS indices");
        }
        for (int32_t cn : grp) {
            const int32_t b = H->row_ptr[cn], d = H->row_ptr[cn + 1] - b;
            vcn.push_back(cn);
            const size_t rec = vw.size();
            vw.resize(rec + W, 0u);
            for (int32_t k = 0; k < D; ++k) {
                uint32_t src = (uint32_t)n * 4u, dst = (uint32_t)n * 4u;  // padding edge
                if (k < d) {
                    const int32_t v = H->col_idx[b + k];
                    const int32_t tgt = cnt[v] >= 2 ? ds_start + first_slot[v] + next_fill[v]++ : v;
                    src = (uint32_t)v * 4u;
                    dst = (uint32_t)tgt * 4u;
                }
                vw[rec + k] = src;
                vw[rec + D + k] = dst;
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
    std::vector<uint16_t> syn_col((size_t)m * D, (uint16_t)(n + 1));
    for (int i = 0; i < m; ++i)
        for (int32_t q = H->row_ptr[i]; q < H->row_ptr[i + 1]; ++q)
            syn_col[(size_t)i * D + (q - H->row_ptr[i])] = (uint16_t)H->col_idx[q];

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
    if (e == hipSuccess) {
        int v = 0;
        e = hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, device);
        c->max_lds = (size_t)v;
    }
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
    const size_t lds = lds_bytes(c, kind);
    if (lds > c->max_lds)
        return fail(LDPC_EUNSUPPORTED, "one frame needs " + std::to_string(lds) + " B of LDS, device allows " +
                                           std::to_string(c->max_lds));
    int threads = ((c->max_group_visits + 63) / 64) * 64;
    threads = std::min(1024, std::max(64, threads));

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
    a.n = c->n;
    a.m = c->m;
    a.G = c->G;
    a.max_iter = max_iter;
    a.early_stop = (flags & LDPC_FLAG_EARLY_STOP) ? 1 : 0;
    a.num_frames = num_frames;
    a.ds_start = (int32_t)(p_bytes(c) / 4);
    a.ds_start_b = (uint32_t)p_bytes(c);
    a.dummy_b = (uint32_t)c->n * 4u;
    a.l_offset = (int32_t)(p_bytes(c) + ds_bytes(c));
    a.ymin = (float)(kXMin * kLog2e);
    a.ymax = (float)(kXMax * kLog2e);
    hipError_t e = launch_decode(a, kind, c->D, c->uniform, threads, lds, (hipStream_t)hip_stream);
    if (e != hipSuccess) return hip_fail(e, "decode launch");
    return LDPC_OK;
}

}  // extern "C"
