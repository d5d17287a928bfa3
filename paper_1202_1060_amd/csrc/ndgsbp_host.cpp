// C ABI of the NDGSBP decoder: validation, code tables, launch selection.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "ndgsbp.h"
#include "ndgsbp_code.h"
#include "ndgsbp_hbm.h"
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

void free_tables(ldpc_code* c) {
    DeviceTables& t = c->dev;
    (void)hipFree(t.vcn);
    (void)hipFree(t.vfirst);
    (void)hipFree(t.vdfirst);
    (void)hipFree(c->hbm_ws);
    c->hbm_ws = nullptr;
    c->hbm_ws_bytes = 0;
    if (c->hbm_last) (void)hipEventDestroy(c->hbm_last);
    c->hbm_last = nullptr;
    (void)hipFree(t.visit_ptr);
    (void)hipFree(t.fix);
    (void)hipFree(t.fix_ptr);
    (void)hipFree(t.work);
    t = DeviceTables{};
    for (Layout& l : c->lay) {
        (void)hipFree(l.vw);
        (void)hipFree(l.syn_col);
        l = Layout{};
    }
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
    // iteration blocks: all groups, or groups_per_iteration at a time
    const int gpi = g->groups_per_iteration;
    if (gpi < 0) return fail(LDPC_EINVAL, "groups_per_iteration < 0");
    if (gpi > 0 && g->kind != LDPC_GROUPS_EXPLICIT)
        return fail(LDPC_EINVAL, "groups_per_iteration needs explicit groups");
    const int per = gpi > 0 ? gpi : (int)out.size();
    if ((int)out.size() % per) return fail(LDPC_EINVAL, "num_groups is not a multiple of groups_per_iteration");
    // no CN twice in a group; every CN in some group of every iteration block
    std::vector<int32_t> stamp(m, -1);
    std::vector<int32_t> covered(m, -1);
    for (size_t k = 0; k < out.size(); ++k) {
        if (out[k].empty()) return fail(LDPC_EINVAL, "empty group");
        const int32_t blk = (int32_t)(k / per);
        for (int32_t c : out[k]) {
            if (stamp[c] == (int32_t)k) return fail(LDPC_EINVAL, "CN repeated within a group");
            stamp[c] = (int32_t)k;
            covered[c] = blk;
        }
        if ((k + 1) % per == 0)
            for (int c = 0; c < m; ++c)
                if (covered[c] != blk)
                    return fail(LDPC_EINVAL, "CN " + std::to_string(c) + " belongs to no group" +
                                                 (gpi > 0 ? " of iteration block " + std::to_string(blk) : ""));
    }
    return LDPC_OK;
}

// VN groups (the vertical schedule): `vgroup` = the group of every VN; the
// visits of group g are the CNs adjacent to its VNs, in increasing order.
int expand_vn_groups(const ldpc_h_csr* H, const ldpc_grouping* g, std::vector<int32_t>& vgroup,
                     std::vector<std::vector<int32_t>>& out) {
    const int m = H->m, n = H->n;
    if (g->num_groups < 1) return fail(LDPC_EINVAL, "num_groups must be >= 1");
    if (!g->group_ptr || !g->group_cn) return fail(LDPC_EINVAL, "VN grouping needs group_ptr/group_cn");
    if (g->group_ptr[0] != 0) return fail(LDPC_EINVAL, "group_ptr[0] must be 0");
    if (g->groups_per_iteration != 0) return fail(LDPC_EINVAL, "groups_per_iteration needs CN groups");
    vgroup.assign(n, -1);
    for (int k = 0; k < g->num_groups; ++k) {
        if (g->group_ptr[k + 1] < g->group_ptr[k]) return fail(LDPC_EINVAL, "group_ptr not monotone");
        if (g->group_ptr[k + 1] == g->group_ptr[k]) return fail(LDPC_EINVAL, "empty group");
        for (int32_t q = g->group_ptr[k]; q < g->group_ptr[k + 1]; ++q) {
            const int32_t v = g->group_cn[q];
            if (v < 0 || v >= n) return fail(LDPC_EINVAL, "group VN out of range");
            if (vgroup[v] >= 0) return fail(LDPC_EINVAL, "VN " + std::to_string(v) + " in two groups");
            vgroup[v] = k;
        }
    }
    for (int v = 0; v < n; ++v)
        if (vgroup[v] < 0) return fail(LDPC_EINVAL, "VN " + std::to_string(v) + " belongs to no group");
    out.assign(g->num_groups, {});
    std::vector<int32_t> last(m, -1);
    for (int c = 0; c < m; ++c)
        for (int32_t q = H->row_ptr[c]; q < H->row_ptr[c + 1]; ++q) {
            const int32_t k = vgroup[H->col_idx[q]];
            if (last[c] == k) continue;  // rows are scanned in CN order, so
            last[c] = k;                 // each group's list stays sorted
            if (out[k].empty() || out[k].back() != c) out[k].push_back(c);
        }
    // a group whose VNs have no edge has nothing to visit: drop it and
    // renumber the others
    std::vector<int32_t> renum(out.size(), -1);
    size_t kept = 0;
    for (size_t k = 0; k < out.size(); ++k)
        if (!out[k].empty()) {
            renum[k] = (int32_t)kept;
            if (kept != k) out[kept].swap(out[k]);
            ++kept;
        }
    out.resize(kept);
    if (out.empty()) return fail(LDPC_EINVAL, "no group has an edge");
    for (int v = 0; v < n; ++v) vgroup[v] = renum[vgroup[v]];
    return LDPC_OK;
}

// LDS of a workgroup (layout in ndgsbp_internal.h).
size_t float_bytes(const ldpc_code* c) { return align16((size_t)(c->ds_start + c->max_slots) * 4); }
size_t msg_bytes(const ldpc_code* c, const Layout& l, MsgKind kind) {
    return align16((size_t)c->m * message_row_bytes(kind, l.D, l.H));
}
size_t lds_bytes(const ldpc_code* c, const Layout& l, MsgKind kind) {
    return float_bytes(c) + msg_bytes(c, l, kind) + 16;
}

int threads_for(const ldpc_code* c, const Layout& l) {
    const int cap = max_threads_for_degree(l.D);
    int t = ((l.H * c->max_group_visits + 63) / 64) * 64;
    return std::max(64, std::min(t, cap));
}

// Padded degree of the kernel variant for h lanes per CN (a multiple of h).
int pick_degree(int d, int h) {
    static const int kD[] = {4, 6, 7, 8, 10, 12, 16, 24, 32};
    for (int x : kD)
        if (d <= x && x % h == 0) return x;
    return -1;
}

// Lanes per CN visit that a mapping may use.
bool valid_lanes(int h) { return h == 1 || h == 2 || h == 4; }

// Lanes per CN visit before the device is known: the mapping that wastes the
// fewest lane-edge slots in the CN phase (idle lanes of the last wave plus
// padding edges), two lanes on a tie; ldpc_code_tune overrides it.
int pick_lanes(const ldpc_code* c, int max_visits, int64_t max_edges) {
    double best_eff = -1.0;
    int best = 1;
    for (int h : {2, 1}) {
        if (!c->lay[h - 1].valid) continue;
        const int D = c->lay[h - 1].D;
        const int lanes = std::min(1024, ((h * max_visits + 63) / 64) * 64);
        const double eff = (double)max_edges / ((double)lanes * (D / h));
        if (eff > best_eff + 1e-9) {
            best_eff = eff;
            best = h;
        }
    }
    return best;
}

// The same choice once the device is known, per message format, among the
// mappings whose frame fits in LDS. Each lane of a visit pays a fixed cost
// besides its edges (DPP exchanges, row address), counted as half an edge
// with four lanes; a mapping is scored by its edges per paid lane-edge slot
// (all passes of a group counted) times its residency, min(1, waves per
// SIMD / 4): with fewer waves the CN phase waits on LDS round trips and
// barriers instead of issuing. When every mapping leaves one workgroup per
// CU, each barrier idles the CU and the mapping with the widest workgroup
// is taken whatever its padding (measured faster on codes of n = 4608 and
// 8064). Two lanes on a tie; 0 when no mapping fits in LDS (the HBM tier
// decodes such codes).
int pick_lanes_resident(const ldpc_code* c, MsgKind kind, int64_t max_edges) {
    constexpr double kWavesToHide = 4.0;
    double best_score = -1.0;
    int best = 0, widest = 0, widest_threads = 0;
    bool all_alone = true;
    for (int h : {2, 1, 4}) {
        const Layout& l = c->lay[h - 1];
        if (!l.valid || (c->vertical && h > 2)) continue;
        const size_t lds = lds_bytes(c, l, kind);
        if (lds > c->max_lds) continue;
        const int threads = threads_for(c, l);
        int per_cu = 0;
        if (decode_occupancy(kind, l.D, l.uniform, h, c->vertical ? 2 : 0, threads, lds, &per_cu) != hipSuccess ||
            per_cu < 1)
            continue;
        const int64_t lane_visits = (int64_t)h * c->max_group_visits;
        const int64_t passes = (lane_visits + threads - 1) / threads;
        const double fixed = h == 4 ? 0.5 : 0.0;
        const double eff = (double)max_edges / ((double)passes * threads * (l.D / h + fixed));
        const double waves = (double)per_cu * (threads / 64) / 4.0;
        const double score = eff * std::min(1.0, waves / kWavesToHide);
        if (score > best_score + 1e-9) {
            best_score = score;
            best = h;
        }
        if (per_cu > 1) all_alone = false;
        if (threads > widest_threads) {
            widest_threads = threads;
            widest = h;
        }
    }
    return best && all_alone ? widest : best;
}

#ifndef NDGSBP_LDS_BANKS
#define NDGSBP_LDS_BANKS 32
#endif
#ifndef NDGSBP_BANK_VISITS
#define NDGSBP_BANK_VISITS 16
#endif

// Edge order of every CN in the mapping with `lanes` lanes per CN visit
// (order[c * D + k] = the edge of CN c, by its position in the CSR row, at
// row position k; -1 for padding). Lane h of a visit reads the posteriors
// at positions h*DH .. h*DH + DH - 1, one per LDS instruction, so one
// instruction of a run of 32 lanes (32 / lanes consecutive visits) gathers
// 32 posteriors, which collide when they fall in one of the
// NDGSBP_LDS_BANKS banks. At its first visit each CN takes the order that
// adds the fewest collisions with the CNs already placed in its run (every
// permutation up to degree 6, else position by position). The order is
// kept for all of the CN's visits, since its message row persists between
// them; it changes results only by the rounding order of eq. (1).
void edge_order(const ldpc_h_csr* H, int lanes, int D, const std::vector<int32_t>& vcn,
                const std::vector<int32_t>& visit_ptr, std::vector<int32_t>& order) {
    const int m = H->m, DH = D / lanes, B = NDGSBP_LDS_BANKS, RUN = 32 / lanes;
    order.assign((size_t)m * D, -1);
    std::vector<char> placed(m, 0);
    std::vector<int32_t> cnt((size_t)DH * B);
    std::vector<int> perm(D), best(D);
    auto bank = [&](int c, int q) { return (int)(H->col_idx[H->row_ptr[c] + q] % B); };
    for (size_t g = 0; g + 1 < visit_ptr.size(); ++g) {
        for (int32_t s = visit_ptr[g]; s < visit_ptr[g + 1]; s += RUN) {
            const int32_t e = std::min(visit_ptr[g + 1], s + RUN);
            std::fill(cnt.begin(), cnt.end(), 0);
            auto add = [&](int c) {
                for (int k = 0; k < D; ++k) {
                    const int q = order[(size_t)c * D + k];
                    if (q >= 0) ++cnt[(size_t)(k % DH) * B + bank(c, q)];
                }
            };
            for (int32_t j = s; j < e; ++j)
                if (placed[vcn[j]]) add(vcn[j]);
            for (int32_t j = s; j < e; ++j) {
                const int c = vcn[j];
                if (placed[c]) continue;
                const int d = H->row_ptr[c + 1] - H->row_ptr[c];
                // position k holds edge perm[k] (>= d: padding, one shared word)
                auto cost = [&](const std::vector<int>& p) {
                    int x = 0;
                    for (int k = 0; k < DH; ++k)
                        for (int h = 0; h < lanes; ++h) {
                            const int q = p[h * DH + k];
                            if (q >= d) continue;
                            const int b = bank(c, q);
                            x += cnt[(size_t)k * B + b];
                            for (int h2 = 0; h2 < h; ++h2) {
                                const int q2 = p[h2 * DH + k];
                                if (q2 < d && bank(c, q2) == b) ++x;
                            }
                        }
                    return x;
                };
                for (int k = 0; k < D; ++k) perm[k] = k;
                if (D <= 6) {
                    int bc = -1;
                    do {
                        const int x = cost(perm);
                        if (bc < 0 || x < bc) {
                            bc = x;
                            best = perm;
                        }
                    } while (std::next_permutation(perm.begin(), perm.end()));
                } else {
                    // position by position: the unused edge whose bank is least used
                    std::vector<char> used(D, 0);
                    std::vector<int32_t> local((size_t)DH * B, 0);
                    for (int k = 0; k < DH; ++k)
                        for (int h = 0; h < lanes; ++h) {
                            int pick = -1, pc = 0;
                            for (int q = 0; q < D; ++q) {
                                if (used[q]) continue;
                                const int x = q < d ? cnt[(size_t)k * B + bank(c, q)] + local[(size_t)k * B + bank(c, q)] : 0;
                                if (pick < 0 || x < pc) {
                                    pick = q;
                                    pc = x;
                                }
                            }
                            used[pick] = 1;
                            if (pick < d) ++local[(size_t)k * B + bank(c, pick)];
                            best[h * DH + k] = pick;
                        }
                }
                for (int k = 0; k < D; ++k) order[(size_t)c * D + k] = best[k] < d ? best[k] : -1;
                placed[c] = 1;
                add(c);
            }
        }
    }
}

MsgKind msg_kind(uint32_t flags) {
    return (flags & LDPC_FLAG_MSG_FP16) ? kMsgF16 : (flags & LDPC_FLAG_MSG_BF16) ? kMsgBF16 : kMsgF32;
}

int check_flags(uint32_t flags) {
    const uint32_t known =
        LDPC_FLAG_EARLY_STOP | LDPC_FLAG_MSG_FP16 | LDPC_FLAG_MSG_BF16 | LDPC_FLAG_OUT_PACKED | LDPC_FLAG_TIER_HBM;
    if (flags & ~known) return fail(LDPC_EINVAL, "unknown flag bits");
    if ((flags & LDPC_FLAG_MSG_FP16) && (flags & LDPC_FLAG_MSG_BF16))
        return fail(LDPC_EINVAL, "MSG_FP16 and MSG_BF16 are exclusive");
    return LDPC_OK;
}

int check_lds(const ldpc_code* c, const Layout& lay, MsgKind kind) {
    if (lds_bytes(c, lay, kind) > c->max_lds)
        return fail(LDPC_EUNSUPPORTED, "one frame needs " + std::to_string(lds_bytes(c, lay, kind)) +
                                           " B of LDS, device allows " + std::to_string(c->max_lds));
    return LDPC_OK;
}

// Persistent workgroups of a launch: as many as can be resident, at most one
// per frame.
int set_blocks(MsgKind kind, int D, bool uniform, bool table, int num_cus, int64_t frames, LaunchShape& shape) {
    int per_cu = 0;
    const int mode = table ? 1 : shape.vertical ? 2 : 0;
    hipError_t oe = decode_occupancy(kind, D, uniform, shape.lanes, mode, shape.threads, shape.lds_bytes, &per_cu);
    if (oe != hipSuccess) return hip_fail(oe, "occupancy query");
    if (per_cu < 1) return fail(LDPC_EUNSUPPORTED, "kernel variant cannot be resident");
    shape.blocks = (int)std::min<int64_t>((int64_t)per_cu * num_cus, frames);
    return LDPC_OK;
}

Problem make_problem(const ldpc_code* c, const Layout& lay, const float* llr, int32_t num_frames, int32_t max_iter,
                     uint8_t* hard, float* post, int32_t* iters, uint8_t* syn_ok) {
    Problem p{};
    p.vcn = c->dev.vcn;
    p.vw = lay.vw;
    p.visit_ptr = c->dev.visit_ptr;
    p.fix = c->dev.fix;
    p.fix_ptr = c->dev.fix_ptr;
    p.syn_col = lay.syn_col;
    p.llr = llr;
    p.hard = hard;
    p.post = post;
    p.iters = iters;
    p.syn_ok = syn_ok;
    p.n = c->n;
    p.m = c->m;
    p.G = c->G;
    p.R = c->R;
    p.max_iter = max_iter;
    p.first = 0;
    p.num_frames = num_frames;
    p.ds_start_b = 4u * (uint32_t)c->ds_start;
    p.pad_b = 4u * (uint32_t)c->n;
    p.l_offset = (int32_t)float_bytes(c);
    return p;
}

void set_launch_constants(DecodeArgs& a, uint32_t flags, size_t lds) {
    a.early_stop = (flags & LDPC_FLAG_EARLY_STOP) ? 1 : 0;
    a.packed = (flags & LDPC_FLAG_OUT_PACKED) ? 1 : 0;
    a.sh_offset = (int32_t)(lds - 16);
    a.ymax = (float)(kXMax * kLog2e);
}

// Launch class of a batched problem: kernel variant, and with size
// splitting the power of two at or above its LDS need.
struct ClassKey {
    int D = 0, H = 1;
    bool uniform = false;
    int size_class = 0;
    bool operator<(const ClassKey& o) const {
        if (D != o.D) return D < o.D;
        if (H != o.H) return H < o.H;
        if (uniform != o.uniform) return uniform < o.uniform;
        return size_class < o.size_class;
    }
};

int size_class(size_t lds) {
    int k = 0;
    while (((size_t)1 << k) < lds) ++k;
    return k;
}

struct BatchClass {
    ClassKey key;
    int32_t table_offset = 0;
    int32_t nprob = 0;
    int32_t total_frames = 0;
    double work_estimate = 0.0;
    LaunchShape shape{};
    DecodeArgs args{};
};

constexpr int kMaxBatchStreams = 8;

ldpc_batch_options default_batch_options() {
    ldpc_batch_options o;
    o.lanes_per_cn = 0;
    o.split_by_size = 1;
    o.max_threads = 0;
    o.streams = 4;
    return o;
}

}  // namespace

struct ldpc_batch {
    int32_t device = -1;
    MsgKind kind = kMsgF32;
    int32_t num_problems = 0;
    int64_t total_frames = 0;
    std::vector<BatchClass> classes;
    Problem* table = nullptr;  // device: every class's problems
    uint32_t* work = nullptr;  // device: a counter pair per class
    std::vector<hipStream_t> streams;  // streams besides the caller's
    std::vector<hipEvent_t> events;    // fork, then one join per extra stream
};

namespace {

void free_batch(ldpc_batch* b) {
    for (hipEvent_t ev : b->events) (void)hipEventDestroy(ev);
    for (hipStream_t st : b->streams) (void)hipStreamDestroy(st);
    b->events.clear();
    b->streams.clear();
    (void)hipFree(b->table);
    (void)hipFree(b->work);
    b->table = nullptr;
    b->work = nullptr;
}

int check_options(const ldpc_batch_options& o) {
    if (o.lanes_per_cn != 0 && !valid_lanes(o.lanes_per_cn))
        return fail(LDPC_EINVAL, "lanes_per_cn must be 0, 1, 2 or 4");
    if (o.max_threads < 0 || o.max_threads % 64 || o.max_threads > 1024)
        return fail(LDPC_EINVAL, "max_threads must be 0 or a multiple of 64 up to 1024");
    if (o.streams < 0 || o.streams > kMaxBatchStreams) return fail(LDPC_EINVAL, "streams must be in 0..8");
    return LDPC_OK;
}

// Launch classes of a set of problems (validated), their problem table in
// class order, and the device they run on.
struct ClassPlan {
    std::vector<BatchClass> classes;
    std::vector<Problem> table;
    int32_t device = -1;
    int num_cus = 0;
    int64_t total_frames = 0;
};

int form_classes(const ldpc_problem* probs, int32_t count, MsgKind kind, const ldpc_batch_options& o,
                 ClassPlan& plan) {
    if (count < 0) return fail(LDPC_EINVAL, "count < 0");
    if (count > 0 && !probs) return fail(LDPC_EINVAL, "probs is NULL");
    struct Item {
        int idx;
        const Layout* lay;
        ClassKey key;
        size_t lds;
        int threads;
    };
    std::vector<Item> items;
    for (int i = 0; i < count; ++i) {
        const ldpc_problem& q = probs[i];
        const std::string at = "problem " + std::to_string(i) + ": ";
        if (!q.code) return fail(LDPC_EINVAL, at + "code is NULL");
        if (q.num_frames < 0) return fail(LDPC_EINVAL, at + "num_frames < 0");
        if (q.max_iter < 1) return fail(LDPC_EINVAL, at + "max_iter < 1");
        if (plan.device < 0) {
            plan.device = q.code->device;
            plan.num_cus = q.code->num_cus;
        } else if (q.code->device != plan.device) {
            return fail(LDPC_EINVAL, at + "codes of one batch must be on one device");
        }
        if (q.num_frames == 0) continue;
        if (!q.llr || !q.hard || !q.iters) return fail(LDPC_EINVAL, at + "llr, hard and iters are required");
        if (q.code->vertical) return fail(LDPC_EUNSUPPORTED, at + "codes with VN groups are not batched");
        const int h = o.lanes_per_cn ? o.lanes_per_cn : q.code->lanes_for[kind];
        const Layout& lay = q.code->lay[h - 1];
        if (!lay.valid) return fail(LDPC_EUNSUPPORTED, at + "no kernel variant with that mapping");
        int rc = check_lds(q.code, lay, kind);
        if (rc) return fail(rc, at + g_last_error + " (batches run the LDS tier; ldpc_decode takes the HBM tier)");
        Item it;
        it.idx = i;
        it.lay = &lay;
        it.lds = lds_bytes(q.code, lay, kind);
        it.threads = threads_for(q.code, lay);
        it.key.D = lay.D;
        it.key.H = lay.H;
        it.key.uniform = lay.uniform;
        it.key.size_class = o.split_by_size ? size_class(it.lds) : 0;
        items.push_back(it);
    }
    // classes: one persistent launch each
    std::stable_sort(items.begin(), items.end(), [](const Item& x, const Item& y) { return x.key < y.key; });
    for (size_t s = 0; s < items.size();) {
        size_t e = s;
        while (e < items.size() && !(items[s].key < items[e].key) && !(items[e].key < items[s].key)) ++e;
        BatchClass bc;
        bc.key = items[s].key;
        bc.table_offset = (int32_t)plan.table.size();
        size_t lds = 0;
        int threads = 64;
        int64_t frames = 0;
        double work = 0.0;
        for (size_t k = s; k < e; ++k) {
            const ldpc_problem& q = probs[items[k].idx];
            if (frames + q.num_frames > INT32_MAX)
                return fail(LDPC_EUNSUPPORTED, "more than 2^31 - 1 frames in one launch class");
            plan.table.push_back(make_problem(q.code, *items[k].lay, q.llr, q.num_frames, q.max_iter, q.hard,
                                              q.post, q.iters, q.syn_ok));
            plan.table.back().first = (int32_t)frames;
            frames += q.num_frames;
            work += (double)q.num_frames * (double)q.code->edge_updates * q.max_iter;
            lds = std::max(lds, items[k].lds);
            threads = std::max(threads, items[k].threads);
        }
        if (o.max_threads) threads = std::min(threads, o.max_threads);
        bc.nprob = (int32_t)(e - s);
        bc.total_frames = (int32_t)frames;
        bc.work_estimate = work;
        bc.shape.lanes = bc.key.H;
        bc.shape.threads = threads;
        bc.shape.lds_bytes = lds;
        plan.total_frames += frames;
        plan.classes.push_back(bc);
        s = e;
    }
    // the longest launches first, so that short ones fill the tails
    std::stable_sort(plan.classes.begin(), plan.classes.end(),
                     [](const BatchClass& x, const BatchClass& y) { return x.work_estimate > y.work_estimate; });
    return LDPC_OK;
}

void finish_class_args(BatchClass& bc, const std::vector<Problem>& table, const Problem* dev_table, uint32_t* work,
                       uint32_t flags) {
    DecodeArgs& a = bc.args;
    a = DecodeArgs{};
    a.p0 = table[bc.table_offset];
    a.table = dev_table + bc.table_offset;
    a.nprob = bc.nprob;
    a.total_frames = bc.total_frames;
    a.work = work;
    set_launch_constants(a, flags, bc.shape.lds_bytes);
}

// Enqueues the classes: class k on stream k mod S of {main, extra...}, the
// extra streams forked from and joined back into `main` with evs[0] (fork)
// and evs[1..] (joins); evs holds extra.size() + 1 events.
hipError_t launch_classes(const std::vector<BatchClass>& classes, MsgKind kind, hipStream_t main,
                          const std::vector<hipStream_t>& extra, const std::vector<hipEvent_t>& evs) {
    const int ns = (int)extra.size() + 1;
    hipError_t e = hipSuccess;
    if (ns > 1) {
        e = hipEventRecord(evs[0], main);
        for (int k = 1; k < ns && e == hipSuccess; ++k) e = hipStreamWaitEvent(extra[k - 1], evs[0], 0);
    }
    for (size_t k = 0; k < classes.size() && e == hipSuccess; ++k) {
        const BatchClass& bc = classes[k];
        hipStream_t st = k % ns == 0 ? main : extra[k % ns - 1];
        e = launch_decode(bc.args, kind, bc.key.D, bc.key.uniform, bc.shape, st);
    }
    for (int k = 1; k < ns && e == hipSuccess; ++k) {
        e = hipEventRecord(evs[k], extra[k - 1]);
        if (e == hipSuccess) e = hipStreamWaitEvent(main, evs[k], 0);
    }
    return e;
}

// Staging ring of the asynchronous ldpc_decode_batched, one per device, kept
// for the life of the process: each slot holds a pinned host and a device
// copy of a problem table, work counters, fork/join events and the streams
// its launch classes fork onto (per slot, so that calls in flight at the
// same time, e.g. from a serving loop on several caller streams, do not
// queue behind each other's classes); a slot is reused once the call that
// last used it has finished on the device.
constexpr int kStageRing = 16;
constexpr int kStageClasses = 64;
constexpr int kStageStreams = 4;

struct StageSlot {
    Problem* host = nullptr;  // pinned
    Problem* dev = nullptr;
    size_t cap = 0;           // problems
    uint32_t* work = nullptr; // 2 per class, zero between launches
    hipEvent_t done = nullptr;
    std::vector<hipEvent_t> fork_join;
    std::vector<hipStream_t> streams;  // kStageStreams - 1 fork streams
    bool in_use = false;
};

struct DeviceStage {
    std::mutex mu;
    StageSlot slots[kStageRing];
    unsigned next = 0;
};

std::mutex g_stage_mu;
std::map<int, DeviceStage*> g_stage;

hipError_t get_stage(int device, DeviceStage** out) {
    std::lock_guard<std::mutex> lock(g_stage_mu);
    auto it = g_stage.find(device);
    if (it != g_stage.end()) {
        *out = it->second;
        return hipSuccess;
    }
    DeviceStage* ds = new DeviceStage();
    hipError_t e = hipSuccess;
    for (StageSlot& s : ds->slots) {
        for (int k = 1; k < kStageStreams && e == hipSuccess; ++k) {
            hipStream_t st = nullptr;
            e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
            if (e == hipSuccess) s.streams.push_back(st);
        }
        if (e == hipSuccess) e = hipEventCreateWithFlags(&s.done, hipEventDisableTiming);
        for (int k = 0; k < kStageStreams && e == hipSuccess; ++k) {
            hipEvent_t ev = nullptr;
            e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
            if (e == hipSuccess) s.fork_join.push_back(ev);
        }
        if (e == hipSuccess) e = hipMalloc((void**)&s.work, 2 * sizeof(uint32_t) * kStageClasses);
        if (e == hipSuccess) e = hipMemset(s.work, 0, 2 * sizeof(uint32_t) * kStageClasses);
    }
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) return e;  // the partial ring is leaked; the call fails
    g_stage[device] = ds;
    *out = ds;
    return hipSuccess;
}

// HBM tier (codes beyond LDS, or LDPC_FLAG_TIER_HBM): one-lane tables,
// 64-frame tiles in a workspace. Without `scratch` the workspace is the
// code's own, grown on demand, and the code's HBM-tier launches are ordered
// on the device; with it, the caller's fixed buffer bounds the tiles in
// flight and nothing is allocated or ordered.
int decode_hbm(ldpc_code* c, const float* llr, int32_t num_frames, int32_t max_iter, uint32_t flags, uint8_t* hard,
               float* post, int32_t* iters, uint8_t* syn_ok, const Scratch* scratch, hipStream_t stream) {
    const MsgKind kind = msg_kind(flags);
    const Layout& lay = c->lay[0];
    if (!lay.valid) return fail(LDPC_EUNSUPPORTED, "no one-lane tables for the HBM tier");
    if (c->R > 1)
        return fail(LDPC_EUNSUPPORTED, "the HBM tier decodes its 64 frames of a tile at different iterations: "
                                       "one grouping for every iteration only");
    const int slots = hbm_slots();
    const int waves = std::max(1, std::min(hbm_max_threads(lay.D) / 64, c->max_group_visits));
    const int threads = 64 * waves;
    // the tile's sign words live in LDS when they fit, and its delta slots
    // too when both fit
    const size_t sgn_bytes = hbm_sign_bytes(c->n);
    const size_t slot_bytes = hbm_slot_bytes(c->max_slots);
    const bool sgn = sgn_bytes <= c->max_lds - kHbmStaticLds;
    const bool dl = sgn && sgn_bytes + slot_bytes <= c->max_lds - kHbmStaticLds;
    const size_t lds = (sgn ? sgn_bytes : 0) + (dl ? slot_bytes : 0);
    int per_cu = 0;
    hipError_t e = hbm_occupancy(kind, lay.D, lay.uniform, threads, lds, &per_cu);
    if (e != hipSuccess) return hip_fail(e, "occupancy query (HBM tier)");
    if (per_cu < 1) return fail(LDPC_EUNSUPPORTED, "HBM-tier kernel cannot be resident");
    const int64_t tiles_needed = (num_frames + slots - 1) / slots;
    int blocks = (int)std::min<int64_t>((int64_t)per_cu * c->num_cus, tiles_needed);
    const uint64_t frows = (uint64_t)c->ds_start + (uint64_t)c->max_slots;
    const uint64_t fws_tile = frows * slots;
    const uint64_t mws_tile = (uint64_t)c->m * lay.D * slots;
    const size_t msg_size = kind == kMsgF32 ? 4 : 2;
    const size_t ftile_bytes = (fws_tile * 4 + 255) & ~(size_t)255;
    const size_t tile_bytes = ftile_bytes + ((mws_tile * msg_size + 255) & ~(size_t)255);

    HbmArgs a{};
    a.p = make_problem(c, lay, llr, num_frames, max_iter, hard, post, iters, syn_ok);
    a.vfirst = c->dev.vfirst;
    a.vdfirst = c->dev.vdfirst;
    a.sgn_lds = sgn ? 1 : 0;
    a.dslot_lds = dl ? 1 : 0;
    a.max_slots = c->max_slots;
    a.fws_tile = ftile_bytes / 4;
    a.mws_tile = mws_tile;
    a.early_stop = (flags & LDPC_FLAG_EARLY_STOP) ? 1 : 0;
    a.packed = (flags & LDPC_FLAG_OUT_PACKED) ? 1 : 0;
    a.ymax = (float)(kXMax * kLog2e);
    if (scratch) {
        const int64_t fit = (int64_t)(scratch->hbm_bytes / tile_bytes);
        if (fit < 1)
            return fail(LDPC_EUNSUPPORTED, "one HBM-tier tile of this code needs " + std::to_string(tile_bytes) +
                                               " B, more than the " + std::to_string(scratch->hbm_bytes) +
                                               " B of the fixed scratch buffer");
        blocks = (int)std::min<int64_t>(blocks, fit);
        a.fws = reinterpret_cast<float*>(scratch->hbm);
        a.mws = reinterpret_cast<unsigned char*>(scratch->hbm) + (size_t)blocks * ftile_bytes;
        a.work = scratch->work;
        e = launch_hbm(a, kind, lay.D, lay.uniform, blocks, threads, stream);
        return e == hipSuccess ? LDPC_OK : hip_fail(e, "HBM-tier decode launch");
    }
    const size_t need = (size_t)blocks * tile_bytes;

    std::lock_guard<std::mutex> lock(c->hbm_mu);
    if (!c->hbm_last) {
        e = hipEventCreateWithFlags(&c->hbm_last, hipEventDisableTiming);
        if (e != hipSuccess) return hip_fail(e, "HBM-tier event");
    }
    if (need > c->hbm_ws_bytes) {
        // no earlier HBM-tier launch of this code may still use the old one
        if (c->hbm_used) {
            e = hipEventSynchronize(c->hbm_last);
            if (e != hipSuccess) return hip_fail(e, "HBM-tier workspace wait");
        }
        (void)hipFree(c->hbm_ws);
        c->hbm_ws = nullptr;
        c->hbm_ws_bytes = 0;
        e = hipMalloc(&c->hbm_ws, need);
        if (e != hipSuccess)
            return e == hipErrorOutOfMemory ? fail(LDPC_ENOMEM, "HBM-tier workspace of " + std::to_string(need) + " B")
                                            : hip_fail(e, "HBM-tier workspace");
        c->hbm_ws_bytes = need;
    }
    a.fws = reinterpret_cast<float*>(c->hbm_ws);
    a.mws = reinterpret_cast<unsigned char*>(c->hbm_ws) + (size_t)blocks * ftile_bytes;
    a.work = c->dev.work + 2 * (c->next_work.fetch_add(1) % kWorkRing);
    if (c->hbm_used) {
        e = hipStreamWaitEvent(stream, c->hbm_last, 0);
        if (e != hipSuccess) return hip_fail(e, "HBM-tier ordering");
    }
    e = launch_hbm(a, kind, lay.D, lay.uniform, blocks, threads, stream);
    if (e == hipSuccess) e = hipEventRecord(c->hbm_last, stream);
    if (e != hipSuccess) return hip_fail(e, "HBM-tier decode launch");
    c->hbm_used = true;
    return LDPC_OK;
}

// Grows a slot's tables to hold `n` problems (allocates only on growth).
hipError_t reserve_slot(StageSlot& s, size_t n) {
    if (n <= s.cap) return hipSuccess;
    size_t cap = std::max<size_t>(n, 2 * s.cap);
    (void)hipHostFree(s.host);
    (void)hipFree(s.dev);
    s.host = nullptr;
    s.dev = nullptr;
    s.cap = 0;
    hipError_t e = hipHostMalloc((void**)&s.host, cap * sizeof(Problem), hipHostMallocDefault);
    if (e == hipSuccess) e = hipMalloc((void**)&s.dev, cap * sizeof(Problem));
    if (e == hipSuccess) s.cap = cap;
    return e;
}

}  // namespace

namespace ndgsbp {

int record_error(int code, const char* msg) { return fail(code, msg); }

// ldpc_decode, with the work counter and HBM-tier workspace taken from
// `scratch` when it is given (the code's own otherwise).
int decode_enqueue(ldpc_code* c, const float* llr, int32_t num_frames, int32_t max_iter, uint32_t flags,
                   uint8_t* hard, float* post, int32_t* iters, uint8_t* syn_ok, const Scratch* scratch,
                   void* hip_stream) {
    g_last_error.clear();
    if (!c) return fail(LDPC_EINVAL, "code is NULL");
    if (num_frames < 0) return fail(LDPC_EINVAL, "num_frames < 0");
    if (max_iter < 1) return fail(LDPC_EINVAL, "max_iter < 1");
    int rc = check_flags(flags);
    if (rc) return rc;
    if (num_frames == 0) return LDPC_OK;
    if (!llr || !hard || !iters) return fail(LDPC_EINVAL, "llr, hard and iters are required");
    const MsgKind kind = msg_kind(flags);
    const Layout& lay = c->lay[c->lanes_for[kind] - 1];

    DeviceGuard guard(c->device);
    if (!guard.ok) return fail(LDPC_EHIP, "cannot select the code's device");
    if (c->vertical) {
        if ((flags & LDPC_FLAG_TIER_HBM) || lds_bytes(c, lay, kind) > c->max_lds)
            return fail(LDPC_EUNSUPPORTED, "the vertical schedule runs in the LDS tier only");
        if (kind == kMsgBF16 || lay.H > 2)
            return fail(LDPC_EUNSUPPORTED, "the vertical schedule takes FP32 or FP16 messages, one or two lanes");
    } else if ((flags & LDPC_FLAG_TIER_HBM) || lds_bytes(c, lay, kind) > c->max_lds) {
        return decode_hbm(c, llr, num_frames, max_iter, flags, hard, post, iters, syn_ok, scratch,
                          (hipStream_t)hip_stream);
    }
    LaunchShape shape;
    shape.vertical = c->vertical;
    shape.lanes = lay.H;
    shape.threads = threads_for(c, lay);
    shape.lds_bytes = lds_bytes(c, lay, kind);
    rc = set_blocks(kind, lay.D, lay.uniform, false, c->num_cus, num_frames, shape);
    if (rc) return rc;

    DecodeArgs a{};
    a.p0 = make_problem(c, lay, llr, num_frames, max_iter, hard, post, iters, syn_ok);
    a.table = nullptr;
    a.nprob = 1;
    a.total_frames = num_frames;
    a.work = scratch ? scratch->work : c->dev.work + 2 * (c->next_work.fetch_add(1) % kWorkRing);
    set_launch_constants(a, flags, shape.lds_bytes);
    hipError_t e = launch_decode(a, kind, lay.D, lay.uniform, shape, (hipStream_t)hip_stream);
    if (e != hipSuccess) return hip_fail(e, "decode launch");
    return LDPC_OK;
}

}  // namespace ndgsbp

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
    // vertical schedule: the group of every VN; each VN group becomes the
    // visits of the CNs adjacent to it, whose edges into other groups are
    // inputs only
    const bool vertical = grouping && grouping->kind == LDPC_GROUPS_VN;
    std::vector<int32_t> vgroup;
    int rc = vertical ? expand_vn_groups(H, grouping, vgroup, groups) : expand_groups(grouping, m, groups);
    if (rc) return rc;

    ldpc_code* c = new (std::nothrow) ldpc_code();
    if (!c) return fail(LDPC_ENOMEM, "host allocation failed");
    c->device = device;
    c->m = m;
    c->n = n;
    c->nnz = H->nnz;
    c->R = (grouping->groups_per_iteration > 0) ? (int32_t)groups.size() / grouping->groups_per_iteration : 1;
    c->G = (int32_t)groups.size() / c->R;
    c->max_cn_degree = maxd;
    c->vertical = vertical;
    c->max_vn_degree = n ? *std::max_element(vdeg.begin(), vdeg.end()) : 0;

    // float index of the first delta slot: right after the posteriors
    // (n real, one scratch for padding edges, one zero for syndrome padding)
    const int32_t ds_start = n + 2;
    c->ds_start = ds_start;

    // visits, edge source/target indices and fix-up tables (mapping-free)
    std::vector<int32_t> vcn;
    std::vector<uint32_t> esrc, edst;  // per visit edge, in row order
    std::vector<uint8_t> efirst;       // per visit edge: it writes its VN's first delta slot
    std::vector<int32_t> vdeg_of(1, 0);  // prefix over visits of their degree
    std::vector<int32_t> visit_ptr(1, 0), fix_ptr(1, 0);
    std::vector<uint2> fix;
    std::vector<int32_t> cnt(n, 0), first_slot(n, -1), next_fill(n, 0);
    std::vector<int32_t> seen_order;
    int64_t max_edges = 0;
    c->cn_visits = 0;
    c->edge_updates = 0;
    c->max_group_visits = 0;
    c->max_slots = 0;
    for (size_t gidx = 0; gidx < groups.size(); ++gidx) {
        const auto& grp = groups[gidx];
        // an edge is an input only when its VN is outside a vertical group
        auto input_only = [&](int32_t v) { return vertical && vgroup[v] != (int32_t)gidx; };
        // multiplicity of each VN inside the group
        seen_order.clear();
        for (int32_t cn : grp)
            for (int32_t q = H->row_ptr[cn]; q < H->row_ptr[cn + 1]; ++q) {
                const int32_t v = H->col_idx[q];
                if (input_only(v)) continue;
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
        int64_t edges = 0, outputs = 0;
        for (int32_t cn : grp) {
            const int32_t b = H->row_ptr[cn], d = H->row_ptr[cn + 1] - b;
            vcn.push_back(cn);
            for (int32_t k = 0; k < d; ++k) {
                const int32_t v = H->col_idx[b + k];
                // input-only edges add back into the scratch word n
                const bool multi = !input_only(v) && cnt[v] >= 2;
                const int32_t tgt = input_only(v) ? n : multi ? ds_start + first_slot[v] + next_fill[v]++ : v;
                esrc.push_back((uint32_t)v);
                edst.push_back((uint32_t)tgt);
                efirst.push_back(multi && next_fill[v] == 1 ? 1 : 0);
                outputs += input_only(v) ? 0 : 1;
            }
            vdeg_of.push_back(vdeg_of.back() + d);
            edges += d;
        }
        for (int32_t v : seen_order) {
            cnt[v] = 0;
            first_slot[v] = -1;
            next_fill[v] = 0;
        }
        c->edge_updates += outputs;
        max_edges = std::max(max_edges, edges);
        c->cn_visits += (int64_t)grp.size();
        c->max_group_visits = std::max<int32_t>(c->max_group_visits, (int32_t)grp.size());
        c->max_slots = std::max(c->max_slots, slots);
        visit_ptr.push_back((int32_t)vcn.size());
        fix_ptr.push_back((int32_t)fix.size());
    }

    // per-mapping tables: edge half-records padded to D, syndrome rows
    std::vector<uint32_t> vw_h[4], syn_h[4];
    std::vector<uint32_t> vdfirst;  // one-lane layout: bit k = edge at position k writes a first delta slot
    std::vector<int32_t> order_h[4];  // per mapping: row position -> edge of the CN
    for (int h : {1, 2, 4}) {
        Layout& l = c->lay[h - 1];
        const int D = pick_degree(std::max(1, maxd), h);
        if (D < 0 || D % h) continue;
        l.valid = true;
        l.H = h;
        l.D = D;
        l.uniform = true;
        for (int i = 0; i < m; ++i)
            if (H->row_ptr[i + 1] - H->row_ptr[i] != D) l.uniform = false;
        const int DH = D / h;
        const int W = (2 * DH + 3) / 4 * 4;  // words per half-record
        std::vector<int32_t>& order = order_h[h - 1];
        edge_order(H, h, D, vcn, visit_ptr, order);
        std::vector<uint32_t>& vw = vw_h[h - 1];
        vw.assign(vcn.size() * (size_t)h * W, 0u);
        if (h == 1) vdfirst.assign(vcn.size(), 0u);
        for (size_t j = 0; j < vcn.size(); ++j) {
            const int32_t e0 = vdeg_of[j], d = vdeg_of[j + 1] - e0;
            for (int k = 0; k < D; ++k) {
                uint32_t src = 4u * (uint32_t)n, dst = 4u * (uint32_t)n;  // padding edge
                const int32_t q = order[(size_t)vcn[j] * D + k];
                if (q >= 0) {
                    src = 4u * esrc[e0 + q];
                    dst = 4u * edst[e0 + q];
                    if (h == 1 && efirst[e0 + q]) vdfirst[j] |= 1u << k;
                }
                const size_t half = (j * h + (size_t)(k / DH)) * W;
                vw[half + k % DH] = src;
                vw[half + DH + k % DH] = dst;
            }
            // a half-record with a spare word (DH odd) carries the lane's
            // message row, so that the kernel needs no vcn read for it
            if (W > 2 * DH)
                for (int hh = 0; hh < h; ++hh) vw[(j * h + (size_t)hh) * W + 2 * DH] = (uint32_t)(vcn[j] * h + hh);
        }
        const int SD = (D + 3) / 4 * 4;  // syndrome row stride
        std::vector<uint32_t>& syn = syn_h[h - 1];
        syn.assign((size_t)m * SD, 4u * (uint32_t)(n + 1));
        // A check's entries may sit in any order (its parity is a XOR). Lane
        // t checks c = t (+ multiples of the workgroup size), one entry per
        // LDS instruction, so 32 consecutive checks are read together: each
        // check of such a run puts its VNs at the free positions whose bank
        // is least used in the run so far (padding reads one shared word).
        // Positions D .. SD - 1 stay padding: the kernels do not read them.
        {
            const int B = NDGSBP_LDS_BANKS;
            std::vector<int32_t> used((size_t)SD * B);
            for (int r0 = 0; r0 < m; r0 += 32) {
                std::fill(used.begin(), used.end(), 0);
                for (int i = r0; i < std::min(m, r0 + 32); ++i) {
                    uint32_t* row = &syn[(size_t)i * SD];
                    std::vector<char> taken(D, 0);
                    for (int32_t q = H->row_ptr[i]; q < H->row_ptr[i + 1]; ++q) {
                        const int b = H->col_idx[q] % B;
                        int pick = -1;
                        for (int k = 0; k < D; ++k)
                            if (!taken[k] && (pick < 0 || used[(size_t)k * B + b] < used[(size_t)pick * B + b])) pick = k;
                        taken[pick] = 1;
                        ++used[(size_t)pick * B + b];
                        row[pick] = 4u * (uint32_t)H->col_idx[q];
                    }
                }
            }
        }
    }
    // Provisional mappings until the device's LDS and occupancy are known
    // (pick_lanes_resident below): FP32 the slot-count choice, 16-bit one
    // lane per visit.
    const int lanes0 = pick_lanes(c, c->max_group_visits, max_edges);
    const int lanes16 = c->lay[0].valid ? 1 : lanes0;
    c->lanes_for[kMsgF32] = c->lanes_default[kMsgF32] = lanes0;
    c->lanes_for[kMsgF16] = c->lanes_default[kMsgF16] = lanes16;
    c->lanes_for[kMsgBF16] = c->lanes_default[kMsgBF16] = lanes16;

    DeviceGuard guard(device);
    if (!guard.ok) {
        delete c;
        return fail(LDPC_EHIP, "cannot select device " + std::to_string(device));
    }
    hipError_t e = hipSuccess;
    // first visit of each CN within an iteration (the HBM tier treats its
    // old message as the initial 0 in a frame's first iteration)
    std::vector<uint32_t> vfirst(vcn.size(), 0u);
    {
        std::vector<char> seen(m, 0);
        for (size_t j = 0; j < vcn.size(); ++j) {
            vfirst[j] = seen[vcn[j]] ? 0u : 1u;
            seen[vcn[j]] = 1;
        }
    }
    if (e == hipSuccess) e = upload(&c->dev.vcn, vcn);
    if (e == hipSuccess) e = upload(&c->dev.vfirst, vfirst);
    if (e == hipSuccess) e = upload(&c->dev.vdfirst, vdfirst);
    if (e == hipSuccess) e = upload(&c->dev.visit_ptr, visit_ptr);
    if (e == hipSuccess) e = upload(&c->dev.fix, fix);
    if (e == hipSuccess) e = upload(&c->dev.fix_ptr, fix_ptr);
    for (int h : {1, 2, 4}) {
        if (e != hipSuccess) break;
        if (!c->lay[h - 1].valid) continue;
        e = upload(&c->lay[h - 1].vw, vw_h[h - 1]);
        if (e == hipSuccess) e = upload(&c->lay[h - 1].syn_col, syn_h[h - 1]);
    }
    if (e == hipSuccess) e = hipMalloc((void**)&c->dev.work, sizeof(uint32_t) * 2 * kWorkRing);
    if (e == hipSuccess) e = hipMemset(c->dev.work, 0, sizeof(uint32_t) * 2 * kWorkRing);
    if (e == hipSuccess) {
        int v = 0;
        e = hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, device);
        c->max_lds = (size_t)v;
    }
    if (e == hipSuccess) e = hipDeviceGetAttribute(&c->num_cus, hipDeviceAttributeMultiprocessorCount, device);
    // set-up of ldpc_decode_noalloc's fixed scratch on this device (once)
    if (e == hipSuccess) e = noalloc_setup(device);
    if (e == hipSuccess) {
        for (MsgKind k : {kMsgF32, kMsgF16, kMsgBF16}) {
            const int h = pick_lanes_resident(c, k, max_edges);
            if (h) c->lanes_for[k] = c->lanes_default[k] = h;
        }
    }
    if (e != hipSuccess) {
        free_tables(c);
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
        free_tables(code);
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
    info->num_groups = c->G * c->R;
    info->cn_visits = c->cn_visits / c->R;
    info->edge_updates = c->edge_updates / c->R;
    info->groups_per_iteration = c->G;
    info->max_cn_degree = c->max_cn_degree;
    info->max_vn_degree = c->max_vn_degree;
    info->device = c->device;
    info->lds_bytes_fp32 = (int64_t)lds_bytes(c, c->lay[c->lanes_for[kMsgF32] - 1], kMsgF32);
    info->lds_bytes_16 = (int64_t)lds_bytes(c, c->lay[c->lanes_for[kMsgF16] - 1], kMsgF16);
    info->lds_limit = (int64_t)c->max_lds;
    info->lanes_fp32 = c->lanes_for[kMsgF32];
    info->lanes_fp16 = c->lanes_for[kMsgF16];
    info->lanes_bf16 = c->lanes_for[kMsgBF16];
    return LDPC_OK;
}

int ldpc_code_tune(ldpc_code_t c, uint32_t msg_flags, int32_t lanes_per_cn) {
    g_last_error.clear();
    if (!c) return fail(LDPC_EINVAL, "code is NULL");
    if (msg_flags & ~(LDPC_FLAG_MSG_FP16 | LDPC_FLAG_MSG_BF16)) return fail(LDPC_EINVAL, "msg_flags: message format bits only");
    if ((msg_flags & LDPC_FLAG_MSG_FP16) && (msg_flags & LDPC_FLAG_MSG_BF16))
        return fail(LDPC_EINVAL, "MSG_FP16 and MSG_BF16 are exclusive");
    const MsgKind kind = msg_kind(msg_flags);
    if (lanes_per_cn == 0) {
        c->lanes_for[kind] = c->lanes_default[kind];
        return LDPC_OK;
    }
    if (!valid_lanes(lanes_per_cn)) return fail(LDPC_EINVAL, "lanes_per_cn must be 0, 1, 2 or 4");
    if (!c->lay[lanes_per_cn - 1].valid) return fail(LDPC_EUNSUPPORTED, "no kernel variant with that mapping");
    c->lanes_for[kind] = lanes_per_cn;
    return LDPC_OK;
}

int ldpc_decode(ldpc_code_t c, const float* llr, int32_t num_frames, int32_t max_iter, uint32_t flags,
                uint8_t* hard, float* post, int32_t* iters, uint8_t* syn_ok, void* hip_stream) {
    return ndgsbp::decode_enqueue(c, llr, num_frames, max_iter, flags, hard, post, iters, syn_ok, nullptr,
                                  hip_stream);
}

int ldpc_batch_create(const ldpc_problem* probs, int32_t count, uint32_t flags, const ldpc_batch_options* opt,
                      ldpc_batch_t* out) {
    g_last_error.clear();
    if (!out) return fail(LDPC_EINVAL, "out is NULL");
    *out = nullptr;
    int rc = check_flags(flags);
    if (rc) return rc;
    ldpc_batch_options o = default_batch_options();
    if (opt) o = *opt;
    rc = check_options(o);
    if (rc) return rc;
    if (flags & LDPC_FLAG_TIER_HBM) return fail(LDPC_EUNSUPPORTED, "batches run the LDS tier only");
    const MsgKind kind = msg_kind(flags);
    ClassPlan plan;
    rc = form_classes(probs, count, kind, o, plan);
    if (rc) return rc;

    ldpc_batch* b = new (std::nothrow) ldpc_batch();
    if (!b) return fail(LDPC_ENOMEM, "host allocation failed");
    b->device = plan.device;
    b->kind = kind;
    b->num_problems = count;
    b->total_frames = plan.total_frames;
    b->classes = std::move(plan.classes);
    if (b->classes.empty()) {
        *out = b;
        return LDPC_OK;
    }
    DeviceGuard guard(b->device);
    if (!guard.ok) {
        delete b;
        return fail(LDPC_EHIP, "cannot select the batch's device");
    }
    for (BatchClass& bc : b->classes) {
        rc = set_blocks(kind, bc.key.D, bc.key.uniform, true, plan.num_cus, bc.total_frames, bc.shape);
        if (rc) {
            delete b;
            return rc;
        }
    }
    hipError_t e = upload(&b->table, plan.table);
    if (e == hipSuccess) e = hipMalloc((void**)&b->work, 2 * sizeof(uint32_t) * b->classes.size());
    if (e == hipSuccess) e = hipMemset(b->work, 0, 2 * sizeof(uint32_t) * b->classes.size());
    const int nstreams = std::min<int>(std::max(1, o.streams), (int)b->classes.size());
    for (int k = 1; k < nstreams && e == hipSuccess; ++k) {
        hipStream_t st = nullptr;
        e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
        if (e == hipSuccess) b->streams.push_back(st);
    }
    for (int k = 0; k < nstreams && e == hipSuccess; ++k) {
        hipEvent_t ev = nullptr;
        e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
        if (e == hipSuccess) b->events.push_back(ev);
    }
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) {
        free_batch(b);
        delete b;
        return hip_fail(e, "batch tables");
    }
    for (size_t k = 0; k < b->classes.size(); ++k)
        finish_class_args(b->classes[k], plan.table, b->table, b->work + 2 * k, flags);
    *out = b;
    return LDPC_OK;
}

int ldpc_batch_query(ldpc_batch_t b, ldpc_batch_info* info) {
    g_last_error.clear();
    if (!b || !info) return fail(LDPC_EINVAL, "batch or info is NULL");
    info->num_launches = (int32_t)b->classes.size();
    info->num_problems = b->num_problems;
    info->num_streams = (int32_t)b->streams.size() + 1;
    info->total_frames = b->total_frames;
    return LDPC_OK;
}

int ldpc_batch_launch(ldpc_batch_t b, void* hip_stream) {
    g_last_error.clear();
    if (!b) return fail(LDPC_EINVAL, "batch is NULL");
    if (b->classes.empty()) return LDPC_OK;
    DeviceGuard guard(b->device);
    if (!guard.ok) return fail(LDPC_EHIP, "cannot select the batch's device");
    hipError_t e = launch_classes(b->classes, b->kind, (hipStream_t)hip_stream, b->streams, b->events);
    if (e != hipSuccess) return hip_fail(e, "batch launch");
    return LDPC_OK;
}

int ldpc_batch_destroy(ldpc_batch_t b) {
    g_last_error.clear();
    if (!b) return LDPC_OK;
    if (b->table || b->work || !b->streams.empty() || !b->events.empty()) {
        DeviceGuard guard(b->device);
        free_batch(b);
    }
    delete b;
    return LDPC_OK;
}

int ldpc_decode_batched(const ldpc_problem* probs, int32_t count, uint32_t flags, void* hip_stream) {
    g_last_error.clear();
    int rc = check_flags(flags);
    if (rc) return rc;
    if (flags & LDPC_FLAG_TIER_HBM) return fail(LDPC_EUNSUPPORTED, "batches run the LDS tier only");
    const MsgKind kind = msg_kind(flags);
    const ldpc_batch_options o = default_batch_options();
    ClassPlan plan;
    rc = form_classes(probs, count, kind, o, plan);
    if (rc) return rc;
    if (plan.classes.empty()) return LDPC_OK;
    if (plan.classes.size() > (size_t)kStageClasses)
        return fail(LDPC_EUNSUPPORTED, "more than " + std::to_string(kStageClasses) + " launch classes in one call");
    DeviceGuard guard(plan.device);
    if (!guard.ok) return fail(LDPC_EHIP, "cannot select the problems' device");
    for (BatchClass& bc : plan.classes) {
        rc = set_blocks(kind, bc.key.D, bc.key.uniform, true, plan.num_cus, bc.total_frames, bc.shape);
        if (rc) return rc;
    }
    DeviceStage* ds = nullptr;
    hipError_t e = get_stage(plan.device, &ds);
    if (e != hipSuccess) return hip_fail(e, "staging ring");
    hipStream_t main = (hipStream_t)hip_stream;
    std::lock_guard<std::mutex> lock(ds->mu);
    StageSlot& slot = ds->slots[ds->next++ % kStageRing];
    // the slot's previous call must be done with its buffers
    if (slot.in_use) {
        e = hipEventSynchronize(slot.done);
        if (e != hipSuccess) return hip_fail(e, "staging slot wait");
    }
    e = reserve_slot(slot, plan.table.size());
    if (e != hipSuccess) return hip_fail(e, "staging slot");
    std::memcpy(slot.host, plan.table.data(), plan.table.size() * sizeof(Problem));
    e = hipMemcpyAsync(slot.dev, slot.host, plan.table.size() * sizeof(Problem), hipMemcpyHostToDevice, main);
    for (size_t k = 0; k < plan.classes.size(); ++k)
        finish_class_args(plan.classes[k], plan.table, slot.dev, slot.work + 2 * k, flags);
    const int ns = std::min<int>(kStageStreams, (int)plan.classes.size());
    std::vector<hipStream_t> extra(slot.streams.begin(), slot.streams.begin() + (ns - 1));
    std::vector<hipEvent_t> evs(slot.fork_join.begin(), slot.fork_join.begin() + ns);
    if (e == hipSuccess) e = launch_classes(plan.classes, kind, main, extra, evs);
    if (e == hipSuccess) e = hipEventRecord(slot.done, main);
    slot.in_use = true;
    if (e != hipSuccess) return hip_fail(e, "batched decode");
    return LDPC_OK;
}

}  // extern "C"
