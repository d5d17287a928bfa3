/*
 * ndgsbp.h - C ABI of the MI355X (gfx950) NDGSBP LDPC decoder.
 *
 * Method: non-disjoint group-shuffled belief propagation (Hsu, Chang, Su,
 * Weng, "A Non-Disjoint Group Shuffled Decoding for LDPC Codes"). The check
 * nodes (CNs) of H are split into groups that may share CNs (Sec. II-A);
 * each iteration visits the groups in order, and for each group runs the CN
 * update of eq. (1) for every CN of the group followed by the VN update of
 * eq. (2) for every VN the group touches (Sec. II-C, Step 2). After every
 * iteration the total LLR of eq. (3) gives hard decisions whose syndrome
 * may stop the decode (Steps 3-4).
 *
 * Conventions for every entry point:
 *   - returns LDPC_OK (0) or a negative LDPC_E* code; nothing is thrown
 *     across the ABI; ldpc_last_error() gives a thread-local message;
 *   - "host" pointers are read during the call only; "device" pointers
 *     must be device memory of the code's device and stay valid until the
 *     enqueued work completes;
 *   - decode calls are asynchronous on the caller's HIP stream (NULL = the
 *     legacy default stream); argument errors are reported synchronously,
 *     launch errors through the return code of the call that enqueued them.
 */
#ifndef NDGSBP_H
#define NDGSBP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LDPC_OK 0
#define LDPC_EINVAL (-1)       /* malformed argument, H or grouping      */
#define LDPC_ENOMEM (-2)       /* device or host allocation failed       */
#define LDPC_EHIP (-3)         /* a HIP runtime call failed              */
#define LDPC_EUNSUPPORTED (-4) /* valid, but beyond every kernel variant */

#define LDPC_GROUPS_WINDOWS 0
#define LDPC_GROUPS_EXPLICIT 1
#define LDPC_GROUPS_VN 2 /* VN groups: the vertical shuffled schedule (a baseline) */

#define LDPC_FLAG_EARLY_STOP 0x1u /* stop a frame at its first zero syndrome (Step 4b) */
#define LDPC_FLAG_MSG_FP16 0x2u   /* store CN->VN messages as IEEE binary16           */
#define LDPC_FLAG_MSG_BF16 0x4u   /* store CN->VN messages as bfloat16                */
#define LDPC_FLAG_OUT_PACKED 0x8u /* hard decisions 8 per byte: see ldpc_decode        */
#define LDPC_FLAG_TIER_HBM 0x10u  /* ldpc_decode: HBM tier even if the code fits LDS    */

typedef struct ldpc_code* ldpc_code_t;

/* Parity-check matrix H (M x N, Sec. II-B) in CSR form, host memory.
 * Row i lists N(i): col_idx[row_ptr[i] .. row_ptr[i+1]), each VN at most
 * once per row. row_ptr[0] = 0, row_ptr[m] = nnz. */
typedef struct {
    int32_t m;
    int32_t n;
    int64_t nnz;
    const int32_t* row_ptr; /* host, m + 1 entries */
    const int32_t* col_idx; /* host, nnz entries   */
} ldpc_h_csr;

/* CN grouping (Sec. II-A, Step 1), processed in this order every iteration
 * (or, with groups_per_iteration, a new grouping every iteration).
 * WINDOWS: group g = CNs start_g .. start_g + len_g - 1 with
 *   start_g = floor(g*m/G), len_g = start_{g+1} - start_g + overlap,
 *   indices mod m when wrap != 0 (the last window then overlaps the first);
 *   with wrap == 0 the last window ends at m.
 * EXPLICIT: group g = group_cn[group_ptr[g] .. group_ptr[g+1]) (host).
 *   groups_per_iteration = Gp > 0 splits the groups into R = num_groups / Gp
 *   blocks; iteration l (from 1) processes block (l - 1) mod R, so each
 *   iteration can use a fresh grouping (Step 4 returns to Step 1). 0: all
 *   groups every iteration. Decodes with R > 1 run in the LDS tier only.
 * Every CN must appear in some group (of every block) and at most once
 * within a group.
 * VN: the vertical group-shuffled schedule that Sec. I cites as prior art,
 *   for comparison: group_ptr/group_cn list VN ids, each VN in exactly one
 *   group; for group g, every CN->VN message into its VNs is computed from
 *   the VN->CN messages as they stood before the group (eq. (1)), then
 *   those VNs' posteriors are updated (eq. (2)-(3)). One grouping for every
 *   iteration; LDS tier only; not in batches; FP32 or FP16 messages. */
typedef struct {
    int32_t kind;
    int32_t num_groups;
    int32_t overlap;           /* WINDOWS only */
    int32_t wrap;              /* WINDOWS only */
    const int32_t* group_ptr;  /* EXPLICIT and VN, host, num_groups + 1 */
    const int32_t* group_cn;   /* EXPLICIT (CN ids) and VN (VN ids), host */
    int32_t groups_per_iteration; /* EXPLICIT only; 0 = num_groups   */
} ldpc_grouping;

/* Sizes of a created code, for callers that size buffers or count work. */
typedef struct {
    int32_t m, n;
    int64_t nnz;
    int32_t num_groups;
    int64_t cn_visits;       /* CN updates per iteration (mean over blocks)   */
    int64_t edge_updates;    /* edge updates per iteration (mean over blocks) */
    int32_t max_cn_degree;
    int32_t max_vn_degree;
    int32_t device;
    int64_t lds_bytes_fp32;  /* per-frame LDS of the FP32-message kernel      */
    int64_t lds_bytes_16;    /* per-frame LDS of the FP16-message kernel      */
    int64_t lds_limit;       /* LDS per workgroup on the device; codes above
                                it decode in the HBM tier                     */
    int32_t lanes_fp32;      /* lanes per CN visit (1, 2, 4) with FP32 messages */
    int32_t lanes_fp16;      /* ... with FP16 messages                        */
    int32_t lanes_bf16;      /* ... with BF16 messages                        */
    int32_t groups_per_iteration;
} ldpc_code_info;

/* Validate H and the grouping, build the device tables and upload them to
 * `device`. On success *out owns them until ldpc_code_destroy. Apart from
 * ldpc_code_tune the handle is read-only and may be used from any thread and
 * stream.
 * Errors: EINVAL (bad CSR, VN out of range, duplicate VN in a row, CN out
 * of range or repeated within a group, CN in no group, window longer than
 * m), EUNSUPPORTED (n > 65533, CN degree > 32), ENOMEM, EHIP. */
int ldpc_code_create(const ldpc_h_csr* H, const ldpc_grouping* grouping, int32_t device,
                     ldpc_code_t* out);

/* Free the device tables. The caller guarantees that no enqueued decode
 * still uses the code. NULL is accepted. */
int ldpc_code_destroy(ldpc_code_t code);

int ldpc_code_query(ldpc_code_t code, ldpc_code_info* info);

/* Choose the CN-phase mapping of later decodes of `code` with the message
 * format in msg_flags (0, LDPC_FLAG_MSG_FP16 or LDPC_FLAG_MSG_BF16): one lane
 * per CN visit (1), or two or four lanes sharing it (2, 4; the padded degree
 * is then a multiple of the lane count); 0 restores the built-in choice
 * (made at create from the device's LDS size and the occupancy of each
 * mapping's kernel, per message format; any of 1, 2, 4). For tuners: the mappings compute eq. (1) with the same operations
 * in a different summation order, so results agree up to float rounding.
 * Not synchronised with decodes in flight on other threads.
 * Errors: EINVAL (bad flags or value), EUNSUPPORTED (no kernel variant
 * with that mapping for the code's CN degree). */
int ldpc_code_tune(ldpc_code_t code, uint32_t msg_flags, int32_t lanes_per_cn);

/* Decode num_frames frames (Sec. II-C, Steps 2-4).
 *   llr    device, float [num_frames][n]: channel LLRs L_n = 2 y_n / sigma^2
 *   hard   device, uint8 [num_frames][n]: d_n = 1 iff total LLR < 0 (Step 4a);
 *          with LDPC_FLAG_OUT_PACKED uint8 [num_frames][(n + 7) / 8], bit k of
 *          byte q = d_{8q+k}, bits past n zero
 *   post   device, float [num_frames][n]: total LLR of eq. (3), or NULL
 *   iters  device, int32 [num_frames]: iterations run, in [1, max_iter]
 *   syn_ok device, uint8 [num_frames]: 1 iff D H^T = 0 at the end, or NULL
 * Messages start at L_{m->n} = 0. CN updates inside a group all read the
 * messages as they stood before the group. With LDPC_FLAG_EARLY_STOP a frame
 * stops after the first iteration whose syndrome is zero; otherwise every
 * frame runs max_iter iterations. At most one of MSG_FP16 / MSG_BF16.
 * Tiers: a frame's posteriors and messages stay in LDS for its whole decode
 * when they fit (lds_bytes_* <= lds_limit); otherwise (or with
 * LDPC_FLAG_TIER_HBM) they live in a frame-interleaved workspace in device
 * memory that the code allocates on first use and grows when a larger launch
 * needs it (the one case in which ldpc_decode allocates); HBM-tier decodes
 * of one code run one after another on the device (each waits for the
 * previous one). Both tiers compute the same values: the HBM tier equals the
 * LDS tier with one lane per CN visit, bit for bit.
 * Each call takes the next of 1024 work counters of the code (a ring, reset
 * on the device by the call's last workgroup): at most 1024 decodes of one
 * code may be executing at the same time (calls on one stream never
 * overlap).
 * Errors: EINVAL (NULL code/llr/hard/iters, num_frames < 0, max_iter < 1,
 * bad flags), EUNSUPPORTED (no kernel variant fits the code), ENOMEM (HBM
 * workspace), EHIP. */
int ldpc_decode(ldpc_code_t code, const float* llr, int32_t num_frames, int32_t max_iter,
                uint32_t flags, uint8_t* hard, float* post, int32_t* iters, uint8_t* syn_ok,
                void* hip_stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the same
 * decode as ldpc_decode, same arguments, results and errors, bit for bit
 * equal to it, but it allocates nothing. Its kernels take their work
 * counter and, in the HBM tier, their workspace from one fixed device array
 * of 64 MiB per GPU that the library holds from the first ldpc_code_create
 * on that GPU until the process ends (bytes 0..255 the counters, the rest
 * the workspace). HBM-tier decodes run as many 64-frame tiles at once as
 * the array holds; a code one of whose tiles does not fit (e.g. n = 65000
 * with four edges per VN and FP32 messages) is refused with
 * LDPC_EUNSUPPORTED. Every call on a GPU shares that GPU's array and leaves
 * its contents behind: calls on one stream are ordered, but calls that
 * overlap on one GPU (other streams, other threads) race and give wrong
 * results. Each call clears the counters with a small kernel on hip_stream
 * before the decode, so it needs no memset and may be captured. */
int ldpc_decode_noalloc(ldpc_code_t code, const float* llr, int32_t num_frames, int32_t max_iter,
                        uint32_t flags, uint8_t* hard, float* post, int32_t* iters, uint8_t* syn_ok,
                        void* hip_stream);

/* ---- Batched decoding: many problems (codes, frame counts) per launch ----
 *
 * A batch decodes every frame of every problem with the schedule of
 * ldpc_decode (Sec. II-C, Steps 2-4), each problem with its own code,
 * grouping and iteration cap; the results of a problem equal those of
 * ldpc_decode on it alone with the same message format and CN-lane mapping
 * (bit for bit: the same arithmetic runs per frame). Problems are split into
 * launch classes (kernel variant, optionally LDS size); each class is one
 * persistent launch whose workgroups take frames of any of its problems from
 * one work counter, and the classes run concurrently on forked streams. */
typedef struct ldpc_batch* ldpc_batch_t;

/* One problem. Buffers as in ldpc_decode (device memory of the code's
 * device, [num_frames][n] frame-major); num_frames may be 0. */
typedef struct {
    ldpc_code_t code;
    const float* llr;
    int32_t num_frames;
    int32_t max_iter;
    uint8_t* hard;
    float* post;     /* or NULL */
    int32_t* iters;
    uint8_t* syn_ok; /* or NULL */
} ldpc_problem;

/* Launch choices of a batch (the autotuner's knobs). */
typedef struct {
    int32_t lanes_per_cn;  /* 0: each code's mapping for the message format
                              (ldpc_code_tune); 1, 2 or 4: that mapping for
                              all                                           */
    int32_t split_by_size; /* nonzero: one launch per power-of-two LDS size
                              within a kernel variant (workgroups sized for
                              their problems); 0: one launch per variant    */
    int32_t max_threads;   /* workgroup size cap, multiple of 64, <= 1024;
                              0: the size that gives every CN visit of the
                              largest group its own lanes                   */
    int32_t streams;       /* launch classes run on up to this many streams
                              at once (1..8; 0 = 1)                          */
} ldpc_batch_options;

typedef struct {
    int32_t num_launches;
    int32_t num_problems;
    int32_t num_streams;
    int64_t total_frames;
} ldpc_batch_info;

/* Validate the problems, form the launch classes and upload the problem
 * table to the codes' device. Pointers in `probs` are copied: the codes and
 * buffers must stay valid while the batch is launched; `probs` itself is
 * read during the call only. opt NULL = {0, 1, 0, 4}. flags as in
 * ldpc_decode, for every problem. Synchronous.
 * Errors: EINVAL (NULL code or required buffer, negative frames, max_iter
 * < 1, codes on different devices, bad flags or options), EUNSUPPORTED (a
 * code beyond every kernel variant, more than 2^31 - 1 frames in a class),
 * ENOMEM, EHIP. */
int ldpc_batch_create(const ldpc_problem* probs, int32_t count, uint32_t flags,
                      const ldpc_batch_options* opt, ldpc_batch_t* out);

/* Enqueue the batch on hip_stream (and on the batch's own streams, forked
 * from and joined back into hip_stream): asynchronous, no allocation, no
 * host synchronisation and no memset, so it may be captured into a HIP
 * graph. Launches of one batch must not overlap in time (they share its
 * work counters): keep them on one stream or otherwise ordered. */
int ldpc_batch_launch(ldpc_batch_t batch, void* hip_stream);

int ldpc_batch_query(ldpc_batch_t batch, ldpc_batch_info* info);

/* The caller guarantees that no enqueued launch still uses the batch. */
int ldpc_batch_destroy(ldpc_batch_t batch);

/* One-shot form with default options, asynchronous on hip_stream like
 * ldpc_decode: the problem table is staged through a per-device ring of 16
 * pinned-host/device slots that the library keeps for the life of the
 * process, so a call allocates nothing once its slot is large enough (the
 * 17th call in flight waits on the host for the 1st to finish). Each slot
 * has its own streams for the launch classes it forks from hip_stream, so
 * calls in flight at once on different caller streams do not wait behind
 * each other's classes. At most 64 launch classes per call. Not for graph
 * capture (use ldpc_batch_launch).
 * Errors: as ldpc_batch_create, plus EUNSUPPORTED for too many classes. */
int ldpc_decode_batched(const ldpc_problem* probs, int32_t count, uint32_t flags, void* hip_stream);

/* Message of the last failed call on this thread ("" if none). */
const char* ldpc_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* NDGSBP_H */
