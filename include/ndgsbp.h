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

#define LDPC_FLAG_EARLY_STOP 0x1u /* stop a frame at its first zero syndrome (Step 4b) */
#define LDPC_FLAG_MSG_FP16 0x2u   /* store CN->VN messages as IEEE binary16           */
#define LDPC_FLAG_MSG_BF16 0x4u   /* store CN->VN messages as bfloat16                */

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

/* CN grouping (Sec. II-A, Step 1), processed in this order every iteration.
 * WINDOWS: group g = CNs start_g .. start_g + len_g - 1 with
 *   start_g = floor(g*m/G), len_g = start_{g+1} - start_g + overlap,
 *   indices mod m when wrap != 0 (the last window then overlaps the first);
 *   with wrap == 0 the last window ends at m.
 * EXPLICIT: group g = group_cn[group_ptr[g] .. group_ptr[g+1]) (host).
 * Every CN must appear in some group and at most once within a group. */
typedef struct {
    int32_t kind;
    int32_t num_groups;
    int32_t overlap;           /* WINDOWS only */
    int32_t wrap;              /* WINDOWS only */
    const int32_t* group_ptr;  /* EXPLICIT only, host, num_groups + 1 */
    const int32_t* group_cn;   /* EXPLICIT only, host                 */
} ldpc_grouping;

/* Sizes of a created code, for callers that size buffers or count work. */
typedef struct {
    int32_t m, n;
    int64_t nnz;
    int32_t num_groups;
    int64_t cn_visits;       /* sum of group sizes: CN updates per iteration  */
    int64_t edge_updates;    /* sum of CN degrees over all visits             */
    int32_t max_cn_degree;
    int32_t max_vn_degree;
    int32_t device;
    int64_t lds_bytes_fp32;  /* per-frame LDS of the FP32-message kernel      */
    int64_t lds_bytes_16;    /* per-frame LDS of the FP16-message kernel      */
    int32_t lanes_fp32;      /* lanes per CN visit used with FP32 messages    */
    int32_t lanes_fp16;      /* ... with FP16 messages                        */
    int32_t lanes_bf16;      /* ... with BF16 messages                        */
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
 * per CN visit (1) or two lanes sharing it (2); 0 restores the built-in
 * choice. For tuners: the mappings compute eq. (1) with the same operations
 * in a different summation order, so results agree up to float rounding.
 * Not synchronised with decodes in flight on other threads.
 * Errors: EINVAL (bad flags or value), EUNSUPPORTED (no kernel variant
 * with that mapping for the code's CN degree). */
int ldpc_code_tune(ldpc_code_t code, uint32_t msg_flags, int32_t lanes_per_cn);

/* Decode num_frames frames (Sec. II-C, Steps 2-4).
 *   llr    device, float [num_frames][n]: channel LLRs L_n = 2 y_n / sigma^2
 *   hard   device, uint8 [num_frames][n]: d_n = 1 iff total LLR < 0 (Step 4a)
 *   post   device, float [num_frames][n]: total LLR of eq. (3), or NULL
 *   iters  device, int32 [num_frames]: iterations run, in [1, max_iter]
 *   syn_ok device, uint8 [num_frames]: 1 iff D H^T = 0 at the end, or NULL
 * Messages start at L_{m->n} = 0. CN updates inside a group all read the
 * messages as they stood before the group. With LDPC_FLAG_EARLY_STOP a frame
 * stops after the first iteration whose syndrome is zero; otherwise every
 * frame runs max_iter iterations. At most one of MSG_FP16 / MSG_BF16.
 * Errors: EINVAL (NULL code/llr/hard/iters, num_frames < 0, max_iter < 1,
 * bad flags), EUNSUPPORTED (no kernel variant fits the code), EHIP. */
int ldpc_decode(ldpc_code_t code, const float* llr, int32_t num_frames, int32_t max_iter,
                uint32_t flags, uint8_t* hard, float* post, int32_t* iters, uint8_t* syn_ok,
                void* hip_stream);

/* Message of the last failed call on this thread ("" if none). */
const char* ldpc_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* NDGSBP_H */
