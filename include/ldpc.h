/*
 * ldpc.h -- C ABI of the single-scan min-sum LDPC decoder for AMD Instinct
 * MI355X (gfx950).
 *
 * Method: X. Huang, "Single-Scan Min-Sum Algorithms for Fast Decoding of LDPC
 * Codes", ITW 2006.  The library decodes binary LDPC codes with normalised /
 * offset min-sum (Sec. III) in the single-scan form of Sec. IV (Eq. 3): each
 * iteration is one pass over the check-to-variable addressing that rebuilds
 * the variable-to-check message as Z_{n'} - L_{mn'} and accumulates the new
 * posteriors Z_n in the same pass.  Messages can be 6-bit fixed point (int8),
 * the compressed "1-bit" form of Sec. V (a sign bit per edge plus A_m, B_m and
 * the position n~_m per check), or binary32.  The standard two-scan schedule
 * (Sec. III, Eqs. 1-2) is available as a baseline.
 *
 * Conventions
 *  - All functions are plain C, thread-safe for distinct handles, and return
 *    an ldpc_status; on failure ldpc_last_error() gives a message (per thread).
 *  - "host" pointers are ordinary CPU memory; "device" pointers are GPU memory
 *    on the device the code was created for (e.g. from hipMalloc or a torch
 *    tensor).  The library never takes ownership of caller buffers.
 *  - Layouts are row-major; [F][N] means frame-major, N contiguous values per
 *    frame.
 */
#ifndef LDPC_H
#define LDPC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ldpc_code ldpc_code; /* opaque, owned by the library */

typedef enum {
    LDPC_OK = 0,
    LDPC_EINVAL = 1,        /* bad argument (null pointer, range, size) */
    LDPC_EBADCODE = 2,      /* parity-check matrix rejected */
    LDPC_ENOMEM = 3,        /* device or host allocation failed */
    LDPC_EDEVICE = 4,       /* HIP runtime error (launch, copy, device) */
    LDPC_EUNSUPPORTED = 5   /* valid request with no kernel for it */
} ldpc_status;

/* Message representation (Sec. V uses b = 6..8 bit fixed point). */
typedef enum {
    LDPC_MSG_FP32 = 0, /* binary32 messages and posteriors */
    LDPC_MSG_INT8 = 1, /* b-bit fixed point held in int8 (b = msg_bits, default 6: extrinsics
                          saturated to +-31) */
    LDPC_MSG_1BIT = 2  /* Sec. V: per-edge sign bit + per-check (A, B, n~), 6-bit values */
} ldpc_msg;

typedef enum {
    LDPC_SINGLE_SCAN = 0, /* Sec. IV, Eq. (3) (and Sec. V for LDPC_MSG_1BIT) */
    LDPC_TWO_SCAN = 1     /* Sec. III, Eqs. (1)-(2): baseline; FP32 and INT8 only */
} ldpc_sched;

/* flags */
#define LDPC_F_CHECK_INPUT 0x1u /* validate llr_in on the device first (synchronises the stream) */
#define LDPC_F_LAYOUT_SHIFT 8   /* bits 8..11: force a layout (LDPC_LAYOUT_*), 0 = automatic */
#define LDPC_LAYOUT_AUTO 0
#define LDPC_LAYOUT_LDS 1       /* messages in LDS (must fit) */
#define LDPC_LAYOUT_HBM 2       /* messages in the caller's workspace (device memory) */
#define LDPC_LAYOUT_REG 3       /* messages in registers, one workgroup per frame (single-scan
                                   INT8/1BIT; codes with an instantiated shape, see
                                   ldpc_code_info.reg_* / pk_*); INT8 and 1BIT use the packed
                                   two-rows-per-lane kernel (pk_threads per workgroup) when it
                                   has a shape, else the one-row
                                   kernel (1024 threads).  AUTO picks, for fixed point: the
                                   packed kernel from 16 rows per thread (M > 8192; 1BIT from
                                   8 rows per thread), for rows
                                   wider than 8 slots (INT8) and with 256-thread shapes for
                                   small codes; the one-row register kernel otherwise; the
                                   LDS-resident kernels for the remaining codes with M <= 1024 */
#define LDPC_LAYOUT_REG1 4      /* as LDPC_LAYOUT_REG, one row at a time (no packing) */
#define LDPC_LAYOUT_FRAMES 5    /* single-scan FP32 and the two-scan baseline (INT8, FP32):
                                   frames across the lanes of a wavefront, messages and
                                   posteriors in the caller's workspace (frame-minor, so every
                                   access is a whole-wavefront line); each lane takes four
                                   consecutive frames once a call chunk holds 256 frames and
                                   rows have at most 16 entries, otherwise one frame per
                                   lane.  AUTO takes it for these
                                   paths when their per-edge arrays do not fit in LDS.  The
                                   workspace then covers the whole call and depends on
                                   max_iter: ask ldpc_decode_workspace_size() */

/*
 * Decoding parameters (Sec. III: normalisation lambda_k = alpha, offset
 * beta_k = beta, both constant over iterations; iteration cap max_iter).
 *  alpha      in (0, 1]; |L| = max(alpha * m - beta, 0) where m is the
 *             check-node minimum (alpha = 1, beta = 0: plain min-sum).
 *  beta       >= 0, in LLR units.
 *  llr_step   LLR value of one fixed-point unit for INT8 / 1BIT (0.5 for the
 *             6-bit range +-15.5).  Fixed point uses a8 = round(256 alpha),
 *             b = round(min(beta / llr_step, 255)) (half away from zero; 255
 *             steps already zero every message) and
 *             |L| = max(((m*a8 + 128) >> 8) - b, 0).
 *  early_stop nonzero: stop a frame after the first iteration k >= 1 whose
 *             hard decision satisfies H x^T = 0 (Sec. III decoding step).
 *  weights    NULL, or device float32 [weight_iters][C][2]: per iteration k
 *             (row min(k, weight_iters) - 1) and check-degree class c the
 *             pair (a, b) replacing (alpha, beta) (Sec. III indexes lambda
 *             and beta by the iteration).  C is set by weight_classes.
 *             FP32 single-scan takes either form (it then runs frames across
 *             lanes); fixed-point single-scan (INT8, 1BIT, every layout but
 *             FRAMES) takes one pair per iteration, converted per iteration
 *             like alpha and beta: a8 = round(256 a), b = round(b / llr_step),
 *             clamped to [0, 256] and [0, 255] (pairs are device data and are
 *             not validated; keep 0 < a <= 1, b >= 0 for the method's
 *             meaning).  Two-scan returns LDPC_EUNSUPPORTED.
 *  weight_iters rows of `weights` (>= 1 when weights is set).
 *  weight_classes 0: C = the code's check-degree classes (the distinct row
 *             degrees ascending, see ldpc_learn.h; FP32 only unless the code
 *             has one class); 1: C = 1, one pair per iteration for all rows.
 *  msg_bits   fixed-point message width b of Sec. V: 0 or 6 (default), 7 or 8.
 *             Extrinsics saturate to Q = 2^(b-1) - 1 (31, 63, 127) and INT8
 *             inputs range over [-Q, Q] in units of llr_step.  7 and 8 bits:
 *             INT8 single-scan on the LDS/HBM kernel only (AUTO picks it;
 *             REG, REG1 and FRAMES return LDPC_EUNSUPPORTED); 1BIT and
 *             two-scan are 6-bit only.  Ignored for FP32 when 0 or 6.
 */
typedef struct {
    int32_t max_iter;
    float alpha;
    float beta;
    int32_t early_stop;
    int32_t msg;   /* ldpc_msg */
    int32_t sched; /* ldpc_sched */
    float llr_step;
    uint32_t flags;
    const float *weights;
    int32_t weight_iters;
    int32_t weight_classes;
    int32_t msg_bits;
} ldpc_decode_params;

/* Facts about a code handle and its planned device layouts. */
typedef struct {
    int32_t M, N;
    int64_t E;                  /* nonzeros of H (edges of the Tanner graph) */
    int32_t min_row_deg, max_row_deg, max_col_deg;
    int32_t slots_per_row;      /* padded row width used on the device */
    int32_t rows_padded;        /* rows rounded up to a multiple of 64 */
    int32_t device;
    int64_t addr_bytes_single;  /* check-to-variable addressing (all single-scan kernels) */
    int64_t addr_bytes_two;     /* plus the variable-to-check index (two-scan, FP32 sum) */
    int64_t msg_bits_int8;      /* b * E with b = 8 (int8 message store, Sec. V) */
    int64_t msg_bits_1bit;      /* E sign bits + M * (5 + 5 + ceil(log2 d_c)) state bits */
    int32_t lds_bytes_per_cu;   /* LDS available to one workgroup on this device */
    int32_t reg_slots;          /* register-resident shape: slots per row (0 = none) */
    int32_t reg_rows_per_thread;
    int32_t reg_zpack;          /* posterior accumulator fields per 32-bit LDS word */
    int32_t pk_slots;           /* packed (two rows per lane) shape: slots per lane (0 = none);
                                   rows longer than that span a lane pair (max_row_deg
                                   > pk_slots: each lane holds half of every row) */
    int32_t pk_rows_per_thread; /* rows per thread, or per lane pair when rows span two */
    int32_t pk_threads;         /* threads per workgroup (one frame) of the packed kernel */

    /* Degree distributions (Sec. II: |N(m)| and |M(n)|): row_deg_hist[d] rows
     * of degree d (d <= 64, the largest accepted); col_deg_hist[d] columns of
     * degree d for d < 64, col_deg_hist[64] columns of degree 64 or more. */
    int32_t row_deg_hist[65];
    int32_t col_deg_hist[65];

    /* Structure found in H (bit set of LDPC_STRUCT_*; 0 = none found). */
    int32_t structure;
    int32_t qc_lift;            /* LDPC_STRUCT_QC: the largest Z >= 2 for which H is an array of
                                   Z x Z blocks, each empty or one circulant permutation */
    int32_t ira_group;          /* LDPC_STRUCT_IRA_GROUPS: the largest Q for which information
                                   column j of every group of Q columns hits the rows of the
                                   group's first column shifted by j * M / Q (mod M); 0 if none */
    int32_t reserved;           /* 0 */

    /* Per-frame storage of the stored values each form keeps (Secs. IV-V):
     *  var_values_single  N: one posterior Z_n per variable (single-scan)
     *  var_values_two     E = N x mean column degree: one Z_mn per edge (two-scan)
     * and bytes per frame of each message type's per-edge / per-check state
     * and of the posteriors, as the library stores them: */
    int64_t var_values_single;
    int64_t var_values_two;
    int64_t msg_bytes_int8;     /* E: one b-bit message (b = 6..8) per byte */
    int64_t msg_bytes_1bit;     /* ceil(E / 8) sign bytes + 2 M bytes of (A, B, n~) state */
    int64_t msg_bytes_fp32;     /* 4 E */
    int64_t post_bytes_int;     /* 2 N: one int16 posterior per variable */
    int64_t post_bytes_fp32;    /* 4 N */
    /* Bytes per frame and iteration that a decoder streaming every per-frame
     * array through device memory moves (the algorithmic traffic model):
     * single-scan int8 2E + 5N (messages read and written, Z_old read and
     * Z_new written as int16, Z(0) read), 1-bit 2 ceil(E/8) + 4M + 5N,
     * binary32 8E + 12N; two-scan int8 4E + 3N, two-scan binary32 16E + 8N. */
    int64_t stream_bytes_int8;
    int64_t stream_bytes_1bit;
    int64_t stream_bytes_fp32;
    int64_t stream_bytes_two_int8;
    int64_t stream_bytes_two_fp32;
} ldpc_code_info;

/* ldpc_code_info.structure bits */
#define LDPC_STRUCT_QC 0x1         /* circulant-permutation blocks, lift qc_lift */
#define LDPC_STRUCT_IRA 0x2        /* the last M columns are a dual-diagonal staircase: column
                                      N - M + p hits rows p and p + 1 (the last one row M - 1) */
#define LDPC_STRUCT_IRA_GROUPS 0x4 /* and the information columns come in cyclic groups of
                                      ira_group columns (repeat-accumulate codes in the form of
                                      the DVB-S2 tables) */

/*
 * Create a code handle from a sparse parity-check matrix H (M x N over GF(2),
 * Sec. II) in CSR form.
 *  row_ptr  host, M+1 entries, row_ptr[0] = 0, nondecreasing, row_ptr[M] = nnz.
 *  col_idx  host, nnz entries; row m lists N(m) in the order messages are
 *           indexed inside the check (ties of the 1-bit argmax go to the first).
 *  device   HIP device ordinal; the handle keeps its own device copies.  A
 *           negative ordinal makes a host-only handle (no device memory, LDS
 *           budget of one gfx950 CU) for queries and workspace sizing; decoding
 *           with it returns LDPC_EINVAL.
 * Rejected with LDPC_EBADCODE: a row of degree < 2 (the minimum over N(m)\n
 * would be empty), a repeated column inside a row, an index outside [0, N).
 * LDPC_EUNSUPPORTED: a row degree above 64.
 */
ldpc_status ldpc_code_create(int32_t M, int32_t N, int64_t nnz, const int32_t *row_ptr,
                             const int32_t *col_idx, int32_t device, ldpc_code **out);

/* Free a handle and its device memory.  NULL is accepted. */
ldpc_status ldpc_code_destroy(ldpc_code *code);

/* Fill *out with the facts above.  Host only; the structure is found once,
 * when the handle is created. */
ldpc_status ldpc_code_query(const ldpc_code *code, ldpc_code_info *out);

/*
 * Bytes of device workspace ldpc_decode_batch needs for n_frames frames with
 * these parameters (0 when every per-frame state fits in LDS).
 */
ldpc_status ldpc_decode_workspace_size(const ldpc_code *code, int32_t n_frames,
                                       const ldpc_decode_params *p, size_t *bytes);

/* The kernel a decode call runs (ldpc_plan_info.kernel). */
typedef enum {
    LDPC_KERNEL_GENERIC_INT = 0,    /* single-scan fixed point (Sec. IV-V), one workgroup per
                                       frame, one thread per row, messages in LDS or workspace */
    LDPC_KERNEL_GENERIC_F32 = 1,    /* single-scan binary32, one workgroup per frame */
    LDPC_KERNEL_TWO_SCAN = 2,       /* two-scan baseline (Sec. III), one workgroup per frame */
    LDPC_KERNEL_REG1 = 3,           /* single-scan fixed point, messages in registers, one row
                                       per lane */
    LDPC_KERNEL_PACKED = 4,         /* single-scan fixed point, messages in registers, two rows
                                       per lane (16-bit halves) */
    LDPC_KERNEL_F32_FRAMES = 5,     /* single-scan binary32, frames across lanes */
    LDPC_KERNEL_TWO_SCAN_FRAMES = 6 /* two-scan baseline, frames across lanes */
} ldpc_kernel;

typedef struct {
    int32_t kernel;          /* ldpc_kernel */
    int32_t layout;          /* the LDPC_LAYOUT_* value that forces this same plan */
    int32_t threads;         /* threads per workgroup of the decoding kernel */
    int32_t lds_bytes;       /* LDS per workgroup of the decoding kernel (0: none) */
    int32_t frames_per_lane; /* frames-across-lanes kernels: frames each lane decodes (1 or
                                4); 0 for the kernels with one workgroup per frame */
    int32_t reserved;        /* 0 */
    size_t workspace_bytes;  /* what ldpc_decode_workspace_size() returns for the same call */
} ldpc_plan_info;

/*
 * The plan ldpc_decode_batch would follow for n_frames frames with these
 * parameters (after AUTO and any layout pinned by ldpc_autotune).  Host only;
 * works with host-only handles.  Errors: as ldpc_decode_workspace_size (a
 * request with no kernel returns LDPC_EUNSUPPORTED); out NULL: LDPC_EINVAL.
 */
ldpc_status ldpc_decode_plan(const ldpc_code *code, int32_t n_frames, const ldpc_decode_params *p,
                             ldpc_plan_info *out);

/*
 * Decode n_frames frames (one parity-check matrix, Sec. III-V).
 *  llr_in      device [F][N]: float32 channel LLRs Z^(0) for LDPC_MSG_FP32;
 *              int8 fixed-point LLRs in [-Q, Q] (units of llr_step; Q = 31 for
 *              the default 6-bit messages) for INT8 and 1BIT (values outside
 *              are saturated).
 *  hard_out    device [F][N] uint8: x_n = 0 if Z_n > 0 else 1.
 *  llr_out     device [F][N] float32 posterior Z_n (fixed point: Z * llr_step,
 *              exact); may be NULL.
 *  iters_out   device [F] int32: iterations run (first k >= 1 whose decision is a
 *              codeword when early_stop, else max_iter; 0 if max_iter == 0).
 *  syndrome_ok device [F] uint8: 1 iff H x^T = 0 for the returned hard_out.
 *  workspace   device, at least ldpc_decode_workspace_size() bytes, 256-byte
 *              aligned; may be NULL when that size is 0.
 *  stream      hipStream_t (NULL = default stream).
 * The call is asynchronous on `stream`, allocates nothing and never
 * synchronises (except with LDPC_F_CHECK_INPUT).  Each frame's result depends
 * only on its own input.  max_iter = 0 returns the channel decisions.
 * Errors: LDPC_EINVAL for n_frames < 0, max_iter < 0, alpha outside (0, 1],
 * beta < 0, llr_step <= 0, a required NULL pointer, a small workspace,
 * weight_iters < 1 with weights, weight_classes outside {0, 1} or msg_bits
 * outside {0, 6, 7, 8}; LDPC_EUNSUPPORTED for LDPC_TWO_SCAN with
 * LDPC_MSG_1BIT, a forced layout that does not fit, weights or message
 * widths on a path that has no kernel for them (see above); LDPC_EDEVICE
 * for a failed launch.
 */
ldpc_status ldpc_decode_batch(const ldpc_code *code, int32_t n_frames, const void *llr_in,
                              const ldpc_decode_params *p, uint8_t *hard_out, float *llr_out,
                              int32_t *iters_out, uint8_t *syndrome_ok, void *workspace,
                              size_t workspace_bytes, void *stream);

/*
 * ldpc_decode_batch for callers that cannot allocate device memory (code
 * under HIP graph capture, serving loops, harnesses that forbid hipMalloc):
 * the same decode, with the workspace taken from a static device array of
 * LDPC_NOALLOC_SCRATCH_BYTES that the library holds on each GPU it runs on
 * until the process ends (its address is looked up once per device, when the
 * first handle on that device is created).  The caller still owns every
 * input and output buffer.  Calls no hipMalloc, hipFree or allocating
 * routine; asynchronous on `stream` like ldpc_decode_batch.
 * Every call on one GPU shares that GPU's array and leaves its contents
 * behind (the kernels initialise what they read), so calls that overlap in
 * time on one GPU (different streams, threads or processes sharing it) race:
 * order them on one stream.
 * Errors: those of ldpc_decode_batch, and LDPC_EUNSUPPORTED when the call's
 * ldpc_decode_workspace_size() exceeds LDPC_NOALLOC_SCRATCH_BYTES.
 */
#define LDPC_NOALLOC_SCRATCH_BYTES (128u << 20)
ldpc_status ldpc_decode_batch_noalloc(const ldpc_code *code, int32_t n_frames, const void *llr_in,
                                      const ldpc_decode_params *p, uint8_t *hard_out, float *llr_out,
                                      int32_t *iters_out, uint8_t *syndrome_ok, void *stream);

/* Message describing the last failure on the calling thread ("" if none). */
const char *ldpc_last_error(void);

/* Library version string. */
const char *ldpc_version(void);

#ifdef __cplusplus
}
#endif
#endif /* LDPC_H */
