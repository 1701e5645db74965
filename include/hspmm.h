/*
 * hspmm -- hybrid CSR + BCSR sparse x dense matrix multiplication on one
 * AMD Instinct MI355X (gfx950).
 *
 * The operation is C = A * B with A sparse (CSR, m x k) and B dense (k x n,
 * row-major), the inner-product definition c_ij = sum_k a_ik b_kj of
 * Sec. 2.1.  The plan splits A into a row-wise CSR-part and a vector-wise
 * BCSR-part made of B_r x 1 column tiles (Sec. 3.2, Alg. 1); a cost model
 * (the analogue of Sec. 3.1 Eq. 1 and Sec. 3.5 Eq. 2-3) decides, per block
 * of B_r rows, which part a row block goes to.  The CSR-part runs as a
 * gather-FMA kernel (the AXPY kernel of Sec. 3.3), the BCSR-part as an MFMA
 * kernel (the outer-product kernel of Sec. 3.3, Alg. 2-3); both parts run
 * in one launch and every row of C has exactly one writer (Sec. 3.4).
 * Backward: dB = A^T * dC through a device-built transposed plan, and
 * dA = SDDMM(dC, B) sampled on A's pattern.
 *
 * Conventions for every entry point
 *  - Array arguments are DEVICE pointers unless stated otherwise; the caller
 *    owns them.  Index arrays are int32, row-major dense matrices use a
 *    leading dimension in elements (ld >= n).
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream);
 *    all device work is ordered on it.
 *  - Every call returns HSPMM_OK (0) or a negative hspmm_status and never
 *    aborts; hybrid_spmm_last_error() then describes the failure.
 */
#ifndef HSPMM_H
#define HSPMM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct hspmm_plan* hspmm_plan_t;

typedef enum {
    HSPMM_OK = 0,
    HSPMM_ERR_ARG = -1,         /* null pointer, negative size, ld < n, bad opts */
    HSPMM_ERR_CSR = -2,         /* row_ptr not monotone / not 0..nnz, column out of range */
    HSPMM_ERR_DTYPE = -3,       /* unsupported dtype value */
    HSPMM_ERR_NO_BACKWARD = -4, /* backward on a plan built without want_backward */
    HSPMM_ERR_HIP = -5,         /* a HIP runtime call failed */
    HSPMM_ERR_OOM = -6,         /* device allocation failed or max_workspace_bytes exceeded */
    HSPMM_ERR_OVERFLOW = -7     /* nnz, padded tile slots or an index would exceed 2^31 - 1 */
} hspmm_status;

/* Precision of the stored A-parts and of the dense operand B (Sec. 3.3:
 * FP64, FP32, FP16; BF16 added).  For F16/BF16, C, dB and dA are FP32 and
 * products accumulate in FP32. */
typedef enum { HSPMM_F64 = 0, HSPMM_F32 = 1, HSPMM_F16 = 2, HSPMM_BF16 = 3 } hspmm_dtype;

/* How row blocks are assigned to the two parts.
 *   AUTO      each B_r-row block goes to the part with the lower predicted
 *             time (byte/time model, row blocks are independent);
 *   CSR_ONLY  every row in the CSR-part (r_boundary = m, the pure-vector mode
 *             of Sec. 4.3);
 *   BCSR_ONLY every row block in the BCSR-part (r_boundary = 0, the pure
 *             matrix-unit mode of Sec. 4.3);
 *   BOUNDARY  contiguous split of Alg. 1: rows [0, r_boundary) CSR, the rest
 *             BCSR; r_boundary = -1 solves Eq. 1 with the cost model's
 *             predicted times, HSPMM_R_MEASURED solves it with throughputs
 *             measured on this matrix at plan time (the warm-up runs of
 *             Sec. 3.1: the forward of the whole matrix is timed once in
 *             the CSR-part and once in the BCSR-part at width n_hint, and
 *             TP = m / time). */
#define HSPMM_R_MEASURED (-2)
typedef enum {
    HSPMM_SPLIT_AUTO = 0,
    HSPMM_SPLIT_CSR_ONLY = 1,
    HSPMM_SPLIT_BCSR_ONLY = 2,
    HSPMM_SPLIT_BOUNDARY = 3
} hspmm_split;

typedef struct {
    uint32_t struct_size;         /* must be sizeof(hspmm_plan_opts) */
    int32_t compute;              /* hspmm_dtype of the A-parts and of B */
    int32_t split;                /* hspmm_split */
    int32_t block_rows;           /* B_r: 16 (0 = 16); the MFMA tile height */
    int64_t r_boundary;           /* BOUNDARY only; -1 = solve Eq. 1 (model),
                                     HSPMM_R_MEASURED = solve it (measured) */
    int32_t n_hint;               /* expected n for the cost model (0 = 128) */
    int32_t want_backward;        /* nonzero: also build the transposed plan */
    uint64_t max_workspace_bytes; /* 0 = unlimited; larger plans fail with OOM */
} hspmm_plan_opts;

/* Host-side description of a built plan (filled by hybrid_spmm_plan_info). */
typedef struct {
    uint32_t struct_size;         /* must be sizeof(hspmm_plan_info) */
    int32_t compute;
    int64_t m, k, nnz_input, nnz;  /* nnz = canonical entries (duplicates summed) */
    int32_t block_rows;
    int32_t canonical_input;      /* 1: input already sorted and duplicate-free */
    int64_t rows_csr;             /* rows in the CSR-part */
    int64_t nnz_csr;              /* entries in the CSR-part */
    int64_t long_rows;            /* CSR rows split across several waves */
    int64_t rb_bcsr;              /* row blocks in the BCSR-part */
    int64_t nblk;                 /* non-empty B_r x 1 tiles in the BCSR-part */
    int64_t nblk_padded;          /* tiles incl. zero tiles that pad the MFMA K */
    int64_t nnz_bcsr;             /* entries in the BCSR-part */
    double  fill;                 /* nnz_bcsr / (nblk * B_r) */
    double  pred_us_csr, pred_us_bcsr; /* cost-model time of each part at n_hint */
    int64_t r_boundary;           /* BOUNDARY mode: rows in the CSR-part */
    int64_t bytes_device;         /* device memory held by the plan */
    double  plan_ms;              /* wall time of hybrid_spmm_plan */
    int32_t has_backward;
    int64_t t_rows_csr, t_rb_bcsr, t_nblk; /* same split figures for A^T */
    /* cost-model time of the whole matrix in each part at n_hint, whatever
     * the split: the inputs of Eq. 1 (BOUNDARY with r_boundary < 0 uses
     * TP_csr = m / pred_us_csr_all and TP_bcsr = m / pred_us_bcsr_all with
     * t_csr = t_bcsr = 1) */
    double  pred_us_csr_all, pred_us_bcsr_all;
    /* groups of BCSR row blocks sharing columns (FP32 / FP64 plans): the
     * group kernels stage each group's shared columns in LDS once */
    int64_t ngroups;              /* 0: the BCSR-part runs ungrouped */
    int64_t grp_staged_tiles;     /* tiles that read their B row from the stage */
    int64_t grp_stage_rows;       /* staged rows summed over the groups */
    /* HSPMM_R_MEASURED plans: the measured forward time of the whole matrix
     * in each part at n_hint, the inputs of the measured Eq. 1 (0 otherwise) */
    double  meas_us_csr_all, meas_us_bcsr_all;
} hspmm_plan_info;

/* Build a plan for A (m x k, nnz entries, CSR) -- Alg. 1 plus the cost model.
 *   row_ptr[m+1], col_idx[nnz]: device int32; columns may be unsorted and
 *     may repeat inside a row (duplicates are summed).
 *   vals[nnz]: device array of vals_dtype (any hspmm_dtype); converted once
 *     to `compute` (FP16/BF16 with one power-of-two scale per B_r-row block,
 *     round-to-nearest-even).
 *   opts: NULL = defaults (F32, AUTO, B_r 16, n_hint 128, no backward).
 * Host-synchronous: returns after the device work on `stream` is complete;
 * the caller may then free the inputs.  The plan owns all derived memory.
 * Errors: ARG, CSR, DTYPE, HIP, OOM, OVERFLOW; *out is NULL on error. */
int hybrid_spmm_plan(hspmm_plan_t* out, int64_t m, int64_t k, int64_t nnz,
                     const int32_t* row_ptr, const int32_t* col_idx,
                     const void* vals, int32_t vals_dtype,
                     const hspmm_plan_opts* opts, void* stream);

/* C = A * B (Sec. 2.1); C is overwritten (rows without entries become 0).
 *   B: k x n, row-major, leading dimension ldb, dtype = compute.
 *   C: m x n, row-major, leading dimension ldc; FP64 if compute = F64, FP32
 *      otherwise.
 * Asynchronous on `stream`; allocates only if n exceeds every earlier n of
 * this plan (a scratch buffer for split long rows).  Not thread-safe on one
 * plan.  Errors: ARG, HIP, OOM. */
int hybrid_spmm_run(hspmm_plan_t p, int64_t n, const void* B, int64_t ldb,
                    void* C, int64_t ldc, void* stream);

/* The same product as hybrid_spmm_run for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): nothing is allocated, on the host or the
 * device.  The partial rows of split CSR rows go to a static device array
 * of HSPMM_NOALLOC_SCRATCH_BYTES bytes per GPU, held from the library's
 * first use of it on that GPU until the process ends, instead of the plan's
 * growable buffer.  Arguments, layout and results are those of
 * hybrid_spmm_run (bitwise: the same kernels); C is overwritten.
 * Every call on one GPU shares that GPU's array, so calls that overlap on
 * one GPU (other streams, other plans, other threads) race: order them.
 * The array needs no clearing: each call writes every slot it reads.
 * Errors: ARG; OOM when the split rows need more than the static array at
 * this n (n_partials * n * 4 bytes, 8 for F64 plans; nothing is launched);
 * HIP. */
#define HSPMM_NOALLOC_SCRATCH_BYTES 33554432u /* 32 MiB */
int hybrid_spmm_run_noalloc(hspmm_plan_t p, int64_t n, const void* B, int64_t ldb,
                            void* C, int64_t ldc, void* stream);

/* Gradients of L(vals, B) through C = A * B, given dC = dL/dC:
 *   dB = A^T * dC  (k x n, ld lddb; FP64 for F64 plans, FP32 otherwise), or
 *        skipped if dB is NULL;
 *   dA[e] = <dC[row(e),:], B[col(e),:]> for every input entry e in the
 *        original input order (duplicates receive the same value); FP64 for
 *        F64 plans, FP32 otherwise; skipped if dA_vals is NULL.
 *   B: as in hybrid_spmm_run (dtype = compute); dC: m x n, FP64 for F64
 *      plans, FP32 otherwise.
 * F16/BF16 plans compute dB in FP32 from the stored (quantised) values.
 * dA accumulates in FP32; for F16/BF16 plans the BCSR-part's rows (n a
 * multiple of 8, at most 256) first round each 16-row slab of dC to the
 * compute type after an exact power-of-two scale (largest magnitude in
 * [2^14, 2^15)), one rounding per dC element.
 * When both gradients are requested, they are computed in one pass over
 * the transposed plan: each gathered row of dC serves its dB product and
 * the dA dot products of the same entries (Sec. 3.3 product and its
 * gradient; one gather stream instead of two).  This applies for n up to
 * 256 (FP32 dC) / 128 (FP64) with n, ldb, lddc, lddb multiples of 16 bytes
 * and 16-byte aligned dC, dB, B (8-byte B for F16/BF16 plans); a
 * BCSR-part in A^T qualifies for F32/F64 plans only (its dA
 * MFMAs hold B in the compute type) and with at most 2048 tiles per row
 * block, a CSR-part from rows of B of 256 bytes (n * element size; below
 * that the separate SDDMM's own gathers cost less than the one-pass form's
 * scattered dA writes).  dB is then bitwise the separate product's; dA differs only in
 * summation order, and for F16/BF16 plans its dot products run in FP32
 * on the stored B (no rounding of dC).  Errors: ARG, NO_BACKWARD (dB
 * requested without want_backward), HIP, OOM. */
int hybrid_spmm_backward(hspmm_plan_t p, int64_t n, const void* B, int64_t ldb,
                         const void* dC, int64_t lddc, void* dB, int64_t lddb,
                         void* dA_vals, void* stream);

/* Whether hybrid_spmm_backward with these operands and both outputs takes
 * the one-pass path described above (*fused = 1) or runs dB and dA as
 * separate products (*fused = 0).  dB may be NULL to ask about a 16-byte
 * aligned dB (as a fresh allocation is) with the given lddb.  No device
 * work.  Errors: ARG. */
int hybrid_spmm_backward_fused(hspmm_plan_t p, int64_t n, const void* B, int64_t ldb,
                               const void* dC, int64_t lddc, const void* dB, int64_t lddb,
                               int32_t* fused);

/* Replace the values of A (same pattern, original input order, any dtype)
 * and re-pack both parts (and the transposed plan).  Asynchronous.  The
 * FP16/BF16 row-block scales are recomputed.  Errors: ARG, DTYPE, HIP. */
int hybrid_spmm_update_values(hspmm_plan_t p, const void* vals, int32_t vals_dtype,
                              void* stream);

/* Fill a host hspmm_plan_info (info->struct_size must be set). */
int hybrid_spmm_plan_info(hspmm_plan_t p, hspmm_plan_info* info);

/* Copy one array of the built format to host memory, in the canonical
 * layout of Alg. 1 (padding tiles removed, BCSR tile values as [tile][B_r]).
 *   which: 0 = A's plan, 1 = the transposed plan.
 *   field: hspmm_field.  dst: HOST pointer or NULL; *bytes receives the size
 *   of the array; nothing is copied if dst is NULL or capacity < *bytes.
 * Meant for tests and inspection.  Errors: ARG, HIP. */
typedef enum {
    HSPMM_F_RB_CLASS = 0,  /* int32 [nrb]: 0 CSR-part, 1 BCSR-part */
    HSPMM_F_RB_NNZ = 1,    /* int32 [nrb]: stored entries per row block */
    HSPMM_F_RB_NBLK = 2,   /* int32 [nrb]: non-empty tiles per row block */
    HSPMM_F_CSR_ROWS = 3,  /* int32 [rows_csr]: row ids, ascending */
    HSPMM_F_CSR_PTR = 4,   /* int32 [rows_csr+1] */
    HSPMM_F_CSR_COL = 5,   /* int32 [nnz_csr] */
    HSPMM_F_CSR_VAL = 6,   /* compute dtype [nnz_csr] (F16/BF16: value / scale) */
    HSPMM_F_BCSR_RB = 7,   /* int32 [rb_bcsr]: row-block ids, ascending */
    HSPMM_F_BLK_PTR = 8,   /* int32 [rb_bcsr+1] */
    HSPMM_F_BLK_COL = 9,   /* int32 [nblk] */
    HSPMM_F_BLK_VAL = 10,  /* compute dtype [nblk][B_r] */
    HSPMM_F_RB_SCALE = 11, /* FP64 [nrb]: power-of-two scale (1 for F32/F64) */
    HSPMM_F_GRP_PTR = 12,  /* int32 [ngroups+1]: groups as ranges of GRP_RB */
    HSPMM_F_GRP_RB = 13,   /* int32 [rb_bcsr]: row blocks in the group kernels' order */
    HSPMM_F_GRP_UPTR = 14, /* int32 [ngroups+1]: groups as ranges of GRP_UCOL */
    HSPMM_F_GRP_UCOL = 15, /* int32: each group's staged columns, ascending */
    HSPMM_F_BLK_BSRC = 16  /* int32 [nblk], tiles as BLK_COL: stage row >= 0, or
                              -(column + 1) for a tile gathered directly */
} hspmm_field;

int hybrid_spmm_export(hspmm_plan_t p, int32_t which, int32_t field, void* dst,
                       int64_t capacity, int64_t* bytes);

/* Calibration of the workgroup partition of the fused forward launch, the
 * analogue of the thread split (t_neon, t_sme) of Sec. 3.5: the forward is
 * timed on `stream` at a candidate set of partitions (x, y) = (workgroups
 * of the CSR-part, workgroups of the BCSR-part, both in units of 8) with
 * x + y <= T, T = the workgroups the GPU holds at once / 8; Eq. 2
 * perf(x, y) = a0 + a1 x + a2 y + a3 x^2 + a4 y^2 (GFLOP/s) is fitted by
 * least squares (terms of an empty part dropped) and Eq. 3 picks the
 * argmax over all integer x + y <= T.  The chosen partition is applied to
 * later runs if it measures at least as fast as the default launch (one
 * workgroup per work unit); otherwise the default is kept.
 *   B, C, n, ldb, ldc: as in hybrid_spmm_run (C is overwritten);
 *   reps: timed launches per candidate (>= 1); info: host output.
 * Host-synchronous.  Errors: ARG, HIP. */
#define HSPMM_CALIB_MAX 32
typedef struct {
    uint32_t struct_size;            /* must be sizeof(hspmm_calib_info) */
    int32_t T;                       /* partition units available (x + y <= T) */
    int32_t x_max, y_max;            /* units each part can use (0: part empty) */
    int32_t n_candidates;
    int32_t cand_x[HSPMM_CALIB_MAX]; /* CSR-part workgroups / 8 */
    int32_t cand_y[HSPMM_CALIB_MAX]; /* BCSR-part workgroups / 8 */
    double cand_gflops[HSPMM_CALIB_MAX];
    double coef[5];                  /* a0..a4 of Eq. 2 (dropped terms are 0) */
    int32_t best_x, best_y;          /* Eq. 3 argmax */
    double best_gflops;              /* measured at (best_x, best_y) */
    double default_gflops;           /* measured with the default launch */
    int32_t applied;                 /* 1: (best_x, best_y) is used by later runs */
} hspmm_calib_info;

int hybrid_spmm_calibrate(hspmm_plan_t p, int64_t n, const void* B, int64_t ldb, void* C, int64_t ldc,
                          int32_t reps, hspmm_calib_info* info, void* stream);

/* Kernel timing for callers that measure the products (benchmarks,
 * profilers): while set, every product this thread launches (run, the dB
 * and dA halves of backward, run_noalloc) records `start` (a hipEvent_t) as
 * its first kernel begins and `stop` as its last kernel ends, from the
 * kernels' own dispatch timestamps, so no marker separates the kernels of
 * consecutive calls.  NULL, NULL clears them.  The events must have been
 * created with timing enabled; this thread only.  A start event delays the
 * dispatch of the kernel that carries it by about 4.5 us (measured), and a
 * stop event costs nothing measurable: to time a sequence of products, give
 * its first product the start event and its last the stop event.  Errors:
 * none. */
int hybrid_spmm_set_timing_events(void* start, void* stop);

/* Release the plan and all its device memory (NULL-safe).  Waits for all
 * work queued on the device first (hipFree does so in any case): the
 * products record no per-call event to wait on, since such an event delays
 * the next kernel on its stream. */
void hybrid_spmm_destroy(hspmm_plan_t p);

/* Message of the last failed call on this thread ("" if none); valid until
 * the next call on this thread. */
const char* hybrid_spmm_last_error(void);

/* Library version string. */
const char* hybrid_spmm_version(void);

#ifdef __cplusplus
}
#endif
#endif /* HSPMM_H */
