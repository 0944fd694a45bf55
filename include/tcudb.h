/*
 * tcudb.h -- C ABI of libtcudb.so: the join-aggregate-as-GEMM operator of
 * TCUDB (Hu, Li, Tseng, SIGMOD 2022) on AMD Instinct MI355X (gfx950).
 *
 * The operator answers the matrix multiplication query of Section 2.3 and,
 * generally, the group-by aggregate over a two-way join of Section 3.3
 * (Lemma Q3, queries Q3/Q4): for relation A of records (g, k, v) and relation
 * B of records (k, h, w),
 *
 *     C[g,h] = sum over pairs (a, b) with a.k == b.k, a.g == g, b.h == h of a.v * b.w
 *
 * computed as in Sections 3.1 and 3.3: encode X[g,k] = sum of a.v (M x K),
 * Y[k,h] = sum of b.w (K x N), then one matrix product C = X * Y (M x N).
 *
 * Conventions shared by every call:
 *  - Array pointers are DEVICE pointers owned by the caller.  The library never
 *    allocates, frees or keeps caller memory.  Its only global state is one
 *    internal non-blocking stream per device (tcu_join_agg_bwd), created on
 *    first use and kept for the life of the process, and the device array
 *    that tcu_join_agg_fwd_noalloc uses as its workspace.
 *  - Work is enqueued on the caller's stream and is asynchronous unless a call
 *    says otherwise; results are valid once the stream has reached that point.
 *    Work a call puts on an internal stream is ordered after the caller's
 *    earlier work and before its later work by events, so every call stays
 *    stream-ordered with respect to the caller's stream.  The device whose
 *    memory a call uses must be current.
 *  - Matrices are dense row-major with the leading dimension equal to the
 *    column count, unless a call takes explicit leading dimensions.
 *  - Host-side argument errors return a negative status and enqueue nothing.
 *  - Records with a key or group outside its range are never written out of
 *    bounds: they are skipped and counted in a status block at the start of
 *    the workspace, which tcu_sync_status() reads back.
 *  - A NULL value column means COUNT: every value is 1 (Section 3.3).
 *  - Calls that share one workspace must not overlap (same stream or ordered).
 */
#ifndef TCUDB_H
#define TCUDB_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    TCU_OK = 0,
    TCU_ERR_ARG = -1,        /* NULL required pointer, bad size or enum        */
    TCU_ERR_KEY_RANGE = -2,  /* device: a record had an out-of-range key/group */
    TCU_ERR_WORKSPACE = -3,  /* workspace NULL, misaligned or too small        */
    TCU_ERR_INFEASIBLE = -4, /* mixed form: tolerance not reachable            */
    TCU_ERR_NONFINITE = -5,  /* mixed form: NaN or infinity in an encoding     */
    TCU_ERR_HIP = -6,        /* a HIP runtime call failed                      */
    TCU_ERR_COUNT_RANGE = -7 /* device: a pair count exceeded INT32_MAX        */
} tcu_status;

typedef enum { TCU_F64 = 0, TCU_F32 = 1 } tcu_dtype;

typedef enum {
    TCU_PREC_FP64 = 0,       /* FP64 encodings, FP64 matrix-core product       */
    TCU_PREC_SPLIT_BF16 = 1, /* FP64 encodings cut into 7-bit integer digits
                                held in BF16, BF16 matrix cores with exact
                                FP32 partial sums, FP64 combination          */
    TCU_PREC_SPLIT_I8 = 2,   /* the same digits held in int8, int8 matrix
                                cores with exact int32 partial sums          */
    TCU_PREC_CRT_I8 = 3      /* FP64 encodings truncated to integers of
                                `bits` bits per line, residues modulo L small
                                coprime moduli on the int8 matrix cores (one
                                exact GEMM per modulus), the integer product
                                recovered by the Chinese remainder theorem */
} tcu_precision;

/* Largest slice count of the mixed forms (8 digits of 7 bits). */
#define TCU_MAX_SLICES 8
#define TCU_MAX_MODULI 15

/* Relation flags. */
#define TCU_REL_UNIQUE_CELLS 1u /* no two records share a (group, key) pair, as
                                   for a table that stores a matrix (the MM
                                   query); the encoding then uses plain stores
                                   instead of atomics.  If the promise is
                                   broken, one of the duplicates' values is
                                   kept (no memory is touched out of bounds). */

/* One relation, struct of arrays with n records.
 * For A: group = g in [0,M) (A.col_num of the MM query), key = k in [0,K)
 *        (A.row_num).
 * For B: group = h in [0,N) (B.row_num), key = k in [0,K) (B.col_num).
 * val: n values of `dtype`, or NULL for COUNT.
 * flags: TCU_REL_* bits. */
typedef struct {
    int64_t n;
    const int32_t *group;
    const int32_t *key;
    const void *val;
    tcu_dtype dtype;
    uint32_t flags;
} tcu_relation;

/* Flags for tcu_workspace_bytes. */
#define TCU_WS_BACKWARD 1 /* size for tcu_join_agg_bwd as well               */
#define TCU_WS_COUNT 2    /* size for the optional pair-count output         */

/* Flags for tcu_join_agg_bwd. */
#define TCU_BWD_SAVED_ENCODINGS 1 /* ws still holds X and Y written by the last
                                     tcu_join_agg_fwd on these same relations,
                                     shapes and precision (saved activations):
                                     skip re-encoding.  Without the flag X and
                                     Y are rebuilt from the records
                                     (activation checkpointing). */

/* Status block read back by tcu_sync_status (host copy). */
typedef struct {
    uint32_t flags;        /* TCU_FLAG_* bits                                 */
    uint32_t slices;       /* mixed forms: digit slices (or moduli) of the
                              last product; 0 when it ran in FP64            */
    uint64_t skipped_a;    /* records of A skipped by the last call           */
    uint64_t skipped_b;    /* records of B skipped by the last call           */
    uint32_t bits;         /* residue form: truncation width of the last
                              product                                        */
    uint32_t need;         /* mixed forms: the last product certificate's
                              largest per-cell need in its form (bits or
                              digits; 255: a cell it could not bound)        */
    uint32_t exceptions;   /* residue form: cells of the last product whose
                              need exceeded `bits` (or that the certificate
                              could not bound), recomputed one by one      */
} tcu_status_info;

#define TCU_FLAG_KEY_RANGE 1u /* a record had an out-of-range key or group    */
#define TCU_FLAG_NONFINITE 2u /* a mixed form met NaN or infinity             */
#define TCU_FLAG_FALLBACK 4u  /* a mixed-form product had no certified plan
                                 and ran in FP64 instead                      */
#define TCU_FLAG_COUNT_RANGE 8u /* a pair count exceeded INT32_MAX (stored as
                                   INT32_MAX)                                 */

/* Bytes of device workspace the calls below need for these shapes (Section
 * 3.3 encodings X and Y, plus the status block; with TCU_WS_BACKWARD the two
 * gradient matrices; in the mixed forms the certificate's planes, digit
 * slices or residues; in the FP64 form, for products with too few output
 * tiles to fill the chip, the partial products of their split contraction).  Given the relations (A and B not NULL), the size also
 * holds the scratch with which an encoding of 1 GiB or more runs window by
 * window (tcu_encode); a workspace sized without it (A or B NULL) is still
 * accepted and encodes in one pass.  The workspace must be 256-byte aligned.
 * Returns 0 for invalid shapes. */
size_t tcu_workspace_bytes(const tcu_relation *A, const tcu_relation *B, int32_t M, int32_t K,
                           int32_t N, tcu_precision p, int flags);

/* Step a1, the encoding of Sections 3.1/3.3 ("fill"): out (rows x cols,
 * FP64, row-major, leading dimension cols) is overwritten with
 *   transpose == 0: out[group, key] = sum of val   (A -> X, rows = M, cols = K)
 *   transpose == 1: out[key, group] = sum of val   (B -> Y, rows = K, cols = N)
 * Duplicate coordinates add up (FP64 atomics: order-dependent rounding);
 * unique coordinates give the values bit for bit (with TCU_REL_UNIQUE_CELLS
 * through plain stores).  Out-of-range records are
 * skipped and counted as A's skips in the workspace status block.
 * ws: 256-byte aligned, at least 256 bytes (the status block).  With
 * tcu_encode_workspace_bytes(R, rows, cols) bytes, a matrix of 1 GiB or more
 * is filled one window of rows at a time (about 128 MiB each: the records are
 * first partitioned by window, then each window is zeroed and filled while it
 * stays in the last-level cache); with less, in one pass.  Same result. */
tcu_status tcu_encode(const tcu_relation *R, int transpose, int32_t rows, int32_t cols,
                      double *out, void *ws, size_t ws_bytes, hipStream_t stream);

/* Workspace bytes with which tcu_encode fills this matrix window by window:
 * 256 plus, for matrices of at least 1 GiB, a scratch of about (4 + value
 * size) bytes per record (the records' cell offsets and values, ordered by
 * window).  Returns 256 where the one-pass fill is used anyway, 0 for
 * invalid arguments. */
size_t tcu_encode_workspace_bytes(const tcu_relation *R, int32_t rows, int32_t cols);

/* Step a0 host part, the mixed forms' precision plan (the feasibility test
 * of Section 4.2.1 retargeted: a cheap look at the operands' magnitudes
 * decides the narrow type's width, or refuses).  Every mixed-form product
 * C = X Y (contraction length k) is planned from a certificate computed on
 * the device from the two operands themselves:
 *   per line (row g of X, column h of Y): the exponent e with 2^(e-1) <=
 *     max |z| < 2^e, the normalised sum s = sum |z| 2^-e (rounded up), and
 *     the magnitude codes q = floor(|z| 2^(7-e)) in [0, 127];
 *   per cell: T = (Q_X Q_Y)[g,h] by one int8 GEMM, so that
 *     D_lo = 2^(e_g + f_h - 14) T <= (|X||Y|)[g,h];
 *   the truncation of both operands to b-bit integers per line (residue
 *     form) moves C[g,h] by at most 2^(e_g + f_h - b) (s_g + s_h), and S
 *     digits of 7 bits with the pairs past the first S anti-diagonals
 *     dropped (digit forms) by at most 2^(e_g + f_h - 7S) (s_g + s_h +
 *     (S - 1) k);
 *   the cell's need is the smallest b (or S) whose bound plus the FP64
 *     rounding of the combination stays within tol * D_lo (0 when row g or
 *     column h is all zero: every term of the cell is then 0).
 * need: the largest per-cell need over C (255 for a cell with T = 0 but a
 * nonzero bound: not certifiable); u: the smaller of the two operands'
 * largest normalised line sums (then |sum_k x'y'| < 2^(2b) min(u, k)).
 * Returns the digit count S = max(need, 1) (TCU_PREC_SPLIT_*, at most 8), or
 * for TCU_PREC_CRT_I8 the modulus count L, the smallest with
 * log2(prod m_i) > 2b + log2(min(max(u, 1), k)) + 1 + 1e-6 (so that prod m_i
 * > 2 |P| (1 + 2^-38), which the reconstruction's rounding of P / prod m_i
 * needs), b = max(need, 1) <= 53 written to
 * *bits (moduli 256, 255, 253, 251, 247, 241, 239, 233, 229, 227, 223, 217,
 * 211, 199, 197); TCU_ERR_INFEASIBLE when no plan exists (then the product
 * runs in FP64 and TCU_FLAG_FALLBACK is set), tol < 2^-50, or the residue
 * form with k > 131071 (int32 sums); TCU_ERR_ARG for a bad precision or
 * k < 1.  tol <= 0 means 1e-12.  Host only: touches no device. */
int tcu_mixed_plan(tcu_precision p, int32_t k, double tol, uint32_t need, double u,
                   int32_t *bits);

/* Step a0 device part alone: the per-line scale exponents and S digit slices
 * of a dense FP64 matrix Z (rows x cols, leading dimension ld).
 * axis == 0: lines are rows (length cols); 1: lines are columns (length rows).
 * For a line with largest magnitude mx, e = the exponent with
 * 2^(e-1) <= mx < 2^e (0 for an all-zero line), r_0 = z 2^-e and for
 * p = 1..S: t = r_{p-1} 2^7, d_p = trunc(t), r_p = t - d_p.
 * exps[line] = e (int32, `lines` entries); digits d_p are written as int8
 * (TCU_PREC_SPLIT_I8) or BF16 (TCU_PREC_SPLIT_BF16) in the blocked layout
 *   slices[p][t / KSTEP][(t % KSTEP) / HALF][line][t % HALF],
 *   KSTEP = 32 (int8) or 16 (BF16) digits, HALF = KSTEP / 2,
 * lines padded with zero digits to lines_pad (multiple of 128, >= lines) and
 * positions t to len_pad (multiple of 64, >= line length); slice p starts at
 * element p * lines_pad * len_pad.  NaN/Inf values give digits 0 and set
 * TCU_ERR_NONFINITE in the status block.  ws: >= 256 + 8 * lines_pad bytes. */
tcu_status tcu_split(const double *Z, int32_t rows, int32_t cols, int64_t ld, int axis,
                     tcu_precision p, int32_t S, void *slices, int32_t lines_pad,
                     int32_t len_pad, int32_t *exps, void *ws, size_t ws_bytes,
                     hipStream_t stream);

/* Step a2 alone, the contraction of Section 3.3: C = op(A) * op(B) in FP64 on
 * the matrix cores, op(A) m x k, op(B) k x n, C m x n (leading dimension ldc).
 * trans_a == 0: A is m x k row-major (lda >= k); 1: A is k x m (lda >= m).
 * trans_b == 0: B is k x n row-major (ldb >= n); 1: B is n x k (ldb >= k).
 * C is overwritten.  k == 0 gives C = 0. */
tcu_status tcu_gemm_f64(int trans_a, int trans_b, int32_t m, int32_t n, int32_t k,
                        const double *A, int64_t lda, const double *B, int64_t ldb,
                        double *C, int64_t ldc, hipStream_t stream);

/* tcu_gemm_f64 for outputs too small to fill the chip, such as the literal
 * Lemma-Q3 product 1^T C of Section 3.3 (one output row, a long
 * contraction): the contraction is cut into chunks that run as separate
 * workgroups, their partial products land in ws, and a second kernel adds
 * them in chunk order, the same on every run (results are reproducible bit
 * for bit).  When the output has enough tiles (or k < 1024) this is
 * tcu_gemm_f64 and ws is not touched.
 * ws: device, 256-byte aligned, at least tcu_gemm_f64_workspace_bytes(m, n,
 * k) bytes (0: no workspace needed; ws may then be NULL).
 * Errors as tcu_gemm_f64, plus TCU_ERR_WORKSPACE. */
size_t tcu_gemm_f64_workspace_bytes(int32_t m, int32_t n, int32_t k);
tcu_status tcu_gemm_f64_ws(int trans_a, int trans_b, int32_t m, int32_t n, int32_t k,
                           const double *A, int64_t lda, const double *B, int64_t ldb, double *C,
                           int64_t ldc, void *ws, size_t ws_bytes, hipStream_t stream);

/* Steps a1-a3, the operator (Sections 2.3, 3.3): C (M x N FP64 row-major,
 * rows g ascending, columns h ascending) = the join-aggregate above.
 * count (M x N int32, or NULL): exact number of joined pairs per (g,h); SQL's
 * result holds exactly the cells with count > 0 (a dense C shows 0 elsewhere).
 * With TCU_REL_UNIQUE_CELLS on both relations (every multiplicity 0 or 1)
 * the counts come from one int8 product of the 0/1 encodings with exact
 * int32 sums; otherwise from the FP64 product of the multiplicity encodings
 * (exact: every partial sum is a non-negative integer no larger than the
 * count).  A count above INT32_MAX is stored as INT32_MAX and flagged
 * (TCU_FLAG_COUNT_RANGE; tcu_sync_status returns TCU_ERR_COUNT_RANGE).  The
 * workspace must be sized with TCU_WS_COUNT.
 * The mixed forms (TCU_PREC_SPLIT_*, TCU_PREC_CRT_I8) guarantee, cell by
 * cell,
 *   |C - exact| <= tol * (|X||Y|)[g,h]
 * (tol <= 0 means 1e-12): the plan is certified for every cell of the
 * product from the operands (tcu_mixed_plan), and a product without a
 * certified plan runs in FP64 instead (TCU_FLAG_FALLBACK), whose error is
 * at most about K 2^-53 (|X||Y|)[g,h].  The residue form may instead take
 * a width b below the largest need when few cells (at most 4096) need more
 * than b or cannot be bounded and the narrower width saves moduli: those
 * cells are then recomputed one by one after the reconstruction as
 * compensated FP64 dot products (within about 2^-53 |C|), and their number
 * is reported (tcu_status_info.exceptions).  Planning reads the certificate
 * back to the host, so a mixed-form call SYNCHRONISES the stream once per
 * product (twice when the residue form looks for such cells); the FP64
 * form never does.  TCU_ERR_INFEASIBLE (launching nothing) for
 * tol < 2^-50 or, in the residue form, K > 131071.  The count output is
 * exact in every form.
 * Device-side conditions (out-of-range records, NaN/Inf in the mixed forms)
 * are reported by tcu_sync_status. */
tcu_status tcu_join_agg_fwd(const tcu_relation *A, const tcu_relation *B, int32_t M, int32_t K,
                            int32_t N, tcu_precision p, double tol, double *C, int32_t *count,
                            void *ws, size_t ws_bytes, hipStream_t stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * forward of tcu_join_agg_fwd with the same arguments and results, whose
 * workspace is the library's own device array of TCU_NOALLOC_MAX_BYTES
 * bytes instead of a caller buffer.  Each device the library runs on holds
 * one such array from module load until the process ends.  The call itself
 * allocates nothing (no hipMalloc, no library routine that allocates).
 * Returns TCU_ERR_WORKSPACE, launching nothing, when these shapes and this
 * precision need more than TCU_NOALLOC_MAX_BYTES (tcu_workspace_bytes with
 * flags 0 tells), e.g. beyond M = K = N = 2048 in the FP64 form.
 * status: NULL, or a 256-byte aligned device buffer of 256 bytes that
 *    receives the call's status block, which tcu_sync_status(status, ...)
 *    then reads (out-of-range records, non-finite values).
 * All calls on one device share its array and leave their contents in it:
 * calls that may overlap on one device (different streams, or host threads
 * without ordering) race and give wrong results.  Every call clears and
 * rewrites what it reads, so ordered calls are independent. */
#define TCU_NOALLOC_MAX_BYTES ((64u << 20) + (64u << 10))
tcu_status tcu_join_agg_fwd_noalloc(const tcu_relation *A, const tcu_relation *B, int32_t M,
                                    int32_t K, int32_t N, tcu_precision p, double tol, double *C,
                                    int32_t *count, void *status, hipStream_t stream);

/* Step a4, the adjoint of the operator for L = sum_{g,h} dC[g,h] C[g,h]:
 *   dA_val[i] = sum_{b: b.k == a_i.k} dC[a_i.g, b.h] * b.w = (dC Y^T)[a_i.g, a_i.k]
 *   dB_val[j] = sum_{a: a.k == b_j.k} dC[a.g, b_j.h] * a.v = (X^T dC)[b_j.k, b_j.h]
 * By default X and Y are re-encoded from the records (activation
 * checkpointing: nothing of the forward is kept); with
 * TCU_BWD_SAVED_ENCODINGS the forward's X and Y in ws are used.  Either
 * output may be NULL.  Skipped records get 0.  Gradients are FP64 whatever
 * the value dtype.  In the mixed forms each product (dX = dC Y^T over N,
 * dY = X^T dC over M) is certified and planned on its own operands as in
 * the forward, so |dX - exact| <= tol (|dC||Y^T|)[g,k] and |dY - exact| <=
 * tol (|X^T||dC|)[k,h] cell by cell, and the call synchronises once per
 * product.  Needs a
 * workspace sized with TCU_WS_BACKWARD.  With both outputs, the gather of
 * dA_val (and, when re-encoding, the encoding of X) runs on the device's
 * internal stream beside the products on the caller's stream; in the FP64
 * form a dY product that fills more than one round of workgroups is cut
 * into two row blocks, and the gather of the first block's dB_val entries
 * joins that stream beside the second block's product.  The call joins the
 * internal stream back before returning control of the stream. */
tcu_status tcu_join_agg_bwd(const tcu_relation *A, const tcu_relation *B, int32_t M, int32_t K,
                            int32_t N, tcu_precision p, double tol, const double *dC,
                            double *dA_val, double *dB_val, int flags, void *ws,
                            size_t ws_bytes, hipStream_t stream);

/* ---- Measurement (instrumentation, not a step of the method) -------------
 *
 * Launch records of the matrix-core product kernels, for timing the
 * dominant kernel inside a timed region with HIP events.  While recording
 * is on for the calling host thread, every launch of one of these kernels
 * that a call made on this thread issues is bracketed by hipEventRecord of
 * the next record's `begin` and `end` events, on the stream the kernel runs
 * on (the caller's or the library's internal one), and the record receives
 * the kernel, its shape and its algorithmic operation count:
 *   TCU_KERNEL_GEMM_F64    FP64 product, ops = 2 m n k FLOP
 *   TCU_KERNEL_GEMM_CRT    residue products, planes = L moduli,
 *                          ops = L * 2 m n k int8 operations
 *   TCU_KERNEL_CERTIFY     the certificate's int8 product, ops = 2 m n k
 *   TCU_KERNEL_GEMM_SPLIT  digit products, planes = S digits,
 *                          ops = S (S + 1) / 2 * 2 m n k
 *   TCU_KERNEL_ENCODE      one relation's scatter into an m x n matrix,
 *                          ops = algorithmic bytes (group, key and value
 *                          read, one 8-byte cell written per record)
 *   TCU_KERNEL_GATHER      an adjoint's gather (or a row range of it),
 *                          ops = 24 bytes per record of the relation
 *   TCU_KERNEL_COUNT       the pair counts' int8 product, ops = 2 m n k
 * The caller creates the events (timing enabled) and, once the work has
 * run, reads each launch's duration with hipEventElapsedTime.
 * records: the caller's host array of `capacity` records; count: a host
 * int32 that is set to 0 now and counts every launch seen (launches beyond
 * `capacity` are counted, not recorded).  count == NULL stops recording.
 * The arrays must stay valid while recording is on.  TCU_ERR_ARG for a
 * negative capacity or a NULL array with a positive one. */
typedef enum {
    TCU_KERNEL_GEMM_F64 = 1,
    TCU_KERNEL_GEMM_CRT = 2,
    TCU_KERNEL_CERTIFY = 3,
    TCU_KERNEL_GEMM_SPLIT = 4,
    TCU_KERNEL_ENCODE = 5,
    TCU_KERNEL_GATHER = 6,
    TCU_KERNEL_COUNT = 7
} tcu_kernel_id;
typedef struct {
    hipEvent_t begin, end;  /* the caller's events                         */
    int32_t kernel;         /* tcu_kernel_id                               */
    int32_t m, n, k;        /* output rows, columns, contraction length    */
    int32_t planes;         /* moduli or digit slices (1 for FP64); for an
                               encoding, its row windows (1: one pass)     */
    double ops;             /* algorithmic operations of the launch        */
} tcu_launch_record;
tcu_status tcu_trace_launches(tcu_launch_record *records, int32_t capacity, int32_t *count);

/* Measured matrix-core peaks, the rates the roofline is read against beside
 * the published ones (not a step of the method).  One launch of a
 * register-only loop: kind 0 runs FP64 16x16x4 MFMAs, kind 1 int8 32x32x32
 * MFMAs on uniformly random bytes (the residue form's operands), kind 2
 * int8 on near-constant bytes; iters >= 1 rounds of eight independent
 * instructions per wave, 2048 workgroups of 256 threads.  out: device
 * buffer of at least tcu_mfma_peak_out_bytes() bytes (per-thread checksums).
 * tcu_mfma_peak_ops(kind, iters) is the launch's operation count (FLOPs or
 * integer ops), to divide by the launch's duration.  Asynchronous on the
 * stream; TCU_ERR_ARG for a bad kind, iters < 1 or a NULL buffer. */
size_t tcu_mfma_peak_out_bytes(void);
double tcu_mfma_peak_ops(int kind, int32_t iters);
tcu_status tcu_mfma_peak(int kind, int32_t iters, void *out, hipStream_t stream);

/* Dictionary encoding for the encodings of Section 3.1: dom(ID) is the union
 * of two columns' values, with k distinct values v_1 < ... < v_k (sorted,
 * signed 64-bit).  codes_a[i] = the rank of a[i] in that list (0-based), and
 * likewise codes_b; dict (capacity n_a + n_b) receives v_1..v_k and *k (a
 * host pointer) receives k.  Codes are independent of record order.  The
 * call SYNCHRONISES the stream once (to size the sort of the distinct
 * values).  n_a + n_b must not exceed 2^31 - 1.  ws: at least
 * tcu_dict_workspace_bytes(n_a + n_b) bytes, 256-byte aligned (about 24
 * bytes per value); errors are returned, not recorded in ws. */
size_t tcu_dict_workspace_bytes(int64_t n);
tcu_status tcu_dict_encode(const int64_t *a, int64_t n_a, const int64_t *b, int64_t n_b,
                           int32_t *codes_a, int32_t *codes_b, int64_t *dict, int64_t *k,
                           void *ws, size_t ws_bytes, hipStream_t stream);

/* Queries Q3 and Q4 of Section 3.3 in re-associated form: A forms a single
 * group (Lemma Q3's 1^{1 x n} factor: A's group column is ignored), so
 *   c[h] = sum over joined pairs (a, b) with b.group == h of a.val * b.val
 *        = sum_{b: b.group == h} hA[b.key] * b.val,  hA[k] = sum_{a: a.key == k} a.val,
 * computed from the records in two streaming passes without forming X or Y.
 * count (N entries, or NULL) receives the exact number of joined pairs per
 * group, so SUM / COUNT is the AVG of Section 3.3.  N = 1 with every B record
 * in group 0 is Q4.  c is FP64 (N entries).  Records with a key outside
 * [0,K) (or a B group outside [0,N)) are skipped and counted in the status
 * block at the start of ws (tcu_sync_status).  Floating-point sums use
 * atomics (order-dependent last bits); counts are exact.  ws: at least
 * tcu_join_agg_row_workspace_bytes(K, N) bytes, 256-byte aligned. */
size_t tcu_join_agg_row_workspace_bytes(int32_t K, int32_t N);
tcu_status tcu_join_agg_row(const tcu_relation *A, const tcu_relation *B, int32_t K, int32_t N,
                            double *c, uint64_t *count, void *ws, size_t ws_bytes,
                            hipStream_t stream);

/* ---- Block-sparse form (Section 4.2.4: TCU-SpMM) ------------------------
 *
 * The operator of tcu_join_agg_fwd (same relations, same C) evaluated on
 * 16 x 16 block-sparse encodings: X and Y are cut into 16 x 16 tiles, tiles
 * holding no record are neither stored nor multiplied, and every pair of
 * stored tiles that meet on a key tile runs on the FP64 matrix cores.  Meant
 * for large, sparse key domains (K much larger than the keys any group
 * touches), where the dense product would multiply mostly zeros.
 *
 * C: [M*N] FP64 row-major, every cell written (exactly 0 where no pair
 *    joins).  With A->val == NULL and B->val == NULL, C is the pair count.
 * Cost: building the tiles makes ONE host synchronisation per relation (to
 *    size the sort of its distinct tile keys), so the call blocks until the
 *    stream has reached that point.
 * Records out of range are skipped and counted (tcu_sync_status).
 * Duplicate cells add up (FP64 atomics) unless TCU_REL_UNIQUE_CELLS is set.
 * Workspace: tcu_join_agg_bsr_workspace_bytes(); it bounds the tile storage
 *    by 2 KB per record (at most one new tile per record), capped by the
 *    number of tiles of the M x K and K x N grids. */
size_t tcu_join_agg_bsr_workspace_bytes(const tcu_relation *A, const tcu_relation *B,
                                        int32_t M, int32_t K, int32_t N);
tcu_status tcu_join_agg_bsr(const tcu_relation *A, const tcu_relation *B, int32_t M, int32_t K,
                            int32_t N, double *C, void *ws, size_t ws_bytes, hipStream_t stream);

/* The choice between the dense FP64 operator (tcu_join_agg_fwd) and the
 * block-sparse one (tcu_join_agg_bsr), after the paper's switch to TCU-SpMM
 * when the encodings are sparse (Section 4.2.4) and its cost model's
 * comparison of estimated times (Section 4.2.2).  Host only, no device call.
 * Returns 1 when the block-sparse form is predicted faster, 0 when the dense
 * one is, TCU_ERR_ARG on bad arguments.  The model, with constants measured
 * on MI355X on Q1 pair counts (one record per tuple, n = 4096 and 8192,
 * 32 to 16384 distinct keys):
 *   dense        2 M N K / (70 TFLOP/s) + 16 B per cell of X and Y / (3 TB/s)
 *   block-sparse 0.62 ms + 1.7 ns per 16 x 16 tile of C
 *                + 0.14 ns per pair of stored tiles meeting on a key tile,
 * with stored tiles estimated as min(records, tiles of the grid) per side
 * and meetings as their product over the key tiles (keys spread evenly). */
int tcu_block_sparse_preferred(const tcu_relation *A, const tcu_relation *B, int32_t M,
                               int32_t K, int32_t N);

/* ---- Matrix-to-table conversion (Section 3.2: multi-way joins) ----------
 *
 * nonzero(M): the cells (i, j) of a dense rows x cols FP64 matrix (leading
 * dimension ld >= cols) with M[i,j] != 0, in row-major order, i.e. the
 * tuple pairs that survive a join, ready to be re-encoded for the next join
 * of a multi-way join.
 * out_row, out_col: [capacity] int32; entries beyond *count or capacity are
 *    not written.  If *count > capacity, only the first `capacity` pairs
 *    are written: call again with a larger output.
 * col_map, out_key: both NULL, or col_map [cols] int32 and out_key
 *    [capacity] int32 with out_key[p] = col_map[out_col[p]] (the join key of
 *    the next join, e.g. the code of B.ID2 for B tuple out_col[p]).
 * count: host pointer; receives the number of nonzero cells.  The call
 *    SYNCHRONISES the stream to read it.
 * rows, cols < 2^31; M may be NULL only if rows * cols == 0.
 * Workspace: tcu_nonzero_workspace_bytes(rows, cols), 256-byte aligned. */
size_t tcu_nonzero_workspace_bytes(int64_t rows, int64_t cols);
tcu_status tcu_nonzero(const double *M, int64_t rows, int64_t cols, int64_t ld, int32_t *out_row,
                       int32_t *out_col, const int32_t *col_map, int32_t *out_key,
                       int64_t capacity, int64_t *count, void *ws, size_t ws_bytes,
                       hipStream_t stream);

/* ---- Operands larger than device memory (Section 4.2.3) -----------------
 *
 * C (m x n, ldc) = A (m x k, lda) * B (k x n, ldb), FP64 row-major, with A, B
 * and C in HOST memory (allocate them pinned, with hipHostMalloc, for the
 * copies to overlap the products; pageable memory is correct but slow).
 * The device holds only blocks: dev_buf (device memory, 256-byte aligned,
 * dev_bytes long) must hold 6 block^2 doubles.  block: a multiple of 128,
 * or 0 for the largest multiple of 128 that fits dev_bytes.
 * Blocks of A and B stream in on one internal stream while the FP64 matrix
 * cores multiply on `stream` and finished C blocks stream out on another;
 * the call creates and destroys those two streams and SYNCHRONISES all
 * three before it returns (C is complete on return).
 * Host-link traffic: 8 (m k ceil(n / block) + k n ceil(m / block) + m n) bytes.
 * Errors: TCU_ERR_ARG (m, n or k < 0, NULL pointer with a nonzero extent,
 * ld smaller than the row length, block not a multiple of 128),
 * TCU_ERR_WORKSPACE (dev_buf NULL, misaligned, or smaller than 6 block^2
 * doubles), TCU_ERR_HIP. */
tcu_status tcu_gemm_f64_host(int32_t m, int32_t n, int32_t k, const double *A, int64_t lda,
                             const double *B, int64_t ldb, double *C, int64_t ldc, void *dev_buf,
                             size_t dev_bytes, int64_t block, hipStream_t stream);

/* SYNCHRONISES the stream, then reads the workspace status block written by
 * the last call that used `ws`.  Returns TCU_ERR_NONFINITE if the mixed form
 * met NaN/Inf, else TCU_ERR_KEY_RANGE if records were skipped, else
 * TCU_ERR_COUNT_RANGE if a pair count exceeded INT32_MAX, else TCU_OK.
 * info (may be NULL) receives the whole block. */
tcu_status tcu_sync_status(void *ws, hipStream_t stream, tcu_status_info *info);

/* Static description of a status code. */
const char *tcu_status_str(tcu_status s);

/* Library version string. */
const char *tcu_version(void);

#ifdef __cplusplus
}
#endif

#endif /* TCUDB_H */
