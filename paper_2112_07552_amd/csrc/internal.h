// internal.h -- declarations shared by the HIP sources of libtcudb.so.
// Not part of the public ABI (that is include/tcudb.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "tcudb.h"

namespace tcu {

// Workspace status block (first 256 bytes of every workspace).
struct StatusBlock {
    uint32_t flags;                 // kFlag* bits
    uint32_t slices;                // mixed form: slices or moduli of the last product (0: FP64)
    unsigned long long skipped_a;   // records of A skipped
    unsigned long long skipped_b;   // records of B skipped
    uint32_t bits;                  // residue form: truncation width of the last product
    uint32_t need_bits;             // certificate: largest per-cell truncation width needed
    uint32_t need_slices;           // certificate: largest per-cell digit count needed
    uint32_t need;                  // the last product's need in its own form
    unsigned long long umax_a;      // bit pattern of max over lines of sum|z| 2^-e, operand A
    unsigned long long umax_b;      // the same for operand B
    uint32_t need_cert;             // certificate: largest need among the cells it bounds
    uint32_t need_min;              // certificate: smallest nonzero need among those cells
    uint32_t exc_seg[4];            // exception scan: cells listed per segment (kExcThresholds;
                                    // above the segment's capacity: it overflowed)
    uint32_t exceptions;            // residue form: cells of the last product recomputed alone
    uint32_t pad[43];
};
static_assert(sizeof(StatusBlock) == 256, "status block must be 256 bytes");
constexpr int kExcThresholds = 4;  // thresholds the exception scan counts above

constexpr uint32_t kFlagKeyRange = 1u;
constexpr uint32_t kFlagNonFinite = 2u;
constexpr uint32_t kFlagFallback = 4u;   // a mixed-form product ran in FP64 (no certified plan)
constexpr uint32_t kFlagCountRange = 8u; // a pair count exceeded INT32_MAX
constexpr uint32_t kNeedUncertified = 255u;  // a cell the certificate cannot bound
constexpr size_t kAlign = 256;

inline size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// Launch records of the matrix-core product kernels (tcu_trace_launches):
// the calling thread's buffer, or none.  A TraceScope around one launch
// records the begin event before it and the end event after it, on the
// launch's stream.
struct LaunchTrace {
    tcu_launch_record *rec = nullptr;
    int32_t cap = 0;
    int32_t *count = nullptr;
};
LaunchTrace &launch_trace();

class TraceScope {
  public:
    TraceScope(int kernel, int m, int n, int k, int planes, double ops, hipStream_t s) : s_(s) {
        LaunchTrace &t = launch_trace();
        if (t.count == nullptr) return;
        const int32_t i = (*t.count)++;
        if (t.rec == nullptr || i >= t.cap) return;
        r_ = &t.rec[i];
        r_->kernel = kernel;
        r_->m = m;
        r_->n = n;
        r_->k = k;
        r_->planes = planes;
        r_->ops = ops;
        (void)hipEventRecord(r_->begin, s_);
    }
    ~TraceScope() {
        if (r_ != nullptr) (void)hipEventRecord(r_->end, s_);
    }
    TraceScope(const TraceScope &) = delete;
    TraceScope &operator=(const TraceScope &) = delete;

  private:
    tcu_launch_record *r_ = nullptr;
    hipStream_t s_;
};

// api.hip: the body of tcu_join_agg_fwd on a given workspace, and the
// workspace bytes it needs (0 for invalid shapes or precision).
tcu_status join_agg_fwd_ws(const tcu_relation *A, const tcu_relation *B, int32_t M, int32_t K,
                           int32_t N, tcu_precision p, double tol, double *C, int32_t *count,
                           void *ws, size_t ws_bytes, hipStream_t stream);
size_t join_agg_fwd_ws_bytes(const tcu_relation *A, const tcu_relation *B, int32_t M,
                             int32_t K, int32_t N, tcu_precision p, bool with_count);

// encode.hip
hipError_t launch_zero_f64(double *p, size_t n, hipStream_t s);
hipError_t launch_clear_status(StatusBlock *st, hipStream_t s, uint32_t slices = 0);
// status words of a mixed-form product: cleared before its certificate, and
// the plan it ran with (slices = 0 and the fallback flag: FP64; exceptions:
// cells the residue form recomputed alone)
hipError_t launch_reset_plan(StatusBlock *st, hipStream_t s);
hipError_t launch_set_plan(StatusBlock *st, uint32_t slices, uint32_t bits, uint32_t need,
                           bool fallback, hipStream_t s, uint32_t exceptions = 0);
hipError_t launch_encode(const tcu_relation &R, int transpose, int rows, int cols, double *out,
                         StatusBlock *st, int which, hipStream_t s);
// The whole encoding of one relation: out zeroed, then the records placed.
// Matrices of at least 1 GiB go window by window when `scratch` holds
// encode_scratch_bytes(R, rows, cols) bytes (256-byte aligned); otherwise
// (scratch NULL or too small, or a smaller matrix) one zero pass and one
// scatter.  Same result either way.
size_t encode_scratch_bytes(const tcu_relation &R, int rows, int cols);
hipError_t launch_encode_zeroed(const tcu_relation &R, int transpose, int rows, int cols,
                                double *out, StatusBlock *st, int which, void *scratch,
                                size_t scratch_bytes, hipStream_t s);
// dst[i] = src[row_i, col_i] for the records whose row lies in [r0, r1)
// (r1 < 0: all rows); the launch with r0 = 0 also writes 0 for records
// outside the matrix.
hipError_t launch_gather(const tcu_relation &R, int transpose, int rows, int cols,
                         const double *src, double *dst, hipStream_t s, int r0 = 0,
                         int r1 = -1);
// counts held in FP64 to int32; values above INT32_MAX are stored as
// INT32_MAX and set kFlagCountRange
hipError_t launch_f64_to_i32(const double *src, int32_t *dst, size_t n, StatusBlock *st,
                             hipStream_t s);

// split.hip: per-line max |z| (axis 0: rows, 1: columns) into maxbits (bit
// patterns of non-negative doubles), the sums of |z| (sums may be NULL), and
// the digit slices of Z.  Row sums land in sums[row]; column sums in
// col_sum_parts(rows) partial sums sums[part * cols + col], which
// line_abs_sum adds in order (sums then holds kColParts * cols doubles).
constexpr int kColParts = 32;
int col_sum_chunk(int rows);
int col_sum_parts(int rows);
hipError_t launch_line_max(const double *Z, int rows, int cols, int64_t ld, int axis,
                           unsigned long long *maxbits, double *sums, StatusBlock *st,
                           hipStream_t s);
// Lines are rows (axis 0, lines_pad >= rows, len_pad >= cols) or columns
// (axis 1, lines_pad >= cols, len_pad >= rows); lines_pad % 128 == 0,
// len_pad % 64 == 0.  Layout: slices[p][t / KSTEP][(t % KSTEP) / HALF][line][t % HALF]
// with KSTEP = 32 / sizeof(digit), HALF = KSTEP / 2.
hipError_t launch_split(const double *Z, int rows, int cols, int64_t ld, int axis,
                        const unsigned long long *maxbits, int S, int digit_bf16, void *out,
                        int lines_pad, int len_pad, int *exps, hipStream_t s);

// gemm_split.hip: C (m x n, ldc) = 2^(ex[g] + ey[h]) * sum over digit pairs
// (p, q) with p + q <= S + 1 of 2^(-7(p+q)) X_p Y_q, digits from launch_split
// (X lines = rows of op(A), Y lines = columns of op(B), both of length k).
hipError_t launch_gemm_split(int m, int n, int k, int S, int digit_bf16, const void *xs,
                             int x_lines_pad, const void *ys, int y_lines_pad, int len_pad,
                             const int *ex, const int *ey, double *C, int64_t ldc,
                             hipStream_t s);
// k-steps per exact integer chunk of the split GEMM (host side of its plan).
int split_chunk_steps(int S, int digit_bf16);

// gemm_f64.hip: C (m x n, ldc) = op(A) * op(B), FP64 matrix cores; with
// accumulate != 0, C += op(A) * op(B).
hipError_t launch_gemm_f64(int trans_a, int trans_b, int m, int n, int k, const double *A,
                           int64_t lda, const double *B, int64_t ldb, double *C, int64_t ldc,
                           hipStream_t s, int accumulate = 0);
// The same product with the contraction split into chunks whose partial
// products go to `part` and are summed in chunk order, when the output has
// too few tiles to fill the chip (gemm_f64_split_bytes > 0); otherwise (or
// part == NULL) launch_gemm_f64.  part: gemm_f64_split_bytes(m, n, k) bytes.
size_t gemm_f64_split_bytes(int m, int n, int k);
hipError_t launch_gemm_f64_split(int trans_a, int trans_b, int m, int n, int k, const double *A,
                                 int64_t lda, const double *B, int64_t ldb, double *C,
                                 int64_t ldc, double *part, hipStream_t s);
// Rows m1 (a multiple of the tile height, 0 < m1 < m) at which an m x n FP64
// product can be cut into two launches that together take no more rounds of
// concurrently resident workgroups than one launch; 0 when no such cut exists
// or the product fills at most one round.
int gemm_f64_row_cut(int m, int n);

// dict.hip: dictionary encoding (ranks in the sorted union of two columns).
size_t dict_workspace_bytes(int64_t n);
hipError_t run_dict_encode(const long long *a, int64_t n_a, const long long *b, int64_t n_b,
                           int *codes_a, int *codes_b, long long *dict, int64_t *k_out,
                           void *ws, hipStream_t s);

// reassoc.hip: Q3/Q4 in re-associated form (histogram of A by key, then one
// pass over B grouped by B's group column).
size_t row_workspace_bytes(int K, int N);
hipError_t run_join_agg_row(const tcu_relation &A, const tcu_relation &B, int K, int N,
                            double *c, unsigned long long *count, void *ws, hipStream_t s);

// bsr.hip: the join-aggregate on 16 x 16 block-sparse encodings (tiles
// without records skipped); C dense M x N FP64.
size_t bsr_workspace_bytes(int64_t na, int64_t nb, int M, int K, int N);
hipError_t run_join_agg_bsr(const tcu_relation &A, const tcu_relation &B, int M, int K, int N,
                            double *C, void *ws, hipStream_t s);

// compact.hip: nonzero() of a dense matrix in row-major order (three-pass
// stream compaction); *count receives the total (host synchronisation).
size_t nonzero_workspace_bytes(int64_t rows, int64_t cols);
hipError_t run_nonzero(const double *M, int64_t rows, int64_t cols, int64_t ld, int32_t *out_row,
                       int32_t *out_col, const int32_t *col_map, int32_t *out_key,
                       int64_t capacity, int64_t *count, void *ws, hipStream_t s);

// ooc.hip: C = A * B with A, B, C in host memory, streamed through a device
// buffer of 6 block^2 doubles (blocked, pipelined over three streams).
int64_t ooc_block(size_t dev_bytes);
hipError_t run_gemm_f64_host(int m, int n, int k, const double *A, int64_t lda, const double *B,
                             int64_t ldb, double *C, int64_t ldc, void *dev_buf,
                             size_t dev_bytes, int64_t block, hipStream_t s);

// peak.hip: register-only matrix-core loops (kind 0: FP64 16x16x4; 1: int8
// 32x32x32 on hashed random bytes; 2: int8 on near-constant bytes).
double mfma_peak_ops(int kind, int iters);
size_t mfma_peak_out_bytes();
hipError_t launch_mfma_peak(int kind, int iters, void *out, hipStream_t s);

// crt.hip: the CRT form.  Residues of each line's `bits`-bit truncation
// modulo the first L moduli, int8, in the slice layout with lines_pad a
// multiple of 256; the GEMM writes per-modulus residues of the product into
// res (L planes of crt_residue_plane(m, n) int8) and reconstructs C (m x n,
// ldc) from them.
// The certificate of a mixed-form product (crt.hip): magnitude planes of
// both operands (int8, the residue layout; lines_pad a multiple of 256,
// len_pad of crt_len_align()) with their lines' normalised sums of |z|, then
// one int8 GEMM whose epilogue folds every cell's need into need_bits
// (residue form: truncation width) or need_slices (digit forms: digits).
struct CertArgs {
    const double *sx, *sy;  // normalised sums of the lines of A and B (rounded up)
    double tcrt;            // residue form: tolerance left for the truncation
    double kterm;           // 2^14 K
    double tdig[TCU_MAX_SLICES + 1];  // digit forms: tolerance left, per digit count
    uint32_t *need_bits, *need_slices;
    // residue form: the need of every cell (bytes, the residue planes'
    // layout, crt_residue_plane(m, n)), and the largest need and smallest
    // nonzero need among the cells the certificate bounds; may be NULL
    uint8_t *need_plane;
    uint32_t *need_cert, *need_min;
};
hipError_t launch_mag_plane(const double *Z, int rows, int cols, int64_t ld, int axis,
                            const unsigned long long *maxbits, const double *sums, double *shat,
                            unsigned long long *umax, int8_t *out, int lines_pad, int len_pad,
                            hipStream_t s);
hipError_t launch_certify(int m, int n, int k, const int8_t *qa, int a_lines_pad,
                          const int8_t *qb, int b_lines_pad, int len_pad, const CertArgs &ca,
                          bool digits, hipStream_t s);
// The count path (crt.hip): the 0/1 plane of a relation with unique cells
// (line = group, position = key; the rest zero), then one int8 product with
// exact int32 sums written to count (m x n, leading dimension ldc).
hipError_t launch_count_planes(const tcu_relation &R, int lines, int len, int8_t *plane,
                               int lines_pad, int len_pad, hipStream_t s);
hipError_t launch_count_product(int m, int n, int k, const int8_t *qa, int a_lines_pad,
                                const int8_t *qb, int b_lines_pad, int len_pad, int32_t *count,
                                int64_t ldc, hipStream_t s);
double crt_modulus_bits(int L);
int crt_max_moduli();
int64_t crt_residue_plane(int64_t m, int64_t n);
int crt_len_align();  // the residue planes' length is a multiple of this
// columns of the int8 products' tiles for an output n wide: the right
// operand's planes hold a multiple of this many lines
int crt_tile_cols(int64_t n);
hipError_t launch_crt_split(const double *Z, int rows, int cols, int64_t ld, int axis,
                            const unsigned long long *maxbits, int L, int bits, int8_t *out,
                            int lines_pad, int len_pad, int *exps, hipStream_t s);
hipError_t launch_gemm_crt(int m, int n, int k, int L, int bits, const int8_t *xs, int x_lines_pad,
                           const int8_t *ys, int y_lines_pad, int len_pad, int8_t *res,
                           const int *ex, const int *ey, double *C, int64_t ldc, int accumulate,
                           hipStream_t s);
// Exceptions of the residue form (crt.hip).  Thresholds t[0] > t[1] > ...
// (unused ones 255) cut the cells of the need plane into segments: a cell
// belongs to the first j with need > t[j], and cells at or below every
// threshold to none.  The scan lists segment j's cells, {row, col, need, 0},
// at list + j * cap, and counts them in st->exc_seg[j]; a count above cap
// means the segment overflowed (its list is incomplete).  The fix-up
// recomputes every cell of segments 0 .. last as a compensated FP64 dot
// product of its row of op(A) and column of op(B) and stores it into C.  An
// operand with axis 0 is stored line by line (A: m x k; B: n x k), with
// axis 1 position by position (A: k x m; B: k x n), leading dimension ld.
struct ExcThresholds {
    uint32_t t[4];
};
hipError_t launch_need_scan(const uint8_t *plane, int m, int n, ExcThresholds thr, int4 *list,
                            uint32_t cap, StatusBlock *st, hipStream_t s);
hipError_t launch_exception_fixup(const int4 *list, const StatusBlock *st, uint32_t cap, int last,
                                  int k, const double *Za, int64_t lda, int axa, const double *Zb,
                                  int64_t ldb, int axb, double *C, int64_t ldc, hipStream_t s);

}  // namespace tcu
