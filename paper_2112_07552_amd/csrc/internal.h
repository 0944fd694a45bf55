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
    uint32_t flags;                 // bit 0: out-of-range record, bit 1: non-finite
    uint32_t slices;                // mixed form: slice count used
    unsigned long long skipped_a;   // records of A skipped
    unsigned long long skipped_b;   // records of B skipped
    int32_t exp_lo, exp_hi;         // mixed form: exponent range seen by the stats pass
    uint32_t pad[56];
};
static_assert(sizeof(StatusBlock) == 256, "status block must be 256 bytes");

constexpr uint32_t kFlagKeyRange = 1u;
constexpr uint32_t kFlagNonFinite = 2u;
constexpr size_t kAlign = 256;

inline size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// api.hip: the body of tcu_join_agg_fwd on a given workspace, and the
// workspace bytes it needs (0 for invalid shapes or precision).
tcu_status join_agg_fwd_ws(const tcu_relation *A, const tcu_relation *B, int32_t M, int32_t K,
                           int32_t N, tcu_precision p, double tol, double *C, int32_t *count,
                           void *ws, size_t ws_bytes, hipStream_t stream);
size_t join_agg_fwd_ws_bytes(int32_t M, int32_t K, int32_t N, tcu_precision p);

// encode.hip
hipError_t launch_zero_f64(double *p, size_t n, hipStream_t s);
hipError_t launch_clear_status(StatusBlock *st, hipStream_t s, uint32_t slices = 0);
hipError_t launch_encode(const tcu_relation &R, int transpose, int rows, int cols, double *out,
                         StatusBlock *st, int which, hipStream_t s);
// dst[i] = src[row_i, col_i] for the records whose row lies in [r0, r1)
// (r1 < 0: all rows); the launch with r0 = 0 also writes 0 for records
// outside the matrix.
hipError_t launch_gather(const tcu_relation &R, int transpose, int rows, int cols,
                         const double *src, double *dst, hipStream_t s, int r0 = 0,
                         int r1 = -1);
hipError_t launch_f64_to_i32(const double *src, int32_t *dst, size_t n, hipStream_t s);

// split.hip: per-line max |z| (axis 0: rows, 1: columns) into maxbits (bit
// patterns of non-negative doubles), and the digit slices of Z.
hipError_t launch_line_max(const double *Z, int rows, int cols, int64_t ld, int axis,
                           unsigned long long *maxbits, StatusBlock *st, hipStream_t s);
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
double crt_modulus_bits(int L);
int crt_max_moduli();
int64_t crt_residue_plane(int64_t m, int64_t n);
int crt_len_align();  // the residue planes' length is a multiple of this
hipError_t launch_crt_split(const double *Z, int rows, int cols, int64_t ld, int axis,
                            const unsigned long long *maxbits, int L, int bits, int8_t *out,
                            int lines_pad, int len_pad, int *exps, hipStream_t s);
hipError_t launch_gemm_crt(int m, int n, int k, int L, int bits, const int8_t *xs, int x_lines_pad,
                           const int8_t *ys, int y_lines_pad, int len_pad, int8_t *res,
                           const int *ex, const int *ey, double *C, int64_t ldc, int accumulate,
                           hipStream_t s);

}  // namespace tcu
