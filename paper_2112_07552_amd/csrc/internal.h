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

// encode.hip
hipError_t launch_zero_f64(double *p, size_t n, hipStream_t s);
hipError_t launch_clear_status(StatusBlock *st, hipStream_t s);
hipError_t launch_encode(const tcu_relation &R, int transpose, int rows, int cols, double *out,
                         StatusBlock *st, int which, hipStream_t s);
hipError_t launch_gather(const tcu_relation &R, int transpose, int rows, int cols,
                         const double *src, double *dst, hipStream_t s);
hipError_t launch_f64_to_i32(const double *src, int32_t *dst, size_t n, hipStream_t s);

// gemm_f64.hip: C (m x n, ldc) = op(A) * op(B), FP64 matrix cores.
hipError_t launch_gemm_f64(int trans_a, int trans_b, int m, int n, int k, const double *A,
                           int64_t lda, const double *B, int64_t ldb, double *C, int64_t ldc,
                           hipStream_t s);

}  // namespace tcu
