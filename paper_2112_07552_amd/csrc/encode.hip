// encode.hip -- step a1 (encoding, Sections 3.1 and 3.3 of TCUDB) and the
// record gathers of the adjoint.
//
// The encoding places every record's value at its (group, key) cell of a
// dense row-major matrix; duplicate cells add up.  It is a scatter bound by
// random-access throughput: per record it reads 4 + 4 + sizeof(val) bytes
// and performs one 8-byte FP64 atomic add (no return) into the matrix,
// which the zero pass wrote beforehand, or one plain store when the caller
// declares the cells unique.  Unique coordinates (the measured workload)
// give the record values bit for bit, since 0 + v == v.
#include "internal.h"

namespace tcu {
namespace {

constexpr int kThreads = 256;

__global__ void __launch_bounds__(kThreads) zero_f64_kernel(double *__restrict__ p, size_t n,
                                                            int vec) {
    const size_t stride = (size_t)gridDim.x * kThreads;
    const size_t t0 = (size_t)blockIdx.x * kThreads + threadIdx.x;
    if (vec) {
        // p is 16-byte aligned: 16-byte stores over the even prefix, then the odd tail
        const size_t n2 = n / 2;
        double2 *p2 = reinterpret_cast<double2 *>(p);
        for (size_t i = t0; i < n2; i += stride) p2[i] = make_double2(0.0, 0.0);
        if (t0 == 0 && (n & 1)) p[n - 1] = 0.0;
    } else {
        for (size_t i = t0; i < n; i += stride) p[i] = 0.0;
    }
}

__global__ void zero_status_kernel(StatusBlock *st, uint32_t slices) {
    uint32_t *w = reinterpret_cast<uint32_t *>(st);
    w[threadIdx.x] = threadIdx.x == 1 ? slices : 0u;  // 64 threads x 4 bytes; word 1 = slices
}

// The plan words of the status block before a mixed-form product's
// certificate: needs and normalised-sum maxima to zero.
__global__ void reset_plan_kernel(StatusBlock *st) {
    st->need_bits = 0;
    st->need_slices = 0;
    st->umax_a = 0;
    st->umax_b = 0;
}

// The plan a mixed-form product ran with (slices = 0: FP64 fallback).
__global__ void set_plan_kernel(StatusBlock *st, uint32_t slices, uint32_t bits, uint32_t need,
                                int fallback) {
    st->slices = slices;
    st->bits = bits;
    st->need = need;
    if (fallback) st->flags |= kFlagFallback;
}

// Counts this wave's invalid records and adds them to the status block once
// (st == nullptr: a repeated pass whose skips were already counted).
__device__ inline void report_skips(bool bad, StatusBlock *st, int which) {
    const unsigned long long mask = __ballot(bad);
    if (st != nullptr && mask != 0ull && (threadIdx.x & 63) == 0) {
        atomicOr(&st->flags, kFlagKeyRange);
        atomicAdd(which == 0 ? &st->skipped_a : &st->skipped_b,
                  (unsigned long long)__popcll(mask));
    }
}

// UNIQUE: the caller promised unique (group, key) cells, so a plain store
// replaces the atomic add (random 8-byte stores run about 3x faster than
// device-scope FP64 atomics, which fetch the whole line first).
template <typename T, bool UNIQUE>
__global__ void __launch_bounds__(kThreads)
encode_kernel(int64_t n, const int32_t *__restrict__ grp, const int32_t *__restrict__ key,
              const T *__restrict__ val, int transpose, int rows, int cols,
              double *__restrict__ out, StatusBlock *st, int which) {
    const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    bool bad = false;
    if (i < n) {
        const int g = grp[i], k = key[i];
        const int r = transpose ? k : g;
        const int c = transpose ? g : k;
        if ((unsigned)r < (unsigned)rows && (unsigned)c < (unsigned)cols) {
            const double v = val ? (double)val[i] : 1.0;
            double *dst = out + (size_t)r * (size_t)cols + c;
            if (UNIQUE) *dst = v;
            else unsafeAtomicAdd(dst, v);
        } else {
            bad = true;
        }
    }
    report_skips(bad, st, which);
}

__global__ void __launch_bounds__(kThreads)
gather_kernel(int64_t n, const int32_t *__restrict__ grp, const int32_t *__restrict__ key,
              int transpose, int rows, int cols, int r0, int r1, const double *__restrict__ src,
              double *__restrict__ dst) {
    const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (i >= n) return;
    const int g = grp[i], k = key[i];
    const int r = transpose ? k : g;
    const int c = transpose ? g : k;
    const bool valid = (unsigned)r < (unsigned)rows && (unsigned)c < (unsigned)cols;
    // a launch covers the records whose row lies in [r0, r1); the one that
    // starts at row 0 also writes the zeros of records outside the matrix
    if (valid ? (r < r0 || r >= r1) : r0 != 0) return;
    dst[i] = valid ? src[(size_t)r * (size_t)cols + c] : 0.0;
}

__global__ void __launch_bounds__(kThreads)
f64_to_i32_kernel(const double *__restrict__ src, int32_t *__restrict__ dst, size_t n,
                  StatusBlock *st) {
    const size_t stride = (size_t)gridDim.x * kThreads;
    bool over = false;
    for (size_t i = (size_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += stride) {
        const double v = src[i];
        const bool big = !(v <= 2147483647.0);
        over |= big;
        dst[i] = big ? 2147483647 : (int32_t)v;
    }
    if (__ballot(over) != 0ull && (threadIdx.x & 63) == 0) atomicOr(&st->flags, kFlagCountRange);
}

inline unsigned grid_for(int64_t n) { return (unsigned)((n + kThreads - 1) / kThreads); }

inline unsigned capped_grid(size_t n) {
    size_t g = (n + kThreads - 1) / kThreads;
    const size_t cap = 256 * 64;  // 64 blocks per CU is plenty for a stream
    return (unsigned)(g < 1 ? 1 : (g > cap ? cap : g));
}

}  // namespace

hipError_t launch_zero_f64(double *p, size_t n, hipStream_t s) {
    if (n == 0) return hipSuccess;
    const int vec = ((uintptr_t)p & 15) == 0;
    zero_f64_kernel<<<capped_grid(vec ? n / 2 + 1 : n), kThreads, 0, s>>>(p, n, vec);
    return hipGetLastError();
}

hipError_t launch_clear_status(StatusBlock *st, hipStream_t s, uint32_t slices) {
    zero_status_kernel<<<1, 64, 0, s>>>(st, slices);
    return hipGetLastError();
}

hipError_t launch_reset_plan(StatusBlock *st, hipStream_t s) {
    reset_plan_kernel<<<1, 1, 0, s>>>(st);
    return hipGetLastError();
}

hipError_t launch_set_plan(StatusBlock *st, uint32_t slices, uint32_t bits, uint32_t need,
                           bool fallback, hipStream_t s) {
    set_plan_kernel<<<1, 1, 0, s>>>(st, slices, bits, need, fallback ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_encode(const tcu_relation &R, int transpose, int rows, int cols, double *out,
                         StatusBlock *st, int which, hipStream_t s) {
    if (R.n == 0) return hipSuccess;
    const unsigned grid = grid_for(R.n);
    // algorithmic bytes: the record (group, key, value) in, one 8-byte cell out
    const double vbytes = R.val == nullptr ? 0.0 : (R.dtype == TCU_F32 ? 4.0 : 8.0);
    TraceScope ts(TCU_KERNEL_ENCODE, rows, cols, 0, 1, (double)R.n * (16.0 + vbytes), s);
    const bool unique = (R.flags & TCU_REL_UNIQUE_CELLS) != 0;
    const float *vf = static_cast<const float *>(R.val);
    const double *vd = static_cast<const double *>(R.val);
    if (R.dtype == TCU_F32) {
        if (unique)
            encode_kernel<float, true><<<grid, kThreads, 0, s>>>(R.n, R.group, R.key, vf,
                                                                 transpose, rows, cols, out, st,
                                                                 which);
        else
            encode_kernel<float, false><<<grid, kThreads, 0, s>>>(R.n, R.group, R.key, vf,
                                                                  transpose, rows, cols, out, st,
                                                                  which);
    } else {
        if (unique)
            encode_kernel<double, true><<<grid, kThreads, 0, s>>>(R.n, R.group, R.key, vd,
                                                                  transpose, rows, cols, out, st,
                                                                  which);
        else
            encode_kernel<double, false><<<grid, kThreads, 0, s>>>(R.n, R.group, R.key, vd,
                                                                   transpose, rows, cols, out,
                                                                   st, which);
    }
    return hipGetLastError();
}

hipError_t launch_gather(const tcu_relation &R, int transpose, int rows, int cols,
                         const double *src, double *dst, hipStream_t s, int r0, int r1) {
    if (R.n == 0) return hipSuccess;
    if (r1 < 0) r1 = rows;
    // algorithmic bytes: group and key in, one 8-byte cell in, 8 bytes out
    TraceScope ts(TCU_KERNEL_GATHER, rows, cols, 0, 1, (double)R.n * 24.0, s);
    gather_kernel<<<grid_for(R.n), kThreads, 0, s>>>(R.n, R.group, R.key, transpose, rows, cols,
                                                     r0, r1, src, dst);
    return hipGetLastError();
}

hipError_t launch_f64_to_i32(const double *src, int32_t *dst, size_t n, StatusBlock *st,
                             hipStream_t s) {
    if (n == 0) return hipSuccess;
    f64_to_i32_kernel<<<capped_grid(n), kThreads, 0, s>>>(src, dst, n, st);
    return hipGetLastError();
}

}  // namespace tcu
