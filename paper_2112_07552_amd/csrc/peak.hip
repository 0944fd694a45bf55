// peak.hip -- register-only matrix-core loops that measure the rates the
// roofline is compared with beside the published peaks: under sustained
// matrix load the chip does not hold the clock the published figures
// assume, and the int8 rate depends on the operand bits (uniformly random
// bytes, such as residues, draw more power than near-constant ones).
//
// Each wave keeps eight independent accumulators and issues nothing but
// matrix instructions in its loop; 2048 workgroups of 256 threads cover
// every SIMD many times over.  The instructions are written as inline
// assembly on accumulators pinned in VGPRs: through the builtins the
// compiler copies every accumulator between VGPRs and AGPRs in each round,
// and the copies, not the matrix cores, then set the rate.  The s_nop
// blocks cover the VALU-write -> matrix-read hazard on entry and the
// matrix-write -> VALU-read hazard on exit (at most 18 wait states).
#include "internal.h"

namespace tcu {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef int i4 __attribute__((ext_vector_type(4)));
typedef int i16v __attribute__((ext_vector_type(16)));

constexpr int kPeakThreads = 256;
constexpr int kPeakBlocks = 2048;
constexpr int kAcc = 8;
// the nop blocks name every accumulator (and, on entry, the operands),
// which keeps them between the last VALU write of those registers and the
// first matrix read, and between the last matrix write and the first VALU read
#define ACC_OPERANDS : "+v"(acc[0]), "+v"(acc[1]), "+v"(acc[2]), "+v"(acc[3]), "+v"(acc[4]), "+v"(acc[5]), "+v"(acc[6]), "+v"(acc[7])

__device__ inline unsigned mix32(unsigned x) {
    x ^= x >> 16;
    x *= 0x7feb352du;
    x ^= x >> 15;
    x *= 0x846ca68bu;
    x ^= x >> 16;
    return x;
}

__global__ void __launch_bounds__(kPeakThreads) fp64_peak_kernel(int iters, double *out) {
    d4 acc[kAcc];
#pragma unroll
    for (int j = 0; j < kAcc; ++j) acc[j] = d4{0.0, 0.0, 0.0, 0.0};
    double a = 1.0 + 1e-3 * threadIdx.x, b = 0.5 + 1e-3 * blockIdx.x;
    asm volatile("s_nop 7" ACC_OPERANDS, "+v"(a), "+v"(b));
    for (int it = 0; it < iters; ++it)
#pragma unroll
        for (int j = 0; j < kAcc; ++j)
            asm volatile("v_mfma_f64_16x16x4_f64 %0, %1, %2, %0" : "+v"(acc[j]) : "v"(a), "v"(b));
    asm volatile("s_nop 7\n\ts_nop 7\n\ts_nop 7" ACC_OPERANDS);
    double s = 0.0;
#pragma unroll
    for (int j = 0; j < kAcc; ++j) s += acc[j][0] + acc[j][1] + acc[j][2] + acc[j][3];
    out[(size_t)blockIdx.x * kPeakThreads + threadIdx.x] = s;
}

// random != 0: operands are hashed bytes (uniform over all 256 values);
// otherwise small near-constant values
__global__ void __launch_bounds__(kPeakThreads) int8_peak_kernel(int iters, int random, int *out) {
    i16v acc[kAcc];
#pragma unroll
    for (int j = 0; j < kAcc; ++j) acc[j] = i16v{};
    const unsigned g = blockIdx.x * kPeakThreads + threadIdx.x;
    i4 a, b;
    if (random) {
        a = i4{(int)mix32(4 * g), (int)mix32(4 * g + 1), (int)mix32(4 * g + 2), (int)mix32(4 * g + 3)};
        b = i4{(int)mix32(~(4 * g)), (int)mix32(~(4 * g + 1)), (int)mix32(~(4 * g + 2)),
               (int)mix32(~(4 * g + 3))};
    } else {
        a = i4{(int)(threadIdx.x & 3), 1, 2, 3};
        b = i4{1, 3, 2, 1};
    }
    asm volatile("s_nop 7" ACC_OPERANDS, "+v"(a), "+v"(b));
    for (int it = 0; it < iters; ++it)
#pragma unroll
        for (int j = 0; j < kAcc; ++j)
            asm volatile("v_mfma_i32_32x32x32_i8 %0, %1, %2, %0" : "+v"(acc[j]) : "v"(a), "v"(b));
    asm volatile("s_nop 7\n\ts_nop 7\n\ts_nop 7" ACC_OPERANDS);
    int s = 0;
#pragma unroll
    for (int j = 0; j < kAcc; ++j)
#pragma unroll
        for (int i = 0; i < 16; ++i) s ^= acc[j][i];
    out[g] = s;
}

}  // namespace

double mfma_peak_ops(int kind, int iters) {
    const double mfmas = (double)kPeakBlocks * (kPeakThreads / 64) * iters * kAcc;
    return mfmas * (kind == 0 ? 2.0 * 16 * 16 * 4 : 2.0 * 32 * 32 * 32);
}

size_t mfma_peak_out_bytes() { return (size_t)kPeakBlocks * kPeakThreads * sizeof(double); }

hipError_t launch_mfma_peak(int kind, int iters, void *out, hipStream_t s) {
    if (kind == 0)
        fp64_peak_kernel<<<kPeakBlocks, kPeakThreads, 0, s>>>(iters, static_cast<double *>(out));
    else
        int8_peak_kernel<<<kPeakBlocks, kPeakThreads, 0, s>>>(iters, kind == 1,
                                                              static_cast<int *>(out));
    return hipGetLastError();
}

}  // namespace tcu
